"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module generates inputs only: grid sizes, the node field kappa, right-hand
sides and random choices.  It holds none of the solver's arithmetic (no edge
weights, no stencil, no elimination), so the oracle and the HIP path can both
draw from it without sharing any part of the method.

Conventions (used by every caller):
  * The grid has n2 rows (the interface length) and n1 columns (the slab
    direction) of interior unknowns; the Dirichlet ring adds one node on each
    side.  Node (c, r) of the interior, 0 <= c < n1, 0 <= r < n2, sits at
    x = (c+1) h, y = (r+1) h with h = 1/(n2+1).
  * The coefficient field is stored on the nodes including the ring, shape
    (n1+2, n2+2), the row index r fastest: kappa[c+1, r+1] belongs to node
    (c, r).
  * Right-hand sides have shape (nrhs, n1, n2), r fastest.

The coefficient field is exp(g) with g a Gaussian random field with the
squared-exponential covariance k(d) = sigma^2 exp(-d^2 / (2 l^2)), l = 0.05,
sigma^2 = 1.  It is sampled exactly from the separable covariance
K = Kx (x) Ky: g = Fx Z Fy^T with F = V sqrt(max(lambda, 0)) from the
symmetric eigendecomposition of each 1-D covariance matrix (a Cholesky
factor does not exist: the 1-D matrices are numerically singular).
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field

import numpy as np

GRF_LENGTH = 0.05
GRF_VARIANCE = 1.0

# Seeds of the synthetic workloads.
SEED_KAPPA = 0
SEED_KAPPA_OBS = 1
SEED_RHS = 100
SEED_NOISE = 200
SEED_FD_NODES = 300
SEED_BATCH = 400
SEED_SKETCH = 500


def default_h(n2: int) -> float:
    """Grid spacing: n2 interior rows between y = 0 and y = 1."""
    return 1.0 / (n2 + 1)


@functools.lru_cache(maxsize=32)
def _grf_factor(npts: int, h: float, length: float) -> np.ndarray:
    x = np.arange(npts, dtype=np.float64) * h
    d = x[:, None] - x[None, :]
    k = np.exp(-(d * d) / (2.0 * length * length))
    lam, v = np.linalg.eigh(k)
    return np.ascontiguousarray(v * np.sqrt(np.maximum(lam, 0.0))[None, :])


def grf(n2: int, n1: int, seed: int, h: float | None = None,
        length: float = GRF_LENGTH, variance: float = GRF_VARIANCE) -> np.ndarray:
    """Gaussian random field on the (n1+2) x (n2+2) nodes (ring included)."""
    if h is None:
        h = default_h(n2)
    fx = _grf_factor(n1 + 2, float(h), float(length))
    fy = _grf_factor(n2 + 2, float(h), float(length))
    z = np.random.default_rng(seed).standard_normal((n1 + 2, n2 + 2))
    return np.sqrt(variance) * (fx @ z @ fy.T)


def kappa_lognormal(n2: int, n1: int, seed: int, h: float | None = None) -> np.ndarray:
    return np.exp(grf(n2, n1, seed, h))


def kappa_const(n2: int, n1: int, value: float = 1.0) -> np.ndarray:
    return np.full((n1 + 2, n2 + 2), float(value))


def rhs_uniform(n2: int, n1: int, nrhs: int, seed: int = SEED_RHS) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (nrhs, n1, n2))


def rhs_normal(n2: int, n1: int, nrhs: int, seed: int = SEED_RHS) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((nrhs, n1, n2))


@dataclass
class Workload:
    """One synthetic problem: grid, slab width, coefficient field and loads."""
    name: str
    n2: int
    n1: int
    b: int
    nrhs: int
    kappa_kind: str          # "const" or "lognormal"
    rhs_kind: str            # "uniform" or "normal"
    kappa_seed: int = SEED_KAPPA
    rhs_seed: int = SEED_RHS
    extra: dict = field(default_factory=dict)

    @property
    def h(self) -> float:
        return default_h(self.n2)

    @property
    def m(self) -> int:
        return self.n1 // (self.b + 1)

    @property
    def N(self) -> int:
        return self.n1 * self.n2

    def kappa(self) -> np.ndarray:
        if self.kappa_kind == "const":
            return kappa_const(self.n2, self.n1)
        return kappa_lognormal(self.n2, self.n1, self.kappa_seed, self.h)

    def rhs(self, nrhs: int | None = None) -> np.ndarray:
        k = self.nrhs if nrhs is None else nrhs
        if self.rhs_kind == "normal":
            return rhs_normal(self.n2, self.n1, k, self.rhs_seed)
        return rhs_uniform(self.n2, self.n1, k, self.rhs_seed)

    def shift(self) -> np.ndarray | None:
        """Helmholtz diagonal term for workloads with extra["ppw"], else None."""
        if "ppw" not in self.extra:
            return None
        return helmholtz_shift(self.n2, self.n1, self.extra["ppw"], self.h)


# The five synthetic workloads: Poisson 64x64 (b=7, 8 slabs); lognormal
# diffusion 1024x1024 (b=31); lognormal diffusion 2048 rows x 4096 columns
# (b=31, 128 slabs, 16 normal RHS); the 512x512 differentiation case (b=15);
# the batch of uneven problems is drawn by batch_problems().
POISSON_64 = Workload("poisson_64x64_b7", 64, 64, 7, 1, "const", "uniform")
DIFFUSION_1024 = Workload("diffusion_1024x1024_b31", 1024, 1024, 31, 1, "lognormal", "uniform")
DIFFUSION_2048x4096 = Workload("diffusion_2048x4096_b31", 2048, 4096, 31, 16, "lognormal", "normal")
ADJOINT_512 = Workload("adjoint_512x512_b15", 512, 512, 15, 1, "lognormal", "uniform")
# Helmholtz -Laplace u - k^2 u at 40 points per wavelength on 1024 x 1024 (25.6
# wavelengths across, 2018 eigenvalues below k^2): slabs of 16 columns are
# under half a wavelength, so only the reduced matrix is indefinite
HELMHOLTZ_1024 = Workload("helmholtz_1024x1024_b15_ppw40", 1024, 1024, 15, 1, "const", "uniform",
                          extra={"ppw": 40.0})
# 2048 x 2048 at 20 points per wavelength (102 wavelengths across): slabs of 32
# columns span 1.6 wavelengths, so the slab interiors are indefinite as well
HELMHOLTZ_2048 = Workload("helmholtz_2048x2048_b31_ppw20", 2048, 2048, 31, 1, "const", "uniform",
                          extra={"ppw": 20.0})


# The differentiation workload: 16 coefficient fields theta_i = log kappa_i on
# the 512x512 grid (GRF seeds 10..25), one shared uniform load, an observation
# made from a second field (seed SEED_KAPPA_OBS) plus 1% Gaussian noise, and
# central differences at 32 random interior nodes.
DIFF_THETA_SEEDS = tuple(range(10, 26))
DIFF_NOISE_LEVEL = 0.01


def noise_normal(n2: int, n1: int, nrhs: int, seed: int = SEED_NOISE) -> np.ndarray:
    """Standard normal samples of the shape of a right-hand side block."""
    return np.random.default_rng(seed).standard_normal((nrhs, n1, n2))


def helmholtz_shift(n2: int, n1: int, ppw: float, h: float | None = None) -> np.ndarray:
    """Diagonal term c = -k^2 of the constant-coefficient Helmholtz operator
    -Laplace u - k^2 u with k chosen for `ppw` grid points per wavelength
    (k h = 2 pi / ppw), on the (n1, n2) interior nodes."""
    if h is None:
        h = default_h(n2)
    k = 2.0 * np.pi / (ppw * h)
    return np.full((n1, n2), -k * k)


def bessel_field(n2: int, n1: int, k: float, h: float | None = None,
                 source=(-0.1, 0.5)) -> np.ndarray:
    """J0(k |x - source|) on the grid with its ring, in the layout of kappa:
    shape (n1+2, n2+2), entry [i, j] at x = (i h, j h) (column i, row j; the
    interior nodes are 1..n1 and 1..n2).  The exact solution of the
    constant-coefficient Helmholtz benchmark -Laplace u - k^2 u = 0 with
    Dirichlet data u = J0 on the boundary of the unit square."""
    from scipy.special import j0
    if h is None:
        h = default_h(n2)
    x1 = np.arange(n1 + 2)[:, None] * h
    x2 = np.arange(n2 + 2)[None, :] * h
    return j0(k * np.hypot(x1 - source[0], x2 - source[1]))


def gaussian_test_vectors(m: int, ncols: int, n2: int, seed: int = SEED_SKETCH) -> np.ndarray:
    """ncols standard normal interface vectors, shape (m, ncols, n2): block j
    of column k is interface j's part (the test vectors of a sketch of T)."""
    return np.random.default_rng(seed).standard_normal((m, ncols, n2))


def fd_nodes(n2: int, n1: int, count: int = 32, seed: int = SEED_FD_NODES) -> np.ndarray:
    """Distinct random interior nodes as (c, r) pairs, shape (count, 2)."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n1 * n2, size=count, replace=False)
    return np.stack([flat // n2, flat % n2], axis=1)


def batch_problems(count: int = 256, seed: int = SEED_BATCH) -> list[Workload]:
    """Uneven batch: n2 in {128,...,1024}, n1 in {128,...,2048}, b in {7,15,31}, 1-16 RHS.

    n1 is rounded down to a multiple of b+1 so that the slabs tile the grid.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n2 = int(rng.choice([128, 256, 512, 1024]))
        n1 = int(rng.choice([128, 256, 512, 1024, 2048]))
        b = int(rng.choice([7, 15, 31]))
        nrhs = int(rng.integers(1, 17))
        n1 = (n1 // (b + 1)) * (b + 1)
        out.append(Workload(f"batch_{i}", n2, n1, b, nrhs, "lognormal", "uniform",
                            kappa_seed=1000 + i, rhs_seed=2000 + i))
    return out
