"""FP64 CPU oracle of the SlabLU hot path.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The GPU library never calls it
and shares no code with it.

Plain, slow, obviously correct: each function follows one passage of Yesypenko
& Martinsson, "SlabLU: a two-level sparse direct solver for elliptic PDEs"
(arXiv 2211.07572), cited by section / equation / algorithm.  Arithmetic is
float64 throughout; LAPACK (through SciPy) supplies the banded and dense
factorizations, nothing is blocked, fused or reordered beyond the paper.

Problem (Sec. 1.1, eq. (Au=f)): -div(kappa grad u) = f on a uniform grid with
n2 rows and n1 columns of interior nodes, Dirichlet u = 0 on the ring around
them, spacing h.  Readings of the paper used here (where it is silent or
garbled):
  * 5-point conservative stencil (generalising eq. (discretization) to a
    variable coefficient): every edge e = (p, q) between neighbouring nodes
    carries w_e = (kappa_p + kappa_q) / (2 h^2); (A u)_p = sum_e w_e (u_p - u_q)
    with u_q = 0 on the ring.  This is the positive-definite sign.
  * Clustering (Sec. 2.2, Fig. 1): columns are grouped with period b+1; in each
    period the first b columns are the interior of a slab and the last column
    is an interface.  Slab s owns columns s(b+1) .. s(b+1)+b-1, interface j is
    column j(b+1)+b; there are m = n1/(b+1) slabs and m interfaces, the last
    interface borders the right Dirichlet side.  In the paper's numbering slab
    s is I_{2s} (slab 0 is an extra I_0 in front of I_1) and interface j is
    I_{2j+1}.
  * Inside a slab the unknowns are ordered grid row by grid row, the b columns
    fastest: local index r*b + k.  Interface j is ordered by row r.
  * Eq. (T31) and (T35) carry index slips; the forms used are
    T31 = A31 - A32 A22^-1 A21 and T35 = A35 - A34 A44^-1 A45, and the entry
    T_57 in the fourth row of eq. (dell3) is T_75.
  * Alg. 1's loop bounds skip S_3; the sweep used is S_0 = T_00,
    S_j = T_jj - T_{j,j-1} S_{j-1}^-1 T_{j-1,j} for j = 1 .. m-1.
  * Odd-even order (Remark in Sec. 4, concluding section; no formulas given):
    at every level the interfaces at even positions of the remaining list are
    eliminated together and those at odd positions are kept (see
    odd_even_build).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.linalg.lapack as lapack
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# Clustering of the nodes (Sec. 2.2, Fig. 1) -- integer maps.
# ---------------------------------------------------------------------------

def check_dims(n2: int, n1: int, b: int) -> int:
    if n2 < 1 or n1 < 2 or b < 1 or n1 % (b + 1) != 0:
        raise ValueError(f"bad grid: n2={n2} n1={n1} b={b} (need n1 % (b+1) == 0)")
    return n1 // (b + 1)


def index_maps(n2: int, n1: int, b: int) -> dict:
    """Index vectors I_1, I_2, ... of Sec. 2.2 as flat natural indices.

    Natural index of node (c, r) is c*n2 + r.  Returns
      col_kind[c]     1 for an interface column, 0 for a slab-interior column
      slab_of_col[c]  slab (or interface) number s = c // (b+1)
      local_of_col[c] position k = c % (b+1) inside the period
      perm_even       slab interiors concatenated, slab s at [s*n2*b, (s+1)*n2*b),
                      entry r*b + k -> natural index of node (s(b+1)+k, r)
      perm_odd        interfaces concatenated, interface j at [j*n2, (j+1)*n2),
                      entry r -> natural index of node (j(b+1)+b, r)
    """
    m = check_dims(n2, n1, b)
    period = b + 1
    c = np.arange(n1)
    col_kind = (c % period == b).astype(np.int32)
    slab_of_col = (c // period).astype(np.int32)
    local_of_col = (c % period).astype(np.int32)
    s = np.arange(m)[:, None, None]
    r = np.arange(n2)[None, :, None]
    k = np.arange(b)[None, None, :]
    perm_even = ((s * period + k) * n2 + r).reshape(-1).astype(np.int64)
    j = np.arange(m)[:, None]
    rr = np.arange(n2)[None, :]
    perm_odd = ((j * period + b) * n2 + rr).reshape(-1).astype(np.int64)
    return dict(col_kind=col_kind, slab_of_col=slab_of_col, local_of_col=local_of_col,
                perm_even=perm_even, perm_odd=perm_odd, m=m)


def slab_index(maps: dict, n2: int, b: int, s: int) -> np.ndarray:
    """I_{2s}: natural indices of slab s's interior, in local order r*b + k."""
    ne = n2 * b
    return maps["perm_even"][s * ne:(s + 1) * ne]


def interface_index(maps: dict, n2: int, j: int) -> np.ndarray:
    """I_{2j+1}: natural indices of interface j, in row order."""
    return maps["perm_odd"][j * n2:(j + 1) * n2]


# ---------------------------------------------------------------------------
# Discretization (Sec. 2.1, eq. (discretization)) -- edge weights and A.
# ---------------------------------------------------------------------------

def edge_weights(kappa: np.ndarray, n2: int, n1: int, h: float):
    """Edge weights w_e = (kappa_p + kappa_q) / (2 h^2).

    wh[c, r], c = 0..n1: edge between node (c-1, r) and (c, r) (columns -1 and
    n1 are the ring).  wv[c, r], r = 0..n2: edge between (c, r-1) and (c, r).
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    assert kappa.shape == (n1 + 2, n2 + 2)
    wh = 0.5 * (kappa[0:n1 + 1, 1:n2 + 1] + kappa[1:n1 + 2, 1:n2 + 1]) / (h * h)
    wv = 0.5 * (kappa[1:n1 + 1, 0:n2 + 1] + kappa[1:n1 + 1, 1:n2 + 2]) / (h * h)
    return wh, wv


def assemble_A(wh: np.ndarray, wv: np.ndarray, n2: int, n1: int) -> sp.csr_matrix:
    """Sparse A in natural order: (A u)_p = sum over edges w_e (u_p - u_q)."""
    N = n1 * n2
    c, r = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    p = (c * n2 + r).reshape(-1)
    diag = (wh[:-1, :] + wh[1:, :] + wv[:, :-1] + wv[:, 1:]).reshape(-1)
    rows = [p]
    cols = [p]
    vals = [diag]
    # horizontal neighbours: (c, r) -- (c+1, r), weight wh[c+1, r]
    hc, hr = np.meshgrid(np.arange(n1 - 1), np.arange(n2), indexing="ij")
    a = (hc * n2 + hr).reshape(-1)
    bb = a + n2
    w = wh[1:n1, :].reshape(-1)
    rows += [a, bb]
    cols += [bb, a]
    vals += [-w, -w]
    # vertical neighbours: (c, r) -- (c, r+1), weight wv[c, r+1]
    vc, vr = np.meshgrid(np.arange(n1), np.arange(n2 - 1), indexing="ij")
    a = (vc * n2 + vr).reshape(-1)
    bb = a + 1
    w = wv[:, 1:n2].reshape(-1)
    rows += [a, bb]
    cols += [bb, a]
    vals += [-w, -w]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


@dataclass
class Problem:
    n2: int
    n1: int
    b: int
    h: float
    kappa: np.ndarray
    maps: dict
    wh: np.ndarray
    wv: np.ndarray
    A: sp.csr_matrix

    @property
    def m(self) -> int:
        return self.maps["m"]

    @property
    def N(self) -> int:
        return self.n1 * self.n2

    def I_e(self, s: int) -> np.ndarray:
        return slab_index(self.maps, self.n2, self.b, s)

    def I_o(self, j: int) -> np.ndarray:
        return interface_index(self.maps, self.n2, j)

    def block(self, I, J) -> sp.csr_matrix:
        """A_{IJ} = A[I, J] (eq. (dell1) blocks)."""
        return self.A[I][:, J]


def make_problem(kappa, n2: int, n1: int, b: int, h: float | None = None,
                 shift: np.ndarray | None = None) -> Problem:
    """shift: optional diagonal term c on the interior nodes, shape (n1, n2):
    (A u)_p gains c_p u_p.  The Helmholtz operator of eq. (var_helm),
    -Laplace u - k^2 b(x) u (the paper calls the wavenumber kappa), is kappa = 1
    with c = -k^2 b(x); every factorization here pivots (banded and dense
    LAPACK LU), so indefinite shifts are handled."""
    if h is None:
        h = 1.0 / (n2 + 1)
    maps = index_maps(n2, n1, b)
    wh, wv = edge_weights(kappa, n2, n1, h)
    A = assemble_A(wh, wv, n2, n1)
    if shift is not None:
        c = np.asarray(shift, dtype=np.float64)
        assert c.shape == (n1, n2)
        A = (A + sp.diags(c.reshape(-1))).tocsr()
    return Problem(n2, n1, b, float(h), np.asarray(kappa, dtype=np.float64), maps, wh, wv, A)


def apply_A(prob: Problem, u: np.ndarray) -> np.ndarray:
    """A u for u of shape (nrhs, n1, n2) (or (n1, n2))."""
    flat = u.reshape(-1, prob.N)
    out = (prob.A @ flat.T).T
    return out.reshape(u.shape)


def dirichlet_load(prob: Problem, g: np.ndarray) -> np.ndarray:
    """Load of Dirichlet data (eq. (bvp): u = g on the boundary) on the
    right-hand side of eq. (Au=f): an edge e from interior node p to a ring
    node q carries w_e (u_p - g_q), so w_e g_q moves to f_p.  g has the layout
    of kappa, shape (n1+2, n2+2) or (nrhs, n1+2, n2+2); only its ring is read.
    Returns the load alone, shape (nrhs, n1, n2) (or (n1, n2))."""
    n1, n2 = prob.n1, prob.n2
    g3 = np.asarray(g, dtype=np.float64).reshape(-1, n1 + 2, n2 + 2)
    f = np.zeros((g3.shape[0], n1, n2))
    f[:, 0, :] += prob.wh[0, :] * g3[:, 0, 1:n2 + 1]              # left ring column
    f[:, n1 - 1, :] += prob.wh[n1, :] * g3[:, n1 + 1, 1:n2 + 1]   # right ring column
    f[:, :, 0] += prob.wv[:, 0] * g3[:, 1:n1 + 1, 0]              # ring row below
    f[:, :, n2 - 1] += prob.wv[:, n2] * g3[:, 1:n1 + 1, n2 + 1]   # ring row above
    return f if np.ndim(g) == 3 else f[0]


def relres(prob: Problem, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """relerr_res = ||A u - f||_2 / ||f||_2 per right-hand side (Sec. 5.1)."""
    r = apply_A(prob, u) - f
    r = r.reshape(-1, prob.N)
    f2 = f.reshape(-1, prob.N)
    return np.linalg.norm(r, axis=1) / np.linalg.norm(f2, axis=1)


# ---------------------------------------------------------------------------
# Stage one (Sec. 3.1): slab factorizations, Schur complements, reduced RHS.
# ---------------------------------------------------------------------------

def _to_lapack_band(M: sp.spmatrix, bw: int) -> np.ndarray:
    """Banded (sparse) matrix -> LAPACK general band storage with room for fill.

    Row (2*bw + i - j) of the result holds a_ij, as dgbtrf expects for kl = ku = bw.
    """
    n = M.shape[0]
    ab = np.zeros((3 * bw + 1, n))
    for d in range(-bw, bw + 1):
        diag = M.diagonal(d)
        if d >= 0:
            ab[2 * bw - d, d:] = diag
        else:
            ab[2 * bw - d, :n + d] = diag
    return ab


class SlabFactor:
    """Factorization of one slab interior A_{2s,2s} (Alg. 3, first loop).

    A_{2s,2s} is banded with half-bandwidth b in the local ordering; it is
    factored by LAPACK's banded LU (dgbtrf) and applied by dgbtrs.
    """

    def __init__(self, Aee: sp.spmatrix, b: int):
        Aee = sp.csr_matrix(Aee)
        self.n = Aee.shape[0]
        self.b = b
        outside = sp.triu(Aee, b + 1).nnz + sp.tril(Aee, -(b + 1)).nnz
        assert outside == 0, "slab block is not banded with half-bandwidth b"
        lu, piv, info = lapack.dgbtrf(_to_lapack_band(Aee, b), b, b)
        if info != 0:
            raise np.linalg.LinAlgError(f"banded LU breakdown, info={info}")
        self.lu, self.piv = lu, piv

    def solve(self, rhs: np.ndarray, trans: int = 0) -> np.ndarray:
        """A_{2s,2s}^{-1} rhs (trans=1: A_{2s,2s}^{-T} rhs) for a vector or columns."""
        x, info = lapack.dgbtrs(self.lu, self.b, self.b, np.asarray(rhs, dtype=np.float64),
                                self.piv, trans=trans)
        assert info == 0
        return x


@dataclass
class StageOne:
    factors: list          # SlabFactor per slab
    T_diag: list           # T_{jj}, n2 x n2, j = 0..m-1
    T_up: list             # T_{j,j+1}, j = 0..m-2
    T_lo: list             # T_{j+1,j}, j = 0..m-2


def slab_contributions(prob: Problem, s: int, factor: "SlabFactor | None" = None,
                       transpose: bool = False) -> dict:
    """Schur-complement pieces that slab s (I_{2s}) adds to the reduced blocks.

    Returns {(jr, jc): C} with C = A_{o(jr),2s} A_{2s,2s}^-1 A_{2s,o(jc)} for the
    interfaces jr, jc in {s-1, s} that exist (eq. (T11_detailed)).
    """
    A = prob.A.T.tocsr() if transpose else prob.A
    Ie = prob.I_e(s)
    if factor is None:
        factor = SlabFactor(A[Ie][:, Ie], prob.b)
    nbrs = [j for j in (s - 1, s) if 0 <= j < prob.m]
    out = {}
    for jc in nbrs:
        X = factor.solve(A[Ie][:, prob.I_o(jc)].toarray())     # A_{2s,2s}^-1 A_{2s, o(jc)}
        for jr in nbrs:
            out[(jr, jc)] = A[prob.I_o(jr)][:, Ie] @ X
    return out


def interface_blocks(prob: Problem, j: int) -> tuple:
    """T_jj and (for j < m-1) T_{j,j+1} from the two slabs touching interface j only."""
    A = prob.A
    Tjj = A[prob.I_o(j)][:, prob.I_o(j)].toarray()
    Tup = None
    for s in (j, j + 1):
        if s >= prob.m:
            continue
        C = slab_contributions(prob, s)
        Tjj -= C[(j, j)]
        if s == j + 1:
            Tup = A[prob.I_o(j)][:, prob.I_o(j + 1)].toarray() - C[(j, j + 1)]
    return Tjj, Tup


_POOL_STATE = {}


def _pool_init(prob: Problem, transpose: bool):
    # one BLAS thread per worker process: the workers already fill the cores
    # (multithreaded BLAS pools in every worker oversubscribe them and have
    # stalled the pool)
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    _POOL_STATE["prob"], _POOL_STATE["transpose"] = prob, transpose


def _pool_slab(s: int):
    """Worker of stage_one(workers > 1): factor slab s and form its pieces."""
    prob, transpose = _POOL_STATE["prob"], _POOL_STATE["transpose"]
    A = prob.A.T.tocsr() if transpose else prob.A
    fac = SlabFactor(A[prob.I_e(s)][:, prob.I_e(s)], prob.b)
    return fac, slab_contributions(prob, s, fac, transpose)


def stage_one(prob: Problem, transpose: bool = False, workers: int = 1) -> StageOne:
    """Eliminate every slab interior and form the block-tridiagonal T (eq. (dell3)).

    For interface j (index set I_{2j+1}) with slab j on its left (I_{2j}) and
    slab j+1 on its right (I_{2j+2}):
      T_jj     = A_oo - A_{o,2j} A_{2j,2j}^-1 A_{2j,o} - A_{o,2j+2} A_{2j+2,2j+2}^-1 A_{2j+2,o}
      T_{j,j+1} = A_{o(j),o(j+1)} - A_{o(j),2j+2} A_{2j+2,2j+2}^-1 A_{2j+2,o(j+1)}
      T_{j+1,j} = A_{o(j+1),o(j)} - A_{o(j+1),2j+2} A_{2j+2,2j+2}^-1 A_{2j+2,o(j)}
    (eqs. (T11)-(T35) with the index slips read as stated in the module
    docstring).  With transpose=True every block of A is replaced by the
    corresponding block of A^T, which gives the reduced system of A^T.
    """
    A = prob.A.T.tocsr() if transpose else prob.A
    m = prob.m

    def blk(I, J):
        return A[I][:, J]

    if workers > 1:
        # the slabs are independent (Sec. 3.1): spread them over processes
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"),
                                    initializer=_pool_init, initargs=(prob, transpose)) as ex:
            done = list(ex.map(_pool_slab, range(m)))
        factors = [d[0] for d in done]
        pieces = [d[1] for d in done]
    else:
        factors = [SlabFactor(blk(prob.I_e(s), prob.I_e(s)), prob.b) for s in range(m)]
        pieces = None
    T_diag = [blk(prob.I_o(j), prob.I_o(j)).toarray() for j in range(m)]
    T_up = [blk(prob.I_o(j), prob.I_o(j + 1)).toarray() for j in range(m - 1)]
    T_lo = [blk(prob.I_o(j + 1), prob.I_o(j)).toarray() for j in range(m - 1)]
    for s in range(m):
        C_s = pieces[s] if pieces is not None else slab_contributions(prob, s, factors[s], transpose)
        for (jr, jc), C in C_s.items():
            if jr == jc:
                T_diag[jr] -= C
            elif jc == jr + 1:
                T_up[jr] -= C
            else:
                T_lo[jc] -= C
    return StageOne(factors, T_diag, T_up, T_lo)


def reduced_rhs(prob: Problem, s1: StageOne, f: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Equivalent body load on the interfaces, eqs. (f1)-(f5).

    f~_j = f_{o(j)} - A_{o(j),2j} A_{2j,2j}^-1 f_{2j} - A_{o(j),2j+2} A_{2j+2,2j+2}^-1 f_{2j+2}.
    f: (nrhs, n1, n2).  Returns (nrhs, m, n2).
    """
    A = prob.A.T.tocsr() if transpose else prob.A
    m, n2 = prob.m, prob.n2
    F = f.reshape(-1, prob.N)
    out = np.empty((F.shape[0], m, n2))
    for j in range(m):
        out[:, j, :] = F[:, prob.I_o(j)]
    for s in range(m):
        Ie = prob.I_e(s)
        y = s1.factors[s].solve(F[:, Ie].T)        # A_{2s,2s}^-1 f_{2s}, columns = rhs
        for j in (s - 1, s):
            if 0 <= j < m:
                out[:, j, :] -= (A[prob.I_o(j)][:, Ie] @ y).T
    return out


def interior_solve(prob: Problem, s1: StageOne, f: np.ndarray, uo: np.ndarray,
                   transpose: bool = False) -> np.ndarray:
    """Slab interiors from the interface values, eq. (usol_even).

    u_{2s} = A_{2s,2s}^-1 (f_{2s} - A_{2s,o(s-1)} u_{o(s-1)} - A_{2s,o(s)} u_{o(s)}).
    Returns the full solution (nrhs, n1, n2).
    """
    A = prob.A.T.tocsr() if transpose else prob.A
    m = prob.m
    F = f.reshape(-1, prob.N)
    U = np.zeros_like(F)
    for j in range(m):
        U[:, prob.I_o(j)] = uo[:, j, :]
    for s in range(m):
        Ie = prob.I_e(s)
        rhs = F[:, Ie].T.copy()
        for j in (s - 1, s):
            if 0 <= j < m:
                rhs -= A[Ie][:, prob.I_o(j)] @ uo[:, j, :].T
        U[:, Ie] = s1.factors[s].solve(rhs).T
    return U.reshape(f.shape)


# ---------------------------------------------------------------------------
# Stage two (Sec. 4): Alg. 1 (sweeping build) and Alg. 2 (sweeping solve).
# ---------------------------------------------------------------------------

@dataclass
class StageTwo:
    S: list        # S_j before factorization (recorded for comparison)
    lu: list       # LAPACK LU factors of each S_j ("compute and store S_j^-1")


def sweeping_build(s1: StageOne) -> StageTwo:
    """Alg. 1: S_0 = T_00; S_j = T_jj - T_{j,j-1} S_{j-1}^-1 T_{j-1,j}."""
    m = len(s1.T_diag)
    S = [s1.T_diag[0].copy()]
    lu = [sla.lu_factor(S[0])]
    for j in range(1, m):
        Sj = s1.T_diag[j] - s1.T_lo[j - 1] @ sla.lu_solve(lu[j - 1], s1.T_up[j - 1])
        S.append(Sj)
        lu.append(sla.lu_factor(Sj))
    return StageTwo(S, lu)


def sweeping_solve(s1: StageOne, s2: StageTwo, ft: np.ndarray) -> np.ndarray:
    """Alg. 2 on f~ of shape (nrhs, m, n2): forward sweep, diagonal solves, backward sweep."""
    m = len(s2.S)
    g = [ft[:, j, :].T.copy() for j in range(m)]      # columns = rhs
    for j in range(1, m):
        g[j] -= s1.T_lo[j - 1] @ sla.lu_solve(s2.lu[j - 1], g[j - 1])
    for j in range(m):
        g[j] = sla.lu_solve(s2.lu[j], g[j])
    for j in range(m - 2, -1, -1):
        g[j] -= sla.lu_solve(s2.lu[j], s1.T_up[j] @ g[j + 1])
    return np.stack([gj.T for gj in g], axis=1)


# ---------------------------------------------------------------------------
# Stage two in odd-even order (the elimination order proposed in the Remark of
# Sec. 4 and in the concluding section: every other interface block is
# eliminated, level by level, instead of the sweep of Alg. 1).
#
# Reading (the paper gives no formulas for it): the interfaces still present
# at a level form a list a_0, a_1, ..., a_{k-1}; the blocks at even positions
# a_0, a_2, ... are eliminated together, those at odd positions stay.  The
# Schur complement that remains is again block tridiagonal in the kept order:
# eliminating e between its neighbours l (before it) and r (after it) changes
#   T_ll -= T_le T_ee^-1 T_el,   T_rr -= T_re T_ee^-1 T_er,
#   T_lr  = -T_le T_ee^-1 T_er,  T_rl  = -T_re T_ee^-1 T_el
# (T_lr and T_rl were zero).  Levels repeat until no interface is left; the
# last one eliminated is the last interface when m is a power of two.
# ---------------------------------------------------------------------------

@dataclass
class Elimination:
    e: int                 # interface eliminated
    l: int | None          # neighbour before it in the list of its level (kept), or None
    r: int | None          # neighbour after it (kept), or None
    D: np.ndarray          # its pivot block T_ee at the time of elimination
    lu: tuple              # LAPACK LU of D
    T_el: np.ndarray | None
    T_le: np.ndarray | None
    T_er: np.ndarray | None
    T_re: np.ndarray | None


@dataclass
class OddEven:
    levels: list           # list of levels, each a list of Elimination

    def pivot(self, j: int) -> np.ndarray:
        for lev in self.levels:
            for el in lev:
                if el.e == j:
                    return el.D
        raise KeyError(j)


def odd_even_build(s1: StageOne) -> OddEven:
    """Odd-even elimination of the block-tridiagonal T (see the comment above)."""
    m = len(s1.T_diag)
    D = {j: s1.T_diag[j].copy() for j in range(m)}
    up = {j: s1.T_up[j].copy() for j in range(m - 1)}   # T_{x, next(x)}
    lo = {j: s1.T_lo[j].copy() for j in range(m - 1)}   # T_{next(x), x}
    active = list(range(m))
    levels = []
    while active:
        level = []
        for p in range(0, len(active), 2):
            e = active[p]
            l = active[p - 1] if p > 0 else None
            r = active[p + 1] if p + 1 < len(active) else None
            level.append(Elimination(e, l, r, D[e].copy(), sla.lu_factor(D[e]),
                                     lo[l] if l is not None else None,
                                     up[l] if l is not None else None,
                                     up[e] if r is not None else None,
                                     lo[e] if r is not None else None))
        for el in level:
            if el.l is not None:
                D[el.l] = D[el.l] - el.T_le @ sla.lu_solve(el.lu, el.T_el)
            if el.r is not None:
                D[el.r] = D[el.r] - el.T_re @ sla.lu_solve(el.lu, el.T_er)
            if el.l is not None and el.r is not None:
                up[el.l] = -el.T_le @ sla.lu_solve(el.lu, el.T_er)
                lo[el.l] = -el.T_re @ sla.lu_solve(el.lu, el.T_el)
        levels.append(level)
        active = active[1::2]
    return OddEven(levels)


def odd_even_solve(oe: OddEven, ft: np.ndarray) -> np.ndarray:
    """Solve T x = f~ with the odd-even elimination: the right-hand side is
    reduced level by level as T was, then the eliminated blocks are recovered
    from the top level down, x_e = T_ee^-1 (g_e - T_el x_l - T_er x_r)."""
    m = ft.shape[1]
    g = [ft[:, j, :].T.copy() for j in range(m)]
    for level in oe.levels:
        for el in level:
            z = sla.lu_solve(el.lu, g[el.e])
            if el.l is not None:
                g[el.l] = g[el.l] - el.T_le @ z
            if el.r is not None:
                g[el.r] = g[el.r] - el.T_re @ z
    x = [None] * m
    for level in reversed(oe.levels):
        for el in level:
            rhs = g[el.e].copy()
            if el.l is not None:
                rhs -= el.T_el @ x[el.l]
            if el.r is not None:
                rhs -= el.T_er @ x[el.r]
            x[el.e] = sla.lu_solve(el.lu, rhs)
    return np.stack([xj.T for xj in x], axis=1)


# ---------------------------------------------------------------------------
# Alg. 3 (factor) and Alg. 4 (solve), and the adjoint.
# ---------------------------------------------------------------------------

@dataclass
class Factorization:
    prob: Problem
    s1: StageOne
    s2: "StageTwo | OddEven"
    transpose: bool = False


def factor(prob: Problem, transpose: bool = False, order: str = "sweep",
           workers: int = 1) -> Factorization:
    """Alg. 3: slab factorizations, reduced blocks T (formed densely), then
    stage two by Alg. 1 (order="sweep") or in odd-even order (order="odd_even").
    workers > 1 runs the independent slabs of stage one in that many processes."""
    s1 = stage_one(prob, transpose, workers)
    if order == "sweep":
        s2 = sweeping_build(s1)
    elif order == "odd_even":
        s2 = odd_even_build(s1)
    else:
        raise ValueError(order)
    return Factorization(prob, s1, s2, transpose)


def solve(fac: Factorization, f: np.ndarray) -> np.ndarray:
    """Alg. 4: reduced RHS, Alg. 2, interior back-substitution.  f: (nrhs, n1, n2)."""
    f = np.asarray(f, dtype=np.float64)
    squeeze = f.ndim == 2
    if squeeze:
        f = f[None]
    ft = reduced_rhs(fac.prob, fac.s1, f, fac.transpose)
    if isinstance(fac.s2, OddEven):
        uo = odd_even_solve(fac.s2, ft)
    else:
        uo = sweeping_solve(fac.s1, fac.s2, ft)
    u = interior_solve(fac.prob, fac.s1, f, uo, fac.transpose)
    return u[0] if squeeze else u


def solve_adjoint(prob: Problem, g: np.ndarray, fac_T: Factorization | None = None,
                  order: str = "sweep") -> np.ndarray:
    """lambda = A^-T g through the same two-level elimination applied to A^T."""
    if fac_T is None:
        fac_T = factor(prob, transpose=True, order=order)
    return solve(fac_T, g)


def apply_T(prob: Problem, x: np.ndarray) -> np.ndarray:
    """T x = A_oo x - A_oe A_ee^-1 A_eo x, the Schur complement of A onto the
    interface unknowns (Sec. 3.1, eq. (T11_detailed)) applied without forming
    it: the product the randomized sketches of T are built from (Alg. 3,
    Sec. 3.3), here for given test vectors.  x and the result have shape
    (m, ncols, n2): block j of column k is interface j's part.  A_ee (all
    slab interiors together) is factored by a sparse LU."""
    m, n2 = prob.m, prob.n2
    Io = np.concatenate([prob.I_o(j) for j in range(m)])
    Ie = np.concatenate([prob.I_e(s) for s in range(m)])
    A = prob.A
    X = np.ascontiguousarray(x.transpose(0, 2, 1).reshape(m * n2, -1))
    lu = spla.splu(A[Ie][:, Ie].tocsc())
    Y = A[Io][:, Io] @ X - A[Io][:, Ie] @ lu.solve(np.asarray(A[Ie][:, Io] @ X))
    return np.ascontiguousarray(Y.reshape(m, n2, -1).transpose(0, 2, 1))


def interface_values(u: np.ndarray, prob: Problem) -> np.ndarray:
    """Restriction of a full solution (nrhs, n1, n2) to I_1, I_3, ... -> (nrhs, m, n2)."""
    flat = u.reshape(-1, prob.N)
    return np.stack([flat[:, prob.I_o(j)] for j in range(prob.m)], axis=1)


# ---------------------------------------------------------------------------
# Gradient of a loss with respect to theta = log(kappa) (adjoint method).
# ---------------------------------------------------------------------------

def kappa_grad(prob: Problem, u: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """dL/dtheta on the (n1+2) x (n2+2) node field, given u = A^-1 f and lambda = A^-T dL/du.

    L depends on kappa only through A, so dL/dw_e = -lambda^T (dA/dw_e) u =
    -(lambda_p - lambda_q)(u_p - u_q), with ring values zero; w_e depends on
    its two end nodes with dw_e/dkappa_p = 1/(2h^2); dkappa/dtheta = kappa.
    Summed over right-hand sides.
    """
    n2, n1, h = prob.n2, prob.n1, prob.h
    u = u.reshape(-1, n1, n2)
    lam = lam.reshape(-1, n1, n2)
    U = np.zeros((u.shape[0], n1 + 2, n2 + 2))
    Lm = np.zeros_like(U)
    U[:, 1:-1, 1:-1] = u
    Lm[:, 1:-1, 1:-1] = lam
    # horizontal edges between node columns i and i+1 of the padded field, rows 1..n2
    dUh = U[:, 1:, 1:-1] - U[:, :-1, 1:-1]
    dLh = Lm[:, 1:, 1:-1] - Lm[:, :-1, 1:-1]
    gwh = -(dLh * dUh).sum(axis=0)                  # (n1+1, n2) = dL/dw for wh
    dUv = U[:, 1:-1, 1:] - U[:, 1:-1, :-1]
    dLv = Lm[:, 1:-1, 1:] - Lm[:, 1:-1, :-1]
    gwv = -(dLv * dUv).sum(axis=0)                  # (n1, n2+1) = dL/dw for wv
    gk = np.zeros((n1 + 2, n2 + 2))
    scale = 1.0 / (2.0 * h * h)
    gk[:-1, 1:-1] += gwh * scale
    gk[1:, 1:-1] += gwh * scale
    gk[1:-1, :-1] += gwv * scale
    gk[1:-1, 1:] += gwv * scale
    return gk * prob.kappa


def direct_solve(prob: Problem, f: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Independent cross-check: sparse LU (SuperLU) of A (or A^T) in natural order."""
    lu = spla.splu((prob.A.T if transpose else prob.A).tocsc())
    F = f.reshape(-1, prob.N)
    U = np.stack([lu.solve(F[i]) for i in range(F.shape[0])])
    return U.reshape(f.shape)
