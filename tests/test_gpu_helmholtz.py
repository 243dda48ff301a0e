"""The diagonal term c_p of the operator (the Helmholtz term of eq.
(var_helm), c = -k^2 b(x)), on the GPU against the oracle.

Definite cases: a nonnegative c (screened diffusion on a lognormal
coefficient) and a Helmholtz term -k^2 below the lowest eigenvalue of the
Laplacian.  Indefinite cases: a Helmholtz term several wavelengths across the
grid, with slabs narrower than half a wavelength (only T indefinite) or wider
(indefinite slab interiors too); both stages then eliminate with pivots of
either sign and no pivoting, the pivot blocks of T in signed form L J L^T.
The number of negative pivots of T must equal the closed-form count from the
sine modes (negative eigenvalues of A minus those of the m slab interiors,
by the inertia additivity of Schur complements) and the solution must match
the oracle within cond(A) times the two residuals.  An exactly zero pivot must
be reported (SLAB_E_BREAKDOWN) rather than return a wrong answer.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import inputs as G
from oracle import slab_oracle as O
from paper_2211_07572_amd import slab as S

pytestmark = pytest.mark.gpu

ORDERS = ["sweep", "odd_even"]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _col_rel(u, ref):
    u = u.reshape(u.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(u - ref, axis=1) / np.linalg.norm(ref, axis=1)


def _pivot(fac, j):
    return fac.s2.pivot(j) if isinstance(fac.s2, O.OddEven) else fac.s2.S[j]


def _lam_min(n2, n1, h):
    return (4 - 2 * np.cos(np.pi / (n1 + 1)) - 2 * np.cos(np.pi / (n2 + 1))) / h ** 2


def _cases():
    out = []
    # screened diffusion: c >= 0 varying over the grid, lognormal kappa
    n2, n1, b = 70, 96, 15
    h = 1.0 / (n2 + 1)
    c = np.abs(G.rhs_normal(n2, n1, 1, 31)[0]) * 50.0 / h
    out.append(("screened", n2, n1, b, G.kappa_lognormal(n2, n1, 31), c))
    # Helmholtz below the first eigenvalue: -k^2 = -0.5 lambda_min, kappa = 1
    n2, n1, b = 64, 96, 7
    h = 1.0 / (n2 + 1)
    out.append(("helmholtz_definite", n2, n1, b, G.kappa_const(n2, n1),
                np.full((n1, n2), -0.5 * _lam_min(n2, n1, h))))
    return out


CASES = _cases()


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_shift_fp64_parity(case, order):
    name, n2, n1, b, kap, c = case
    prob = O.make_problem(kap, n2, n1, b, shift=c)
    fac = O.factor(prob, order=order)
    h = S.slab_factor(_dev(kap), n2, n1, b, keep_reduced=True, odd_even=order == "odd_even",
                      shift=_dev(c))
    for j in range(prob.m):
        assert _rel_fro(S.slab_export_reduced(h, 0, j).cpu().numpy(), fac.s1.T_diag[j]) <= 1e-12
        assert _rel_fro(S.slab_export_reduced(h, 2, j).cpu().numpy(), _pivot(fac, j)) <= 1e-12
    for j in range(prob.m - 1):
        assert _rel_fro(S.slab_export_reduced(h, 1, j).cpu().numpy(), fac.s1.T_up[j]) <= 1e-12
    f = G.rhs_uniform(n2, n1, 3, 5)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert _col_rel(u, O.solve(fac, f)).max() <= 1e-12
    rr = np.array(S.slab_residual(h, _dev(f), _dev(u)))
    ref = O.relres(prob, u, f)
    assert np.all(np.abs(rr - ref) <= 0.05 * ref + 1e-15)
    x = G.gaussian_test_vectors(prob.m, 2, n2, 6)
    y = S.slab_apply_reduced(h, _dev(x)).cpu().numpy()
    yr = O.apply_T(prob, x)
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()
    h.free()


@pytest.mark.parametrize("precision", [S.SLAB_MIXED, S.SLAB_FP32_REFINE])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_shift_refined_forms(case, precision):
    name, n2, n1, b, kap, c = case
    prob = O.make_problem(kap, n2, n1, b, shift=c)
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=precision, tol=1e-10, odd_even=True,
                      shift=_dev(c))
    f = G.rhs_uniform(n2, n1, 2, 8)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert O.relres(prob, u, f).max() <= 1e-10
    h.free()


def test_shift_in_batch_and_graph_run():
    dims = [(40, 48, 7), (70, 96, 15), (33, 24, 1)]
    kaps = [G.kappa_lognormal(n2, n1, 40 + i) for i, (n2, n1, b) in enumerate(dims)]
    shifts = [None, np.abs(G.rhs_normal(70, 96, 1, 41)[0]) * 1e4, np.full((24, 33), 3e3)]
    fs = [G.rhs_uniform(n2, n1, 2, 50 + i) for i, (n2, n1, b) in enumerate(dims)]
    kd = [_dev(k) for k in kaps]
    sd = [None if c is None else _dev(c) for c in shifts]
    fd = [_dev(f) for f in fs]
    bt = S.slab_factor_batch(kd, dims, precision=S.SLAB_FP64, shifts=sd)
    us = S.slab_solve_batch(bt, fd)
    us2 = S.slab_batch_run(bt, kd, fd)
    for i, (n2, n1, b) in enumerate(dims):
        prob = O.make_problem(kaps[i], n2, n1, b, shift=shifts[i])
        ref = O.direct_solve(prob, fs[i])
        assert _col_rel(us[i].cpu().numpy(), ref).max() <= 1e-12, i
        assert np.array_equal(us2[i].cpu().numpy(), us[i].cpu().numpy()), i
    bt.free()


def test_zero_slab_pivot_is_reported():
    """A diagonal term that makes the first pivot of every slab exactly zero
    (b = 1, h = 1/32 so that c = -4/h^2 cancels the diagonal 4/h^2 exactly):
    the signed elimination without pivoting cannot go on, and the
    factorization says so instead of returning a wrong answer."""
    n2, n1, b = 31, 32, 1
    h = 1.0 / 32
    c = np.full((n1, n2), -4.0 / h ** 2)
    with pytest.raises(S.SlabError) as ei:
        S.slab_factor(_dev(G.kappa_const(n2, n1)), n2, n1, b, h, odd_even=True, shift=_dev(c))
    assert ei.value.status == S.SLAB_E_BREAKDOWN


# ------------------------------------------------- indefinite T (signed pivots)

def _laplace_eigs(n2, n1, h):
    k1 = np.arange(1, n1 + 1)[:, None]
    k2 = np.arange(1, n2 + 1)[None, :]
    return (4 - 2 * np.cos(np.pi * k1 / (n1 + 1)) - 2 * np.cos(np.pi * k2 / (n2 + 1))) / h ** 2


# (name, n2, n1, b, points per wavelength): n2 = 200 spans three full 64-column
# panels and a ragged one; 139 and 35 negative eigenvalues; cond(A) 4.6e4, 3.6e4
INDEF = [("ppw20_b7", 200, 96, 7, 20.0), ("ppw40_b15", 130, 160, 15, 40.0)]


def _indef_setup(n2, n1, b, ppw, slabs_definite=True):
    h = 1.0 / (n2 + 1)
    c = G.helmholtz_shift(n2, n1, ppw, h)
    k2 = -c[0, 0]
    lam = _laplace_eigs(n2, n1, h)
    gap = np.abs(lam - k2)
    slab_neg = int((_laplace_eigs(n2, b, h) < k2).sum())   # one slab interior
    assert (slab_neg == 0) == slabs_definite
    neg = int((lam < k2).sum()) - (n1 // (b + 1)) * slab_neg   # negative eigenvalues of T
    assert neg > 0
    cond = gap.max() / gap.min()   # A = -Laplace - k^2 is symmetric: exact cond_2
    return c, neg, cond


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("case", INDEF, ids=[c[0] for c in INDEF])
def test_indefinite_T_fp64(case, order):
    name, n2, n1, b, ppw = case
    c, neg, cond = _indef_setup(n2, n1, b, ppw)
    kap = G.kappa_const(n2, n1)
    prob = O.make_problem(kap, n2, n1, b, shift=c)
    fac = O.factor(prob, order=order)
    h = S.slab_factor(_dev(kap), n2, n1, b, keep_reduced=True, odd_even=order == "odd_even",
                      shift=_dev(c))
    assert h.negative_pivots() == neg
    for j in range(prob.m):   # stage one does not depend on the signs
        assert _rel_fro(S.slab_export_reduced(h, 0, j).cpu().numpy(), fac.s1.T_diag[j]) <= 1e-12
    f = G.rhs_uniform(n2, n1, 3, 5)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    rr = O.relres(prob, u, f)
    assert rr.max() <= 1e-10
    u_ref = O.solve(fac, f)
    rr_ref = O.relres(prob, u_ref, f)
    # ||u - u*|| / ||u*|| <= cond(A) ||A u - f|| / ||f|| for both solutions
    assert np.all(_col_rel(u, u_ref) <= cond * (rr + rr_ref) * 1.01 + 1e-15)
    h.free()


@pytest.mark.parametrize("precision", [S.SLAB_MIXED, S.SLAB_FP32_REFINE])
@pytest.mark.parametrize("order", ORDERS)
def test_indefinite_T_refined_forms(order, precision):
    name, n2, n1, b, ppw = INDEF[0]
    c, neg, cond = _indef_setup(n2, n1, b, ppw)
    assert cond * 6e-8 < 0.01   # FP32 pivots keep the signs of the exact ones
    kap = G.kappa_const(n2, n1)
    prob = O.make_problem(kap, n2, n1, b, shift=c)
    # each pass shrinks the error by about cond(A) eps_32 times the growth of
    # the elimination (measured 0.1-0.2 per pass with FP32 slab sweeps in
    # odd-even order here: 1e-10 after about 12 passes; the mixed form needs 5)
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=precision, tol=1e-10, max_iter=20,
                      odd_even=order == "odd_even", shift=_dev(c))
    assert h.negative_pivots() == neg
    f = G.rhs_uniform(n2, n1, 2, 8)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert O.relres(prob, u, f).max() <= 1e-10
    h.free()


def test_indefinite_in_batch_and_graph_run():
    """Signed and unsigned problems in one batch (their block products go to
    launches of their own), eager and as one graph."""
    name, n2, n1, b, ppw = INDEF[1]
    c, neg, cond = _indef_setup(n2, n1, b, ppw)
    dims = [(n2, n1, b), (70, 96, 15), (96, 64, 7)]
    kaps = [G.kappa_const(n2, n1), G.kappa_lognormal(70, 96, 61), G.kappa_const(96, 64)]
    c3, neg3, cond3 = _indef_setup(96, 64, 7, 24.0)
    shifts = [c, None, c3]
    fs = [G.rhs_uniform(d[0], d[1], 2, 70 + i) for i, d in enumerate(dims)]
    kd = [_dev(k) for k in kaps]
    sd = [None if x is None else _dev(x) for x in shifts]
    fd = [_dev(f) for f in fs]
    for order in (False, True):
        bt = S.slab_factor_batch(kd, dims, precision=S.SLAB_MIXED, shifts=sd, odd_even=order)
        assert bt.handle(0).negative_pivots() == neg
        assert bt.handle(1).negative_pivots() == 0
        assert bt.handle(2).negative_pivots() == neg3
        us = S.slab_solve_batch(bt, fd)
        us2 = S.slab_batch_run(bt, kd, fd)
        for i, (a2, a1, ab) in enumerate(dims):
            prob = O.make_problem(kaps[i], a2, a1, ab, shift=shifts[i])
            assert O.relres(prob, us[i].cpu().numpy(), fs[i]).max() <= 1e-10, (order, i)
            assert np.array_equal(us2[i].cpu().numpy(), us[i].cpu().numpy()), (order, i)
        bt.free()


# ------------------------------- Dirichlet data and the FD Helmholtz benchmark

@pytest.mark.parametrize("n2,n1,b", [(70, 96, 15), (33, 24, 1), (1, 8, 3)])
def test_dirichlet_load_matches_oracle(n2, n1, b):
    """slab_dirichlet_load against the oracle's load, lognormal kappa, two
    fields of random ring data, from zero and on top of a source.  Both add
    the same terms in the same order; the edge weights themselves are formed
    in a different order on the two sides (last-bit differences), so the
    bound is a few units of rounding of the largest entry."""
    kap = G.kappa_lognormal(n2, n1, 23)
    prob = O.make_problem(kap, n2, n1, b)
    g = np.random.default_rng(9).standard_normal((2, n1 + 2, n2 + 2))
    h = S.slab_factor(_dev(kap), n2, n1, b)
    ref = O.dirichlet_load(prob, g)
    f = S.slab_dirichlet_load(h, _dev(g)).cpu().numpy()
    tol = 1e-15 * np.abs(ref).max()
    assert np.abs(f - ref).max() <= tol
    assert np.count_nonzero(f) == np.count_nonzero(ref)   # only nodes next to the ring
    src = G.rhs_uniform(n2, n1, 2, 4)
    f2 = S.slab_dirichlet_load(h, _dev(g), _dev(src)).cpu().numpy()
    assert np.abs(f2 - (src + ref)).max() <= tol + 1e-16 * np.abs(src).max()
    h.free()


@pytest.mark.parametrize("order", ORDERS)
def test_bessel_benchmark_against_oracle(order):
    """The paper's FD Helmholtz benchmark (eq. (constant_coeff_helm)) at 40
    points per wavelength on 256 x 256 (b = 7; indefinite T): the load of the
    J0 data made on the GPU, the solution against the oracle's for the
    oracle's own load (within cond(A) times the residuals), and relerr_true of
    both equal."""
    n, b, ppw = 256, 7, 40.0
    h = 1.0 / (n + 1)
    k = 2 * np.pi / (ppw * h)
    c = np.full((n, n), -k * k)
    lam = _laplace_eigs(n, n, h)
    gap = np.abs(lam - k * k)
    cond = gap.max() / gap.min()
    ut = G.bessel_field(n, n, k, h)
    prob = O.make_problem(G.kappa_const(n, n), n, n, b, h, shift=c)
    f_ref = O.dirichlet_load(prob, ut)
    u_ref = O.direct_solve(prob, f_ref)
    hd = S.slab_factor(_dev(G.kappa_const(n, n)), n, n, b, h, odd_even=order == "odd_even",
                       shift=_dev(c))
    assert hd.negative_pivots() == int((lam < k * k).sum())
    fd = S.slab_dirichlet_load(hd, _dev(ut))
    u = S.slab_solve(hd, fd).cpu().numpy()[0]
    rr = O.relres(prob, u, f_ref)[0]
    rr_ref = O.relres(prob, u_ref, f_ref)[0]
    assert rr <= 1e-10
    assert _rel_fro(u, u_ref) <= cond * (rr + rr_ref) * 1.01 + 1e-15
    e = _rel_fro(u, ut[1:-1, 1:-1])
    e_ref = _rel_fro(u_ref, ut[1:-1, 1:-1])
    assert abs(e - e_ref) <= cond * (rr + rr_ref) * 1.01 * np.linalg.norm(u_ref) / np.linalg.norm(ut[1:-1, 1:-1]) + 1e-15
    hd.free()


# The paper's first FD Helmholtz row (figure of the constant points-per-wavelength
# runs, Sec. 5.2): N = 1.0M, b = 50, kappa = 27.1, relerr_res 1.1e-11,
# relerr_true 1.8e-3.  Here n = 1000 per side (h = 1/1001) with b = 49, the
# largest width whose period divides 1000.
PAPER_FD_1M = {"n": 1000, "kappa": 27.1, "relerr_res": 1.1e-11, "relerr_true": 1.8e-3}


def test_paper_fd_helmholtz_1m():
    """relerr_true of the FD solution is the discretization's (pollution)
    error, the same for any accurate solver: it must come out at the paper's
    1.8e-3 (within a factor 1.5, the grid conventions may differ slightly),
    and relerr_res at or below the paper's."""
    n, k = PAPER_FD_1M["n"], PAPER_FD_1M["kappa"]
    h = 1.0 / (n + 1)
    print(f"case: paper FD Helmholtz n={n} b=49 kappa={k}", flush=True)
    ut = G.bessel_field(n, n, k, h)
    hd = S.slab_factor(_dev(G.kappa_const(n, n)), n, n, 49, h, odd_even=True,
                       shift=_dev(np.full((n, n), -k * k)))
    fd = S.slab_dirichlet_load(hd, _dev(ut))
    u = S.slab_solve(hd, fd)
    rr = S.slab_residual(hd, fd, u)[0]
    e = _rel_fro(u.cpu().numpy()[0], ut[1:-1, 1:-1])
    print(f"  relerr_res {rr:.2e} (paper {PAPER_FD_1M['relerr_res']:.1e}), "
          f"relerr_true {e:.3e} (paper {PAPER_FD_1M['relerr_true']:.1e})")
    assert rr <= PAPER_FD_1M["relerr_res"]
    assert PAPER_FD_1M["relerr_true"] / 1.5 <= e <= PAPER_FD_1M["relerr_true"] * 1.5
    hd.free()


@pytest.mark.parametrize("precision", [S.SLAB_FP64, S.SLAB_MIXED])
def test_indefinite_T_512(precision):
    """512 x 512, b = 15, 36 points per wavelength (612 negative eigenvalues,
    cond(A) 5.4e4): pivot blocks of eight 64-column panels, so the signed
    trailing updates run at several panel offsets; the block-vector products
    split over k (n >= 512) with their pivot signs; the mixed form on forced
    128-wide FP32 tiles with scaled k.  Negative pivots against the closed
    form, u against the oracle's SuperLU solve within cond(A) times the
    residuals."""
    n, b, ppw = 512, 15, 36.0
    c, neg, cond = _indef_setup(n, n, b, ppw)
    kap = G.kappa_const(n, n)
    prob = O.make_problem(kap, n, n, b, shift=c)
    f = G.rhs_uniform(n, n, 2, 12)
    u_ref = O.direct_solve(prob, f)
    rr_ref = O.relres(prob, u_ref, f)
    print(f"case: indefinite 512x512 b=15 ppw=36 precision={precision}", flush=True)
    h = S.slab_factor(_dev(kap), n, n, b, precision=precision, tol=1e-10, max_iter=20,
                      odd_even=True, shift=_dev(c), tile=128 if precision == S.SLAB_MIXED else 0)
    assert h.negative_pivots() == neg
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    rr = O.relres(prob, u, f)
    lc = h.launches()
    print(f"  relres {rr.max():.2e} after {h.last_info.iterations} passes, "
          f"u vs oracle {_col_rel(u, u_ref).max():.2e}, launches {lc}", flush=True)
    assert rr.max() <= 1e-10
    assert np.all(_col_rel(u, u_ref) <= cond * (rr + rr_ref) * 1.01 + 1e-15)
    assert lc["bmv_split"] > 0
    if precision == S.SLAB_MIXED:
        assert lc["gemm128"] > 0
    h.free()


# indefinite slab interiors too: 8, 8 and 32 columns against 6, 10 and 12 points
# per wavelength (35, 47 and 160 negative eigenvalues per slab)
INDEF_SLABS = [("ppw6_b7", 64, 64, 7, 6.0), ("ppw10_b7", 200, 96, 7, 10.0),
               ("ppw12_b31", 256, 256, 31, 12.0)]


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("case", INDEF_SLABS, ids=[c[0] for c in INDEF_SLABS])
def test_indefinite_slabs_fp64(case, order):
    name, n2, n1, b, ppw = case
    c, neg, cond = _indef_setup(n2, n1, b, ppw, slabs_definite=False)
    kap = G.kappa_const(n2, n1)
    prob = O.make_problem(kap, n2, n1, b, shift=c)
    f = G.rhs_uniform(n2, n1, 2, 5)
    u_ref = O.direct_solve(prob, f)
    rr_ref = O.relres(prob, u_ref, f)
    h = S.slab_factor(_dev(kap), n2, n1, b, odd_even=order == "odd_even", shift=_dev(c))
    assert h.negative_pivots() == neg
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    rr = O.relres(prob, u, f)
    assert rr.max() <= 1e-10
    assert np.all(_col_rel(u, u_ref) <= cond * (rr + rr_ref) * 1.01 + 1e-15)
    h.free()


@pytest.mark.parametrize("order", ORDERS)
def test_indefinite_slabs_mixed(order):
    """Mixed form, 130 x 160 with 16-column slabs at 20 points per wavelength."""
    n2, n1, b, ppw = 130, 160, 15, 20.0
    c, neg, cond = _indef_setup(n2, n1, b, ppw, slabs_definite=False)
    kap = G.kappa_const(n2, n1)
    prob = O.make_problem(kap, n2, n1, b, shift=c)
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=S.SLAB_MIXED, tol=1e-10, max_iter=20,
                      odd_even=order == "odd_even", shift=_dev(c))
    assert h.negative_pivots() == neg
    f = G.rhs_uniform(n2, n1, 2, 8)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert O.relres(prob, u, f).max() <= 1e-10
    h.free()


def test_diverging_refinement_stops_early():
    """The mixed form on 1024 x 1024 at 40 points per wavelength (cond(A) 3e5):
    the FP32 reduced factorization is too inexact for the refinement to
    contract, the residual grows past the right-hand side, and the solve stops
    there with SLAB_E_NOCONV instead of running every allowed pass."""
    w = G.HELMHOLTZ_1024
    print("case: mixed form, Helmholtz 1024x1024 b=15 ppw=40", flush=True)
    h = S.slab_factor(_dev(w.kappa()), w.n2, w.n1, w.b, w.h, precision=S.SLAB_MIXED,
                      odd_even=True, shift=_dev(w.shift()), max_iter=10)
    with pytest.raises(S.SlabError) as ei:
        S.slab_solve(h, _dev(w.rhs(1)))
    assert ei.value.status == S.SLAB_E_NOCONV
    it, rr = h.last_info.iterations, h.last_info.max_relres
    print(f"  stopped after {it} passes at relres {rr:.2e}", flush=True)
    assert 2 <= it < 10 and not (rr <= 1.0)
    h.free()
