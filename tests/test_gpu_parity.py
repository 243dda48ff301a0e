"""GPU parity of the HIP slab solver against the FP64 CPU oracle.

Every test calls the C ABI through the thin binding and compares with the
oracle on the same seeded inputs.  Tolerances: FP64 results within 1e-12
relative (per block / per column); mixed precision is judged by the
relative residual 1e-10 recomputed on the host with the oracle's A.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import inputs as G
from oracle import slab_oracle as O
from paper_2211_07572_amd import slab as S

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _col_rel(u, ref):
    u = u.reshape(u.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(u - ref, axis=1) / np.linalg.norm(ref, axis=1)


# (n2, n1, b): ragged interface lengths over 64-wide tiles, every padded block
# order (16, 32) and b = 1, a single slab, and the 1-D case n2 = 1.
CASES = [
    (200, 80, 7),
    (130, 128, 31),
    (70, 96, 15),
    (33, 24, 1),
    (45, 40, 3),
    (5, 4, 3),
    (1, 8, 1),
    (64, 64, 7),
    (40, 128, 63),
    (70, 96, 47),
    (300, 48, 15),  # pivot blocks over two 128-column panels (GEMM updates at two depths)
]
# odd-even order: odd m and a deeper level tree on top of the cases above
CASES_OE = CASES + [(40, 52, 3), (64, 256, 7)]
ORDERS = ["sweep", "odd_even"]


def _pivot(fac, j):
    return fac.s2.pivot(j) if isinstance(fac.s2, O.OddEven) else fac.s2.S[j]


def _cases(order):
    return CASES_OE if order == "odd_even" else CASES


ORDER_CASES = [(o,) + c for o in ORDERS for c in _cases(o)]


@pytest.mark.parametrize("n2,n1,b", [(64, 64, 7), (1, 2, 1), (1024, 1024, 31), (2048, 4096, 31),
                                     (7, 30, 4)])
def test_index_maps_bit_exact(n2, n1, b):
    got = S.slab_index_maps(n2, n1, b)
    ref = O.index_maps(n2, n1, b)
    assert got["m"] == ref["m"]
    for key in ("col_kind", "slab_of_col", "local_of_col", "perm_even", "perm_odd"):
        g = got[key].cpu().numpy()
        assert g.dtype in (np.int32, np.int64)
        assert np.array_equal(g, ref[key]), key


@pytest.mark.parametrize("order,n2,n1,b", ORDER_CASES)
def test_fp64_reduced_blocks_and_solve(order, n2, n1, b):
    print(f"case fp64 {order} n2={n2} n1={n1} b={b}", flush=True)
    kap = G.kappa_lognormal(n2, n1, 3)
    prob = O.make_problem(kap, n2, n1, b)
    fac = O.factor(prob, order=order)
    h = S.slab_factor(_dev(kap), n2, n1, b, keep_reduced=True, odd_even=order == "odd_even")
    for j in range(prob.m):
        T = S.slab_export_reduced(h, 0, j).cpu().numpy()
        assert _rel_fro(T, fac.s1.T_diag[j]) <= 1e-12, ("T_jj", j)
        Sj = S.slab_export_reduced(h, 2, j).cpu().numpy()
        assert _rel_fro(Sj, _pivot(fac, j)) <= 1e-12, ("pivot", j)
    for j in range(prob.m - 1):
        Tu = S.slab_export_reduced(h, 1, j).cpu().numpy()
        assert _rel_fro(Tu, fac.s1.T_up[j]) <= 1e-12, ("T_j,j+1", j)
    f = G.rhs_uniform(n2, n1, 3, 7)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    u_ref = O.solve(fac, f)
    assert _col_rel(u, u_ref).max() <= 1e-12
    assert O.relres(prob, u, f).max() <= 1e-12
    assert h.last_info.iterations == 1
    h.free()


@pytest.mark.parametrize("precision", [S.SLAB_FP32_REFINE, S.SLAB_MIXED])
@pytest.mark.parametrize("order,n2,n1,b", ORDER_CASES)
def test_fp32_refinement(order, n2, n1, b, precision):
    print(f"case precision={precision} {order} n2={n2} n1={n1} b={b}", flush=True)
    kap = G.kappa_lognormal(n2, n1, 4)
    prob = O.make_problem(kap, n2, n1, b)
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=precision, tol=1e-10,
                      keep_reduced=True, odd_even=order == "odd_even")
    f = G.rhs_normal(n2, n1, 4, 8)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    rr = O.relres(prob, u, f)
    assert rr.max() <= 1e-10, rr
    assert h.last_info.max_relres <= 1e-10
    assert 1 <= h.last_info.iterations <= 6
    if precision == S.SLAB_MIXED:
        # the reduced solve is refined against the FP64 reduced matrix, so the
        # FP64 slab solves need no second pass
        assert h.last_info.iterations == 1
    # FP32 slab work with an FP64 sum gives T to about 1e-6; FP64 slab work gives
    # T to FP64 accuracy (the block factorization itself runs in FP32 in both)
    fac = O.factor(prob, order=order)
    errT = max(_rel_fro(S.slab_export_reduced(h, 0, j).cpu().numpy(), fac.s1.T_diag[j])
               for j in range(prob.m))
    assert errT <= (1e-5 if precision == S.SLAB_FP32_REFINE else 1e-12), errT
    errS = max(_rel_fro(S.slab_export_reduced(h, 2, j).cpu().numpy(), _pivot(fac, j))
               for j in range(prob.m))
    assert errS <= 1e-4, errS
    h.free()


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("n2,n1,b", [(200, 80, 7), (70, 96, 15), (33, 24, 1)])
def test_adjoint_matches_oracle(n2, n1, b, order):
    kap = G.kappa_lognormal(n2, n1, 5)
    prob = O.make_problem(kap, n2, n1, b)
    h = S.slab_factor(_dev(kap), n2, n1, b, odd_even=order == "odd_even")
    g = G.rhs_normal(n2, n1, 2, 9)
    lam = S.slab_solve_adjoint(h, _dev(g)).cpu().numpy()
    lam_ref = O.solve_adjoint(prob, g, order=order)
    assert _col_rel(lam, lam_ref).max() <= 1e-12
    u = S.slab_solve(h, _dev(g)).cpu().numpy()
    assert _col_rel(lam, u).max() <= 1e-12          # A is symmetric
    f = G.rhs_uniform(n2, n1, 2, 10)
    uf = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert abs(np.sum(uf * g) - np.sum(f * lam)) <= 1e-11 * abs(np.sum(uf * g))
    h.free()


def _write_block_inverses(h, values):
    """Overwrite the handle's stored block inverses Gl_r (slab_query 8) with
    values (a device tensor of the stored element type and count)."""
    L = S.load_library()
    L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    L.hipMemcpy.restype = ctypes.c_int
    L.hipDeviceSynchronize.restype = ctypes.c_int
    torch.cuda.synchronize()
    nbytes = values.numel() * values.element_size()
    # hipMemcpyDefault (4): the direction follows from the addresses
    assert L.hipMemcpy(ctypes.c_void_p(h.query(8)), ctypes.c_void_p(values.data_ptr()), nbytes, 4) == 0
    assert L.hipDeviceSynchronize() == 0


def _read_block_inverses(h, count, dtype):
    L = S.load_library()
    L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    L.hipMemcpy.restype = ctypes.c_int
    out = torch.empty(count, dtype=dtype, device=DEV)
    torch.cuda.synchronize()
    assert L.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(h.query(8)),
                       out.numel() * out.element_size(), 4) == 0
    torch.cuda.synchronize()
    return out


def _perturb_block_inverses(h, n2, n1, b, precision, seed=31):
    """Add seeded non-symmetric noise to every stored Gl_r of handle h
    (entries of 0.05 max|Gl| / sqrt(b): the perturbation's norm stays near a
    tenth of the blocks', so the row recursions of the sweeps do not grow
    beyond the FP32 range over n2 rows)."""
    m, BP = n1 // (b + 1), (16 if b <= 16 else (32 if b <= 32 else 64))
    dt = torch.float32 if precision == S.SLAB_FP32_REFINE else torch.float64
    gl = _read_block_inverses(h, m * n2 * BP * BP, dt).view(m, n2, BP, BP)
    rng = np.random.default_rng(seed)
    scale = float(gl[:, :, :b, :b].abs().amax())
    pert = torch.as_tensor(rng.standard_normal((m, n2, b, b)), dtype=dt, device=DEV)
    gl[:, :, :b, :b] += 0.05 / np.sqrt(b) * scale * pert
    _write_block_inverses(h, gl.reshape(-1))


def _transpose_errors(Mf, Ma):
    """(|M_adj - M^T|, |M - M^T|) relative to max |M|."""
    assert np.isfinite(Mf).all() and np.isfinite(Ma).all()
    norm = np.abs(Mf).max()
    return np.abs(Ma - Mf.T).max() / norm, np.abs(Mf - Mf.T).max() / norm


# The operator is symmetric, so its slab block inverses are too and a slip
# between Gl_r and its transpose in the transposed sweeps would not change any
# adjoint result.  Here the stored Gl_r are replaced by non-symmetric ones:
# one solve pass is then a fixed linear map M of the right-hand side, and the
# adjoint solve must apply exactly M^T.  Both maps are formed column by column
# on every grid node (identity right-hand sides).
@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("precision,tol", [(S.SLAB_FP64, 1e-12), (S.SLAB_MIXED, 1e-5),
                                           (S.SLAB_FP32_REFINE, 1e-5)])
@pytest.mark.parametrize("n2,n1,b", [(40, 32, 7), (40, 32, 15), (36, 64, 31), (20, 96, 47)])
def test_adjoint_is_transpose_with_nonsymmetric_block_inverses(n2, n1, b, precision, tol, order):
    kap = G.kappa_lognormal(n2, n1, 21)
    # one pass per solve: u = M f, lambda = M^T g, whatever the residual
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=precision, tol=1e300, max_iter=1,
                      odd_even=order == "odd_even")
    _perturb_block_inverses(h, n2, n1, b, precision)
    N = n1 * n2
    E = torch.eye(N, dtype=torch.float64, device=DEV).view(N, n1, n2)
    Mf = S.slab_solve(h, E).reshape(N, N).cpu().numpy()           # row k = (M e_k)^T
    Ma = S.slab_solve_adjoint(h, E).reshape(N, N).cpu().numpy()   # row k = (M^T e_k)^T
    err, asym = _transpose_errors(Mf, Ma)
    print(f"\n  case: n2={n2} n1={n1} b={b} precision={precision} {order}: "
          f"|M_adj - M^T| {err:.2e}, |M - M^T| {asym:.2e} (relative to max |M|)")
    assert asym >= 100 * tol, asym    # the perturbation is seen by the check
    assert err <= tol, err
    h.free()


# The same through the batched entry points: three problems of the three
# padded block orders in the grouped launches of one batch.
@pytest.mark.parametrize("precision,tol", [(S.SLAB_FP64, 1e-12), (S.SLAB_FP32_REFINE, 1e-5)])
def test_batch_adjoint_is_transpose_with_nonsymmetric_block_inverses(precision, tol):
    dims = [(40, 32, 7), (36, 64, 31), (20, 96, 47)]
    kaps = [_dev(G.kappa_lognormal(n2, n1, 22 + i)) for i, (n2, n1, _) in enumerate(dims)]
    bt = S.slab_factor_batch(kaps, dims, precision=precision, tol=1e300, max_iter=1)
    for i, (n2, n1, b) in enumerate(dims):
        _perturb_block_inverses(bt.handle(i), n2, n1, b, precision, seed=40 + i)
    Es = [torch.eye(n1 * n2, dtype=torch.float64, device=DEV).view(n1 * n2, n1, n2)
          for n2, n1, _ in dims]
    Mfs = S.slab_solve_batch(bt, Es)
    Mas = S.slab_solve_adjoint_batch(bt, Es)
    for (n2, n1, b), Mf, Ma in zip(dims, Mfs, Mas):
        N = n1 * n2
        err, asym = _transpose_errors(Mf.reshape(N, N).cpu().numpy(), Ma.reshape(N, N).cpu().numpy())
        print(f"\n  case: batch n2={n2} n1={n1} b={b} precision={precision}: "
              f"|M_adj - M^T| {err:.2e}, |M - M^T| {asym:.2e} (relative to max |M|)")
        assert asym >= 100 * tol, asym
        assert err <= tol, err
    bt.free()


def test_gradient_kernel_matches_oracle():
    n2, n1, b = 40, 48, 7
    theta = G.grf(n2, n1, 12)
    prob = O.make_problem(np.exp(theta), n2, n1, b)
    f = G.rhs_uniform(n2, n1, 2, 11)
    fac = O.factor(prob)
    u = O.solve(fac, f)
    lam = O.solve_adjoint(prob, u - 0.5)
    ref = O.kappa_grad(prob, u, lam)
    h = S.slab_factor(_dev(theta), n2, n1, b, coef_log=True)
    g1 = S.slab_kappa_grad(h, _dev(u), _dev(lam), mode=1).cpu().numpy()
    assert np.abs(g1 - ref).max() <= 1e-12 * np.abs(ref).max()
    g0 = S.slab_kappa_grad(h, _dev(u), _dev(lam), mode=0).cpu().numpy()
    assert np.abs(g0 * np.exp(theta) - ref).max() <= 1e-12 * np.abs(ref).max()
    h.free()


def test_autograd_gradient_vs_central_fd():
    n2, n1, b = 14, 16, 3
    h_ = 1.0 / (n2 + 1)
    theta0 = G.grf(n2, n1, 13, h_)
    f = _dev(G.rhs_uniform(n2, n1, 1, 12))
    u_obs = _dev(O.solve(O.factor(O.make_problem(np.exp(G.grf(n2, n1, 1, h_)), n2, n1, b)),
                         G.rhs_uniform(n2, n1, 1, 12)))

    def loss(th):
        u = S.solve_theta(th, f, n2, n1, b)
        return 0.5 * ((u - u_obs) ** 2).sum()

    th = _dev(theta0).requires_grad_(True)
    L = loss(th)
    (grad,) = torch.autograd.grad(L, th)
    grad = grad.cpu().numpy()
    rng = np.random.default_rng(G.SEED_FD_NODES)
    eps = 1e-6
    gmax = np.abs(grad).max()
    for _ in range(12):
        i, j = int(rng.integers(1, n1 + 1)), int(rng.integers(1, n2 + 1))
        tp = theta0.copy(); tp[i, j] += eps
        tm = theta0.copy(); tm[i, j] -= eps
        with torch.no_grad():
            fd = (loss(_dev(tp)).item() - loss(_dev(tm)).item()) / (2 * eps)
        assert abs(fd - grad[i, j]) <= 1e-5 * gmax, (i, j, fd, grad[i, j])


def test_poisson_64_closed_form():
    """kappa = 1 on 64 x 64, b = 7: T against the sine-mode closed form."""
    n2 = n1 = 64
    b = 7
    h = 1.0 / 65
    hd = S.slab_factor(_dev(G.kappa_const(n2, n1)), n2, n1, b, h, keep_reduced=True)
    i = np.arange(1, n2 + 1)
    Q = np.sqrt(2.0 / (n2 + 1)) * np.sin(np.pi * np.outer(i, i) / (n2 + 1))
    a = 4 - 2 * np.cos(np.pi * i / (n2 + 1))
    x = a / 2
    U = [np.ones_like(x), 2 * x]
    for _ in range(b):
        U.append(2 * x * U[-1] - U[-2])
    both = Q @ np.diag(a - 2 * U[b - 1] / U[b]) @ Q / h ** 2
    last = Q @ np.diag(a - U[b - 1] / U[b]) @ Q / h ** 2
    off = -Q @ np.diag(1 / U[b]) @ Q / h ** 2
    for j in range(8):
        ref = both if j < 7 else last
        assert _rel_fro(S.slab_export_reduced(hd, 0, j).cpu().numpy(), ref) <= 1e-13
    for j in range(7):
        assert _rel_fro(S.slab_export_reduced(hd, 1, j).cpu().numpy(), off) <= 1e-13
    f = G.rhs_uniform(n2, n1, 1, G.SEED_RHS)
    u = S.slab_solve(hd, _dev(f)).cpu().numpy()
    u_ref = O.solve(O.factor(O.make_problem(G.kappa_const(n2, n1), n2, n1, b, h)), f)
    assert _col_rel(u, u_ref).max() <= 1e-12
    hd.free()


def test_error_paths():
    n2, n1, b = 16, 16, 3
    kap = G.kappa_lognormal(n2, n1, 0)
    bad = kap.copy(); bad[5, 5] = 0.0
    with pytest.raises(S.SlabError) as e:
        S.slab_factor(_dev(bad), n2, n1, b)
    assert e.value.status == S.SLAB_E_INVALID
    bad = kap.copy(); bad[3, 7] = np.nan
    with pytest.raises(S.SlabError) as e:
        S.slab_factor(_dev(bad), n2, n1, b)
    assert e.value.status == S.SLAB_E_INVALID
    # one FP32 pass cannot reach 1e-14: non-convergence is reported, u is the iterate
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=S.SLAB_FP32_REFINE, tol=1e-14, max_iter=1)
    f = _dev(G.rhs_uniform(n2, n1, 1, 1))
    with pytest.raises(S.SlabError) as e:
        S.slab_solve(h, f)
    assert e.value.status == S.SLAB_E_NOCONV
    assert h.last_info.iterations == 1 and h.last_info.max_relres > 1e-14
    h.free()


def test_run_to_run_determinism():
    n2, n1, b = 130, 128, 31
    kap = _dev(G.kappa_lognormal(n2, n1, 6))
    f = _dev(G.rhs_normal(n2, n1, 3, 2))
    outs = []
    for _ in range(2):
        h = S.slab_factor(kap, n2, n1, b, precision=S.SLAB_FP32_REFINE)
        outs.append(S.slab_solve(h, f).cpu().numpy())
        h.free()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("order", ORDERS)
def test_many_rhs_column_groups(order):
    """nrhs = 40 crosses the 16-column sweep and product column groups."""
    n2, n1, b = 70, 48, 7
    kap = G.kappa_lognormal(n2, n1, 7)
    prob = O.make_problem(kap, n2, n1, b)
    h = S.slab_factor(_dev(kap), n2, n1, b, odd_even=order == "odd_even")
    f = G.rhs_uniform(n2, n1, 40, 3)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert _col_rel(u, O.solve(O.factor(prob), f)).max() <= 1e-12
    h.free()


# ---------------------------------------------------- batches of uneven problems

BATCH_DIMS = [(40, 48, 7, 2), (70, 96, 15, 1), (130, 128, 31, 3), (33, 24, 1, 4), (64, 64, 7, 5),
              (5, 4, 3, 1), (96, 160, 15, 2)]


def _batch_inputs(dims, seed0):
    kaps = [G.kappa_lognormal(n2, n1, seed0 + i) for i, (n2, n1, b, _) in enumerate(dims)]
    fs = [G.rhs_uniform(n2, n1, nr, seed0 + 50 + i) for i, (n2, n1, b, nr) in enumerate(dims)]
    return kaps, fs


@pytest.mark.parametrize("order", ORDERS)
def test_batch_fp64_matches_oracle(order):
    """Uneven problems (three padded block orders, 1-5 right-hand sides) factored
    and solved as one batch equal the oracle problem by problem."""
    kaps, fs = _batch_inputs(BATCH_DIMS, 20)
    bt = S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in BATCH_DIMS],
                             precision=S.SLAB_FP64, odd_even=order == "odd_even",
                             keep_reduced=True)
    us = S.slab_solve_batch(bt, [_dev(f) for f in fs])
    for i, (n2, n1, b, nr) in enumerate(BATCH_DIMS):
        print(f"batch problem {i}: n2={n2} n1={n1} b={b} nrhs={nr}", flush=True)
        prob = O.make_problem(kaps[i], n2, n1, b)
        fac = O.factor(prob, order=order)
        assert _col_rel(us[i].cpu().numpy(), O.solve(fac, fs[i])).max() <= 1e-12, i
        h = bt.handle(i)
        for j in range(prob.m):
            Sj = S.slab_export_reduced(h, 2, j).cpu().numpy()
            assert _rel_fro(Sj, _pivot(fac, j)) <= 1e-12, (i, j)
    bt.free()


@pytest.mark.parametrize("precision", [S.SLAB_FP32_REFINE, S.SLAB_MIXED])
def test_batch_refinement(precision):
    kaps, fs = _batch_inputs(BATCH_DIMS, 40)
    bt = S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in BATCH_DIMS],
                             precision=precision, tol=1e-10)
    us = S.slab_solve_batch(bt, [_dev(f) for f in fs])
    for i, (n2, n1, b, nr) in enumerate(BATCH_DIMS):
        prob = O.make_problem(kaps[i], n2, n1, b)
        rr = O.relres(prob, us[i].cpu().numpy(), fs[i])
        assert rr.max() <= 1e-10, (i, rr)
        assert 1 <= bt.last_infos[i].iterations <= 6
    bt.free()


def test_batch_graph_replays_match_eager():
    """The captured refinement passes, replayed on later calls with eager work
    and synchronizations in between, give exactly the eager batch's results."""
    dims = BATCH_DIMS[:5]
    kaps, fs = _batch_inputs(dims, 60)
    kd = [_dev(k) for k in kaps]
    fd = [_dev(f) for f in fs]
    eager = S.slab_factor_batch(kd, [d[:3] for d in dims], precision=S.SLAB_MIXED)
    ref = [u.cpu().numpy() for u in S.slab_solve_batch(eager, fd)]
    ref_it = [inf.iterations for inf in eager.last_infos]
    eager.free()
    bt = S.slab_factor_batch(kd, [d[:3] for d in dims], precision=S.SLAB_MIXED, graph=True)
    outs = [torch.empty_like(f) for f in fd]
    for rep in range(3):
        for o in outs:
            o.fill_(float(rep + 1))          # eager work between the replays
        torch.cuda.synchronize()
        us = S.slab_solve_batch(bt, fd, outs=outs)
        torch.cuda.synchronize()
        for i in range(len(dims)):
            assert np.array_equal(us[i].cpu().numpy(), ref[i]), (rep, i)
            assert bt.last_infos[i].iterations == ref_it[i]
    bt.free()


def test_batch_graph_after_workspace_regrow():
    """A call with more right-hand sides on one problem of a graph batch gives
    that problem a new solve workspace; the next batch solve must not replay a
    graph that still points at the old one."""
    dims = BATCH_DIMS[:3]
    kaps, fs = _batch_inputs(dims, 70)
    fd = [_dev(f) for f in fs]
    bt = S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in dims],
                             precision=S.SLAB_MIXED, graph=True)
    S.slab_solve_batch(bt, fd)
    n2, n1, b, nr = dims[0]
    fbig = G.rhs_uniform(n2, n1, nr + 1, 71)
    ubig = np.zeros_like(fbig)
    rr0 = S.slab_residual(bt.handle(0), _dev(fbig), _dev(ubig))   # grows problem 0's workspace
    assert np.allclose(rr0, 1.0)
    us = S.slab_solve_batch(bt, fd)
    for i, (n2, n1, b, nr) in enumerate(dims):
        rr = O.relres(O.make_problem(kaps[i], n2, n1, b), us[i].cpu().numpy(), fs[i])
        assert rr.max() <= 1e-10, (i, rr)
        assert bt.last_infos[i].max_relres <= 1e-10, i
    bt.free()


def test_batch_reports_failing_problem():
    dims = BATCH_DIMS[:3]
    kaps, _ = _batch_inputs(dims, 80)
    kaps[1] = kaps[1].copy()
    kaps[1][3, 4] = -1.0
    with pytest.raises(S.SlabError) as ei:
        S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in dims])
    assert ei.value.status == S.SLAB_E_INVALID
    assert "problem 1" in str(ei.value)


# ------------------------------------------------------------------- autotuner

def test_autotune_width_is_fastest_measured_and_used():
    n2, n1 = 96, 256
    kap = G.kappa_lognormal(n2, n1, 90)
    b, times = S.slab_autotune(_dev(kap), n2, n1, precision=S.SLAB_MIXED, odd_even=True)
    measured = {w: t for w, t in times.items() if t is not None}
    assert b in measured and measured[b] == min(measured.values())
    assert all(n1 % (w + 1) == 0 for w in measured)
    h = S.slab_factor(_dev(kap), n2, n1, 0, precision=S.SLAB_MIXED, odd_even=True)
    assert h.b == b
    f = G.rhs_uniform(n2, n1, 2, 91)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert O.relres(O.make_problem(kap, n2, n1, b), u, f).max() <= 1e-10
    h.free()


def test_batch_with_autotuned_widths():
    dims = [(40, 64, 0, 1), (64, 96, 7, 2), (33, 128, 0, 3)]
    kaps, fs = _batch_inputs(dims, 95)
    bt = S.slab_factor_batch([_dev(k) for k in kaps], [d[:3] for d in dims],
                             precision=S.SLAB_MIXED)
    us = S.slab_solve_batch(bt, [_dev(f) for f in fs])
    for i, (n2, n1, b, nr) in enumerate(dims):
        bi = bt.handle(i).b
        assert bi > 0 and n1 % (bi + 1) == 0
        if b:
            assert bi == b
        rr = O.relres(O.make_problem(kaps[i], n2, n1, bi), us[i].cpu().numpy(), fs[i])
        assert rr.max() <= 1e-10, (i, rr)
    bt.free()


# ------------------------------------------------- segmented slab recursion

SEG_CASES = [(130, 128, 7), (300, 48, 15), (200, 96, 31), (97, 64, 3)]


@pytest.mark.parametrize("warm", [None, "1"])
@pytest.mark.parametrize("n2,n1,b", SEG_CASES)
def test_segmented_slab_factor(monkeypatch, n2, n1, b, warm):
    """The slab recursion cut into segments of 32 row steps that start early
    from a zero inverse (warm-up of 6 (b+1) steps): T, the pivot blocks and u
    equal the oracle's to 1e-12.  With a one-step warm-up the segments cannot
    agree with their predecessors, so every segmented chain must be caught by
    the check and recomputed in one piece; the results are still exact."""
    monkeypatch.setenv("SLAB_FACTOR_SEG", "32")
    if warm:
        monkeypatch.setenv("SLAB_FACTOR_WARM", warm)
    kap = G.kappa_lognormal(n2, n1, 7)
    prob = O.make_problem(kap, n2, n1, b)
    fac = O.factor(prob, order="odd_even")
    h = S.slab_factor(_dev(kap), n2, n1, b, keep_reduced=True, odd_even=True)
    for j in range(prob.m):
        assert _rel_fro(S.slab_export_reduced(h, 0, j).cpu().numpy(), fac.s1.T_diag[j]) <= 1e-12
        assert _rel_fro(S.slab_export_reduced(h, 2, j).cpu().numpy(), fac.s2.pivot(j)) <= 1e-12
    for j in range(prob.m - 1):
        assert _rel_fro(S.slab_export_reduced(h, 1, j).cpu().numpy(), fac.s1.T_up[j]) <= 1e-12
    f = G.rhs_uniform(n2, n1, 2, 9)
    u = S.slab_solve(h, _dev(f)).cpu().numpy()
    assert _col_rel(u, O.solve(fac, f)).max() <= 1e-12
    h.free()
