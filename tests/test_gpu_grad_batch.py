"""Batched differentiation on the GPU: B coefficient fields theta_i = log
kappa_i on one grid, factored and solved together, the adjoint solves and the
coefficient gradients of the loss L_i = 1/2 ||u_i - u_obs||^2 as batches.

* 512 x 512, b = 15, 16 fields (GRF seeds 10..25), one shared uniform load,
  u_obs from a second field plus 1% noise (computed by the oracle's sparse
  direct solve): the gradient of fields 0 and 15 against the oracle's
  adjoint gradient (u and lambda from sparse direct solves of A and A^T), and
  every field against central differences (step 1e-6 on theta) at 32 random
  interior nodes, the perturbed losses evaluated by batched GPU solves.
* A small uneven batch: the batched adjoint solves equal the single-handle
  ones and the oracle's transposed elimination; the batched gradient kernel
  equals the oracle's formula on the same u and lambda.
* The batched autograd function equals the explicit calls.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import inputs as G
from oracle import slab_oracle as O
from paper_2211_07572_amd import slab as S

pytestmark = pytest.mark.gpu

DEV = "cuda"
W = G.ADJOINT_512
FD_EPS = 1e-6
# Central differences err by a truncation of O(eps^2) plus the rounding error
# of the two loss values divided by 2 eps.  With u accurate to 1e-13 relative
# (asserted against the oracle below) a loss value is off by at most
# ~1e-13 ||u|| ||u - u_obs||, which bounds the rounding term; on this
# workload it is ~1e-3 of max|g| at eps = 1e-6 (measured: 5e-5; the measured
# error falls as 1/eps down to 3e-8 at eps = 1e-3, so rounding dominates).
# A second pass at eps = 1e-3, where truncation dominates, checks 1e-6.
FD_SOLVE_REL = 1e-13
FD_EPS_COARSE = 1e-3
FD_TOL_COARSE = 1e-6
# end-to-end gradient (GPU u and lambda vs sparse direct ones): the solutions
# agree to ~1e-13 relative; the edge products difference neighbouring values,
# which can cost a few digits
GRAD_E2E_TOL = 1e-9


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def c4():
    print("oracle: observation u_obs for the 512x512 differentiation workload", flush=True)
    f = G.rhs_uniform(W.n2, W.n1, 1, G.SEED_RHS)
    kap_obs = G.kappa_lognormal(W.n2, W.n1, G.SEED_KAPPA_OBS, W.h)
    u_clean = O.direct_solve(O.make_problem(kap_obs, W.n2, W.n1, W.b, W.h), f)
    rms = np.sqrt(np.mean(u_clean ** 2))
    u_obs = u_clean + G.DIFF_NOISE_LEVEL * rms * G.noise_normal(W.n2, W.n1, 1)
    thetas = np.stack([G.grf(W.n2, W.n1, s, W.h) for s in G.DIFF_THETA_SEEDS])
    return thetas, f, u_obs


def _losses(thetas, f_dev, uobs_dev):
    """L_i for a stack of fields, by one batched factor + solve (FP64)."""
    B = thetas.shape[0]
    th = [thetas[i] for i in range(B)]
    bt = S.slab_factor_batch(th, [(W.n2, W.n1, W.b, W.h)] * B, precision=S.SLAB_FP64,
                             coef_log=True)
    us = S.slab_solve_batch(bt, [f_dev] * B)
    out = torch.stack([0.5 * ((u - uobs_dev) ** 2).sum() for u in us]).cpu().numpy()
    bt.free()
    return out


def test_c4_batch_gradient(c4):
    thetas, f, u_obs = c4
    B = thetas.shape[0]
    f_dev, uobs_dev = _dev(f), _dev(u_obs)
    theta = _dev(thetas).requires_grad_(True)
    u = S.solve_theta_batch(theta, f_dev, W.n2, W.n1, W.b, W.h)
    loss = 0.5 * ((u - uobs_dev) ** 2).sum()
    loss.backward()
    g = theta.grad.cpu().numpy()
    u_np = u.detach().cpu().numpy()
    print(f"512x512 batch of {B}: loss {loss.item():.6e}", flush=True)
    # oracle: fields 0 and B-1
    for i in (0, B - 1):
        prob = O.make_problem(np.exp(thetas[i]), W.n2, W.n1, W.b, W.h)
        u_or = O.direct_solve(prob, f)
        lam_or = O.direct_solve(prob, u_or - u_obs, transpose=True)
        g_or = O.kappa_grad(prob, u_or, lam_or)
        eu = np.linalg.norm(u_np[i] - u_or) / np.linalg.norm(u_or)
        eg = np.abs(g[i] - g_or).max() / np.abs(g_or).max()
        print(f"  field {i}: u error {eu:.2e}, gradient error {eg:.2e} (max-norm relative)",
              flush=True)
        assert eu <= 1e-12
        assert eg <= GRAD_E2E_TOL
    # central differences at 32 interior nodes of every field
    nodes = G.fd_nodes(W.n2, W.n1, 32)
    for eps in (FD_EPS, FD_EPS_COARSE):
        worst = 0.0
        for i in range(B):
            pert = []
            for (c, r) in nodes:
                for sgn in (1.0, -1.0):
                    t = thetas[i].copy()
                    t[c + 1, r + 1] += sgn * eps
                    pert.append(t)
            L = _losses(_dev(np.stack(pert)), f_dev, uobs_dev).reshape(-1, 2)
            fd = (L[:, 0] - L[:, 1]) / (2 * eps)
            ad = np.array([g[i][c + 1, r + 1] for (c, r) in nodes])
            gmax = np.abs(g[i]).max()
            if eps == FD_EPS:
                rounding = FD_SOLVE_REL * np.linalg.norm(u_np[i]) * np.linalg.norm(u_np[i] - u_obs)
                tol = (rounding / eps) / gmax
            else:
                tol = FD_TOL_COARSE
            err = np.abs(fd - ad).max() / gmax
            worst = max(worst, err / tol)
            assert err <= tol, (i, eps, err, tol)
        print(f"  central differences (eps {eps:g}), {B} fields x 32 nodes: worst error "
              f"{worst:.2e} of its bound", flush=True)


def test_batch_adjoint_and_gradient_kernel():
    dims = [(40, 48, 7), (70, 96, 15), (33, 24, 1)]
    kaps = [G.kappa_lognormal(n2, n1, 20 + i) for i, (n2, n1, b) in enumerate(dims)]
    bt = S.slab_factor_batch([_dev(k) for k in kaps], dims, precision=S.SLAB_FP64)
    gs = [G.rhs_normal(n2, n1, 1 + i, 30 + i) for i, (n2, n1, b) in enumerate(dims)]
    lams = S.slab_solve_adjoint_batch(bt, [_dev(x) for x in gs])
    us = S.slab_solve_batch(bt, [_dev(x) for x in gs])
    grads = S.slab_kappa_grad_batch(bt, us, lams, mode=1)
    for i, (n2, n1, b) in enumerate(dims):
        prob = O.make_problem(kaps[i], n2, n1, b)
        ref = O.solve_adjoint(prob, gs[i])
        lam = lams[i].cpu().numpy()
        assert np.abs(lam - ref).max() <= 1e-12 * np.abs(ref).max()
        single = S.slab_solve_adjoint(bt.handle(i), _dev(gs[i])).cpu().numpy()
        assert np.array_equal(single, lam)
        g_ref = O.kappa_grad(prob, us[i].cpu().numpy(), lam)
        gi = grads[i].cpu().numpy()
        assert np.abs(gi - g_ref).max() <= 1e-12 * np.abs(g_ref).max()
    bt.free()


def test_autograd_batch_equals_explicit_calls():
    n2, n1, b, B = 48, 64, 7, 3
    h = 1.0 / (n2 + 1)
    thetas = np.stack([G.grf(n2, n1, 40 + i, h) for i in range(B)])
    f = G.rhs_uniform(n2, n1, 2, 41)
    target = G.rhs_normal(n2, n1, 2, 42) * 1e-3
    theta = _dev(thetas).requires_grad_(True)
    fd = _dev(f).requires_grad_(True)
    u = S.solve_theta_batch(theta, fd, n2, n1, b, h)
    loss = 0.5 * ((u - _dev(target)) ** 2).sum()
    loss.backward()
    for i in range(B):
        prob = O.make_problem(np.exp(thetas[i]), n2, n1, b, h)
        u_or = O.solve(O.factor(prob), f)
        lam_or = O.solve_adjoint(prob, u_or - target)
        g_or = O.kappa_grad(prob, u_or, lam_or)
        gi = theta.grad[i].cpu().numpy()
        assert np.abs(gi - g_or).max() <= 1e-10 * np.abs(g_or).max()
    # dL/df = sum_i lambda_i for the shared load
    lam_sum = sum(O.solve_adjoint(O.make_problem(np.exp(thetas[i]), n2, n1, b, h),
                                  O.solve(O.factor(O.make_problem(np.exp(thetas[i]), n2, n1, b, h)), f)
                                  - target) for i in range(B))
    gf = fd.grad.cpu().numpy()
    assert np.abs(gf - lam_sum).max() <= 1e-10 * np.abs(lam_sum).max()
