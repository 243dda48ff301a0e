"""slab_solve_noalloc: the allocation-free variant of slab_solve (its solve
buffers and plan tables live in the library's fixed device scratch array)
against slab_solve on the same handle and right-hand sides, through the C ABI.

Two calls in a row, the second on a smaller problem, so the second call runs
in an array that still holds the first call's contents; a request larger than
the array is refused on the host before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import inputs as G
from paper_2211_07572_amd import slab as S

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _col_rel(u, ref):
    u = u.reshape(u.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(u - ref, axis=1) / np.linalg.norm(ref, axis=1)


CASES = [
    # (n2, n1, b, precision, odd_even, nrhs, seed): the second is smaller
    (512, 512, 15, S.SLAB_FP64, True, 2, 0),
    (130, 128, 31, S.SLAB_MIXED, False, 1, 3),
]


def test_noalloc_matches_slab_solve_two_calls():
    handles = []
    for n2, n1, b, prec, oe, nrhs, seed in CASES:
        print(f"noalloc case: n2={n2} n1={n1} b={b} precision={prec} odd_even={oe} nrhs={nrhs}",
              flush=True)
        kap = _dev(G.kappa_lognormal(n2, n1, seed))
        h = S.slab_factor(kap, n2, n1, b, precision=prec, tol=1e-10, odd_even=oe)
        handles.append(h)
        f = _dev(G.rhs_uniform(n2, n1, nrhs, G.SEED_RHS + seed))
        u_ref = S.slab_solve(h, f)
        info_ref = (h.last_info.iterations, h.last_info.max_relres)
        out = torch.full_like(f, float("nan"))
        u = S.slab_solve_noalloc(h, f, out=out)
        info = (h.last_info.iterations, h.last_info.max_relres)
        torch.cuda.synchronize()
        a, r = u.cpu().numpy(), u_ref.cpu().numpy()
        err = _col_rel(a, r).max()
        print(f"  max column difference {err:.2e}, bit-equal {np.array_equal(a, r)}, "
              f"passes {info} vs {info_ref}", flush=True)
        assert err <= 1e-12
        assert info[0] == info_ref[0]
        assert info[1] == pytest.approx(info_ref[1], rel=1e-6, abs=1e-15)
        # the handle's own workspace is untouched: slab_solve still agrees
        u2 = S.slab_solve(h, f).cpu().numpy()
        assert np.array_equal(u2, r)
    for h in handles:
        h.free()


def test_noalloc_refuses_oversize_request():
    n2, n1, b = 512, 512, 15
    kap = _dev(G.kappa_lognormal(n2, n1, 0))
    h = S.slab_factor(kap, n2, n1, b, odd_even=True)
    f = torch.zeros((40, n1, n2), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SlabError) as ei:
        S.slab_solve_noalloc(h, f, out=torch.empty_like(f))
    assert ei.value.status == S.SLAB_E_INVALID
    assert "scratch array" in str(ei.value)
    # the handle still solves normally afterwards
    f1 = _dev(G.rhs_uniform(n2, n1, 1, G.SEED_RHS))
    S.slab_solve(h, f1)
    h.free()


def test_noalloc_signed_factorization():
    """A Helmholtz term with indefinite slabs and T (pivots of either sign,
    pivot signs kept by the handle): the allocation-free solve matches
    slab_solve on the same handle."""
    n2, n1, b = 96, 96, 7
    print("noalloc case: Helmholtz 96x96 b=7, 10 points per wavelength", flush=True)
    c = G.helmholtz_shift(n2, n1, 10.0)
    h = S.slab_factor(_dev(G.kappa_const(n2, n1)), n2, n1, b, odd_even=True, shift=_dev(c))
    assert h.negative_pivots() > 0
    f = _dev(G.rhs_uniform(n2, n1, 2, 21))
    r = S.slab_solve(h, f).cpu().numpy()
    a = S.slab_solve_noalloc(h, f, out=torch.full_like(f, float("nan"))).cpu().numpy()
    assert _col_rel(a, r).max() <= 1e-12
    h.free()
