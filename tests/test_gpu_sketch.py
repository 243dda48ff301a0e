"""Matrix-free products with the reduced matrix T (slab_apply_reduced):
y = A_oo x - A_oe A_ee^-1 A_eo x through the stored slab factors, the product
the paper's randomized sketches of T are formed from, against the oracle's
matrix-free product (a sparse LU of all slab interiors) on Gaussian test
vectors.

* Shapes covering every padded block order, b = 1, one slab, a ragged n2.
* FP64 and mixed precision (FP64 slab sweeps): 1e-12 relative per column;
  all-FP32: 1e-5.
* 512 x 512, b = 15 (the differentiation grid): a sketch with s = 6b = 90
  test vectors, FP64, against the oracle; and against T assembled by the
  factorization (exported blocks) applied to the same vectors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import inputs as G
from oracle import slab_oracle as O
from paper_2211_07572_amd import slab as S

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _col_rel(y, ref):
    a = y.transpose(1, 0, 2).reshape(y.shape[1], -1)
    r = ref.transpose(1, 0, 2).reshape(ref.shape[1], -1)
    return np.linalg.norm(a - r, axis=1) / np.linalg.norm(r, axis=1)


CASES = [(40, 48, 7), (70, 96, 15), (130, 128, 31), (33, 24, 1), (97, 64, 63), (50, 16, 15)]


@pytest.mark.parametrize("precision,tol", [(S.SLAB_FP64, 1e-12), (S.SLAB_MIXED, 1e-12),
                                           (S.SLAB_FP32_REFINE, 1e-5)])
@pytest.mark.parametrize("n2,n1,b", CASES)
def test_apply_reduced_matches_oracle(n2, n1, b, precision, tol):
    kap = G.kappa_lognormal(n2, n1, 17)
    prob = O.make_problem(kap, n2, n1, b)
    x = G.gaussian_test_vectors(prob.m, 5, n2, 3)
    ref = O.apply_T(prob, x)
    h = S.slab_factor(_dev(kap), n2, n1, b, precision=precision, odd_even=True)
    y = S.slab_apply_reduced(h, _dev(x)).cpu().numpy()
    err = _col_rel(y, ref).max()
    assert err <= tol, err
    h.free()


def test_sketch_512():
    W = G.ADJOINT_512
    theta = G.grf(W.n2, W.n1, 10, W.h)
    prob = O.make_problem(np.exp(theta), W.n2, W.n1, W.b, W.h)
    s = 6 * W.b
    x = G.gaussian_test_vectors(prob.m, s, W.n2)
    print(f"oracle: matrix-free T on {s} test vectors, 512x512 b=15", flush=True)
    ref = O.apply_T(prob, x)
    h = S.slab_factor(_dev(theta), W.n2, W.n1, W.b, W.h, coef_log=True, keep_reduced=True,
                      odd_even=True)
    y = S.slab_apply_reduced(h, _dev(x)).cpu().numpy()
    err = _col_rel(y, ref).max()
    # the same product from the assembled blocks of the factorization
    yb = np.zeros_like(x)
    for j in range(prob.m):
        Tjj = S.slab_export_reduced(h, 0, j).cpu().numpy()
        yb[j] += x[j] @ Tjj.T
        if j + 1 < prob.m:
            Tup = S.slab_export_reduced(h, 1, j).cpu().numpy()
            yb[j] += x[j + 1] @ Tup.T
            yb[j + 1] += x[j] @ Tup
    errb = _col_rel(y, yb).max()
    print(f"512x512 sketch of {s} columns: vs oracle {err:.2e}, vs assembled T {errb:.2e}",
          flush=True)
    assert err <= 1e-12
    assert errb <= 1e-12
    h.free()
