"""Host-side checks of the C ABI: the library loads, exports every function of
include/slab.h, and rejects bad arguments before any HIP call (these tests
need no GPU)."""
import ctypes
import subprocess

import pytest

from paper_2211_07572_amd import slab as S


@pytest.fixture(scope="module")
def lib():
    return S.load_library()


def test_header_declares_the_four_calls():
    names = S.header_functions()
    for n in ("slab_factor", "slab_solve", "slab_solve_adjoint", "slab_free"):
        assert n in names
    assert len(names) == len(set(names))


def test_every_header_symbol_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in S.header_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


@pytest.mark.parametrize("n2,n1,b,h,code", [
    (16, 64, 7, 0.1, S.SLAB_OK),
    (16, 63, 7, 0.1, S.SLAB_E_INVALID),   # n1 not a multiple of b+1
    (0, 64, 7, 0.1, S.SLAB_E_INVALID),    # empty interface
    (16, 64, -1, 0.1, S.SLAB_E_INVALID),  # b < 0
    (16, 64, 0, 0.1, S.SLAB_OK),          # b = 0: chosen by the autotuner
    (16, 66, 0, 0.1, S.SLAB_E_INVALID),   # b = 0 needs n1 % 4 == 0
    (16, 128, 127, 0.1, S.SLAB_E_INVALID),  # b > 63
    (16, 64, 7, 0.0, S.SLAB_E_INVALID),   # h <= 0
    (16, 64, 7, float("nan"), S.SLAB_E_INVALID),
    (1, 2, 1, 0.5, S.SLAB_OK),            # smallest grid
])
def test_check_problem_dims(n2, n1, b, h, code):
    assert S.slab_check_problem(n2, n1, b, h) == code


def test_check_problem_options():
    assert S.slab_check_problem(8, 16, 7, 0.1, precision=7) == S.SLAB_E_INVALID
    assert S.slab_check_problem(8, 16, 7, 0.1, tol=0.0) == S.SLAB_E_INVALID
    assert S.slab_check_problem(8, 16, 7, 0.1, max_iter=0) == S.SLAB_E_INVALID
    assert S.slab_check_problem(8, 16, 7, 0.1, flags=64) == S.SLAB_E_INVALID
    assert S.slab_check_problem(8, 16, 7, 0.1, kappa_ptr=0) == S.SLAB_E_INVALID
    assert S.slab_check_problem(8, 16, 7, 0.1, precision=S.SLAB_FP32_REFINE,
                                flags=S.SLAB_KEEP_REDUCED | S.SLAB_COEF_LOG) == S.SLAB_OK


def test_factor_rejects_before_device_work(lib):
    prob = S.slab_problem(63, 16, 7, 0.1, ctypes.c_void_p(1))
    opts = S.slab_options(S.SLAB_FP64, 1e-10, 10, 0)
    out = ctypes.c_void_p(123)
    rc = lib.slab_factor(ctypes.byref(prob), ctypes.byref(opts), None, ctypes.byref(out), None)
    assert rc == S.SLAB_E_INVALID
    assert out.value is None
    assert b"multiple" in lib.slab_last_error()
    rc = lib.slab_factor(ctypes.byref(prob), ctypes.byref(opts), None, None, None)
    assert rc == S.SLAB_E_INVALID


def test_null_handles(lib):
    assert lib.slab_free(None) == S.SLAB_OK
    assert lib.slab_solve(None, ctypes.c_void_p(8), ctypes.c_void_p(16), 1, 1, None, None) == S.SLAB_E_INVALID
    assert lib.slab_solve_adjoint(None, ctypes.c_void_p(8), ctypes.c_void_p(16), 1, 1, None, None) == S.SLAB_E_INVALID
    v = ctypes.c_int64()
    assert lib.slab_query(None, 0, ctypes.byref(v)) == S.SLAB_E_INVALID
    assert lib.slab_export_reduced(None, 0, 0, ctypes.c_void_p(8), None) == S.SLAB_E_INVALID
    assert lib.slab_kappa_grad(None, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, 0, ctypes.c_void_p(8), None) == S.SLAB_E_INVALID
    arr = (ctypes.c_double * 1)()
    assert lib.slab_residual(None, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, arr, None) == S.SLAB_E_INVALID
    assert lib.slab_index_maps(10, 4, 3, None, None, None, None, None, None) == S.SLAB_E_INVALID


def test_autotune_rejects_before_device_work(lib):
    b = ctypes.c_int32(-7)
    prob = S.slab_problem(66, 16, 0, 0.1, ctypes.c_void_p(1))
    assert lib.slab_autotune(ctypes.byref(prob), None, 1, None, ctypes.byref(b), None) == S.SLAB_E_INVALID
    prob = S.slab_problem(64, 16, 0, 0.1, ctypes.c_void_p(1))
    assert lib.slab_autotune(ctypes.byref(prob), None, 0, None, ctypes.byref(b), None) == S.SLAB_E_INVALID
    assert lib.slab_autotune(None, None, 1, None, ctypes.byref(b), None) == S.SLAB_E_INVALID
    assert b.value == -7


def test_batch_rejects_before_device_work(lib):
    out = ctypes.c_void_p(5)
    probs = (S.slab_problem * 2)(S.slab_problem(64, 16, 7, 0.1, ctypes.c_void_p(1)),
                                 S.slab_problem(63, 16, 7, 0.1, ctypes.c_void_p(1)))
    assert lib.slab_factor_batch(probs, 2, None, None, ctypes.byref(out), None) == S.SLAB_E_INVALID
    assert out.value is None
    assert b"problem 1" in lib.slab_last_error()
    assert lib.slab_factor_batch(probs, 0, None, None, ctypes.byref(out), None) == S.SLAB_E_INVALID
    assert lib.slab_batch_free(None) == S.SLAB_OK
