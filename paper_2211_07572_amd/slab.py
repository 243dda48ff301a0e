"""Python binding of the slab solver's C ABI (include/slab.h).

Argument marshalling only: every step of factor and solve runs in the HIP
library libslab.so built in this package.  PyTorch supplies device memory and
the current stream.  If the library is missing the import of this module
still works, but every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libslab.so")
HEADER = os.path.join(os.path.dirname(PKG_DIR), "include", "slab.h")

SLAB_OK = 0
SLAB_E_INVALID = -1
SLAB_E_NOMEM = -2
SLAB_E_BREAKDOWN = -3
SLAB_E_NOCONV = -4
SLAB_E_HIP = -5

SLAB_FP64 = 0
SLAB_FP32_REFINE = 1
SLAB_MIXED = 2

SLAB_KEEP_REDUCED = 1
SLAB_COEF_LOG = 2
SLAB_ODD_EVEN = 4
SLAB_GRAPH = 8

_STATUS_NAMES = {0: "SLAB_OK", -1: "SLAB_E_INVALID", -2: "SLAB_E_NOMEM", -3: "SLAB_E_BREAKDOWN",
                 -4: "SLAB_E_NOCONV", -5: "SLAB_E_HIP"}


class SlabError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class slab_problem(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("b", ctypes.c_int32),
                ("h", ctypes.c_double), ("kappa", ctypes.c_void_p), ("shift", ctypes.c_void_p)]


class slab_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tile", ctypes.c_int32)]


class slab_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("max_relres", ctypes.c_double),
                ("failed_block", ctypes.c_int32)]


_lib = None


def header_functions() -> list[str]:
    """Names of the functions declared in include/slab.h."""
    text = open(HEADER).read()
    return re.findall(r"^\s*(?:int|const char\*)\s+(slab_\w+)\s*\(", text, flags=re.M)


def load_library(path: str = LIB_PATH):
    """Load libslab.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with python -m paper_2211_07572_amd.build_lib")
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.slab_last_error.restype = ctypes.c_char_p
    L.slab_last_error.argtypes = []
    L.slab_check_problem.argtypes = [ctypes.POINTER(slab_problem), ctypes.POINTER(slab_options)]
    L.slab_factor.argtypes = [ctypes.POINTER(slab_problem), ctypes.POINTER(slab_options), vp,
                              ctypes.POINTER(vp), ctypes.POINTER(slab_solve_info)]
    L.slab_solve.argtypes = [vp, vp, vp, i32, i64, vp, ctypes.POINTER(slab_solve_info)]
    L.slab_solve_adjoint.argtypes = [vp, vp, vp, i32, i64, vp, ctypes.POINTER(slab_solve_info)]
    L.slab_solve_noalloc.argtypes = [vp, vp, vp, i32, i64, vp, ctypes.POINTER(slab_solve_info)]
    L.slab_free.argtypes = [vp]
    L.slab_index_maps.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp]
    L.slab_kappa_grad.argtypes = [vp, vp, vp, i32, i64, i32, vp, vp]
    L.slab_residual.argtypes = [vp, vp, vp, i32, i64, ctypes.POINTER(dp), vp]
    L.slab_dirichlet_load.argtypes = [vp, vp, vp, i32, i64, vp]
    L.slab_export_reduced.argtypes = [vp, i32, i32, vp, vp]
    L.slab_apply_reduced.argtypes = [vp, vp, vp, i32, vp]
    L.slab_query.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.slab_factor_batch.argtypes = [ctypes.POINTER(slab_problem), i32, ctypes.POINTER(slab_options),
                                    vp, ctypes.POINTER(vp), ctypes.POINTER(slab_solve_info)]
    L.slab_solve_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(i32), ctypes.POINTER(i64), vp,
                                   ctypes.POINTER(slab_solve_info)]
    L.slab_solve_adjoint_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(i32), ctypes.POINTER(i64), vp,
                                           ctypes.POINTER(slab_solve_info)]
    L.slab_kappa_grad_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(i32), ctypes.POINTER(i64), i32,
                                        ctypes.POINTER(vp), vp]
    L.slab_batch_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                 ctypes.POINTER(i32), ctypes.POINTER(i64), vp,
                                 ctypes.POINTER(slab_solve_info)]
    L.slab_batch_handle.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.slab_batch_query.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.slab_batch_free.argtypes = [vp]
    L.slab_release_cache.argtypes = []
    L.slab_autotune.argtypes = [ctypes.POINTER(slab_problem), ctypes.POINTER(slab_options), i32, vp,
                                ctypes.POINTER(i32), ctypes.POINTER(dp)]
    for name in header_functions():
        if name != "slab_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != SLAB_OK:
        raise SlabError(rc, load_library().slab_last_error().decode(errors="replace"))


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class SlabHandle:
    """One factorization (an opaque slab_handle); owned unless it belongs to a batch."""

    def __init__(self, ptr, n2, n1, b, h, precision, owned=True):
        self._ptr = ptr
        self.n2, self.n1, self.b, self.h, self.precision = n2, n1, b, h, precision
        self.m = n1 // (b + 1)
        self.last_info = slab_solve_info()
        self._owned = owned

    @property
    def ptr(self):
        if not self._ptr:
            raise ValueError("handle already freed")
        return self._ptr

    def free(self):
        if self._ptr:
            if self._owned:
                load_library().slab_free(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        _check(load_library().slab_query(self.ptr, what, ctypes.byref(v)))
        return v.value

    def phase_us(self) -> dict:
        names = ["slab_factor", "boundary_columns", "schur", "assemble", "block_factor",
                 "block_products"]
        return {n: self.query(10 + i) for i, n in enumerate(names)}

    def negative_pivots(self) -> int:
        """Negative pivots of the signed block factorization of T (factored
        with a diagonal term; 0 otherwise): the number of negative eigenvalues
        of T, i.e. those of A less those of the slab interiors."""
        return self.query(7)

    LAUNCH_KINDS = ("gemm128", "gemm64", "gemm_cprefetch", "bmv_split", "bmv")

    def launches(self) -> dict:
        """Kernel launches issued for this handle so far, by kind."""
        return {n: self.query(20 + i) for i, n in enumerate(self.LAUNCH_KINDS)}


def _vec_shape(t, n2, n1):
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.shape[1] != n1 or t.shape[2] != n2:
        raise ValueError(f"expected shape (nrhs, {n1}, {n2}), got {tuple(t.shape)}")
    return t


def slab_factor(kappa, n2: int, n1: int, b: int, h: float | None = None, precision: int = SLAB_FP64,
                tol: float = 1e-10, max_iter: int = 10, keep_reduced: bool = False,
                coef_log: bool = False, odd_even: bool = False, tile: int = 0,
                shift=None, stream=None) -> SlabHandle:
    """Alg. 3 on the device field kappa (or theta = log kappa), shape (n1+2, n2+2).
    tile: FP32 block-product tile (0 automatic, 64 or 128).  shift: optional
    diagonal term c_p on the interior nodes, shape (n1, n2) (c = -k^2 b(x): the
    Helmholtz term)."""
    L = load_library()
    if h is None:
        h = 1.0 / (n2 + 1)
    if tuple(kappa.shape) != (n1 + 2, n2 + 2):
        raise ValueError(f"kappa must have shape {(n1 + 2, n2 + 2)}")
    sh = None
    if shift is not None:
        if tuple(shift.shape) != (n1, n2):
            raise ValueError(f"shift must have shape {(n1, n2)}")
        sh = _dev_f64(shift, "shift")
    prob = slab_problem(n1, n2, b, float(h), _dev_f64(kappa, "kappa"), sh)
    flags = ((SLAB_KEEP_REDUCED if keep_reduced else 0) | (SLAB_COEF_LOG if coef_log else 0)
             | (SLAB_ODD_EVEN if odd_even else 0))
    opts = slab_options(precision, float(tol), int(max_iter), flags, int(tile))
    out = ctypes.c_void_p()
    info = slab_solve_info()
    _check(L.slab_factor(ctypes.byref(prob), ctypes.byref(opts), _stream_ptr(stream),
                         ctypes.byref(out), ctypes.byref(info)))
    handle = SlabHandle(out, n2, n1, b, h, precision)
    if b == 0:  # width chosen by the autotuner
        handle.b = handle.query(3)
        handle.m = n1 // (handle.b + 1)
    return handle


def _solve(fn, handle: SlabHandle, f, out=None, stream=None, check=True):
    import torch
    f3 = _vec_shape(f, handle.n2, handle.n1)
    if not f3.is_contiguous():
        f3 = f3.contiguous()
    u = torch.empty_like(f3) if out is None else _vec_shape(out, handle.n2, handle.n1)
    info = slab_solve_info()
    rc = fn(handle.ptr, _dev_f64(f3, "f"), _dev_f64(u, "u"), f3.shape[0], handle.n1 * handle.n2,
            _stream_ptr(stream), ctypes.byref(info))
    handle.last_info = info
    if check:
        _check(rc)
    return u.view(f.shape) if f.dim() == 2 else u


def slab_solve(handle: SlabHandle, f, out=None, stream=None, check=True):
    """Alg. 4: u = A^-1 f for f of shape (nrhs, n1, n2) (or (n1, n2)), CUDA float64."""
    return _solve(load_library().slab_solve, handle, f, out, stream, check)


def slab_solve_adjoint(handle: SlabHandle, g, out=None, stream=None, check=True):
    """lambda = A^-T g with the stored factors applied transposed."""
    return _solve(load_library().slab_solve_adjoint, handle, g, out, stream, check)


def slab_solve_noalloc(handle: SlabHandle, f, out=None, stream=None, check=True):
    """slab_solve with its buffers in the library's fixed scratch array (no
    device allocation inside the library call; out must be given to avoid the
    one torch allocation of the result)."""
    return _solve(load_library().slab_solve_noalloc, handle, f, out, stream, check)


def slab_free(handle: SlabHandle):
    handle.free()


def slab_index_maps(n2: int, n1: int, b: int, stream=None) -> dict:
    import torch
    m = n1 // (b + 1) if b + 1 > 0 else 0
    dev = torch.device("cuda")
    out = dict(col_kind=torch.empty(n1, dtype=torch.int32, device=dev),
               slab_of_col=torch.empty(n1, dtype=torch.int32, device=dev),
               local_of_col=torch.empty(n1, dtype=torch.int32, device=dev),
               perm_even=torch.empty(max(m * n2 * b, 1), dtype=torch.int64, device=dev),
               perm_odd=torch.empty(max(m * n2, 1), dtype=torch.int64, device=dev))
    p = {k: ctypes.c_void_p(v.data_ptr()) for k, v in out.items()}
    _check(load_library().slab_index_maps(n1, n2, b, p["col_kind"], p["slab_of_col"],
                                          p["local_of_col"], p["perm_even"], p["perm_odd"],
                                          _stream_ptr(stream)))
    out["perm_even"] = out["perm_even"][:m * n2 * b]
    out["perm_odd"] = out["perm_odd"][:m * n2]
    out["m"] = m
    return out


def slab_kappa_grad(handle: SlabHandle, u, lam, mode: int = 1, stream=None):
    """dL/dkappa (mode 0) or dL/dtheta (mode 1) on the (n1+2, n2+2) field."""
    import torch
    u3 = _vec_shape(u, handle.n2, handle.n1).contiguous()
    l3 = _vec_shape(lam, handle.n2, handle.n1).contiguous()
    grad = torch.empty((handle.n1 + 2, handle.n2 + 2), dtype=torch.float64, device=u3.device)
    _check(load_library().slab_kappa_grad(handle.ptr, _dev_f64(u3, "u"), _dev_f64(l3, "lam"),
                                          u3.shape[0], handle.n1 * handle.n2, mode,
                                          _dev_f64(grad, "grad"), _stream_ptr(stream)))
    return grad


def slab_dirichlet_load(handle: SlabHandle, g, f=None, stream=None):
    """f += load of the Dirichlet data g (ring values of (n1+2, n2+2) fields,
    shape (nrhs, n1+2, n2+2) or (n1+2, n2+2), CUDA float64) on the right-hand
    side of A u = f; f (nrhs, n1, n2) is updated in place, or a new zero one is
    made.  Returns f."""
    import torch
    g3 = g.unsqueeze(0) if g.dim() == 2 else g
    if g3.dim() != 3 or tuple(g3.shape[1:]) != (handle.n1 + 2, handle.n2 + 2):
        raise ValueError(f"g must have shape (nrhs, {handle.n1 + 2}, {handle.n2 + 2})")
    g3 = g3.contiguous()
    if f is None:
        f = torch.zeros((g3.shape[0], handle.n1, handle.n2), dtype=torch.float64,
                        device=g3.device)
    f3 = _vec_shape(f, handle.n2, handle.n1)
    if not f3.is_contiguous() or f3.shape[0] != g3.shape[0]:
        raise ValueError("f must be contiguous with one column per field of g")
    _check(load_library().slab_dirichlet_load(handle.ptr, _dev_f64(g3, "g"), _dev_f64(f3, "f"),
                                              g3.shape[0], handle.n1 * handle.n2,
                                              _stream_ptr(stream)))
    return f


def slab_residual(handle: SlabHandle, f, u, stream=None) -> list[float]:
    f3 = _vec_shape(f, handle.n2, handle.n1).contiguous()
    u3 = _vec_shape(u, handle.n2, handle.n1).contiguous()
    arr = (ctypes.c_double * f3.shape[0])()
    _check(load_library().slab_residual(handle.ptr, _dev_f64(f3, "f"), _dev_f64(u3, "u"),
                                        f3.shape[0], handle.n1 * handle.n2, arr,
                                        _stream_ptr(stream)))
    return list(arr)


def slab_apply_reduced(handle: SlabHandle, x, stream=None):
    """y = T x (matrix-free, through the stored slab factors) for interface
    vectors x of shape (m, ncols, n2), CUDA float64; returns y of that shape."""
    import torch
    if x.dim() != 3 or x.shape[0] != handle.m or x.shape[2] != handle.n2:
        raise ValueError(f"x must have shape ({handle.m}, ncols, {handle.n2})")
    xc = x.contiguous()
    y = torch.empty_like(xc)
    _check(load_library().slab_apply_reduced(handle.ptr, _dev_f64(xc, "x"), _dev_f64(y, "y"),
                                             xc.shape[1], _stream_ptr(stream)))
    return y


def slab_export_reduced(handle: SlabHandle, which: int, j: int, stream=None):
    """FP64 copy of T_jj (which=0), T_{j,j+1} (1) or the pivot block of interface j
    before its factorization (2: S_j of Alg. 1, or the odd-even pivot); needs keep_reduced."""
    import torch
    out = torch.empty((handle.n2, handle.n2), dtype=torch.float64, device="cuda")
    _check(load_library().slab_export_reduced(handle.ptr, which, j, _dev_f64(out, "out"),
                                              _stream_ptr(stream)))
    return out


def slab_check_problem(n2: int, n1: int, b: int, h: float, kappa_ptr: int = 1,
                       precision: int = SLAB_FP64, tol: float = 1e-10, max_iter: int = 10,
                       flags: int = 0, tile: int = 0) -> int:
    """Host-only argument check; returns the status code (no HIP call is made)."""
    prob = slab_problem(n1, n2, b, float(h), ctypes.c_void_p(kappa_ptr))
    opts = slab_options(precision, float(tol), int(max_iter), flags, int(tile))
    return load_library().slab_check_problem(ctypes.byref(prob), ctypes.byref(opts))


# ---------------------------------------------------------------------------
# Differentiable solve: u(theta) = A(exp(theta))^-1 f.
# ---------------------------------------------------------------------------
def _autograd():
    import torch

    class SlabSolveFunction(torch.autograd.Function):
        """Forward: slab_factor (theta = log kappa) + slab_solve.  Backward:
        slab_solve_adjoint for lambda = A^-T dL/du, then the edge-product
        gradient kernel for dL/dtheta; dL/df = lambda."""

        @staticmethod
        def forward(ctx, theta, f, n2, n1, b, h, precision, tol):
            handle = slab_factor(theta.contiguous(), n2, n1, b, h, precision=precision, tol=tol,
                                 coef_log=True)
            u = slab_solve(handle, f.contiguous())
            ctx.handle = handle
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, gu):
            (u,) = ctx.saved_tensors
            handle = ctx.handle
            lam = slab_solve_adjoint(handle, gu.contiguous())
            gtheta = slab_kappa_grad(handle, u, lam, mode=1)
            return gtheta, lam, None, None, None, None, None, None

    return SlabSolveFunction


def _autograd_batch():
    import torch

    class SlabSolveBatchFunction(torch.autograd.Function):
        """Forward: slab_factor_batch of B fields theta_i = log kappa_i (one
        grid) + slab_solve_batch.  Backward: slab_solve_adjoint_batch for
        lambda_i = A_i^-T dL/du_i, then slab_kappa_grad_batch for dL/dtheta_i;
        dL/df = lambda (summed over the batch when f is shared)."""

        @staticmethod
        def forward(ctx, theta, f, n2, n1, b, h, precision, tol):
            B = theta.shape[0]
            thetas = [theta[i].contiguous() for i in range(B)]
            batch = slab_factor_batch(thetas, [(n2, n1, b, h)] * B, precision=precision, tol=tol,
                                      coef_log=True)
            shared = f.dim() == 3
            fs = [f.contiguous() if shared else f[i].contiguous() for i in range(B)]
            us = slab_solve_batch(batch, fs)
            u = torch.stack(us)
            ctx.batch = batch
            ctx.shared = shared
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, gu):
            (u,) = ctx.saved_tensors
            batch = ctx.batch
            B = u.shape[0]
            lams = slab_solve_adjoint_batch(batch, [gu[i].contiguous() for i in range(B)])
            grads = slab_kappa_grad_batch(batch, [u[i] for i in range(B)], lams, mode=1)
            lam = torch.stack(lams)
            gf = lam.sum(0) if ctx.shared else lam
            return torch.stack(grads), gf, None, None, None, None, None, None

    return SlabSolveBatchFunction


_fn = None
_fn_batch = None


def solve_theta_batch(theta, f, n2: int, n1: int, b: int, h: float | None = None,
                      precision: int = SLAB_FP64, tol: float = 1e-10):
    """Differentiable u_i = A(exp theta_i)^-1 f_i for a batch of B coefficient
    fields on one grid: theta of shape (B, n1+2, n2+2); f of shape
    (nrhs, n1, n2) (shared by every field) or (B, nrhs, n1, n2).  Returns u of
    shape (B, nrhs, n1, n2)."""
    global _fn_batch
    if _fn_batch is None:
        _fn_batch = _autograd_batch()
    if h is None:
        h = 1.0 / (n2 + 1)
    return _fn_batch.apply(theta, f, n2, n1, b, h, precision, tol)


def solve_theta(theta, f, n2: int, n1: int, b: int, h: float | None = None,
                precision: int = SLAB_FP64, tol: float = 1e-10):
    """Differentiable u = A(exp theta)^-1 f (a torch.autograd.Function)."""
    global _fn
    if _fn is None:
        _fn = _autograd()
    if h is None:
        h = 1.0 / (n2 + 1)
    return _fn.apply(theta, f, n2, n1, b, h, precision, tol)


# ---- batches -----------------------------------------------------------------

class SlabBatch:
    """Owns the factorizations of a batch of independent problems (slab_batch)."""

    def __init__(self, ptr, dims, precision):
        self._ptr = ptr
        self.dims = list(dims)          # (n2, n1, b, h) per problem
        self.precision = precision
        self.last_infos = [slab_solve_info() for _ in dims]

    @property
    def ptr(self):
        if not self._ptr:
            raise ValueError("batch already freed")
        return self._ptr

    def __len__(self):
        return len(self.dims)

    def handle(self, i: int) -> SlabHandle:
        """Handle of problem i (owned by the batch)."""
        out = ctypes.c_void_p()
        _check(load_library().slab_batch_handle(self.ptr, i, ctypes.byref(out)))
        n2, n1, b, h = self.dims[i]
        hd = SlabHandle(out, n2, n1, b, h, self.precision, owned=False)
        if b == 0:
            hd.b = hd.query(3)
            hd.m = n1 // (hd.b + 1)
        return hd

    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        _check(load_library().slab_batch_query(self.ptr, what, ctypes.byref(v)))
        return v.value

    def phase_us(self) -> dict:
        names = ["slab_factor", "boundary_columns", "schur", "assemble", "block_factor",
                 "block_products"]
        return {n: self.query(10 + i) for i, n in enumerate(names)}

    def free(self):
        if self._ptr:
            load_library().slab_batch_free(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def slab_factor_batch(kappas, dims, precision: int = SLAB_FP64, tol: float = 1e-10,
                      max_iter: int = 10, odd_even: bool = True, graph: bool = False,
                      keep_reduced: bool = False, tile: int = 0, coef_log: bool = False,
                      shifts=None, stream=None) -> SlabBatch:
    """Factor independent problems together.  kappas: CUDA float64 tensors of
    shape (n1+2, n2+2); dims: (n2, n1, b) or (n2, n1, b, h) per problem."""
    L = load_library()
    full = []
    for d in dims:
        n2, n1, b = d[:3]
        h = d[3] if len(d) > 3 else 1.0 / (n2 + 1)
        full.append((int(n2), int(n1), int(b), float(h)))
    if len(kappas) != len(full):
        raise ValueError("one coefficient field per problem")
    arr = (slab_problem * len(full))()
    for i, ((n2, n1, b, h), k) in enumerate(zip(full, kappas)):
        if tuple(k.shape) != (n1 + 2, n2 + 2):
            raise ValueError(f"kappa {i} must have shape {(n1 + 2, n2 + 2)}")
        sh = None
        if shifts is not None and shifts[i] is not None:
            if tuple(shifts[i].shape) != (n1, n2):
                raise ValueError(f"shift {i} must have shape {(n1, n2)}")
            sh = _dev_f64(shifts[i], f"shift[{i}]")
        arr[i] = slab_problem(n1, n2, b, h, _dev_f64(k, f"kappa[{i}]"), sh)
    flags = ((SLAB_ODD_EVEN if odd_even else 0) | (SLAB_GRAPH if graph else 0)
             | (SLAB_KEEP_REDUCED if keep_reduced else 0) | (SLAB_COEF_LOG if coef_log else 0))
    opts = slab_options(precision, float(tol), int(max_iter), flags, int(tile))
    infos = (slab_solve_info * len(full))()
    out = ctypes.c_void_p()
    _check(L.slab_factor_batch(arr, len(full), ctypes.byref(opts), _stream_ptr(stream),
                               ctypes.byref(out), infos))
    return SlabBatch(out, full, precision)


def _batch_vectors(batch: SlabBatch, fs, outs):
    import torch
    cnt = len(batch)
    if len(fs) != cnt:
        raise ValueError("one right-hand side block per problem")
    f3, us = [], []
    for i, f in enumerate(fs):
        n2, n1 = batch.dims[i][0], batch.dims[i][1]
        t = _vec_shape(f, n2, n1)
        if not t.is_contiguous():
            t = t.contiguous()
        f3.append(t)
        us.append(torch.empty_like(t) if outs is None else _vec_shape(outs[i], n2, n1))
    fp = (ctypes.c_void_p * cnt)(*[_dev_f64(t, f"f[{i}]").value for i, t in enumerate(f3)])
    up = (ctypes.c_void_p * cnt)(*[_dev_f64(t, f"u[{i}]").value for i, t in enumerate(us)])
    nr = (ctypes.c_int32 * cnt)(*[t.shape[0] for t in f3])
    ld = (ctypes.c_int64 * cnt)(*[batch.dims[i][0] * batch.dims[i][1] for i in range(cnt)])
    return f3, us, fp, up, nr, ld


def _solve_batch(fn, batch: SlabBatch, fs, outs, stream, check):
    cnt = len(batch)
    _, us, fp, up, nr, ld = _batch_vectors(batch, fs, outs)
    infos = (slab_solve_info * cnt)()
    rc = fn(batch.ptr, fp, up, nr, ld, _stream_ptr(stream), infos)
    batch.last_infos = list(infos)
    if check:
        _check(rc)
    return [u.view(f.shape) if f.dim() == 2 else u for u, f in zip(us, fs)]


def slab_solve_batch(batch: SlabBatch, fs, outs=None, stream=None, check=True):
    """Solve every problem of the batch: fs[i] of shape (nrhs_i, n1_i, n2_i)
    (or (n1_i, n2_i)), CUDA float64.  Returns the list of solutions."""
    return _solve_batch(load_library().slab_solve_batch, batch, fs, outs, stream, check)


def slab_solve_adjoint_batch(batch: SlabBatch, gs, outs=None, stream=None, check=True):
    """lambda_i = A_i^-T g_i for every problem of the batch (stored factors
    applied transposed).  Returns the list of lambda_i."""
    return _solve_batch(load_library().slab_solve_adjoint_batch, batch, gs, outs, stream, check)


def slab_batch_run(batch: SlabBatch, kappas, fs, outs=None, stream=None, check=True):
    """Factor every problem again from kappas[i] (CUDA float64, shape
    (n1_i+2, n2_i+2)) and solve fs[i], as one HIP graph launch (captured on
    the first call, replayed while the tensors are the same).  Returns the
    list of solutions."""
    cnt = len(batch)
    if len(kappas) != cnt:
        raise ValueError("one coefficient field per problem")
    for i, k in enumerate(kappas):
        n2, n1 = batch.dims[i][0], batch.dims[i][1]
        if tuple(k.shape) != (n1 + 2, n2 + 2):
            raise ValueError(f"kappa {i} must have shape {(n1 + 2, n2 + 2)}")
    kp = (ctypes.c_void_p * cnt)(*[_dev_f64(k, f"kappa[{i}]").value for i, k in enumerate(kappas)])
    _, us, fp, up, nr, ld = _batch_vectors(batch, fs, outs)
    infos = (slab_solve_info * cnt)()
    rc = load_library().slab_batch_run(batch.ptr, kp, fp, up, nr, ld, _stream_ptr(stream), infos)
    batch.last_infos = list(infos)
    if check:
        _check(rc)
    return [u.view(f.shape) if f.dim() == 2 else u for u, f in zip(us, fs)]


def slab_kappa_grad_batch(batch: SlabBatch, us, lams, mode: int = 1, stream=None):
    """slab_kappa_grad for every problem: list of (n1_i+2, n2_i+2) gradients."""
    import torch
    cnt = len(batch)
    u3, _, upp, _, nr, ld = _batch_vectors(batch, us, lams)
    l3 = [_vec_shape(l, batch.dims[i][0], batch.dims[i][1]).contiguous()
          for i, l in enumerate(lams)]
    lp = (ctypes.c_void_p * cnt)(*[_dev_f64(t, f"lam[{i}]").value for i, t in enumerate(l3)])
    grads = [torch.empty((n1 + 2, n2 + 2), dtype=torch.float64, device=u3[0].device)
             for (n2, n1, _, _) in batch.dims]
    gp = (ctypes.c_void_p * cnt)(*[_dev_f64(g, f"grad[{i}]").value for i, g in enumerate(grads)])
    _check(load_library().slab_kappa_grad_batch(batch.ptr, upp, lp, nr, ld, int(mode), gp,
                                                _stream_ptr(stream)))
    return grads


def release_cache():
    """Return the library's cached, unused device memory to HIP."""
    _check(load_library().slab_release_cache())


def slab_autotune(kappa, n2: int, n1: int, h: float | None = None, precision: int = SLAB_FP64,
                  tol: float = 1e-10, max_iter: int = 10, odd_even: bool = False, nrhs: int = 1,
                  stream=None):
    """Slab width chosen by measurement for this grid; returns (b, seconds per
    candidate b in (3, 7, 15, 31, 63), None where not tried)."""
    L = load_library()
    if h is None:
        h = 1.0 / (n2 + 1)
    prob = slab_problem(n1, n2, 0, float(h), _dev_f64(kappa, "kappa"))
    opts = slab_options(precision, float(tol), int(max_iter), SLAB_ODD_EVEN if odd_even else 0)
    b = ctypes.c_int32()
    times = (ctypes.c_double * 5)()
    _check(L.slab_autotune(ctypes.byref(prob), ctypes.byref(opts), int(nrhs), _stream_ptr(stream),
                           ctypes.byref(b), times))
    return b.value, {w: (t if t >= 0 else None) for w, t in zip((3, 7, 15, 31, 63), times)}
