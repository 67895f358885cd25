"""Python binding of libmapi.so: MAPI / RPI on one MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C-ABI declared in include/mapi.h.  PyTorch supplies device
memory and the stream.  There is no CPU fallback: if libmapi.so is missing or
cannot be loaded, every call raises.

The function names are those of the C-ABI (mapi_solve, rpi_solve, mapi_mavp,
mapi_quantize, mapi_mingram, mapi_pca_topk, mapi_pagerank, ...).
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# MAPI_CHECKED=1 loads the device-checked build (libmapi_checked.so, built by
# `python -m paper_2110_12065_amd.build` beside libmapi.so)
LIB_PATH = os.path.join(HERE, "libmapi_checked.so" if os.environ.get("MAPI_CHECKED") == "1" else "libmapi.so")

MAPI_F32, MAPI_BF16, MAPI_FP8_E4M3 = 0, 1, 2
OPS = {"min1": 0, "min2": 1, "diamond": 2, "dot": 3}
METHODS = {"mapi": 0, "rpi": 1}
KERNELS = {"mavp": 0, "finalize": 1, "gram": 2, "csr": 3, "deflate": 4, "batched": 5, "minibatch": 6}
WORKSPACE = {"solve": 0, "hybrid": 1, "pagerank": 2, "pagerank_f64": 3, "product": 4, "mingram": 5, "pca": 6,
             "pca_vector": 7, "image": 8, "minibatch": 9, "minibatch_min": 10, "factored": 11}
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_DEGENERATE", 5: "ERR_BUDGET",
          6: "ERR_UNSUPPORTED", 7: "ERR_PENDING", 8: "ERR_TIMEOUT"}


class MapiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Dense(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n_rows", C.c_int64), ("n_cols", C.c_int64), ("ld", C.c_int64),
                ("dtype", C.c_int32), ("row_scale", C.c_void_p)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("tol", C.c_double), ("final_l2", C.c_int32), ("op", C.c_int32),
                ("check_every", C.c_int32), ("stall_iters", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("rows_per_wave", C.c_int32), ("waves", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("unroll", C.c_int32), ("w_in_lds", C.c_int32), ("nontemporal", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double), ("norm", C.c_double),
                ("status", C.c_int32)]

    def as_dict(self):
        return dict(iters=self.iters, converged=bool(self.converged), residual=self.residual, norm=self.norm,
                    status=STATUS.get(self.status, self.status))


_lib = None
_lib_lock = threading.Lock()

# name -> (restype, argtypes)
_SIGS = {
    "mapi_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mapi_destroy": (None, [C.c_void_p]),
    "mapi_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mapi_last_error": (C.c_char_p, []),
    "mapi_version": (C.c_char_p, []),
    "mapi_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "mapi_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "mapi_timing_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "mapi_timing_get": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "mapi_timing_reset": (C.c_int, [C.c_void_p]),
    "mapi_mavp": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_void_p, C.c_void_p, C.c_int32]),
    "mapi_autotune_dense": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_int32, C.c_int32, C.POINTER(Tuning),
                                      C.POINTER(C.c_double)]),
    "mapi_tuning_get": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.POINTER(Tuning)]),
    "mapi_tuning_set": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.POINTER(Tuning)]),
    "mapi_mavp_timed": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_void_p, C.c_void_p, C.c_int32,
                                  C.POINTER(Tuning), C.c_int32, C.POINTER(C.c_double)]),
    "mapi_copy_reference": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32,
                                      C.POINTER(C.c_double)]),
    "mapi_read_reference": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_double)]),
    "mapi_solve": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_void_p, C.c_void_p, C.POINTER(Opts), C.POINTER(Info)]),
    "rpi_solve": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_void_p, C.c_void_p, C.POINTER(Opts), C.POINTER(Info)]),
    "mapi_solve_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_void_p, C.c_void_p, C.POINTER(Opts),
                                     C.POINTER(Info)]),
    "mapi_quantize": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_void_p,
                                C.c_int64, C.c_void_p]),
    "mapi_mingram": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_int32,
                               C.c_void_p, C.c_int64]),
    "mapi_pca_topk": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_double,
                                C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(Opts), C.POINTER(Info)]),
    "mapi_pagerank": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                                C.POINTER(Opts), C.POINTER(Info)]),
    "mapi_pagerank_f64": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.POINTER(Opts), C.POINTER(Info)]),
    "mapi_pagerank_split_config": (C.c_int, [C.c_void_p, C.c_int64]),
    "mapi_pagerank_split_after": (C.c_int, [C.c_void_p, C.c_int32]),
    "mapi_factored_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_double,
                                      C.c_void_p, C.c_void_p, C.POINTER(Opts), C.POINTER(Info)]),
    "mapi_hybrid_solve": (C.c_int, [C.c_void_p, C.POINTER(Dense), C.c_void_p, C.c_void_p, C.POINTER(Opts),
                                    C.POINTER(Opts), C.POINTER(Info), C.POINTER(Info)]),
    "mapi_image_reconstruct": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_int32,
                                         C.c_void_p, C.POINTER(Opts), C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p]),
    "mapi_minibatch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_int32,
                                 C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_void_p]),
}


def lib():
    """The loaded libmapi.so (raises if it is missing)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_12065_amd.build` "
                                   "(there is no CPU fallback)")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


def _check(status):
    if status != 0:
        raise MapiError(status, lib().mapi_last_error().decode(errors="replace"))


# ------------------------------------------------------------------ context
class Context:
    """A libmapi context on one device, enqueuing on torch's current stream."""

    def __init__(self, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: libmapi runs on the GPU only")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._stream = torch.cuda.current_stream(self.device).cuda_stream
        h = C.c_void_p()
        _check(lib().mapi_create(self.device, C.c_void_p(self._stream), C.byref(h)))
        self.handle = h

    # caller-owned device workspace --------------------------------------------
    def workspace_size(self, kind, n, nnz=0):
        """Bytes of workspace a call of `kind` (a WORKSPACE key) needs at size (n, nnz)."""
        b = C.c_size_t()
        _check(lib().mapi_workspace_size(self.handle, WORKSPACE[kind], int(n), int(nnz), C.byref(b)))
        return b.value

    def set_workspace(self, buf):
        """Make every call of this context take its device buffers from `buf` (a device
        tensor, kept alive here); None returns to context-owned memory."""
        if buf is None:
            _check(lib().mapi_set_workspace(self.handle, None, 0))
            self._ws = None
            return
        if not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("the workspace must be a contiguous device tensor")
        _check(lib().mapi_set_workspace(self.handle, C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))
        self._ws = buf

    def sync_stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            _check(lib().mapi_set_stream(self.handle, C.c_void_p(s)))
            self._stream = s

    def close(self):
        if getattr(self, "handle", None):
            lib().mapi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # kernel timing ---------------------------------------------------------
    def timing(self, enable=True):
        _check(lib().mapi_timing_enable(self.handle, int(bool(enable))))

    def timing_reset(self):
        _check(lib().mapi_timing_reset(self.handle))

    def timing_get(self, kind):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().mapi_timing_get(self.handle, KERNELS[kind], C.byref(ms), C.byref(n)))
        return ms.value, n.value


_ctx = {}


def default_context(device=None):
    import torch
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _ctx:
        _ctx[d] = Context(d)
    c = _ctx[d]
    c.sync_stream()
    return c


def _ctx_of(ctx, t):
    c = ctx if ctx is not None else default_context(t.device.index)
    c.sync_stream()
    return c


# ------------------------------------------------------------------ marshalling
def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return MAPI_F32
    if t.dtype in (torch.bfloat16, torch.int16) or str(t.dtype) == "torch.uint16":
        return MAPI_BF16
    if t.dtype == torch.uint8 or t.dtype == getattr(torch, "float8_e4m3fn", None):
        return MAPI_FP8_E4M3
    raise TypeError(f"unsupported matrix dtype {t.dtype}")


def _dense(A, row_scale=None):
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D tensor with unit column stride")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    code = _dtype_code(A)
    rs = None
    if code == MAPI_FP8_E4M3:
        if row_scale is None:
            raise ValueError("FP8 storage needs row_scale")
        rs = row_scale.data_ptr()
    return Dense(A.data_ptr(), A.shape[0], A.shape[1], A.stride(0), code, rs)


def _vec(t, n, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous float32 device tensor of length {n}")
    return t.data_ptr()


def _opts(max_iters, tol, op, final_l2, check_every, stall_iters):
    return Opts(int(max_iters), float(tol), int(bool(final_l2)), OPS[op] if isinstance(op, str) else int(op),
                int(check_every), int(stall_iters))


# ------------------------------------------------------------------ entry points
def mapi_mavp(A, w, op="min1", row_scale=None, y=None, ctx=None):
    """y = A (+) w (one product, no normalisation)."""
    import torch
    c = _ctx_of(ctx, A)
    d = _dense(A, row_scale)
    if y is None:
        y = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    _check(lib().mapi_mavp(c.handle, C.byref(d), C.c_void_p(_vec(w, A.shape[1], "w")),
                           C.c_void_p(_vec(y, A.shape[0], "y")), OPS[op] if isinstance(op, str) else int(op)))
    return y


def _solve(fn, A, w0, max_iters, tol, op, final_l2, check_every, stall_iters, row_scale, w_out, ctx):
    import torch
    c = _ctx_of(ctx, A)
    d = _dense(A, row_scale)
    n = A.shape[0]
    if w_out is None:
        w_out = torch.empty(n, dtype=torch.float32, device=A.device)
    o = _opts(max_iters, tol, op, final_l2, check_every, stall_iters)
    info = Info()
    st = fn(c.handle, C.byref(d), C.c_void_p(_vec(w0, n, "w0")), C.c_void_p(_vec(w_out, n, "w_out")),
            C.byref(o), C.byref(info))
    _check(st)
    return w_out, info.as_dict()


def mapi_solve(A, w0, max_iters=100, tol=0.0, op="min1", final_l2=False, check_every=0, stall_iters=0,
               row_scale=None, w_out=None, ctx=None):
    """MAPI (eq. 6, Algorithm 1) on a square dense matrix.  Returns (w, info)."""
    return _solve(lib().mapi_solve, A, w0, max_iters, tol, op, final_l2, check_every, stall_iters, row_scale,
                  w_out, ctx)


def mapi_solve_noalloc(A, w0, max_iters=100, tol=0.0, op="min1", final_l2=False, check_every=0, stall_iters=0,
                       row_scale=None, w_out=None, ctx=None):
    """mapi_solve with the solve's buffers in the library's static device scratch array (no device
    allocation by the library; w_out is allocated here when not given).  Returns (w, info)."""
    return _solve(lib().mapi_solve_noalloc, A, w0, max_iters, tol, op, final_l2, check_every, stall_iters,
                  row_scale, w_out, ctx)


def rpi_solve(A, w0, max_iters=100, tol=0.0, final_l2=False, check_every=0, stall_iters=0, row_scale=None,
              w_out=None, ctx=None):
    """RPI (eq. 1) on a square dense matrix.  Returns (w, info)."""
    return _solve(lib().rpi_solve, A, w0, max_iters, tol, "dot", final_l2, check_every, stall_iters, row_scale,
                  w_out, ctx)


def mapi_hybrid_solve(A, w0, mapi_iters=100, mapi_tol=0.0, rpi_iters=100, rpi_tol=0.0, op="min1",
                      final_l2=False, check_every=0, stall_iters=0, row_scale=None, w_out=None, ctx=None):
    """MAPI (to mapi_iters / mapi_tol), then RPI from its l2-normalised result (to rpi_iters /
    rpi_tol).  Returns (w, info_mapi, info_rpi)."""
    import torch
    c = _ctx_of(ctx, A)
    d = _dense(A, row_scale)
    n = A.shape[0]
    if w_out is None:
        w_out = torch.empty(n, dtype=torch.float32, device=A.device)
    o1 = _opts(mapi_iters, mapi_tol, op, True, check_every, stall_iters)
    o2 = _opts(rpi_iters, rpi_tol, "dot", final_l2, check_every, stall_iters)
    i1, i2 = Info(), Info()
    _check(lib().mapi_hybrid_solve(c.handle, C.byref(d), C.c_void_p(_vec(w0, n, "w0")),
                                   C.c_void_p(_vec(w_out, n, "w_out")), C.byref(o1), C.byref(o2),
                                   C.byref(i1), C.byref(i2)))
    return w_out, i1.as_dict(), i2.as_dict()


def mapi_image_reconstruct(V, w0, method="mapi", max_iters=100, tol=0.0, check_every=0, stall_iters=0, op="min1",
                           ctx=None):
    """Algorithm 2: V device float32 P x N (column i = corrupted copy i); op "min1" (eq. 3) or
    "min2" (eq. 4) for MAPI.  Returns (R P x N, W P x 2, infos of the two solves)."""
    import torch
    c = _ctx_of(ctx, V)
    if V.dim() != 2 or V.dtype != torch.float32 or V.stride(1) != 1:
        raise ValueError("V must be a float32 P x N tensor with unit column stride")
    P, N = V.shape
    R = torch.empty((P, N), dtype=torch.float32, device=V.device)
    W = torch.empty((2, P), dtype=torch.float32, device=V.device)
    o = _opts(max_iters, tol, op, False, check_every, stall_iters)
    infos = (Info * 2)()
    _check(lib().mapi_image_reconstruct(c.handle, C.c_void_p(V.data_ptr()), int(P), int(N), int(V.stride(0)),
                                        METHODS[method], C.c_void_p(_vec(w0, P, "w0")), C.byref(o),
                                        C.c_void_p(R.data_ptr()), int(N), C.c_void_p(W.data_ptr()), infos))
    return R, W.t(), [i.as_dict() for i in infos]


def mapi_minibatch(X, batches, beta, W0, op="min1", final_l2=False, w_out=None, ctx=None):
    """Mini-batch MAPI with momentum (Algorithm 3).  X: device float32 N x D, samples as rows;
    batches: device int32 (runs, T, s) sample indices; W0: device float32 (runs, D).
    Returns (W (runs, D), infos)."""
    import torch
    c = _ctx_of(ctx, X)
    if X.dim() != 2 or X.dtype != torch.float32 or X.stride(1) != 1:
        raise ValueError("X must be a float32 N x D tensor with unit column stride")
    if batches.dim() != 3 or batches.dtype != torch.int32 or not batches.is_contiguous():
        raise ValueError("batches must be a contiguous int32 tensor of shape (runs, T, s)")
    runs, T, s = batches.shape
    N, D = X.shape
    if tuple(W0.shape) != (runs, D) or W0.dtype != torch.float32 or not W0.is_contiguous():
        raise ValueError("W0 must be a contiguous float32 tensor of shape (runs, D)")
    if w_out is None:
        w_out = torch.empty((runs, D), dtype=torch.float32, device=X.device)
    infos = (Info * runs)()
    _check(lib().mapi_minibatch(c.handle, C.c_void_p(X.data_ptr()), int(N), int(D), int(X.stride(0)),
                                C.c_void_p(batches.data_ptr()), int(s), int(T), float(beta), OPS[op], int(runs),
                                C.c_void_p(W0.data_ptr()), C.c_void_p(w_out.data_ptr()), int(bool(final_l2)), infos))
    return w_out, [i.as_dict() for i in infos]


def mapi_quantize(A, dtype, ctx=None):
    """Reduced storage of a float32 matrix: "bf16" -> uint16 codes; "fp8" -> (uint8 codes, float32 row scales)."""
    import torch
    c = _ctx_of(ctx, A)
    if A.dtype != torch.float32 or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D float32 tensor with unit column stride")
    n, m = A.shape
    if dtype == "bf16":
        ld = (m + 7) // 8 * 8
        out = torch.empty((n, ld), dtype=torch.int16, device=A.device)[:, :m]
        _check(lib().mapi_quantize(c.handle, C.c_void_p(A.data_ptr()), n, m, A.stride(0), MAPI_BF16,
                                   C.c_void_p(out.data_ptr()), ld, None))
        return out, None
    if dtype == "fp8":
        ld = (m + 15) // 16 * 16
        out = torch.empty((n, ld), dtype=torch.uint8, device=A.device)[:, :m]
        scale = torch.empty(n, dtype=torch.float32, device=A.device)
        _check(lib().mapi_quantize(c.handle, C.c_void_p(A.data_ptr()), n, m, A.stride(0), MAPI_FP8_E4M3,
                                   C.c_void_p(out.data_ptr()), ld, C.c_void_p(scale.data_ptr())))
        return out, scale
    raise ValueError(dtype)


def mapi_mingram(X, scale, op="min1", ctx=None):
    """A = scale * X (+) X^T over the rows of X (eq. 5; op "dot" gives eq. 2).  Returns D x D float32."""
    import torch
    c = _ctx_of(ctx, X)
    if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D float32 tensor with unit column stride")
    D, N = X.shape
    A = torch.empty((D, D), dtype=torch.float32, device=X.device)
    _check(lib().mapi_mingram(c.handle, C.c_void_p(X.data_ptr()), D, N, X.stride(0), float(scale),
                              OPS[op], C.c_void_p(A.data_ptr()), D))
    return A


def mapi_pca_topk(X, k, W0=None, method="mapi", scale=None, max_iters=100, tol=0.0, op="min1", check_every=0,
                  stall_iters=0, ctx=None):
    """Top-k principal vectors with deflation.  W0: D x k start vectors (columns), or None
    for the seeded starts (vector i from the generated start vector of seed i).
    Returns (P as a D x k tensor, [info per vector])."""
    import torch
    c = _ctx_of(ctx, X)
    if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D float32 tensor with unit column stride")
    D, N = X.shape
    W0c = None
    if W0 is not None:
        W0c = W0.t().contiguous()          # column i at offset i*D
        if W0c.shape != (k, D) or W0c.dtype != torch.float32:
            raise ValueError("W0 must be a D x k float32 tensor")
    Pc = torch.empty((k, D), dtype=torch.float32, device=X.device)
    o = _opts(max_iters, tol, op, False, check_every, stall_iters)
    infos = (Info * k)()
    _check(lib().mapi_pca_topk(c.handle, C.c_void_p(X.data_ptr()), D, N, X.stride(0), int(k),
                               float(1.0 / N if scale is None else scale), METHODS[method],
                               C.c_void_p(W0c.data_ptr() if W0c is not None else None),
                               C.c_void_p(Pc.data_ptr()), C.byref(o), infos))
    return Pc.t(), [infos[i].as_dict() for i in range(k)]


def mapi_pagerank(row_ptr, col, val, alpha=0.85, method="mapi", w0=None, max_iters=100, tol=0.0, final_l2=False,
                  check_every=0, stall_iters=0, w_out=None, f64=False, ctx=None):
    """Power iteration on G = alpha H + (1 - alpha)/n 1 (eq. 11), H in CSR by destination row.
    Returns (w, info).  f64: float64 iterate (w0 / w_out float64), mapi_pagerank_f64."""
    import torch
    c = _ctx_of(ctx, row_ptr)
    n = row_ptr.numel() - 1
    nnz = col.numel()
    for t, dt, name in ((row_ptr, torch.int32, "row_ptr"), (col, torch.int32, "col"), (val, torch.float32, "val")):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} device tensor")
    if val.numel() != nnz:
        raise ValueError("col and val differ in length")
    H = Csr(n, nnz, row_ptr.data_ptr(), col.data_ptr() if nnz else None, val.data_ptr() if nnz else None)
    wdt = torch.float64 if f64 else torch.float32
    if w_out is None:
        w_out = torch.empty(n, dtype=wdt, device=row_ptr.device)
    for t, name in ((w0, "w0"), (w_out, "w_out")):
        if t is not None and not (t.is_cuda and t.dtype == wdt and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"{name} must be a contiguous {wdt} device tensor of length {n}")
    o = _opts(max_iters, tol, "min1", final_l2, check_every, stall_iters)
    info = Info()
    fn = lib().mapi_pagerank_f64 if f64 else lib().mapi_pagerank
    _check(fn(c.handle, C.byref(H), float(alpha), METHODS[method],
              C.c_void_p(w0.data_ptr()) if w0 is not None else None,
              C.c_void_p(w_out.data_ptr()), C.byref(o), C.byref(info)))
    return w_out, info.as_dict()


def mapi_factored_solve(X, w0, scale=None, max_iters=100, tol=0.0, op="min1", final_l2=False, check_every=0,
                        stall_iters=0, w_out=None, ctx=None):
    """Power iteration with the factored operator X (+) (X^T (+) w) * scale (not a method of the
    paper; see include/mapi.h).  X: device float32 D x N.  Returns (w, info)."""
    import torch
    c = _ctx_of(ctx, X)
    if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D float32 tensor with unit column stride")
    D, N = X.shape
    if w_out is None:
        w_out = torch.empty(D, dtype=torch.float32, device=X.device)
    o = _opts(max_iters, tol, op, final_l2, check_every, stall_iters)
    info = Info()
    _check(lib().mapi_factored_solve(c.handle, C.c_void_p(X.data_ptr()), D, N, X.stride(0),
                                     float(1.0 / N if scale is None else scale), C.c_void_p(_vec(w0, D, "w0")),
                                     C.c_void_p(_vec(w_out, D, "w_out")), C.byref(o), C.byref(info)))
    return w_out, info.as_dict()


def mapi_pagerank_split_config(min_n, ctx=None):
    """PageRank graphs with at least min_n nodes use the column-split product (min_n <= 0: never)."""
    c = ctx if ctx is not None else default_context()
    _check(lib().mapi_pagerank_split_config(c.handle, int(min_n)))


def mapi_pagerank_split_after(iters, ctx=None):
    """Build the column-split layout only after `iters` plain products of a solve (0: before
    the first); see mapi_pagerank_split_config."""
    c = ctx if ctx is not None else default_context()
    _check(lib().mapi_pagerank_split_after(c.handle, int(iters)))


# ------------------------------------------------------------------ launch shapes
def mapi_autotune_dense(A, op="min1", reps=3, row_scale=None, ctx=None):
    """Time every launch shape of the dense product on A and keep the fastest for A's size bucket.
    Returns (shape dict, mean ms)."""
    c = _ctx_of(ctx, A)
    d = _dense(A, row_scale)
    best = Tuning()
    ms = C.c_double()
    _check(lib().mapi_autotune_dense(c.handle, C.byref(d), OPS[op], int(reps), C.byref(best), C.byref(ms)))
    return best.as_dict(), ms.value


def mapi_tuning_get(dtype_code, n_rows, n_cols, ctx=None):
    c = ctx if ctx is not None else default_context()
    t = Tuning()
    _check(lib().mapi_tuning_get(c.handle, int(dtype_code), int(n_rows), int(n_cols), C.byref(t)))
    return t.as_dict()


def mapi_tuning_set(dtype_code, n_rows, n_cols, shape, ctx=None):
    c = ctx if ctx is not None else default_context()
    t = Tuning(**shape)
    _check(lib().mapi_tuning_set(c.handle, int(dtype_code), int(n_rows), int(n_cols), C.byref(t)))


def mapi_mavp_timed(A, w, shape, op="min1", reps=5, row_scale=None, y=None, ctx=None):
    """Mean ms of `reps` products with an explicit launch shape (dict of mapi_tuning fields)."""
    import torch
    c = _ctx_of(ctx, A)
    d = _dense(A, row_scale)
    if y is None:
        y = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    t = Tuning(**shape)
    ms = C.c_double()
    _check(lib().mapi_mavp_timed(c.handle, C.byref(d), C.c_void_p(_vec(w, A.shape[1], "w")),
                                 C.c_void_p(_vec(y, A.shape[0], "y")), OPS[op], C.byref(t), int(reps), C.byref(ms)))
    return ms.value


def mapi_copy_reference(src, dst, reps=5, ctx=None):
    """Mean ms of a plain 16-byte-vector copy of src into dst (the bandwidth reference)."""
    c = _ctx_of(ctx, src)
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst smaller than src")
    ms = C.c_double()
    _check(lib().mapi_copy_reference(c.handle, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                     int(reps), C.byref(ms)))
    return ms.value


def mapi_read_reference(src, reps=5, ctx=None):
    """Mean ms of a plain streaming read of src (non-temporal 16-byte loads): the
    attainable-read-bandwidth reference."""
    c = _ctx_of(ctx, src)
    nbytes = src.numel() * src.element_size()
    ms = C.c_double()
    _check(lib().mapi_read_reference(c.handle, C.c_void_p(src.data_ptr()), nbytes, int(reps), C.byref(ms)))
    return ms.value


# ------------------------------------------------------------------ batched
class Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("method", C.c_int32), ("A", Dense), ("H", Csr), ("alpha", C.c_double),
                ("gen_n", C.c_int64), ("gen_dtype", C.c_int32), ("seed", C.c_uint64), ("w0", C.c_void_p),
                ("w_out", C.c_void_p), ("opts", Opts)]


PROB_DENSE, PROB_CSR, PROB_GENERATED = 0, 1, 2

_SIGS.update({
    "mapi_solve_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem), C.POINTER(Info)]),
    "mapi_solve_batched_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem),
                                                    C.POINTER(C.c_size_t)]),
    "mapi_batched_config": (C.c_int, [C.c_void_p, C.c_int32]),
    "mapi_batched_rows_set": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32]),
    "mapi_batched_rows_get": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_int32)]),
    "mapi_autotune_batched": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "mapi_generate_dense": (C.c_int, [C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p, C.c_int64, C.c_void_p]),
})


def problem_dense(A, method="mapi", w0=None, w_out=None, row_scale=None, max_iters=100, tol=0.0, op="min1",
                  stall_iters=0):
    """Describe a dense instance for mapi_solve_batched (keeps its tensors alive on the object)."""
    import torch
    p = Problem()
    p.kind = PROB_DENSE
    p.method = METHODS[method]
    p.A = _dense(A, row_scale)
    n = A.shape[0]
    w_out = torch.empty(n, dtype=torch.float32, device=A.device) if w_out is None else w_out
    p.w0 = _vec(w0, n, "w0") if w0 is not None else None
    p.w_out = _vec(w_out, n, "w_out")
    p.opts = _opts(max_iters, tol, op, False, 0, stall_iters)
    p._keep = (A, w0, w_out, row_scale)
    p.out = w_out
    p.n = n
    return p


def problem_csr(row_ptr, col, val, alpha=0.85, method="mapi", w0=None, w_out=None, max_iters=100, tol=0.0,
                stall_iters=0):
    import torch
    p = Problem()
    p.kind = PROB_CSR
    p.method = METHODS[method]
    n = row_ptr.numel() - 1
    p.H = Csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
              val.data_ptr() if val.numel() else None)
    p.alpha = float(alpha)
    w_out = torch.empty(n, dtype=torch.float32, device=row_ptr.device) if w_out is None else w_out
    p.w0 = _vec(w0, n, "w0") if w0 is not None else None
    p.w_out = _vec(w_out, n, "w_out")
    p.opts = _opts(max_iters, tol, "min1", False, 0, stall_iters)
    p._keep = (row_ptr, col, val, w0, w_out)
    p.out = w_out
    p.n = n
    return p


def problem_generated(n, seed, dtype="f32", method="mapi", w_out=None, max_iters=100, tol=0.0, op="min1",
                      stall_iters=0, device=None):
    import torch
    p = Problem()
    p.kind = PROB_GENERATED
    p.method = METHODS[method]
    p.gen_n = int(n)
    p.gen_dtype = {"f32": MAPI_F32, "bf16": MAPI_BF16}[dtype]
    p.seed = int(seed)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    w_out = torch.empty(n, dtype=torch.float32, device=dev) if w_out is None else w_out
    p.w0 = None
    p.w_out = _vec(w_out, n, "w_out")
    p.opts = _opts(max_iters, tol, op, False, 0, stall_iters)
    p._keep = (w_out,)
    p.out = w_out
    p.n = int(n)
    return p


def mapi_solve_batched(problems, ctx=None):
    """Solve a ragged list of problems with the persistent batched kernel.
    Returns the list of info dicts; results are in each problem's `.out` tensor."""
    c = ctx if ctx is not None else default_context()
    c.sync_stream()
    k = len(problems)
    arr = (Problem * k)(*problems)
    infos = (Info * k)()
    st = lib().mapi_solve_batched(c.handle, k, arr, infos)
    res = [infos[i].as_dict() for i in range(k)]
    if st not in (0, 4):
        _check(st)
    return res


def mapi_solve_batched_workspace_size(problems, ctx=None):
    """Bytes of the device arena mapi_solve_batched needs for this list of problems."""
    c = ctx if ctx is not None else default_context()
    k = len(problems)
    arr = (Problem * k)(*problems)
    b = C.c_size_t()
    _check(lib().mapi_solve_batched_workspace_size(c.handle, k, arr, C.byref(b)))
    return b.value


def mapi_batched_config(blocks_per_cu, ctx=None):
    c = ctx if ctx is not None else default_context()
    _check(lib().mapi_batched_config(c.handle, int(blocks_per_cu)))


def mapi_batched_rows_set(dtype_code, n, rows, ctx=None):
    c = ctx if ctx is not None else default_context()
    _check(lib().mapi_batched_rows_set(c.handle, int(dtype_code), int(n), int(rows)))


def mapi_batched_rows_get(dtype_code, n, ctx=None):
    c = ctx if ctx is not None else default_context()
    r = C.c_int32()
    _check(lib().mapi_batched_rows_get(c.handle, int(dtype_code), int(n), C.byref(r)))
    return r.value


def mapi_autotune_batched(dtype_code, n, count=32, iters=5, ctx=None):
    """Pick the product tile height of batched dense instances of size n; returns (rows, ms)."""
    c = ctx if ctx is not None else default_context()
    r = C.c_int32()
    ms = C.c_double()
    _check(lib().mapi_autotune_batched(c.handle, int(dtype_code), int(n), int(count), int(iters), C.byref(r),
                                       C.byref(ms)))
    return r.value, ms.value


def mapi_generate_dense(n, seed, ctx=None):
    """The seed-generated problem materialised on the device: (A float32 n x n, w0)."""
    import torch
    c = ctx if ctx is not None else default_context()
    c.sync_stream()
    ld = (n + 3) // 4 * 4
    A = torch.empty((n, ld), dtype=torch.float32, device=torch.device("cuda", c.device))[:, :n]
    w0 = torch.empty(n, dtype=torch.float32, device=A.device)
    _check(lib().mapi_generate_dense(c.handle, int(n), int(seed), C.c_void_p(A.data_ptr()), ld,
                                     C.c_void_p(w0.data_ptr())))
    return A, w0


# ------------------------------------------------------------------ serving
class ServeCfg(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("max_slots", C.c_int32), ("idle_exit_ms", C.c_double)]


class Request(C.Structure):
    _fields_ = [("prob", Problem), ("host_out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double),
                ("norm", C.c_double), ("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double),
                ("t_done_ms", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status"] = STATUS.get(self.status, self.status)
        d["converged"] = bool(self.converged)
        return d


class ServeSummary(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("solves_per_s", C.c_double), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("budget_bytes", C.c_size_t), ("peak_bytes", C.c_size_t),
                ("kernel_launches", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_SIGS.update({
    "mapi_serve_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(ServeCfg), C.POINTER(C.c_void_p)]),
    "mapi_serve_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "mapi_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Result)]),
    "mapi_serve_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int64, C.POINTER(Result)]),
    "mapi_serve_stats": (C.c_int, [C.c_void_p, C.POINTER(ServeSummary)]),
    "mapi_serve_destroy": (None, [C.c_void_p]),
})


def request_generated(n, seed, dtype="f32", method="mapi", max_iters=1000, tol=1e-6, op="min1", stall_iters=0):
    """A device-generated dense request (matrix and start vector from the seed)."""
    p = Problem()
    p.kind = PROB_GENERATED
    p.method = METHODS[method]
    p.gen_n = int(n)
    p.gen_dtype = {"f32": MAPI_F32, "bf16": MAPI_BF16}[dtype]
    p.seed = int(seed)
    p.opts = _opts(max_iters, tol, op, False, 0, stall_iters)
    p.n = int(n)
    return p


def _pinned(a, dtype):
    """A pinned host torch tensor holding `a`: pinned CPU tensors of the right type are used as
    they are; anything else (numpy arrays, pageable tensors) is copied into pinned memory."""
    import numpy as np
    import torch
    if isinstance(a, torch.Tensor) and a.device.type == "cpu" and a.is_pinned() and a.dtype == dtype \
            and a.is_contiguous():
        return a
    t = torch.as_tensor(np.ascontiguousarray(a)) if not isinstance(a, torch.Tensor) else a
    out = torch.empty(t.shape, dtype=dtype, pin_memory=True)
    out.copy_(t.to(dtype))
    return out


def request_csr_host(row_ptr, col, val, alpha=0.85, method="mapi", max_iters=1000, tol=1e-6, stall_iters=0):
    """A PageRank request whose CSR arrays live in pinned host memory, read by the persistent
    kernel at admission.  Pinned CPU torch tensors are used in place; numpy arrays or pageable
    tensors are first copied into pinned memory (kept alive with the request)."""
    import torch
    row_ptr = _pinned(row_ptr, torch.int32)
    col = _pinned(col, torch.int32)
    val = _pinned(val, torch.float32)
    p = Problem()
    p.kind = PROB_CSR
    p.method = METHODS[method]
    n = row_ptr.numel() - 1
    p.H = Csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
              val.data_ptr() if val.numel() else None)
    p.alpha = float(alpha)
    p.opts = _opts(max_iters, tol, "min1", False, 0, stall_iters)
    p._keep = (row_ptr, col, val)
    p.n = n
    return p


class Server:
    """Continuous-batching server (mapi_serve_*) on one device."""

    def __init__(self, budget_bytes, device=0, blocks_per_cu=0, max_slots=0, idle_exit_ms=0.0):
        cfg = ServeCfg(int(blocks_per_cu), int(max_slots), float(idle_exit_ms))
        h = C.c_void_p()
        _check(lib().mapi_serve_create(int(device), int(budget_bytes), C.byref(cfg), C.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, prob, host_out):
        """Queue a request; host_out is a float32 numpy array of length n that receives the result."""
        import numpy as np
        if not (isinstance(host_out, np.ndarray) and host_out.dtype == np.float32 and host_out.flags.c_contiguous
                and host_out.size == prob.n):
            raise ValueError("host_out must be a contiguous float32 array of length n")
        req = Request(prob, host_out.ctypes.data)
        t = C.c_uint64()
        _check(lib().mapi_serve_submit(self.handle, C.byref(req), C.byref(t)))
        self._keep[t.value] = (prob, host_out)
        return t.value

    def poll(self, ticket):
        r = Result()
        st = lib().mapi_serve_poll(self.handle, int(ticket), C.byref(r))
        if st == 7:
            return None
        _check(st)
        self._keep.pop(ticket, None)
        return r.as_dict()

    def wait(self, ticket, timeout_us=-1):
        r = Result()
        st = lib().mapi_serve_wait(self.handle, int(ticket), int(timeout_us), C.byref(r))
        if st == 8:
            return None
        _check(st)
        self._keep.pop(ticket, None)
        return r.as_dict()

    def stats(self):
        s = ServeSummary()
        _check(lib().mapi_serve_stats(self.handle, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().mapi_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
