"""paper_1401_7962_amd -- full-pivot Gauss-Jordan inversion on MI355X.

Thin Python binding over the C ABI of ``libgj.so`` (``include/gj.h``).  The
functions here only marshal arguments: every step of the elimination runs in
the library's HIP kernels.  PyTorch supplies device memory and the stream.
If the library is missing, every call raises: there is no CPU fallback.

Entry points (same names as the C ABI):
    gj_invert, gj_invert_noalloc, gj_invert_batched, gj_det, gj_solve,
    gj_workspace_size, gj_status_string, gj_onchip_max_n, gj_dgemm

Every caller-supplied buffer is checked here (device, dtype, contiguity and
extent) before the library is called, so a short buffer raises GJError
instead of reaching a kernel.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgj.so")

GJ_OK, GJ_E_INVALID_ARG, GJ_E_WORKSPACE, GJ_E_HIP, GJ_E_UNSUPPORTED = 0, -1, -2, -3, -4
GJ_RES_OK, GJ_RES_SINGULAR, GJ_RES_NONFINITE, GJ_RES_REFINE_FALLBACK = 0, 1, 2, 3
GJ_PREC_FP64, GJ_PREC_FP32_REFINED = 0, 1
GJ_FLAG_REUSE_PLAN = 1
GJ_FLAG_PIVOT_PARTIAL = 2   # partial pivoting on |a| (row swaps only)
GJ_FLAG_PIVOT_PROGRAM = 4   # the section-3 program's rule: largest positive value in column k
GJ_FLAG_ACCURATE = 8   # refined path: extra updates with error-free split residuals
GJ_FLAG_BLOCKED = 16   # delayed updates (trailing-block steps, matrix-core products per panel); FP64 or the refined path's FP32 stage
GJ_OP_INVERT, GJ_OP_DET, GJ_OP_INVERT_BATCHED, GJ_OP_SOLVE = 0, 1, 2, 3


class gj_result(ctypes.Structure):
    _fields_ = [
        ("code", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("det_sign", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("det_mant", ctypes.c_double),
        ("det_exp", ctypes.c_int64),
        ("det", ctypes.c_double),
        ("logabsdet", ctypes.c_double),
        ("resid", ctypes.c_double),
    ]


RESULT_BYTES = ctypes.sizeof(gj_result)  # 56


class gj_opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("want_resid", ctypes.c_int32),
        ("max_refine_iters", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("zero_tol", ctypes.c_double),
        ("step_events", ctypes.c_void_p * 2),
    ]


class GJError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgj.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise GJError(f"libgj.so not built ({path}); run __graft_entry__.build()")
    import torch  # noqa: F401  -- make torch's HIP runtime the one the library binds to
    lib = ctypes.CDLL(path)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.gj_invert.argtypes = [I32, P, I64, P, I64, P, P, P, P, P, SZ, P]
    lib.gj_invert.restype = I32
    lib.gj_invert_noalloc.argtypes = [I32, P, I64, P, I64, P, P, P, P, P]
    lib.gj_invert_noalloc.restype = I32
    lib.gj_invert_batched.argtypes = [I32, P, P, P, P, P, P, P, P, P, P, SZ, P]
    lib.gj_invert_batched.restype = I32
    lib.gj_det.argtypes = [I32, P, I64, P, P, P, P, P, SZ, P]
    lib.gj_det.restype = I32
    lib.gj_solve.argtypes = [I32, I32, P, I64, P, I64, P, I64, P, P, P, P, P, SZ, P]
    lib.gj_solve.restype = I32
    lib.gj_workspace_size.argtypes = [I32, I32, P, P]
    lib.gj_workspace_size.restype = SZ
    lib.gj_status_string.argtypes = [I32]
    lib.gj_status_string.restype = ctypes.c_char_p
    D = ctypes.c_double
    lib.gj_dgemm.argtypes = [I32, I32, I32, D, P, I64, P, I64, D, P, I64, D, P, I64, P]
    lib.gj_dgemm.restype = I32
    F = ctypes.c_float
    lib.gj_sgemm.argtypes = [I32, I32, I32, F, P, I64, P, I64, F, P, I64, F, P, I64, P]
    lib.gj_sgemm.restype = I32
    lib.gj_onchip_max_n.argtypes = [I32]
    lib.gj_onchip_max_n.restype = I32
    _lib = lib
    return lib


EXPORTS = ("gj_invert", "gj_invert_noalloc", "gj_invert_batched", "gj_det", "gj_solve",
           "gj_workspace_size", "gj_status_string", "gj_onchip_max_n", "gj_dgemm", "gj_sgemm")

# size of gj_invert_noalloc's built-in scratch array (GJ_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


def make_opts(precision=GJ_PREC_FP64, want_resid=False, max_refine_iters=10, flags=0,
              zero_tol=-1.0, step_events=None) -> gj_opts:
    o = gj_opts()
    o.precision = precision
    o.want_resid = 1 if want_resid else 0
    o.max_refine_iters = max_refine_iters
    o.flags = flags
    o.zero_tol = zero_tol
    if step_events is not None:
        o.step_events[0] = step_events[0]
        o.step_events[1] = step_events[1]
    return o


def _check(status: int):
    if status != GJ_OK:
        raise GJError(gj_status_string(status))


def gj_status_string(code: int) -> str:
    return load_library().gj_status_string(int(code)).decode()


def gj_onchip_max_n(precision: int = GJ_PREC_FP64) -> int:
    return int(load_library().gj_onchip_max_n(precision))


def gj_workspace_size(op: int, n_or_batch: int, n_host=None, opts: gj_opts | None = None) -> int:
    lib = load_library()
    arr = None
    if n_host is not None:
        import numpy as np
        arr = np.ascontiguousarray(n_host, dtype=np.int32)
    return int(lib.gj_workspace_size(op, n_or_batch,
                                      arr.ctypes.data_as(ctypes.c_void_p) if arr is not None else None,
                                      ctypes.byref(opts) if opts is not None else None))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _on(t, name, device):
    import torch
    if not isinstance(t, torch.Tensor):
        raise GJError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.device != device:
        raise GJError(f"{name} must be on {device}")


def _check_matrix(t, name, rows, cols, device):
    """A row-major float64 matrix of at least rows x cols on ``device``."""
    import torch
    _on(t, name, device)
    if t.dtype != torch.float64 or t.dim() != 2:
        raise GJError(f"{name} must be a 2-D float64 tensor")
    if t.shape[0] < rows or t.shape[1] < cols or t.stride(1) != 1 or t.stride(0) < cols:
        raise GJError(f"{name} must be row-major with at least {rows} x {cols} elements")


def _check_vec(t, name, dtype, count, device):
    """A contiguous tensor of ``dtype`` holding at least ``count`` elements."""
    _on(t, name, device)
    if t.dtype != dtype or not t.is_contiguous():
        raise GJError(f"{name} must be a contiguous {dtype} tensor")
    if t.numel() < count:
        raise GJError(f"{name} holds {t.numel()} elements; {count} are needed")


def _check_bytes(t, name, nbytes, device):
    """A contiguous tensor of at least ``nbytes`` bytes."""
    _on(t, name, device)
    if not t.is_contiguous():
        raise GJError(f"{name} must be contiguous")
    if t.numel() * t.element_size() < nbytes:
        raise GJError(f"{name} holds {t.numel() * t.element_size()} bytes; {nbytes} are needed")


def _res_tensor(count: int, device):
    import torch
    return torch.empty(count * RESULT_BYTES, dtype=torch.uint8, device=device)


def results_to_dicts(res_tensor) -> list:
    """Copy device gj_result records to the host as dicts."""
    raw = res_tensor.detach().cpu().numpy().tobytes()
    out = []
    for i in range(len(raw) // RESULT_BYTES):
        r = gj_result.from_buffer_copy(raw[i * RESULT_BYTES:(i + 1) * RESULT_BYTES])
        out.append({name: getattr(r, name) for name, _ in gj_result._fields_})
    return out


def gj_invert(A, X=None, ipiv=None, jpiv=None, res=None, opts: gj_opts | None = None, ws=None,
              stream=None):
    """Invert one square FP64 CUDA tensor.  Returns (X, ipiv, jpiv, res) where
    res is the raw device record (use results_to_dicts)."""
    lib = load_library()
    _check_square(A)
    n = A.shape[0]
    dev = A.device
    X, ipiv, jpiv, res = _single_outputs(n, X, ipiv, jpiv, res, dev)
    need = gj_workspace_size(GJ_OP_INVERT, n, None, opts)
    if need == 0:
        raise GJError("gj_invert: unsupported size or options")
    if ws is None:
        ws = _workspace(need, dev)
    _check_bytes(ws, "ws", need, dev)
    st = lib.gj_invert(n, _ptr(A), A.stride(0), _ptr(X), X.stride(0), _ptr(ipiv), _ptr(jpiv),
                       _ptr(res), ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                       ws.numel() * ws.element_size(), _stream_ptr(stream))
    _check(st)
    return X, ipiv, jpiv, res


def _single_outputs(n, X, ipiv, jpiv, res, dev):
    """Allocate the outputs not given; check the ones given."""
    import torch
    X = torch.empty((n, n), dtype=torch.float64, device=dev) if X is None else X
    ipiv = torch.empty(n, dtype=torch.int32, device=dev) if ipiv is None else ipiv
    jpiv = torch.empty(n, dtype=torch.int32, device=dev) if jpiv is None else jpiv
    res = _res_tensor(1, dev) if res is None else res
    _check_matrix(X, "X", n, n, dev)
    _check_vec(ipiv, "ipiv", torch.int32, n, dev)
    _check_vec(jpiv, "jpiv", torch.int32, n, dev)
    _check_bytes(res, "res", RESULT_BYTES, dev)
    return X, ipiv, jpiv, res


def _check_square(A):
    import torch
    if (not isinstance(A, torch.Tensor) or A.dim() != 2 or A.shape[0] != A.shape[1]
            or A.dtype != torch.float64 or not A.is_cuda):
        raise GJError("A must be a square float64 CUDA tensor")
    if A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise GJError("A must be row-major (unit column stride)")


def gj_invert_noalloc(A, X=None, ipiv=None, jpiv=None, res=None, opts: gj_opts | None = None,
                      stream=None):
    """gj_invert with the library's built-in scratch array instead of a
    workspace (the C entry point allocates nothing; outputs not given are
    allocated here).  Calls that overlap in time on one GPU race on that
    array.  Returns (X, ipiv, jpiv, res)."""
    lib = load_library()
    _check_square(A)
    n = A.shape[0]
    X, ipiv, jpiv, res = _single_outputs(n, X, ipiv, jpiv, res, A.device)
    st = lib.gj_invert_noalloc(n, _ptr(A), A.stride(0), _ptr(X), X.stride(0), _ptr(ipiv),
                               _ptr(jpiv), _ptr(res),
                               ctypes.byref(opts) if opts is not None else None,
                               _stream_ptr(stream))
    _check(st)
    return X, ipiv, jpiv, res


def gj_dgemm(A, B, C=None, D=None, alpha=1.0, beta=0.0, gamma=0.0, stream=None):
    """D = alpha A B + beta C + gamma I on the FP64 matrix cores (2-D float64
    CUDA tensors, unit column stride)."""
    import torch
    lib = load_library()
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise GJError("inner dimensions differ")
    if D is None:
        D = torch.empty((M, N), dtype=torch.float64, device=A.device)
    st = lib.gj_dgemm(M, N, K, float(alpha), _ptr(A), A.stride(0), _ptr(B), B.stride(0),
                      float(beta), _ptr(C) if C is not None else None,
                      C.stride(0) if C is not None else N, float(gamma), _ptr(D), D.stride(0),
                      _stream_ptr(stream))
    _check(st)
    return D


def gj_sgemm(A, B, C=None, D=None, alpha=1.0, beta=0.0, gamma=0.0, stream=None):
    """D = alpha A B + beta C + gamma I on the FP32 matrix cores (2-D float32
    CUDA tensors, unit column stride)."""
    import torch
    lib = load_library()
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise GJError("inner dimensions differ")
    for name, T in (("A", A), ("B", B), ("C", C), ("D", D)):
        if T is not None and (T.dtype != torch.float32 or not T.is_cuda or T.dim() != 2
                              or T.stride(1) != 1):
            raise GJError(f"{name} must be a 2-D float32 CUDA tensor with unit column stride")
    if D is None:
        D = torch.empty((M, N), dtype=torch.float32, device=A.device)
    if D.shape != (M, N) or (C is not None and C.shape != (M, N)):
        raise GJError("C and D must be M x N")
    st = lib.gj_sgemm(M, N, K, float(alpha), _ptr(A), A.stride(0), _ptr(B), B.stride(0),
                      float(beta), _ptr(C) if C is not None else None,
                      C.stride(0) if C is not None else N, float(gamma), _ptr(D), D.stride(0),
                      _stream_ptr(stream))
    _check(st)
    return D


def gj_solve(A, B, X=None, ipiv=None, jpiv=None, res=None, opts: gj_opts | None = None, ws=None,
             stream=None):
    """X = A^-1 B for a square FP64 CUDA tensor A and an n x m FP64 CUDA
    tensor B (both row-major).  Returns (X, ipiv, jpiv, res)."""
    import torch
    lib = load_library()
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.dtype != torch.float64 or not A.is_cuda:
        raise GJError("A must be a square float64 CUDA tensor")
    if B.dim() != 2 or B.shape[0] != A.shape[0] or B.dtype != torch.float64 or not B.is_cuda:
        raise GJError("B must be an n x m float64 CUDA tensor")
    if A.stride(1) != 1 or B.stride(1) != 1:
        raise GJError("A and B must be row-major (unit column stride)")
    n, m = A.shape[0], B.shape[1]
    dev = A.device
    if B.device != dev:
        raise GJError(f"B must be on {dev}")
    X = torch.empty((n, m), dtype=torch.float64, device=dev) if X is None else X
    ipiv = torch.empty(n, dtype=torch.int32, device=dev) if ipiv is None else ipiv
    jpiv = torch.empty(n, dtype=torch.int32, device=dev) if jpiv is None else jpiv
    res = _res_tensor(1, dev) if res is None else res
    _check_matrix(X, "X", n, m, dev)
    _check_vec(ipiv, "ipiv", torch.int32, n, dev)
    _check_vec(jpiv, "jpiv", torch.int32, n, dev)
    _check_bytes(res, "res", RESULT_BYTES, dev)
    need = gj_workspace_size(GJ_OP_SOLVE, n, [m], opts)
    if need == 0:
        raise GJError("gj_solve: unsupported size or options")
    if ws is None:
        ws = _workspace(need, dev)
    _check_bytes(ws, "ws", need, dev)
    st = lib.gj_solve(n, m, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(X), X.stride(0),
                      _ptr(ipiv), _ptr(jpiv), _ptr(res),
                      ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                      ws.numel() * ws.element_size(), _stream_ptr(stream))
    _check(st)
    return X, ipiv, jpiv, res


def gj_det(A, ipiv=None, jpiv=None, res=None, opts: gj_opts | None = None, ws=None, stream=None):
    import torch
    lib = load_library()
    _check_square(A)
    n = A.shape[0]
    dev = A.device
    ipiv = torch.empty(n, dtype=torch.int32, device=dev) if ipiv is None else ipiv
    jpiv = torch.empty(n, dtype=torch.int32, device=dev) if jpiv is None else jpiv
    res = _res_tensor(1, dev) if res is None else res
    _check_vec(ipiv, "ipiv", torch.int32, n, dev)
    _check_vec(jpiv, "jpiv", torch.int32, n, dev)
    _check_bytes(res, "res", RESULT_BYTES, dev)
    need = gj_workspace_size(GJ_OP_DET, n, None, opts)
    if need == 0:
        raise GJError("gj_det: unsupported size or options")
    if ws is None:
        ws = _workspace(need, dev)
    _check_bytes(ws, "ws", need, dev)
    st = lib.gj_det(n, _ptr(A), A.stride(0), _ptr(ipiv), _ptr(jpiv), _ptr(res),
                    ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                    ws.numel() * ws.element_size(), _stream_ptr(stream))
    _check(st)
    return ipiv, jpiv, res


def gj_invert_batched(sizes, offsets, A, X=None, piv_offsets=None, ipiv=None, jpiv=None, res=None,
                      opts: gj_opts | None = None, ws=None, stream=None):
    """Invert a packed batch.  ``sizes``/``offsets``/``piv_offsets`` are host
    arrays; A (and X) are 1-D float64 CUDA tensors holding the members
    row-major at the given element offsets."""
    import numpy as np
    import torch
    lib = load_library()
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    batch = int(sizes.shape[0])
    if piv_offsets is None:
        piv_offsets = np.zeros(batch, dtype=np.int64)
        piv_offsets[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    piv_offsets = np.ascontiguousarray(piv_offsets, dtype=np.int64)
    if batch < 1 or offsets.shape[0] != batch or piv_offsets.shape[0] != batch:
        raise GJError("sizes, offsets and piv_offsets must have one entry per member")
    if (sizes < 1).any() or (offsets < 0).any() or (piv_offsets < 0).any():
        raise GJError("orders must be >= 1 and offsets >= 0")
    if not isinstance(A, torch.Tensor) or not A.is_cuda:
        raise GJError("A must be a CUDA tensor")
    dev = A.device
    span = int((offsets + sizes.astype(np.int64) ** 2).max())
    total_piv = int((piv_offsets + sizes).max())
    X = torch.empty_like(A) if X is None else X
    ipiv = torch.empty(total_piv, dtype=torch.int32, device=dev) if ipiv is None else ipiv
    jpiv = torch.empty(total_piv, dtype=torch.int32, device=dev) if jpiv is None else jpiv
    res = _res_tensor(batch, dev) if res is None else res
    _check_vec(A, "A", torch.float64, span, dev)
    _check_vec(X, "X", torch.float64, span, dev)
    _check_vec(ipiv, "ipiv", torch.int32, total_piv, dev)
    _check_vec(jpiv, "jpiv", torch.int32, total_piv, dev)
    _check_bytes(res, "res", batch * RESULT_BYTES, dev)
    need = gj_workspace_size(GJ_OP_INVERT_BATCHED, batch, sizes, opts)
    if need == 0:
        raise GJError("invalid batch")
    if ws is None:
        ws = _workspace(need, dev)
    _check_bytes(ws, "ws", need, dev)
    st = lib.gj_invert_batched(batch, sizes.ctypes.data_as(ctypes.c_void_p),
                               offsets.ctypes.data_as(ctypes.c_void_p), _ptr(A), _ptr(X),
                               piv_offsets.ctypes.data_as(ctypes.c_void_p), _ptr(ipiv), _ptr(jpiv),
                               _ptr(res), ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                               ws.numel() * ws.element_size(), _stream_ptr(stream))
    _check(st)
    return X, ipiv, jpiv, res, piv_offsets
