"""Python binding of librandutv.so (the gfx950 randUTV library).

Argument marshalling only: every step of the factorization runs in the HIP
kernels behind the C ABI declared in include/randutv.h.  PyTorch supplies
device memory and the current HIP stream.  Matrices are torch float64 CUDA
tensors in column-major layout (stride (1, ld)); `colmajor()` makes one.

There is no CPU fallback: loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librandutv.so")

RANDUTV_FP64, RANDUTV_FP32, RANDUTV_BF16X3, RANDUTV_BF16X3_FP32 = 0, 1, 2, 3
RANDUTV_BF16X3_BF16X6 = 4
PREC = {"fp64": RANDUTV_FP64, "fp32": RANDUTV_FP32, "bf16x3": RANDUTV_BF16X3,
        "bf16x3_fp32": RANDUTV_BF16X3_FP32, "bf16x3_bf16x6": RANDUTV_BF16X3_BF16X6}
# Arithmetic codes of randutv_gemm (a product has one arithmetic).
GEMM_PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 4}
FORM_U, FORM_V, ECON_U, ONE_STREAM = 1, 2, 4, 8

_lib = None


class RandUTVError(RuntimeError):
    pass


def lib():
    """Load librandutv.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RandUTVError(
            f"{LIB_PATH} not found: build it with `python -m paper_1703_00998_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, u32, dbl, vp, sz = (ctypes.c_int64, ctypes.c_int, ctypes.c_uint,
                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t)
    L.randutv_random_steps.argtypes = [i64, i64, i64]
    L.randutv_random_steps.restype = i64
    L.randutv_g_cols.argtypes = [i64, i64, i64]
    L.randutv_g_cols.restype = i64
    L.randutv_workspace_size.argtypes = [i64, i64, i64, i32, i32, u32, ctypes.POINTER(sz)]
    L.randutv_workspace_size.restype = i32
    L.randutv_factor.argtypes = [i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, i64,
                                 i64, dbl, i32, u32, vp, sz, ctypes.POINTER(i64), vp]
    L.randutv_factor.restype = i32
    L.randutv_workspace_size_lower.argtypes = [i64, i64, i64, i32, i32, u32, ctypes.POINTER(sz)]
    L.randutv_workspace_size_lower.restype = i32
    L.randutv_factor_lower.argtypes = [i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, i64,
                                       i64, dbl, i32, u32, vp, sz, ctypes.POINTER(i64), vp]
    L.randutv_factor_lower.restype = i32
    L.randutv_g_cols_p.argtypes = [i64, i64, i64, i64]
    L.randutv_g_cols_p.restype = i64
    L.randutv_workspace_size_p.argtypes = [i64, i64, i64, i64, i32, i32, u32,
                                           ctypes.POINTER(sz)]
    L.randutv_workspace_size_p.restype = i32
    L.randutv_factor_p.argtypes = [i64, i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, i64,
                                   i64, dbl, i32, u32, vp, sz, ctypes.POINTER(i64), vp]
    L.randutv_factor_p.restype = i32
    L.randutv_rsvd_workspace_size.argtypes = [i64, i64, i64, i64, i32, i32, ctypes.POINTER(sz)]
    L.randutv_rsvd_workspace_size.restype = i32
    L.randutv_rsvd.argtypes = [i64, i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, vp, i64,
                               i32, vp, sz, ctypes.POINTER(i32), vp]
    L.randutv_rsvd.restype = i32
    L.randutv_gemm.argtypes = [i32, i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl,
                               vp, i64, vp, sz, vp]
    L.randutv_gemm.restype = i32
    L.randutv_panel_work_size.argtypes = [i64, i64]
    L.randutv_panel_work_size.restype = sz
    L.randutv_panel_qr.argtypes = [i64, i64, vp, i64, vp, vp, i64, ctypes.POINTER(i32), vp, sz,
                                   vp]
    L.randutv_panel_qr.restype = i32
    L.randutv_small_svd_work_size.argtypes = [i64, i64]
    L.randutv_small_svd_work_size.restype = sz
    L.randutv_small_svd.argtypes = [i64, ctypes.POINTER(i32), i64, vp, vp, vp, vp, vp, sz, vp]
    L.randutv_small_svd.restype = i32
    L.randutv_profile_begin.argtypes = []
    L.randutv_profile_begin.restype = i32
    L.randutv_profile_begin_class.argtypes = [i32]
    L.randutv_profile_begin_class.restype = i32
    L.randutv_profile_end.argtypes = [i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                      ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    L.randutv_profile_end.restype = i32
    L.randutv_profile_class_name.argtypes = [i32]
    L.randutv_profile_class_name.restype = ctypes.c_char_p
    L.randutv_approx_tape_size.argtypes = [i64, i64, i64, i64]
    L.randutv_approx_tape_size.restype = sz
    L.randutv_approx_work_size.argtypes = [i64, i64, i64, i32, i64]
    L.randutv_approx_work_size.restype = sz
    L.randutv_approx_backward_work_size.argtypes = [i64, i64, i64, i32, i64]
    L.randutv_approx_backward_work_size.restype = sz
    L.randutv_approx.argtypes = [i64, i64, i64, i32, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                 vp, sz, i32, vp, sz, vp]
    L.randutv_approx.restype = i32
    L.randutv_approx_backward.argtypes = [i64, i64, i64, i32, i64, vp, i64, vp, i64, vp, i64, vp,
                                          sz, vp, i64, vp, i64, i32, vp, sz, vp]
    L.randutv_approx_backward.restype = i32
    L.randutv_factor_noalloc.argtypes = [i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, i64,
                                         i64, dbl, i32, u32, ctypes.POINTER(i64), vp]
    L.randutv_factor_noalloc.restype = i32
    L.randutv_status.argtypes = [vp, sz, ctypes.POINTER(i64), vp]
    L.randutv_status.restype = i32
    L.randutv_strerror.argtypes = [i32]
    L.randutv_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


EXPORTS = ["randutv_random_steps", "randutv_g_cols", "randutv_workspace_size",
           "randutv_factor", "randutv_g_cols_p", "randutv_workspace_size_p", "randutv_factor_p",
           "randutv_workspace_size_lower", "randutv_factor_lower", "randutv_rsvd_workspace_size", "randutv_rsvd", "randutv_gemm",
           "randutv_panel_work_size", "randutv_panel_qr",
           "randutv_small_svd_work_size", "randutv_small_svd", "randutv_strerror",
           "randutv_status", "randutv_factor_noalloc",
           "randutv_profile_begin", "randutv_profile_begin_class", "randutv_profile_end", "randutv_profile_class_name",
           "randutv_approx_tape_size", "randutv_approx_work_size", "randutv_approx",
           "randutv_approx_backward_work_size", "randutv_approx_backward"]


def profile_begin(only=None):
    """Start per-kernel timing; `only` = a class name restricts the events to
    that kernel class."""
    if only is None:
        _check(lib().randutv_profile_begin(), "randutv_profile_begin")
        return
    for c in range(64):
        name = lib().randutv_profile_class_name(c).decode()
        if not name:
            break
        if name == only:
            _check(lib().randutv_profile_begin_class(c), "randutv_profile_begin_class")
            return
    raise RandUTVError(f"unknown kernel class {only}")


def profile_end(max_classes=64):
    """Per kernel class: {name: (milliseconds, algorithmic flops, algorithmic
    bytes, launches)}."""
    ms = (ctypes.c_double * max_classes)()
    fl = (ctypes.c_double * max_classes)()
    by = (ctypes.c_double * max_classes)()
    ln = (ctypes.c_int64 * max_classes)()
    nc = lib().randutv_profile_end(max_classes, ms, fl, by, ln)
    if nc < 0:
        _check(nc, "randutv_profile_end")
    return {lib().randutv_profile_class_name(c).decode(): (ms[c], fl[c], by[c], int(ln[c]))
            for c in range(nc)}


def _check(status, what):
    if status != 0:
        msg = lib().randutv_strerror(status).decode()
        raise RandUTVError(f"{what} failed with status {status}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ld(t, rows):
    """Leading dimension of a column-major 2-D tensor (stride (1, ld))."""
    if t.dim() != 2 or t.dtype != torch.float64 or not t.is_cuda:
        raise RandUTVError("expected a 2-D float64 CUDA tensor")
    if t.shape[0] != rows:
        raise RandUTVError(f"expected {rows} rows, got {t.shape[0]}")
    if t.numel() == 0:
        return max(1, rows)
    if t.shape[0] > 1 and t.stride(0) != 1:
        raise RandUTVError("tensor must be column-major (stride (1, ld))")
    return max(1, rows, t.stride(1) if t.shape[1] > 1 else rows)


def colmajor(x, device="cuda"):
    """Column-major float64 tensor on `device` from a numpy array or tensor."""
    t = torch.as_tensor(x, dtype=torch.float64).to(device)
    return t.T.contiguous().T


def empty_colmajor(m, n, device="cuda"):
    return torch.empty((n, m), dtype=torch.float64, device=device).T


def random_steps(m, n, b):
    return int(lib().randutv_random_steps(m, n, b))


def g_cols(m, n, b, p=0):
    if p:
        return int(lib().randutv_g_cols_p(m, n, b, p))
    return int(lib().randutv_g_cols(m, n, b))


def workspace_size(m, n, b, q=1, prec="fp64", form_u=True, form_v=True, p=0, econ_u=False):
    flags = (FORM_U if form_u else 0) | (FORM_V if form_v else 0) | (ECON_U if econ_u else 0)
    out = ctypes.c_size_t(0)
    if p:
        _check(lib().randutv_workspace_size_p(m, n, b, p, q, PREC[prec], flags,
                                              ctypes.byref(out)), "randutv_workspace_size_p")
    else:
        _check(lib().randutv_workspace_size(m, n, b, q, PREC[prec], flags, ctypes.byref(out)),
               "randutv_workspace_size")
    return int(out.value)


def workspace(nbytes, device="cuda"):
    """Device workspace (torch-allocated, 256-byte aligned)."""
    return torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)


def _aligned_ptr(ws):
    p = ws.data_ptr()
    return ctypes.c_void_p((p + 255) & ~255), ws.numel() - (((p + 255) & ~255) - p)


def randutv_factor(T, G, b, q, U=None, V=None, k_stop=0, tol=0.0, prec="fp64", work=None,
                   sync=True, p=0, one_stream=False):
    """In-place randUTV of T (m x n column-major FP64, overwritten by T).

    U (m x m, or m x min(m, n) for the economy form) and V (n x n) are
    written when given.  p > 0 over-samples
    (randutv_factor_p; G then has b + p columns per randomized step).
    Returns k (the number of leading columns reduced) when sync=True, else
    None (enqueue only).
    """
    m, n = T.shape
    ldt = _ld(T, m)
    gc = g_cols(m, n, b, p)
    ldg = _ld(G, m) if (G is not None and G.numel() > 0) else max(m, 1)
    if gc > 0 and (G is None or G.shape[1] < gc):
        raise RandUTVError(f"G needs {gc} columns")
    ldu = _ld(U, m) if U is not None else m
    ldv = _ld(V, n) if V is not None else n
    econ = U is not None and U.shape[1] == min(m, n) and min(m, n) < m
    if U is not None and U.shape[1] not in (m, min(m, n)):
        raise RandUTVError("U must have m or min(m, n) columns")
    flags = (FORM_U if U is not None else 0) | (FORM_V if V is not None else 0) | \
        (ECON_U if econ else 0) | (ONE_STREAM if one_stream else 0)
    need = workspace_size(m, n, b, q, prec, U is not None, V is not None, p=p, econ_u=econ)
    if work is None:
        work = workspace(need, T.device)
    wp, wbytes = _aligned_ptr(work)
    if wbytes < need:
        raise RandUTVError("workspace too small")
    k = ctypes.c_int64(0)
    kp = ctypes.byref(k) if (sync or tol > 0) else None
    gp = _ptr(G) if gc > 0 else ctypes.c_void_p(0)
    if p:
        st = lib().randutv_factor_p(
            m, n, b, p, q, _ptr(T), ldt, gp, ldg, _ptr(U), ldu, _ptr(V), ldv, int(k_stop),
            float(tol), PREC[prec], flags, wp, wbytes, kp, _stream())
        _check(st, "randutv_factor_p")
    else:
        st = lib().randutv_factor(
            m, n, b, q, _ptr(T), ldt, gp, ldg, _ptr(U), ldu, _ptr(V), ldv, int(k_stop),
            float(tol), PREC[prec], flags, wp, wbytes, kp, _stream())
        _check(st, "randutv_factor")
    return int(k.value) if (sync or tol > 0) else None


def randutv_factor_noalloc(T, G, b, q, U=None, V=None, k_stop=0, tol=0.0, prec="fp64",
                           sync=True):
    """randutv_factor on the library's own device workspace (no allocation by
    the call).  Returns k when sync=True, else None."""
    m, n = T.shape
    ldt = _ld(T, m)
    gc = g_cols(m, n, b)
    ldg = _ld(G, m) if (G is not None and G.numel() > 0) else max(m, 1)
    if gc > 0 and (G is None or G.shape[1] < gc):
        raise RandUTVError(f"G needs {gc} columns")
    ldu = _ld(U, m) if U is not None else m
    ldv = _ld(V, n) if V is not None else n
    flags = (FORM_U if U is not None else 0) | (FORM_V if V is not None else 0)
    k = ctypes.c_int64(0)
    kp = ctypes.byref(k) if (sync or tol > 0) else None
    st = lib().randutv_factor_noalloc(
        m, n, b, q, _ptr(T), ldt, _ptr(G) if gc > 0 else ctypes.c_void_p(0), ldg, _ptr(U), ldu,
        _ptr(V), ldv, int(k_stop), float(tol), PREC[prec], flags, kp, _stream())
    _check(st, "randutv_factor_noalloc")
    return int(k.value) if (sync or tol > 0) else None


def randutv_status(work, raise_on_error=True):
    """Wait for the current stream and return (status, k) of the last
    factorization or randomized SVD enqueued with workspace `work`
    (randutv_status).  Raises on a nonzero status unless
    raise_on_error=False."""
    wp, wbytes = _aligned_ptr(work)
    k = ctypes.c_int64(-1)
    st = lib().randutv_status(wp, wbytes, ctypes.byref(k), _stream())
    if raise_on_error:
        _check(st, "randutv_status")
    return st, int(k.value)


def workspace_size_lower(m, n, b, q=1, prec="fp64", form_u=True, form_v=True):
    flags = (FORM_U if form_u else 0) | (FORM_V if form_v else 0)
    out = ctypes.c_size_t(0)
    _check(lib().randutv_workspace_size_lower(m, n, b, q, PREC[prec], flags, ctypes.byref(out)),
           "randutv_workspace_size_lower")
    return int(out.value)


def randutv_factor_lower(T, G, b, q, U=None, V=None, k_stop=0, tol=0.0, prec="fp64",
                         work=None, sync=True):
    """In-place A = U L V^T with L lower triangular (T: m x n column-major
    FP64, overwritten by L); G is the n x g_cols(n, m, b) Gaussian of the
    transposed problem.  Returns k when sync=True."""
    m, n = T.shape
    ldt = _ld(T, m)
    gc = g_cols(n, m, b)
    ldg = _ld(G, n) if (G is not None and G.numel() > 0) else max(n, 1)
    if gc > 0 and (G is None or G.shape[1] < gc):
        raise RandUTVError(f"G needs {gc} columns")
    ldu = _ld(U, m) if U is not None else m
    ldv = _ld(V, n) if V is not None else n
    flags = (FORM_U if U is not None else 0) | (FORM_V if V is not None else 0)
    if work is None:
        work = workspace(workspace_size_lower(m, n, b, q, prec, U is not None, V is not None),
                         T.device)
    wp, wbytes = _aligned_ptr(work)
    k = ctypes.c_int64(0)
    st = lib().randutv_factor_lower(
        m, n, b, q, _ptr(T), ldt, _ptr(G) if gc > 0 else ctypes.c_void_p(0), ldg, _ptr(U), ldu,
        _ptr(V), ldv, int(k_stop), float(tol), PREC[prec], flags, wp, wbytes,
        ctypes.byref(k) if (sync or tol > 0) else None, _stream())
    _check(st, "randutv_factor_lower")
    return int(k.value) if (sync or tol > 0) else None


def randutv_rsvd(A, G, k, q, p=0, prec="fp64", work=None, sync=True):
    """Rank-k randomized SVD of A (m x n column-major FP64) with the m x (k+p)
    Gaussian G: returns (U m x k, D (k,), V n x k).  sync=True waits and
    checks the SVD's convergence."""
    m, n = A.shape
    out = ctypes.c_size_t(0)
    _check(lib().randutv_rsvd_workspace_size(m, n, k, p, q, PREC[prec], ctypes.byref(out)),
           "randutv_rsvd_workspace_size")
    if work is None:
        work = workspace(int(out.value), A.device)
    wp, wbytes = _aligned_ptr(work)
    if G.shape[1] < k + p:
        raise RandUTVError(f"G needs {k + p} columns")
    U = empty_colmajor(m, k, A.device)
    V = empty_colmajor(n, k, A.device)
    D = torch.empty(k, dtype=torch.float64, device=A.device)
    sw = ctypes.c_int32(0)
    _check(lib().randutv_rsvd(m, n, k, p, q, _ptr(A), _ld(A, m), _ptr(G), _ld(G, m), _ptr(U),
                              _ld(U, m), _ptr(D), _ptr(V), _ld(V, n), PREC[prec], wp, wbytes,
                              ctypes.byref(sw) if sync else None, _stream()),
           "randutv_rsvd")
    return U, D, V


def randutv_gemm(C, A, B, ta=False, tb=False, alpha=1.0, beta=0.0, prec="fp64", work=None):
    """C = alpha op(A) op(B) + beta C on the library's MFMA GEMM."""
    M, N = C.shape
    K = A.shape[0] if ta else A.shape[1]
    lda = _ld(A, A.shape[0])
    ldb = _ld(B, B.shape[0])
    ldc = _ld(C, M)
    wp, wb = (_aligned_ptr(work) if work is not None else (ctypes.c_void_p(0), 0))
    _check(lib().randutv_gemm(GEMM_PREC[prec], int(ta), int(tb), M, N, K, alpha, _ptr(A), lda,
                              _ptr(B), ldb, beta, _ptr(C), ldc, wp, wb, _stream()),
           "randutv_gemm")
    return C


def randutv_panel_qr(P, tau, Tw):
    """In-place Householder QR of the tall panel P; fills tau and Tw.
    Returns True when the column-by-column path ran (ill-conditioned panel)."""
    Mp, nb = P.shape
    need = int(lib().randutv_panel_work_size(Mp, nb))
    if need == 0:
        raise RandUTVError(f"randutv_panel_qr: unsupported panel shape {Mp} x {nb}")
    ws = workspace(need, P.device)
    wp, wb = _aligned_ptr(ws)
    fb = ctypes.c_int32(0)
    _check(lib().randutv_panel_qr(Mp, nb, _ptr(P), _ld(P, Mp), _ptr(tau), _ptr(Tw),
                                  _ld(Tw, Tw.shape[0]), ctypes.byref(fb), wp, wb, _stream()),
           "randutv_panel_qr")
    return bool(fb.value)


def randutv_small_svd(R, nbs):
    """Batched SVD of square blocks: R is (count, ld, ld) column-major stack
    (tensor of shape (count, ld, ld) whose [i] is the transpose view)."""
    count, ld, _ = R.shape
    Us = torch.empty_like(R)
    Vs = torch.empty_like(R)
    D = torch.zeros((count, ld), dtype=torch.float64, device=R.device)
    need = int(lib().randutv_small_svd_work_size(count, ld))
    ws = workspace(need, R.device)
    wp, wb = _aligned_ptr(ws)
    arr = (ctypes.c_int * count)(*[int(x) for x in nbs])
    st = lib().randutv_small_svd(count, arr, ld, _ptr(R), _ptr(Us), _ptr(Vs), _ptr(D), wp, wb,
                                 _stream())
    if st not in (0, 1):
        _check(st, "randutv_small_svd")
    return Us, D, Vs, st


def randutv_approx(A, G, b, q, k, prec="fp64", want_ak=True):
    """Truncated approximation through the C ABI.  A, G: FP64 column-major
    device tensors.  Returns (Ak or None, Uk, tape)."""
    m, n = A.shape
    tb = int(lib().randutv_approx_tape_size(m, n, b, k))
    wb = int(lib().randutv_approx_work_size(m, n, b, q, k))
    if tb == 0 or wb == 0:
        raise RandUTVError(f"randutv_approx: unsupported shape m={m} n={n} b={b} q={q} k={k}")
    tape = torch.empty(tb // 8, dtype=torch.float64, device=A.device)
    ws = workspace(wb, A.device)
    wp, wbytes = _aligned_ptr(ws)
    Uk = empty_colmajor(m, k, A.device)
    Ak = empty_colmajor(m, n, A.device) if want_ak else None
    _check(lib().randutv_approx(m, n, b, q, k, _ptr(A), _ld(A, m), _ptr(G), _ld(G, m),
                                _ptr(Ak) if Ak is not None else None,
                                _ld(Ak, m) if Ak is not None else m, _ptr(Uk), _ld(Uk, m),
                                _ptr(tape), tb, PREC[prec], wp, wbytes, _stream()),
           "randutv_approx")
    return Ak, Uk, tape


def randutv_approx_backward(A, G, b, q, k, Uk, tape, Akbar, prec="fp64"):
    """Abar = J^T Akbar for A -> A_k (G fixed), through the C ABI."""
    m, n = A.shape
    wb = int(lib().randutv_approx_backward_work_size(m, n, b, q, k))
    if wb == 0:
        raise RandUTVError("randutv_approx_backward: unsupported shape")
    ws = workspace(wb, A.device)
    wp, wbytes = _aligned_ptr(ws)
    Abar = empty_colmajor(m, n, A.device)
    _check(lib().randutv_approx_backward(m, n, b, q, k, _ptr(A), _ld(A, m), _ptr(G), _ld(G, m),
                                         _ptr(Uk), _ld(Uk, m), _ptr(tape), tape.numel() * 8,
                                         _ptr(Akbar), _ld(Akbar, m), _ptr(Abar), _ld(Abar, m),
                                         PREC[prec], wp, wbytes, _stream()),
           "randutv_approx_backward")
    return Abar
