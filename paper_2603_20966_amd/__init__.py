"""MI355X (gfx950) library for the sketch Y = A * Omega(seed) with a generated operand.

Python binding of the C ABI in ``include/sketch.h`` (libsketch.so, built by
``paper_2603_20966_amd.build``); the request server of ``include/sketch_serve.h``
is bound in ``paper_2603_20966_amd.serve``.  The functions carry the ABI's names and only
marshal arguments: torch tensors give device pointers and the current HIP
stream; every step of the computation runs in the library's kernels.  There is
no fallback: if the library is not built, every call raises.

Paper: "Communication Lower Bounds and Algorithms for Sketching with Random
Dense Matrices" (SPAA '26): Sec. 4 (B = A*Omega), Alg. 1 (GenRandom, local
product, Reduce-Scatter of a contraction split), Sec. 6.3 (Philox; Omega
generated instead of communicated).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsketch.so")

SK_A_F32, SK_A_BF16, SK_A_FP8_E4M3 = 0, 1, 2
SK_Y_F32, SK_Y_F64 = 0, 1
SK_DIST = {"normal": 0, "uniform": 1, "rademacher": 2}
STATUS = {0: "SK_OK", -1: "SK_EINVAL", -2: "SK_EDTYPE", -3: "SK_EALIGN", -4: "SK_EWORKSPACE",
          -5: "SK_EHIP", -6: "SK_ENOMEM", -7: "SK_EUNSUPPORTED", -8: "SK_EBUDGET",
          -9: "SK_EQUEUE", -10: "SK_ETIMEOUT", -11: "SK_ESCRATCH"}

_lib = None
_lock = threading.Lock()


class SketchError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = sketch_status_string(status) if _lib is not None else ""
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")


def lib() -> ctypes.CDLL:
    """The loaded libsketch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2603_20966_amd.build.build() "
                               "(the HIP library is required; there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, u64, sz, i32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t,
                                ctypes.c_int)
        L.sketch_abi_version.argtypes = []
        L.sketch_abi_version.restype = i32
        L.sketch_status_string.argtypes = [i32]
        L.sketch_status_string.restype = ctypes.c_char_p
        L.sketch_workspace_size.argtypes = [i32, i32, i64, i64, i64, i64]
        L.sketch_workspace_size.restype = sz
        L.sketch_strip_width.argtypes = [i32, i64]
        L.sketch_strip_width.restype = i64
        L.sketch_gen_matmul.argtypes = [P, i32, i64, i64, i64, P, u64, i64, i64, i64, P, i32, i64,
                                        i32, P, sz, P]
        L.sketch_gen_matmul_noalloc.argtypes = [P, i32, i64, i64, i64, P, u64, i64, i64, i64, P,
                                                i32, i64, i32, P]
        L.sketch_gen_matmul_reduce.argtypes = [P, i64, i32, i64, P, P, P, P, u64, i64, i64, P, i32,
                                               i64, i32, P, sz, P]
        L.sketch_gen_omega.argtypes = [u64, i64, i64, i64, i64, P, i64, P]
        L.sketch_gen_matmul_dist.argtypes = [P, i32, i64, i64, i64, P, u64, i32, i64, i64, i64,
                                             P, i32, i64, i32, P, sz, P]
        L.sketch_gen_matmul_reduce_dist.argtypes = [P, i64, i32, i64, P, P, P, P, u64, i32, i64,
                                                    i64, P, i32, i64, i32, P, sz, P]
        L.sketch_gen_omega_dist.argtypes = [u64, i32, i64, i64, i64, i64, P, i64, P]
        L.sketch_gen_matmul_cm.argtypes = [P, i64, i64, i64, u64, i32, i64, i64, i64, P, i32, i64,
                                           i32, i32, P, sz, P]
        L.sketch_gen_tmatmul.argtypes = [P, i64, i64, i64, u64, i32, i64, i64, i64, P, i32, i64,
                                         i32, P, sz, P]
        L.sketch_matmul_omega.argtypes = [P, i32, i64, i64, i64, P, P, i64, i64, P, i32, i64, i32,
                                          P, sz, P]
        L.sketch_philox_raw.argtypes = [P, u64, P, i64, P]
        L.sketch_normal_raw.argtypes = [P, P, i64, P]
        L.sketch_quantize.argtypes = [P, i64, i64, i64, i32, P, i64, P, P]
        L.sketch_trace_events.argtypes = [P, P, P]
        L.sketch_core_pinv_workspace.argtypes = [i64]
        L.sketch_core_pinv_workspace.restype = sz
        L.sketch_core_pinv.argtypes = [P, i32, i64, i64, ctypes.c_double, i32, P, i64, P, P, P, sz,
                                       P]
        L.sketch_nystrom_workspace.argtypes = [i64, i64]
        L.sketch_nystrom_workspace.restype = sz
        L.sketch_nystrom_error.argtypes = [P, i64, i64, P, i64, i64, P, i64, P, P, sz, P]
        L.sketch_nystrom_rows.argtypes = [P, i64, i64, i64, P, i64, i64, i64, P, i64, P, sz, P]
        for f in ("sketch_gen_matmul", "sketch_gen_matmul_noalloc", "sketch_gen_matmul_reduce", "sketch_gen_matmul_dist",
                  "sketch_gen_matmul_reduce_dist", "sketch_gen_omega_dist",
                  "sketch_gen_matmul_cm", "sketch_gen_tmatmul",
                  "sketch_gen_omega", "sketch_matmul_omega", "sketch_philox_raw",
                  "sketch_normal_raw",
                  "sketch_quantize", "sketch_trace_events", "sketch_core_pinv",
                  "sketch_nystrom_error", "sketch_nystrom_rows"):
            getattr(L, f).restype = i32
        _lib = L
        return L


def _check(status: int, where: str) -> None:
    if status != 0:
        raise SketchError(status, where)


def sketch_abi_version() -> int:
    return int(lib().sketch_abi_version())


def sketch_status_string(status: int) -> str:
    return lib().sketch_status_string(int(status)).decode()


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def _adtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return SK_A_F32
    if t.dtype == torch.bfloat16:
        return SK_A_BF16
    if t.dtype in (torch.uint8, torch.float8_e4m3fn):
        return SK_A_FP8_E4M3
    raise TypeError(f"unsupported A dtype {t.dtype}")


def _ydtype(dt) -> int:
    if dt == torch.float32:
        return SK_Y_F32
    if dt == torch.float64:
        return SK_Y_F64
    raise TypeError(f"unsupported Y dtype {dt}")


def _dist(dist) -> int:
    d = SK_DIST.get(dist, dist) if isinstance(dist, str) else int(dist)
    if not isinstance(d, int):
        raise ValueError(f"unknown distribution {dist!r}")
    return d


def _ld(t: torch.Tensor, name: str) -> int:
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return int(t.stride(0))


def _stream(stream, device) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


_ws_cache: dict = {}
_ws_lock = threading.Lock()


def workspace_for(nbytes: int, device, stream_ptr: int) -> tuple[int, int]:
    """A cached workspace of at least nbytes for (device, stream).

    Calls on one stream run one after the other, so they can share it.  The
    buffer is marked as used by that stream (record_stream), so that when a
    larger one replaces it, torch's caching allocator reuses its memory only
    after the work already enqueued there has finished.  The cache is guarded
    by a lock: host threads may share a stream.
    """
    if nbytes == 0:
        return 0, 0
    dev = torch.device(device)
    key = (dev.index, stream_ptr)
    with _ws_lock:
        buf = _ws_cache.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=dev)
            if stream_ptr != torch.cuda.current_stream(dev).cuda_stream:
                buf.record_stream(torch.cuda.ExternalStream(stream_ptr, device=dev))
            _ws_cache[key] = buf
        return int(buf.data_ptr()), int(buf.numel())


# ----------------------------------------------------------------------------
# ABI calls
# ----------------------------------------------------------------------------
def sketch_strip_width(a_dtype: int, k: int) -> int:
    """Columns per FP32 contraction strip for this storage type and sketch width."""
    return int(lib().sketch_strip_width(a_dtype, k))


def sketch_workspace_size(op: int, a_dtype: int, m: int, n: int, k: int, P: int = 1) -> int:
    return int(lib().sketch_workspace_size(op, a_dtype, m, n, k, P))


def _out(Y, m, k, y_dtype, device):
    if Y is None:
        return torch.empty((m, k), dtype=y_dtype, device=device)
    return Y


def sketch_gen_matmul(A: torch.Tensor, seed: int, k: int, *, omega_row0: int = 0,
                      omega_col0: int = 0, Y: torch.Tensor | None = None, beta: int = 0,
                      a_scales: torch.Tensor | None = None, y_dtype=torch.float32,
                      workspace: torch.Tensor | None = None, stream=None,
                      dist="normal") -> torch.Tensor:
    """Y (=|+=) A * Omega(seed)[row0:row0+n, col0:col0+k] (one share, Alg. 1 local product);
    dist: "normal" (default), "uniform" or "rademacher" entries of Omega."""
    m, n = A.shape
    lda = _ld(A, "A") if m > 0 else max(n, 1)
    Y = _out(Y, m, k, y_dtype if Y is None else Y.dtype, A.device)
    ldy = _ld(Y, "Y") if m > 0 else max(k, 1)
    st = _stream(stream, A.device)
    adt = _adtype(A)
    need = sketch_workspace_size(0, adt, m, n, k, 1)
    if workspace is not None:
        wsp, wsb = _ptr(workspace), workspace.numel() * workspace.element_size()
    else:
        wsp, wsb = workspace_for(need, A.device, st)
    _check(lib().sketch_gen_matmul_dist(_ptr(A), adt, m, n, lda, _ptr(a_scales), seed,
                                        _dist(dist), omega_row0, omega_col0, k, _ptr(Y),
                                        _ydtype(Y.dtype), ldy, beta, wsp, wsb, st),
           "sketch_gen_matmul")
    return Y


def sketch_gen_matmul_noalloc(A: torch.Tensor, seed: int, k: int, *, omega_row0: int = 0,
                              omega_col0: int = 0, Y: torch.Tensor | None = None, beta: int = 0,
                              a_scales: torch.Tensor | None = None, y_dtype=torch.float32,
                              stream=None) -> torch.Tensor:
    """sketch_gen_matmul with the library's static scratch instead of a workspace (no device
    allocation inside the call; pass Y to allocate nothing here either)."""
    m, n = A.shape
    lda = _ld(A, "A") if m > 0 else max(n, 1)
    Y = _out(Y, m, k, y_dtype if Y is None else Y.dtype, A.device)
    ldy = _ld(Y, "Y") if m > 0 else max(k, 1)
    _check(lib().sketch_gen_matmul_noalloc(_ptr(A), _adtype(A), m, n, lda, _ptr(a_scales), seed,
                                           omega_row0, omega_col0, k, _ptr(Y), _ydtype(Y.dtype),
                                           ldy, beta, _stream(stream, A.device)),
           "sketch_gen_matmul_noalloc")
    return Y


def sketch_gen_matmul_reduce(blocks, row0s, seed: int, k: int, *, omega_col0: int = 0,
                             Y: torch.Tensor | None = None, beta: int = 0, scales=None,
                             y_dtype=torch.float32, workspace: torch.Tensor | None = None,
                             stream=None, dist="normal") -> torch.Tensor:
    """Y (=|+=) sum_b A_b * Omega[row0_b:row0_b+n_b, col0:col0+k] (1Dred share, device FP64 sum)."""
    P = len(blocks)
    if P == 0 or len(row0s) != P:
        raise ValueError("need one row offset per block")
    m = blocks[0].shape[0]
    dev = blocks[0].device
    adt = _adtype(blocks[0])
    Y = _out(Y, m, k, y_dtype if Y is None else Y.dtype, dev)
    ldy = _ld(Y, "Y") if m > 0 else max(k, 1)
    ptrs = (ctypes.c_void_p * P)(*[b.data_ptr() for b in blocks])
    nb = (ctypes.c_int64 * P)(*[int(b.shape[1]) for b in blocks])
    ld = (ctypes.c_int64 * P)(*[(_ld(b, "A_b") if m > 0 else max(int(b.shape[1]), 1))
                                for b in blocks])
    r0 = (ctypes.c_int64 * P)(*[int(r) for r in row0s])
    sc = None
    if scales is not None:
        sc = (ctypes.c_void_p * P)(*[(s.data_ptr() if s is not None else None) for s in scales])
    st = _stream(stream, dev)
    need = sketch_workspace_size(1, adt, m, sum(int(b.shape[1]) for b in blocks), k, P)
    if workspace is not None:
        wsp, wsb = _ptr(workspace), workspace.numel() * workspace.element_size()
    else:
        wsp, wsb = workspace_for(need, dev, st)
    _check(lib().sketch_gen_matmul_reduce_dist(ptrs, P, adt, m, nb, ld, r0, sc, seed, _dist(dist),
                                               omega_col0, k, _ptr(Y), _ydtype(Y.dtype), ldy,
                                               beta, wsp, wsb, st), "sketch_gen_matmul_reduce")
    return Y


def sketch_gen_omega(seed: int, row0: int, n: int, col0: int, k: int, *,
                     out: torch.Tensor | None = None, device="cuda", stream=None,
                     dist="normal") -> torch.Tensor:
    """Omega(seed)[row0:row0+n, col0:col0+k] materialised (stored-operand alternative)."""
    if out is None:
        out = torch.empty((n, k), dtype=torch.float32, device=device)
    ldo = _ld(out, "Omega") if n > 0 else max(k, 1)
    _check(lib().sketch_gen_omega_dist(seed, _dist(dist), row0, n, col0, k, _ptr(out), ldo,
                                       _stream(stream, out.device)), "sketch_gen_omega")
    return out


def sketch_matmul_omega(A: torch.Tensor, Omega: torch.Tensor, *, Y: torch.Tensor | None = None,
                        beta: int = 0, a_scales: torch.Tensor | None = None,
                        y_dtype=torch.float32, workspace: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
    """Y (=|+=) A * Omega with Omega read from device memory (same order as the generated path)."""
    m, n = A.shape
    k = Omega.shape[1]
    if Omega.shape[0] != n:
        raise ValueError("Omega must have n rows")
    lda = _ld(A, "A") if m > 0 else max(n, 1)
    ldo = _ld(Omega, "Omega") if n > 0 else max(k, 1)
    Y = _out(Y, m, k, y_dtype if Y is None else Y.dtype, A.device)
    ldy = _ld(Y, "Y") if m > 0 else max(k, 1)
    st = _stream(stream, A.device)
    adt = _adtype(A)
    need = sketch_workspace_size(0, adt, m, n, k, 1)
    if workspace is not None:
        wsp, wsb = _ptr(workspace), workspace.numel() * workspace.element_size()
    else:
        wsp, wsb = workspace_for(need, A.device, st)
    _check(lib().sketch_matmul_omega(_ptr(A), adt, m, n, lda, _ptr(a_scales), _ptr(Omega), ldo, k,
                                     _ptr(Y), _ydtype(Y.dtype), ldy, beta, wsp, wsb, st),
           "sketch_matmul_omega")
    return Y


def sketch_gen_matmul_cm(A: torch.Tensor, seed: int, k: int, *, omega_row0: int = 0,
                         omega_col0: int = 0, Y: torch.Tensor | None = None, beta: int = 0,
                         y_trans: bool = False, y_dtype=torch.float32,
                         workspace: torch.Tensor | None = None, stream=None,
                         dist="normal") -> torch.Tensor:
    """Y (=|+=) A * Omega[row0:row0+n, col0:col0+k] for a column-major FP32 A (an m x n
    tensor with stride (1, lda), e.g. the transpose of a row-major n x m tensor).
    y_trans: return Omega^T A^T (k x m) instead of Y (m x k)."""
    m, n = A.shape
    if A.dtype != torch.float32:
        raise TypeError("column-major A must be float32")
    if m > 1 and A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1)")
    lda = int(A.stride(1)) if n > 1 else max(m, 4)
    shape = (k, m) if y_trans else (m, k)
    Y = _out(Y, shape[0], shape[1], y_dtype if Y is None else Y.dtype, A.device)
    ldy = _ld(Y, "Y") if Y.numel() else max(shape[1], 1)
    st = _stream(stream, A.device)
    need = sketch_workspace_size(2, SK_A_F32, m, n, k, 1)
    if workspace is not None:
        wsp, wsb = _ptr(workspace), workspace.numel() * workspace.element_size()
    else:
        wsp, wsb = workspace_for(need, A.device, st)
    _check(lib().sketch_gen_matmul_cm(_ptr(A), m, n, lda, seed, _dist(dist), omega_row0,
                                      omega_col0, k, _ptr(Y), _ydtype(Y.dtype), ldy, int(y_trans),
                                      beta, wsp, wsb, st), "sketch_gen_matmul_cm")
    return Y


def sketch_gen_tmatmul(B: torch.Tensor, seed: int, k: int, *, omega_row0: int = 0,
                       omega_col0: int = 0, C: torch.Tensor | None = None, beta: int = 0,
                       c_dtype=torch.float32, workspace: torch.Tensor | None = None, stream=None,
                       dist="normal") -> torch.Tensor:
    """C (=|+=) Omega[row0:row0+n, col0:col0+k]^T * B (k x p) for a row-major FP32 B (n x p):
    Alg. 2's second product."""
    n, p = B.shape
    if B.dtype != torch.float32:
        raise TypeError("B must be float32")
    ldb = _ld(B, "B") if n > 0 else max(p, 4)
    C = _out(C, k, p, c_dtype if C is None else C.dtype, B.device)
    ldc = _ld(C, "C") if C.numel() else max(p, 1)
    st = _stream(stream, B.device)
    need = sketch_workspace_size(2, SK_A_F32, p, n, k, 1)
    if workspace is not None:
        wsp, wsb = _ptr(workspace), workspace.numel() * workspace.element_size()
    else:
        wsp, wsb = workspace_for(need, B.device, st)
    _check(lib().sketch_gen_tmatmul(_ptr(B), n, p, ldb, seed, _dist(dist), omega_row0, omega_col0,
                                    k, _ptr(C), _ydtype(C.dtype), ldc, beta, wsp, wsb, st),
           "sketch_gen_tmatmul")
    return C


def sketch_core_pinv(C: torch.Tensor, tol: float = 1e-12, *, max_sweeps: int = 16,
                     Cp: torch.Tensor | None = None, eigvals: bool = False,
                     workspace: torch.Tensor | None = None, stream=None):
    """FP64 pseudo-inverse of the symmetric part of the r x r core C (FP32 or FP64,
    row-major), eigenvalues with |lambda| <= tol * max|lambda| dropped (Sec. 5, Alg. 2;
    tolerance of Sec. 6.2).  Returns (Cp, info) or (Cp, info, eigenvalues); info is a
    device int32 pair (sweeps run, converged)."""
    if C.dim() != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("C must be square")
    r = int(C.shape[0])
    cdt = {torch.float32: SK_Y_F32, torch.float64: SK_Y_F64}.get(C.dtype)
    if cdt is None:
        raise TypeError("C must be float32 or float64")
    ldc = _ld(C, "C") if r else 1
    if Cp is None:
        Cp = torch.empty((r, r), dtype=torch.float64, device=C.device)
    ldcp = _ld(Cp, "Cp") if r else 1
    info = torch.zeros(2, dtype=torch.int32, device=C.device)
    eig = torch.empty(r, dtype=torch.float64, device=C.device) if eigvals else None
    st = _stream(stream, C.device)
    need = int(lib().sketch_core_pinv_workspace(r))
    if workspace is not None:
        wsp, wsb = _ptr(workspace), workspace.numel() * workspace.element_size()
    else:
        wsp, wsb = workspace_for(need, C.device, st)
    _check(lib().sketch_core_pinv(_ptr(C), cdt, r, ldc, float(tol), int(max_sweeps), _ptr(Cp), ldcp,
                                  _ptr(eig), _ptr(info), wsp, wsb, st), "sketch_core_pinv")
    return (Cp, info, eig) if eigvals else (Cp, info)


def _nystrom_ws(n, r, device, st, workspace):
    need = int(lib().sketch_nystrom_workspace(n, r))
    if workspace is not None:
        return _ptr(workspace), workspace.numel() * workspace.element_size()
    return workspace_for(need, device, st)


def sketch_nystrom_error(A: torch.Tensor, B: torch.Tensor, Cp: torch.Tensor, *,
                         sums: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
    """Device FP64 (||A - B Cp B^T||_F^2, ||A||_F^2, relative error) for an n x n FP32 A,
    n x r FP32 B and r x r FP64 Cp (Table 2's error of the Nystrom approximation)."""
    n, r = int(B.shape[0]), int(B.shape[1])
    if A.dtype != torch.float32 or B.dtype != torch.float32 or Cp.dtype != torch.float64:
        raise TypeError("A, B float32 and Cp float64")
    if tuple(A.shape) != (n, n) or tuple(Cp.shape) != (r, r):
        raise ValueError("A must be n x n and Cp r x r for B n x r")
    if sums is None:
        sums = torch.zeros(3, dtype=torch.float64, device=B.device)
    st = _stream(stream, B.device)
    wsp, wsb = _nystrom_ws(n, r, B.device, st, workspace)
    _check(lib().sketch_nystrom_error(_ptr(A), n, _ld(A, "A") if n else 1, _ptr(B), r,
                                      _ld(B, "B") if n else r, _ptr(Cp), _ld(Cp, "Cp"),
                                      _ptr(sums), wsp, wsb, st), "sketch_nystrom_error")
    return sums


def sketch_nystrom_rows(B: torch.Tensor, Cp: torch.Tensor, row0: int, mr: int, *,
                        out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
    """Rows [row0, row0 + mr) of A~ = B Cp B^T (FP64, mr x n)."""
    n, r = int(B.shape[0]), int(B.shape[1])
    if B.dtype != torch.float32 or Cp.dtype != torch.float64:
        raise TypeError("B float32 and Cp float64")
    if out is None:
        out = torch.empty((mr, n), dtype=torch.float64, device=B.device)
    st = _stream(stream, B.device)
    wsp, wsb = _nystrom_ws(n, r, B.device, st, workspace)
    _check(lib().sketch_nystrom_rows(_ptr(B), n, r, _ld(B, "B") if n else r, _ptr(Cp),
                                     _ld(Cp, "Cp"), row0, mr, _ptr(out),
                                     _ld(out, "out") if out.numel() else max(n, 1), wsp, wsb, st),
           "sketch_nystrom_rows")
    return out


def sketch_philox_raw(ctr: torch.Tensor, seed: int, *, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """Philox4x32-10 of each row of ctr (N x 4 int32/uint32 device tensor) under key = seed."""
    if ctr.dim() != 2 or ctr.shape[1] != 4 or not ctr.is_contiguous():
        raise ValueError("ctr must be a contiguous N x 4 tensor")
    if out is None:
        out = torch.empty_like(ctr)
    _check(lib().sketch_philox_raw(_ptr(ctr), seed, _ptr(out), ctr.shape[0],
                                   _stream(stream, ctr.device)), "sketch_philox_raw")
    return out


def sketch_normal_raw(words: torch.Tensor, *, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """The generator's FP32 Box-Muller pair of each row of words (N x 2 int32/uint32
    device tensor: even word, odd word) -> N x 2 float32 (rho cos, rho sin)."""
    if words.dim() != 2 or words.shape[1] != 2 or not words.is_contiguous():
        raise ValueError("words must be a contiguous N x 2 tensor")
    if out is None:
        out = torch.empty(words.shape, dtype=torch.float32, device=words.device)
    _check(lib().sketch_normal_raw(_ptr(words), _ptr(out), words.shape[0],
                                   _stream(stream, words.device)), "sketch_normal_raw")
    return out


def sketch_trace_events(ev_begin, ev_mid, ev_end) -> None:
    """Arm per-phase HIP events (raw hipEvent_t handles) for this thread's next product call."""
    _check(lib().sketch_trace_events(ev_begin, ev_mid, ev_end), "sketch_trace_events")


def sketch_quantize(A: torch.Tensor, dst: str, *, stream=None):
    """Low-precision copy of A: ('bf16' -> (Aq bfloat16, None)); ('fp8' -> (Aq uint8 codes, scales))."""
    m, n = A.shape
    lda = _ld(A, "A") if m > 0 else max(n, 1)
    st = _stream(stream, A.device)
    if dst == "bf16":
        Aq = torch.empty((m, n), dtype=torch.bfloat16, device=A.device)
        if n % 8:
            Aq = torch.empty((m, (n + 7) // 8 * 8), dtype=torch.bfloat16, device=A.device)[:, :n]
        _check(lib().sketch_quantize(_ptr(A), m, n, lda, SK_A_BF16, _ptr(Aq),
                                     _ld(Aq, "Aq") if m > 0 else max(n, 1), None, st),
               "sketch_quantize")
        return Aq, None
    if dst == "fp8":
        ldq = (n + 15) // 16 * 16
        Aq = torch.empty((m, max(ldq, 16)), dtype=torch.uint8, device=A.device)[:, :n]
        scales = torch.empty(((m + 127) // 128,), dtype=torch.float32, device=A.device)
        _check(lib().sketch_quantize(_ptr(A), m, n, lda, SK_A_FP8_E4M3, _ptr(Aq), max(ldq, 16),
                                     _ptr(scales), st), "sketch_quantize")
        return Aq, scales
    raise ValueError("dst must be 'bf16' or 'fp8'")


from .serve import SketchServer, make_request, sk_request_footprint  # noqa: E402

__all__ = ["sketch_abi_version", "sketch_status_string", "sketch_workspace_size",
           "sketch_strip_width", "SketchServer", "make_request", "sk_request_footprint",
           "sketch_gen_matmul", "sketch_gen_matmul_noalloc", "sketch_gen_matmul_reduce",
           "sketch_gen_matmul_cm",
           "sketch_gen_tmatmul",
           "sketch_gen_omega", "sketch_matmul_omega", "sketch_philox_raw", "sketch_normal_raw",
           "sketch_quantize", "sketch_core_pinv", "sketch_nystrom_error", "sketch_nystrom_rows",
           "sketch_trace_events", "SketchError", "lib", "LIB_PATH"]
