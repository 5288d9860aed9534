"""CPU oracle for the sketch Y = A * Omega(seed) with a generated random operand.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  The product library
never loads it, and it shares no code with the GPU path.

The arithmetic lives in ``oracle.c`` (plain C, FP64 sums); this module builds
it with gcc and wraps it with ctypes + numpy.  Citations follow the paper:
Sec. 4 (problem statement B = A*Omega), Alg. 1 (GenRandom, local product,
reduction over the contraction split), Sec. 6.3 (Philox, shared seed).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP contraction off)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    u64 = ctypes.c_uint64
    lib.oracle_philox_raw.argtypes = [P, P, P, i64]
    lib.oracle_normal_pair.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P, P]
    lib.oracle_normal_pairs.argtypes = [P, P, P, P, i64]
    lib.oracle_spec_log_batch.argtypes = [P, P, i64]
    lib.oracle_spec_cossin_batch.argtypes = [P, P, P, i64]
    lib.oracle_omega_value.argtypes = [u64, i64, i64]
    lib.oracle_omega_value.restype = ctypes.c_float
    lib.oracle_omega_value_dist.argtypes = [u64, i64, i64, ctypes.c_int]
    lib.oracle_omega_value_dist.restype = ctypes.c_float
    lib.oracle_omega_block_dist.argtypes = [u64, i64, i64, i64, i64, ctypes.c_int, P]
    lib.oracle_gen_matmul_dist_f64.argtypes = [P, i64, i64, i64, u64, i64, i64, i64,
                                               ctypes.c_int, P]
    lib.oracle_gen_matmul_reduce_dist_f64.argtypes = [P, i64, i64, P, P, P, u64, i64, i64,
                                                      ctypes.c_int, P]
    lib.oracle_gen_matmul_cm_f64.argtypes = [P, i64, i64, i64, u64, i64, i64, i64, ctypes.c_int,
                                             P]
    lib.oracle_gen_tmatmul_f64.argtypes = [P, i64, i64, i64, u64, i64, i64, i64, ctypes.c_int, P]
    lib.oracle_omega_f64ref.argtypes = [u64, i64, i64]
    lib.oracle_omega_f64ref.restype = ctypes.c_double
    lib.oracle_omega_block.argtypes = [u64, i64, i64, i64, i64, P]
    lib.oracle_gen_matmul_f64.argtypes = [P, i64, i64, i64, u64, i64, i64, i64, P]
    lib.oracle_gen_matmul_reduce_f64.argtypes = [P, i64, i64, P, P, P, u64, i64, i64, P]
    lib.oracle_matmul_f64.argtypes = [P, i64, i64, i64, P, i64, i64, P]
    lib.oracle_bf16_encode.argtypes = [P, P, i64]
    lib.oracle_bf16_decode.argtypes = [ctypes.c_uint16]
    lib.oracle_bf16_decode.restype = ctypes.c_double
    lib.oracle_fp8e4m3_encode.argtypes = [ctypes.c_double]
    lib.oracle_fp8e4m3_encode.restype = ctypes.c_uint8
    lib.oracle_fp8e4m3_decode.argtypes = [ctypes.c_uint8]
    lib.oracle_fp8e4m3_decode.restype = ctypes.c_double
    lib.oracle_quantize_fp8_rows128.argtypes = [P, i64, i64, i64, P, i64, P]
    lib.oracle_gen_matmul_q_f64.argtypes = [P, ctypes.c_int, i64, i64, i64, P, u64, i64, i64,
                                            i64, P]
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads() -> int:
    """Threads used by the oracle's OpenMP loops."""
    return int(_load().oracle_num_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _rows(A: np.ndarray, dtype) -> tuple[np.ndarray, int]:
    """Return a C-ordered view/copy of a 2-D array and its leading dimension."""
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    if A.dtype != dtype:
        raise TypeError(f"A must be {dtype}")
    if A.strides[1] != A.itemsize or A.strides[0] % A.itemsize:
        A = np.ascontiguousarray(A)
    return A, A.strides[0] // A.itemsize


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 of each row of ctr (N x 4 uint32) under key (2 uint32)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty_like(ctr)
    _load().oracle_philox_raw(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0])
    return out


def normal_pair(r_even: int, r_odd: int) -> tuple[float, float]:
    """FP32 Box-Muller of two Philox words: (rho cos theta, rho sin theta)."""
    zc = ctypes.c_float()
    zs = ctypes.c_float()
    _load().oracle_normal_pair(r_even, r_odd, ctypes.byref(zc), ctypes.byref(zs))
    return zc.value, zs.value


def normal_pairs(r_even: np.ndarray, r_odd: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """FP32 Box-Muller of word pairs, elementwise: (rho cos theta, rho sin theta) arrays."""
    ev = np.ascontiguousarray(r_even, dtype=np.uint32).ravel()
    od = np.ascontiguousarray(r_odd, dtype=np.uint32).ravel()
    if ev.size != od.size:
        raise ValueError("need as many odd words as even words")
    zc = np.empty(ev.size, dtype=np.float32)
    zs = np.empty(ev.size, dtype=np.float32)
    if ev.size:
        _load().oracle_normal_pairs(_ptr(ev), _ptr(od), _ptr(zc), _ptr(zs), ev.size)
    return zc, zs


def spec_log(mo: np.ndarray) -> np.ndarray:
    """FP32 ln(mo * 2^-24) for odd integers mo in [1, 2^24) (the Box-Muller radius step)."""
    mo = np.ascontiguousarray(mo, dtype=np.uint32)
    out = np.empty(mo.shape, dtype=np.float32)
    _load().oracle_spec_log_batch(_ptr(mo), _ptr(out), mo.size)
    return out


def spec_cossin(mo: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """FP32 (cos, sin) of 2 pi mo 2^-24 for odd integers mo in [1, 2^24)."""
    mo = np.ascontiguousarray(mo, dtype=np.uint32)
    c = np.empty(mo.shape, dtype=np.float32)
    s = np.empty(mo.shape, dtype=np.float32)
    _load().oracle_spec_cossin_batch(_ptr(mo), _ptr(c), _ptr(s), mo.size)
    return c, s


DISTS = {"normal": 0, "uniform": 1, "rademacher": 2}


def _dist(dist) -> int:
    return DISTS[dist] if isinstance(dist, str) else int(dist)


def omega_value(seed: int, row: int, col: int, dist="normal") -> float:
    """Omega(row, col) under the given distribution ("normal", "uniform", "rademacher")."""
    return float(_load().oracle_omega_value_dist(seed, row, col, _dist(dist)))


def omega_f64ref(seed: int, row: int, col: int) -> float:
    return float(_load().oracle_omega_f64ref(seed, row, col))


def omega_block(seed: int, row0: int, n: int, col0: int, k: int, dist="normal") -> np.ndarray:
    """Omega[row0:row0+n, col0:col0+k] (FP32, n x k)."""
    out = np.empty((n, k), dtype=np.float32)
    if n and k:
        _load().oracle_omega_block_dist(seed, row0, n, col0, k, _dist(dist), _ptr(out))
    return out


def gen_matmul(A: np.ndarray, seed: int, row0: int, col0: int, k: int,
               dist="normal") -> np.ndarray:
    """Y = A * Omega(seed)[row0:row0+n, col0:col0+k] in FP64 (A is FP32 m x n)."""
    A, lda = _rows(A, np.float32)
    m, n = A.shape
    Y = np.zeros((m, k), dtype=np.float64)
    if m and k:
        _load().oracle_gen_matmul_dist_f64(_ptr(A), m, n, lda, seed, row0, col0, k, _dist(dist),
                                           _ptr(Y))
    return Y


def gen_matmul_reduce(blocks, row0s, seed: int, col0: int, k: int, dist="normal") -> np.ndarray:
    """Y = sum_b A_b * Omega[row0_b : row0_b + n_b, col0:col0+k], blocks in order (FP64)."""
    views = [_rows(b, np.float32) for b in blocks]
    m = views[0][0].shape[0]
    for v, _ in views:
        if v.shape[0] != m:
            raise ValueError("all blocks need the same row count")
    P = len(views)
    ptrs = (ctypes.c_void_p * P)(*[v.ctypes.data for v, _ in views])
    n_b = np.array([v.shape[1] for v, _ in views], dtype=np.int64)
    lda_b = np.array([ld for _, ld in views], dtype=np.int64)
    r0 = np.array(row0s, dtype=np.int64)
    Y = np.zeros((m, k), dtype=np.float64)
    if m and k:
        _load().oracle_gen_matmul_reduce_dist_f64(ptrs, P, m, _ptr(n_b), _ptr(lda_b), _ptr(r0),
                                                  seed, col0, k, _dist(dist), _ptr(Y))
    return Y


def gen_matmul_cm(Acm: np.ndarray, m: int, n: int, lda: int, seed: int, row0: int, col0: int,
                  k: int, dist="normal") -> np.ndarray:
    """Y = A * Omega[row0:row0+n, col0:col0+k] (FP64, m x k) for a column-major FP32 A given
    as its flat storage: element (i, j) at Acm[j * lda + i]."""
    Acm = np.ascontiguousarray(Acm, dtype=np.float32).ravel()
    if n > 0 and Acm.size < (n - 1) * lda + m:
        raise ValueError("A storage too small")
    Y = np.zeros((m, k), dtype=np.float64)
    if m and k:
        _load().oracle_gen_matmul_cm_f64(_ptr(Acm), m, n, lda, seed, row0, col0, k, _dist(dist),
                                         _ptr(Y))
    return Y


def gen_tmatmul(B: np.ndarray, seed: int, row0: int, col0: int, k: int,
                dist="normal") -> np.ndarray:
    """C = Omega[row0:row0+n, col0:col0+k]^T * B (FP64, k x p) for FP32 B (n x p)
    (Alg. 2's second product)."""
    B, ldb = _rows(B, np.float32)
    n, p = B.shape
    C = np.zeros((k, p), dtype=np.float64)
    if k and p:
        _load().oracle_gen_tmatmul_f64(_ptr(B), n, p, ldb, seed, row0, col0, k, _dist(dist),
                                       _ptr(C))
    return C


def matmul(A: np.ndarray, Om: np.ndarray) -> np.ndarray:
    """Y = A * Om in FP64 for FP32 A (m x n) and explicit FP32 Om (n x k)."""
    A, lda = _rows(A, np.float32)
    Om, ldo = _rows(Om, np.float32)
    m, n = A.shape
    k = Om.shape[1]
    if Om.shape[0] != n:
        raise ValueError("shape mismatch")
    Y = np.zeros((m, k), dtype=np.float64)
    if m and k and n:
        _load().oracle_matmul_f64(_ptr(A), m, n, lda, _ptr(Om), ldo, k, _ptr(Y))
    return Y


def bf16_encode(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    _load().oracle_bf16_encode(_ptr(x), _ptr(out), x.size)
    return out


def bf16_decode(codes: np.ndarray) -> np.ndarray:
    lib = _load()
    flat = np.ascontiguousarray(codes, dtype=np.uint16).ravel()
    return np.array([lib.oracle_bf16_decode(int(c)) for c in flat]).reshape(codes.shape)


def fp8_encode(x: float) -> int:
    return int(_load().oracle_fp8e4m3_encode(float(x)))


def fp8_decode(code: int) -> float:
    return float(_load().oracle_fp8e4m3_decode(int(code)))


def fp8_decode_table() -> np.ndarray:
    """FP64 value of each of the 256 E4M3FN codes (NaN for the two NaN codes)."""
    return np.array([fp8_decode(c) for c in range(256)], dtype=np.float64)


def quantize_fp8_rows128(A: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """FP8 E4M3FN codes (m x n uint8) and per-128-row-block scales (FP32)."""
    A, lda = _rows(A, np.float32)
    m, n = A.shape
    Q = np.zeros((m, n), dtype=np.uint8)
    scales = np.zeros(((m + 127) // 128,), dtype=np.float32)
    if m and n:
        _load().oracle_quantize_fp8_rows128(_ptr(A), m, n, lda, _ptr(Q), n, _ptr(scales))
    elif m:
        scales[:] = 1.0
    return Q, scales


def gen_matmul_q(Aq: np.ndarray, dtype: str, scales, seed: int, row0: int, col0: int,
                 k: int) -> np.ndarray:
    """Y = dequant(Aq) * Omega in FP64.  dtype 'bf16' (uint16 codes) or 'fp8' (uint8 codes)."""
    code = {"bf16": (1, np.uint16), "fp8": (2, np.uint8)}[dtype]
    Aq, lda = _rows(Aq, code[1])
    m, n = Aq.shape
    Y = np.zeros((m, k), dtype=np.float64)
    sc = None
    if scales is not None:
        sc = np.ascontiguousarray(scales, dtype=np.float32)
        if sc.size < (m + 127) // 128:
            raise ValueError("need one scale per 128-row block")
    if m and k:
        _load().oracle_gen_matmul_q_f64(_ptr(Aq), code[0], m, n, lda,
                                        _ptr(sc) if sc is not None else None, seed, row0, col0,
                                        k, _ptr(Y))
    return Y


def rel_fro(Y: np.ndarray, Yref: np.ndarray) -> float:
    """Relative Frobenius error ||Y - Yref|| / ||Yref|| in FP64."""
    Y = np.asarray(Y, dtype=np.float64)
    Yref = np.asarray(Yref, dtype=np.float64)
    den = np.linalg.norm(Yref)
    num = np.linalg.norm(Y - Yref)
    return float(num / den) if den > 0 else float(num)
