"""The allocation-free entry point (sketch_gen_matmul_noalloc) against
sketch_gen_matmul, called through the C ABI with raw device pointers.

Both run the same kernels with the same strips and summation order, so Y must
be bitwise equal; two calls in a row (the second smaller) check that the
library's static scratch left over from the first call does not leak into the
second result.  Cases: the streaming kernel (FP32, k = 5, several strips and a
ragged tail), the matrix-core kernel (FP32, k = 40), the low-precision kernel
(BF16, k = 64) and one call whose partials fill the scratch up to its limit
(8192 x 32768 at k = 64: 16 strips x 8192 rows x 64 FP32 partials = 32 MiB).
"""
import ctypes

import pytest
import torch

import paper_2603_20966_amd as sk
from sketch_inputs import normal_matrix, normal_matrix_device

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SCRATCH = 32 << 20


def _with_workspace(A, k, row0, seed):
    L = sk.lib()
    m, n = A.shape
    adt = sk._adtype(A)
    Y = torch.full((m, k), float("nan"), dtype=torch.float32, device=DEV)
    need = L.sketch_workspace_size(0, adt, m, n, k, 1)
    ws = torch.empty(max(need, 16), dtype=torch.uint8, device=DEV)
    st = L.sketch_gen_matmul(A.data_ptr(), adt, m, n, A.stride(0), None, seed, row0, 0, k,
                             Y.data_ptr(), 0, Y.stride(0), 0, ws.data_ptr(), ws.numel(),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return Y


def _noalloc(A, k, row0, seed):
    L = sk.lib()
    m, n = A.shape
    Y = torch.full((m, k), float("nan"), dtype=torch.float32, device=DEV)
    st = L.sketch_gen_matmul_noalloc(A.data_ptr(), sk._adtype(A), m, n, A.stride(0), None, seed,
                                     row0, 0, k, Y.data_ptr(), 0, Y.stride(0), 0,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return Y


def _pair(shapes, k, dtype):
    for (m, n), row0 in shapes:
        if m * n > 1 << 26:
            A = normal_matrix_device(m, n, seed=m + n, device=DEV).to(dtype)
        else:
            A = torch.from_numpy(normal_matrix(m, n, seed=m + n)).to(DEV).to(dtype)
        print(f"noalloc case m={m} n={n} k={k} dtype={dtype} row0={row0}", flush=True)
        got = _noalloc(A, k, row0, 7)
        want = _with_workspace(A, k, row0, 7)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int32), want.view(torch.int32)), (m, n, k)


def test_noalloc_streaming_kernel_two_calls():
    _pair([((777, 9000), 3), ((130, 2100), 0)], 5, torch.float32)


def test_noalloc_matrix_core_kernel_two_calls():
    _pair([((1100, 6000), 0), ((300, 2500), 5)], 40, torch.float32)


def test_noalloc_low_precision_kernel_two_calls():
    _pair([((520, 9000), 0), ((129, 4104), 0)], 64, torch.bfloat16)


def test_noalloc_full_scratch_then_smaller():
    L = sk.lib()
    n, k = 32768, 64                       # matrix cores: 16 strips of 2048 columns
    per_row = L.sketch_workspace_size(0, 0, 2, n, k, 1) - L.sketch_workspace_size(0, 0, 1, n, k, 1)
    base = L.sketch_workspace_size(0, 0, 1, n, k, 1) - per_row    # the packed Omega
    m = (SCRATCH - base) // per_row
    assert L.sketch_workspace_size(0, 0, m, n, k, 1) <= SCRATCH
    _pair([((m, n), 0), ((1000, 5000), 11)], k, torch.float32)
