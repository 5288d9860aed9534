"""GPU parity: the HIP library against the CPU oracle (run on an MI355X).

Bars:
* the Philox stream and the generated Omega: bit-exact;
* Y in FP32: element by element within the rounding-error bound of the
  kernel's summation (VALU path, k <= 8: chains of 16 FP32 products per lane
  and 1024-column chunk, a 6-level lane tree, 4 chunk sums per 4096-column
  strip, FP64 strip sums, one final rounding):
      |Y - Y_ref| <= 80 u sum_j |A_ij Omega_jc| + u |Y_ref|,   u = 2^-24,
  (matrix-core path, k > 8: a 2048-product chain, 2052 u instead of 80 u),
  and the relative Frobenius error <= 1e-5;
* special cases with exact answers (identity, selection, zero, power-of-two
  scaling) and the layout invariants: bitwise.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk
from sketch_inputs import normal_matrix, normal_matrix_device, selection_matrix

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
DEV = "cuda:0"


def to_dev(x: np.ndarray) -> torch.Tensor:
    """Device copy of a 2-D array with its row pitch padded to 16 bytes (the
    library's alignment rule); returns the (m, n) view."""
    x = np.ascontiguousarray(x)
    if x.ndim != 2:
        return torch.from_numpy(x).to(DEV)
    per = 16 // x.itemsize
    ld = max(per, (x.shape[1] + per - 1) // per * per)
    buf = torch.zeros((x.shape[0], ld), dtype=torch.from_numpy(x[:0]).dtype, device=DEV)
    buf[:, :x.shape[1]] = torch.from_numpy(x).to(DEV)
    return buf[:, :x.shape[1]]


def chain(k: int) -> int:
    """Longest FP32 summation chain (+ tree depth) of the kernel that serves width k
    for FP32 A: 16 products per lane + 6 lane levels + 3 chunk sums on the VALU
    path (k <= 8; bound kept at 80), 2048 + 4 on the matrix-core path (k > 8)."""
    return 80 if k <= 8 else 2052


def check_fp32(Y: torch.Tensor, A: np.ndarray, seed, row0, col0, k, rel=1e-5):
    Yg = Y.double().cpu().numpy()
    ref = oracle.gen_matmul(A, seed, row0, col0, k)
    Om = oracle.omega_block(seed, row0, A.shape[1], col0, k)
    mag = oracle.matmul(np.abs(A).astype(np.float32), np.abs(Om))
    bound = chain(k) * U * mag + U * np.abs(ref)
    bad = np.abs(Yg - ref) > bound
    assert not bad.any(), f"{bad.sum()} elements outside the bound; max excess " \
                          f"{(np.abs(Yg - ref) - bound).max()}"
    assert oracle.rel_fro(Yg, ref) <= rel
    return ref


# ----------------------------------------------------------------------------
# Generator
# ----------------------------------------------------------------------------
def test_philox_raw_bit_exact():
    rng = np.random.default_rng(1)
    N = 1 << 16
    ctr = rng.integers(0, 1 << 32, size=(N, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:8] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0],
               [0, 0, 0, 1], [0xFFFFFFFF, 0, 5, 0], [7, 0xFFFFFFFF, 0xFFFFFFFF, 0]]
    for seed in (0, 1, 0xFFFFFFFFFFFFFFFF, 0x123456789ABCDEF):
        out = sk.sketch_philox_raw(to_dev(ctr.view(np.int32)), seed).cpu().numpy().view(np.uint32)
        ref = oracle.philox4x32_10(ctr, [seed & 0xFFFFFFFF, seed >> 32])
        assert np.array_equal(out, ref)


@pytest.mark.parametrize("seed,row0,n,col0,k", [
    (1, 0, 2048, 0, 5), (1, 3, 1001, 2, 7), (0xFFFFFFFFFFFF, (1 << 33) + 1, 517, 100, 16),
    (42, 4095, 9, 0, 1), (7, 0, 64, (1 << 32) - 3, 3)])
def test_gen_omega_bit_exact(seed, row0, n, col0, k):
    Om = sk.sketch_gen_omega(seed, row0, n, col0, k, device=DEV).cpu().numpy()
    ref = oracle.omega_block(seed, row0, n, col0, k)
    assert np.array_equal(Om.view(np.uint32), ref.view(np.uint32))


def test_gen_omega_strided_output():
    out = torch.full((300, 24), -7.0, device=DEV)
    sk.sketch_gen_omega(5, 10, 300, 3, 9, out=out[:, 4:13])
    got = out.cpu().numpy()
    assert np.array_equal(got[:, 4:13].view(np.uint32),
                          oracle.omega_block(5, 10, 300, 3, 9).view(np.uint32))
    assert (got[:, :4] == -7).all() and (got[:, 13:] == -7).all()


# ----------------------------------------------------------------------------
# Y = A Omega, one share
# ----------------------------------------------------------------------------
def test_small_single_block_workload():
    """2048 x 2048 FP32 N(0,1) A from seed 0, Omega 2048 x 5 from seed 1, no reduction."""
    A = normal_matrix(2048, 2048, seed=0)
    Y = sk.sketch_gen_matmul(to_dev(A), 1, 5)
    torch.cuda.synchronize()
    check_fp32(Y, A, 1, 0, 0, 5)


@pytest.mark.parametrize("m,n,k,row0,col0", [
    (300, 5000, 5, 0, 0),       # 5 strips, ragged last strip, ragged rows
    (1, 4, 1, 0, 0),            # smallest
    (65, 1023, 3, 1, 0),        # single ragged strip, unaligned Omega row offset
    (130, 3000, 8, 4098, 11),   # k class 8, unaligned offsets
    (77, 2500, 16, 6, 0),       # widest register tile (strip 512)
    (40, 1500, 13, 0, 2),       # k class 12 ... 16 with unused columns
    (50, 2100, 40, 5, 0),       # three column groups
    (1000, 700, 6, 0, 0),       # many row blocks, one strip
    (129, 9000, 2, 12345, 1),
])
def test_gen_matmul_shapes(m, n, k, row0, col0):
    A = normal_matrix(m, n, seed=m * 7 + n)
    Y = sk.sketch_gen_matmul(to_dev(A), 99, k, omega_row0=row0, omega_col0=col0)
    torch.cuda.synchronize()
    check_fp32(Y, A, 99, row0, col0, k)


def test_strided_A_view_and_output_ld():
    base = normal_matrix(200, 6000, seed=3)
    Ad = to_dev(base)[:, 1000:4300]            # lda = 6000, n = 3300
    Yfull = torch.full((200, 20), 3.0, device=DEV)
    Y = Yfull[:, 7:12]
    sk.sketch_gen_matmul(Ad, 8, 5, omega_row0=1000, Y=Y)
    torch.cuda.synchronize()
    check_fp32(Y, base[:, 1000:4300], 8, 1000, 0, 5)
    rest = Yfull.cpu().numpy()
    assert (rest[:, :7] == 3).all() and (rest[:, 12:] == 3).all()


def test_beta_accumulate_and_f64_output():
    A = normal_matrix(90, 2600, seed=4)
    Ad = to_dev(A)
    Y0 = torch.from_numpy(normal_matrix(90, 5, seed=5)).double().to(DEV)
    Y = Y0.clone()
    sk.sketch_gen_matmul(Ad, 3, 5, Y=Y, beta=1)
    ref = oracle.gen_matmul(A, 3, 0, 0, 5)
    got = Y.cpu().numpy() - Y0.cpu().numpy()
    assert oracle.rel_fro(got, ref) <= 1e-6
    Y64 = sk.sketch_gen_matmul(Ad, 3, 5, y_dtype=torch.float64)
    assert oracle.rel_fro(Y64.cpu().numpy(), ref) <= 1e-6
    # f32 output is the f64 result rounded once
    Y32 = sk.sketch_gen_matmul(Ad, 3, 5)
    assert torch.equal(Y32, Y64.float())


def test_n_zero_and_m_zero():
    Y = torch.full((10, 5), 9.0, device=DEV)
    sk.sketch_gen_matmul(torch.empty((10, 0), device=DEV), 1, 5, Y=Y)
    assert (Y == 0).all()
    Y = torch.full((10, 5), 9.0, device=DEV)
    sk.sketch_gen_matmul(torch.empty((10, 0), device=DEV), 1, 5, Y=Y, beta=1)
    assert (Y == 9).all()
    out = sk.sketch_gen_matmul(torch.empty((0, 100), device=DEV), 1, 5)
    assert out.shape == (0, 5)


# ----------------------------------------------------------------------------
# Exact special cases
# ----------------------------------------------------------------------------
def test_identity_returns_omega_bitwise():
    for n, row0, col0, k in [(1024, 0, 0, 5), (1500, 13, 3, 9), (700, 2, 0, 16)]:
        Y = sk.sketch_gen_matmul(torch.eye(n, device=DEV), 21, k, omega_row0=row0,
                                 omega_col0=col0).cpu().numpy()
        assert np.array_equal(Y.view(np.uint32),
                              oracle.omega_block(21, row0, n, col0, k).view(np.uint32))


def test_selection_scaling_zero_bitwise():
    S, cols = selection_matrix(333, 5000, seed=1)
    row0 = 3 * 4096 + 2
    Y = sk.sketch_gen_matmul(to_dev(S), 17, 6, omega_row0=row0).cpu().numpy()
    ref = np.array([[oracle.omega_value(17, row0 + int(c), j) for j in range(6)] for c in cols],
                   dtype=np.float32)
    assert np.array_equal(Y, ref)
    A = normal_matrix(100, 3000, seed=2)
    Y1 = sk.sketch_gen_matmul(to_dev(A), 4, 5)
    Y2 = sk.sketch_gen_matmul(to_dev(A * np.float32(8.0)), 4, 5)
    assert torch.equal(Y2, Y1 * 8)
    Z = sk.sketch_gen_matmul(torch.zeros((64, 4096), device=DEV), 4, 5)
    assert (Z == 0).all()


def test_deterministic_repeat():
    A = to_dev(normal_matrix(500, 8192, seed=9))
    Y1 = sk.sketch_gen_matmul(A, 1, 5)
    Y2 = sk.sketch_gen_matmul(A, 1, 5)
    assert torch.equal(Y1, Y2)


def test_rows_of_share_equal_rows_of_whole():
    """Row split (Alg. 1, p1 = P): each row block's Y equals those rows of the whole Y."""
    A = to_dev(normal_matrix(1000, 5000, seed=11))
    Yw = sk.sketch_gen_matmul(A, 2, 5)
    for r0, r1 in [(0, 64), (64, 333), (333, 1000)]:
        assert torch.equal(sk.sketch_gen_matmul(A[r0:r1], 2, 5), Yw[r0:r1])


# ----------------------------------------------------------------------------
# Contraction split with device reduction (1Dred)
# ----------------------------------------------------------------------------
def test_reduce_matches_oracle_ragged_blocks():
    m, widths, k = 150, [1000, 2048, 1, 777], 5
    A = normal_matrix(m, sum(widths), seed=12)
    offs = np.cumsum([0] + widths)
    blocks = [to_dev(A[:, offs[b]:offs[b + 1]]) for b in range(len(widths))]
    row0s = [int(o) for o in offs[:-1]]
    Y = sk.sketch_gen_matmul_reduce(blocks, row0s, 31, k)
    ref = oracle.gen_matmul_reduce([A[:, offs[b]:offs[b + 1]] for b in range(len(widths))],
                                   row0s, 31, 0, k)
    assert oracle.rel_fro(Y.cpu().numpy(), ref) <= 1e-5
    check_fp32(Y, A, 31, 0, 0, k)


def test_reduce_equals_row_layout_bitwise():
    """1Dred (column blocks, device sum) == 1Dnored (row blocks) when the blocks
    are whole strips: same FP32 strip partials, same FP64 order."""
    m, n, P, k = 512, 4 * 4096, 4, 5
    Ad = to_dev(normal_matrix(m, n, seed=13))
    w = n // P
    Yred = sk.sketch_gen_matmul_reduce([Ad[:, b * w:(b + 1) * w] for b in range(P)],
                                       [b * w for b in range(P)], 6, k)
    Yrow = torch.cat([sk.sketch_gen_matmul(Ad[i:i + 128], 6, k) for i in range(0, m, 128)])
    assert torch.equal(Yred, Yrow)


def test_stored_omega_equals_generated_bitwise():
    A = to_dev(normal_matrix(300, 5000, seed=14))
    for k, row0 in [(5, 0), (16, 3), (7, 9)]:
        Om = sk.sketch_gen_omega(8, row0, 5000, 0, k, device=DEV)
        Yc = sk.sketch_matmul_omega(A, Om)
        Yg = sk.sketch_gen_matmul(A, 8, k, omega_row0=row0)
        assert torch.equal(Yc, Yg)


# ----------------------------------------------------------------------------
# The full-size share workload: 32768 x 32768 FP32, k = 5, P = 8 emulated
# ----------------------------------------------------------------------------
def test_full_size_shares_sampled_rows():
    N, P, k = 32768, 8, 5
    A = normal_matrix_device(N, N, seed=0, device=DEV)
    w = N // P
    Yrows = torch.cat([sk.sketch_gen_matmul(A[i * w:(i + 1) * w], 1, k) for i in range(P)])
    Yred = sk.sketch_gen_matmul_reduce([A[:, b * w:(b + 1) * w] for b in range(P)],
                                       [b * w for b in range(P)], 1, k)
    torch.cuda.synchronize()
    assert torch.equal(Yrows, Yred)
    rows = np.random.default_rng(0).choice(N, size=24, replace=False)
    rows = np.concatenate([[0, w - 1, w, N - 1], rows])
    Ah = A[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    ref = oracle.gen_matmul(Ah, 1, 0, 0, k)
    got = Yrows[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    Om = oracle.omega_block(1, 0, N, 0, k)
    mag = oracle.matmul(np.abs(Ah), np.abs(Om))
    assert (np.abs(got - ref) <= 80 * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(got, ref) <= 1e-5
    del A
    torch.cuda.empty_cache()


def test_workspace_reused_across_shapes():
    """One workspace serves later calls of any shape that fits, whatever it holds."""
    ws = torch.full((64 << 20,), 0x7F, dtype=torch.uint8, device=DEV)
    shapes = [(2048, 2048, 5), (300, 5000, 5), (1000, 9000, 16), (64, 3000, 3), (2048, 2048, 5)]
    for m, n, k in shapes:
        A = normal_matrix(m, n, seed=m + n + k)
        Y = sk.sketch_gen_matmul(to_dev(A), 5, k, workspace=ws)
        Yfresh = sk.sketch_gen_matmul(to_dev(A), 5, k,
                                      workspace=torch.zeros(64 << 20, dtype=torch.uint8,
                                                            device=DEV))
        assert torch.equal(Y, Yfresh)
        check_fp32(Y, A, 5, 0, 0, k)
