"""GPU parity of the matrix-core path (FP32 A, k > 16): v_mfma_f32_16x16x4f32 over
2048-column strips, FP64 strip sums.

Bars: relative Frobenius <= 1e-5 against the FP64 oracle, and element by element
within the recursive-summation bound of a 2048-product FP32 chain,
    |Y - Y_ref| <= 2052 u sum_j |A_ij Omega_jc| + u |Y_ref|,  u = 2^-24;
exact special cases and layout invariants bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk
from sketch_inputs import normal_matrix, selection_matrix

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
DEV = "cuda:0"


def to_dev(x):
    ld = max(4, (x.shape[1] + 3) // 4 * 4)
    buf = torch.zeros((x.shape[0], ld), dtype=torch.float32, device=DEV)
    buf[:, :x.shape[1]] = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return buf[:, :x.shape[1]]


def check(Y, A, seed, row0, col0, k, rel=1e-5):
    Yg = Y.double().cpu().numpy()
    ref = oracle.gen_matmul(A, seed, row0, col0, k)
    Om = oracle.omega_block(seed, row0, A.shape[1], col0, k)
    mag = oracle.matmul(np.abs(A).astype(np.float32), np.abs(Om))
    bad = np.abs(Yg - ref) > 2052 * U * mag + U * np.abs(ref)
    assert not bad.any(), int(bad.sum())
    err = oracle.rel_fro(Yg, ref)
    assert err <= rel, err
    return err


@pytest.mark.parametrize("m,n,k,row0,col0", [
    (300, 5000, 17, 0, 0),      # smallest matrix-core sketch, ragged strips and rows
    (257, 4096, 64, 0, 0),      # two 2048 strips, one partial 512-row tile
    (513, 4100, 64, 0, 0),      # one row past a 512-row tile, ragged third strip
    (1100, 2100, 256, 3, 0),    # 16-column chunks (8 N-tiles), three row tiles
    (100, 2049, 33, 3, 1),      # unaligned Omega rows, one-column last strip
    (64, 3000, 128, 4097, 0),
    (70, 2500, 129, 1, 5),      # two column blocks, ragged last one
    (40, 1000, 256, 0, 0),      # widest sketch, single strip
    (513, 700, 24, 2, 0),       # k not a multiple of 16, several row tiles
])
def test_mfma_shapes(m, n, k, row0, col0):
    A = normal_matrix(m, n, seed=m + 3 * n + k)
    Y = sk.sketch_gen_matmul(to_dev(A), 7, k, omega_row0=row0, omega_col0=col0)
    torch.cuda.synchronize()
    check(Y, A, 7, row0, col0, k)


def test_mfma_identity_and_selection_bitwise():
    n, k = 300, 40
    Y = sk.sketch_gen_matmul(torch.eye(n, device=DEV), 5, k, omega_row0=6).cpu().numpy()
    assert np.array_equal(Y.view(np.uint32), oracle.omega_block(5, 6, n, 0, k).view(np.uint32))
    S, cols = selection_matrix(200, 4500, seed=3)
    Y = sk.sketch_gen_matmul(to_dev(S), 9, 70, omega_row0=11).cpu().numpy()
    ref = oracle.omega_block(9, 11, 4500, 0, 70)[cols]
    assert np.array_equal(Y.view(np.uint32), ref.view(np.uint32))


def test_mfma_layouts_and_stored_omega_bitwise():
    m, n, k, P = 300, 8192, 64, 4
    Ad = to_dev(normal_matrix(m, n, seed=21))
    w = n // P
    Yrow = sk.sketch_gen_matmul(Ad, 4, k)
    Yred = sk.sketch_gen_matmul_reduce([Ad[:, b * w:(b + 1) * w] for b in range(P)],
                                       [b * w for b in range(P)], 4, k)
    assert torch.equal(Yrow, Yred)
    Yparts = torch.cat([sk.sketch_gen_matmul(Ad[r:r + 100], 4, k) for r in range(0, m, 100)])
    assert torch.equal(Yrow, Yparts)
    Om = sk.sketch_gen_omega(4, 0, n, 0, k, device=DEV)
    assert torch.equal(sk.sketch_matmul_omega(Ad, Om), Yrow)
    assert torch.equal(sk.sketch_gen_matmul(Ad, 4, k), Yrow)     # deterministic


def test_mfma_column_prefix_consistent():
    """Columns of a wide sketch are the same sketch columns as a narrower one."""
    A = normal_matrix(200, 3000, seed=22)
    Ad = to_dev(A)
    Y64 = sk.sketch_gen_matmul(Ad, 8, 64).double().cpu().numpy()
    Y20 = sk.sketch_gen_matmul(Ad, 8, 20).double().cpu().numpy()
    assert oracle.rel_fro(Y20, Y64[:, :20]) <= 1e-6
    Y5 = sk.sketch_gen_matmul(Ad, 8, 5).double().cpu().numpy()
    assert oracle.rel_fro(Y5, Y64[:, :5]) <= 1e-6


def test_mfma_beta_and_f64():
    A = normal_matrix(130, 2500, seed=23)
    Ad = to_dev(A)
    Y0 = torch.randn((130, 48), dtype=torch.float64, device=DEV)
    Y = Y0.clone()
    sk.sketch_gen_matmul(Ad, 2, 48, Y=Y, beta=1)
    ref = oracle.gen_matmul(A, 2, 0, 0, 48)
    assert oracle.rel_fro((Y - Y0).cpu().numpy(), ref) <= 1e-5
    Y64 = sk.sketch_gen_matmul(Ad, 2, 48, y_dtype=torch.float64)
    assert torch.equal(sk.sketch_gen_matmul(Ad, 2, 48), Y64.float())
