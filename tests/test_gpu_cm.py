"""GPU parity of column-major A (the paper's storage order), the transposed form
Omega^T A^T, and Alg. 2's second product C = Omega^T B.

Column-major kernel (k <= 16): each lane sums its own rows over a quarter of a
strip's columns (<= 256 FP32 products), the four waves' sums are added in order,
strips are summed in FP64: element bound (256 + 4) u sum |a w| + u |y|, u = 2^-24.
Matrix-core kernel (k > 16): FP32 chains over 2048-column strips, bound
(2048 + 4) u sum |a w| + u |y|; it forms the row-major matrix-core kernel's sums
in the same order, so its result equals that of the row-major call bit for bit.
Both: relative Frobenius <= 1e-5 against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk
from sketch_inputs import normal_matrix

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
DEV = "cuda:0"


def cm_dev(A, pad=0):
    """Column-major device copy of a host m x n matrix (ld = m rounded up to 4, + pad)."""
    m, n = A.shape
    ld = (m + 3) // 4 * 4 + pad
    buf = torch.full((n, ld), float("nan"), dtype=torch.float32, device=DEV)
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).to(DEV)
    return buf[:, :m].t()                       # m x n, stride (1, ld)


def chain(k):
    return 260 if k <= 16 else 2052


def check(Y, A, seed, row0, col0, k, dist="normal"):
    ref = oracle.gen_matmul(A, seed, row0, col0, k, dist)
    Om = oracle.omega_block(seed, row0, A.shape[1], col0, k, dist)
    mag = oracle.matmul(np.abs(A).astype(np.float32), np.abs(Om))
    assert (np.abs(Y - ref) <= chain(k) * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(Y, ref) <= 1e-5


@pytest.mark.parametrize("m,n,k,row0,col0,pad", [
    (300, 5000, 5, 0, 0, 0),      # several strips, ragged last strip
    (1000, 1025, 16, 3, 2, 4),    # two strips of 512, padded columns
    (257, 777, 3, 1, 0, 0),       # one row past a 256-row tile, one strip
    (5, 9000, 5, 0, 0, 0),        # few rows (second-product shape)
    (130, 3000, 20, 7, 1, 0),     # matrix cores: two 2048 strips, 20 of 32 sketch columns
    (70, 2100, 64, 0, 3, 8),
    (1000, 5000, 64, 5, 0, 0),    # three strips (last 904), rows 512 + 488
    (513, 2049, 17, 2, 9, 4),     # one row past a 512-row tile, one column past a strip
    (600, 4100, 40, 0, 0, 0),     # 40 of 64 sketch columns, ragged chunk (4100 = 2*2048 + 4)
    (3, 5000, 100, 1, 0, 0),      # three rows (one active wave), two 64-column blocks
    (300, 2500, 256, 0, 0, 0),    # two 128-column blocks of 8 N-tiles
])
def test_column_major_products(m, n, k, row0, col0, pad):
    A = normal_matrix(m, n, seed=m + n + k)
    Ad = cm_dev(A, pad)
    Y = sk.sketch_gen_matmul_cm(Ad, 7, k, omega_row0=row0, omega_col0=col0)
    check(Y.double().cpu().numpy(), A, 7, row0, col0, k)
    Yt = sk.sketch_gen_matmul_cm(Ad, 7, k, omega_row0=row0, omega_col0=col0, y_trans=True)
    assert torch.equal(Yt.t(), Y)                # the transposed form holds the same bits


@pytest.mark.parametrize("m,n,k", [(1000, 5000, 64), (513, 2049, 17), (300, 4100, 130)])
def test_column_major_matrix_cores_equal_row_major(m, n, k):
    """Same products in the same order as the row-major matrix-core call: equal bits."""
    A = normal_matrix(m, n, seed=m + k)
    Y = sk.sketch_gen_matmul_cm(cm_dev(A), 3, k, omega_row0=4)
    ld = (n + 3) // 4 * 4                        # row-major copy, rows 16-byte aligned
    Ar = torch.zeros((m, ld), device=DEV)
    Ar[:, :n] = torch.from_numpy(A).to(DEV)
    Yr = sk.sketch_gen_matmul(Ar[:, :n], 3, k, omega_row0=4)
    assert torch.equal(Y, Yr)


@pytest.mark.parametrize("k", [40, 130])
def test_matrix_core_column_blocks_do_not_change_sums(k):
    """The sketch columns per workgroup adapt to the launch (a few-row A gets one
    16-column block per workgroup, a tall A up to 64 or 128); each column's sums are the
    same, so rows of a tall call equal a short call bit for bit."""
    from sketch_inputs import normal_matrix_device

    m, n = 65536, 2100
    Acm = normal_matrix_device(n, m, seed=11, device=DEV).t()    # column-major, lda = m
    Y = sk.sketch_gen_matmul_cm(Acm, 5, k)
    assert torch.equal(Y[:64], sk.sketch_gen_matmul_cm(Acm[:64], 5, k))
    assert torch.equal(Y[-700:], sk.sketch_gen_matmul_cm(Acm[-700:], 5, k))


def test_column_major_special_cases_and_options():
    n = 600
    for k in (9, 40):                            # VALU and matrix-core kernels: I * Omega = Omega
        Y = sk.sketch_gen_matmul_cm(torch.eye(n, device=DEV).t(), 4, k, omega_row0=5).cpu().numpy()
        assert np.array_equal(Y.view(np.uint32), oracle.omega_block(4, 5, n, 0, k).view(np.uint32))
    A = normal_matrix(200, 3000, seed=3)
    Ad = cm_dev(A)
    Y0 = torch.randn((200, 5), dtype=torch.float64, device=DEV)
    Y = Y0.clone()
    sk.sketch_gen_matmul_cm(Ad, 2, 5, Y=Y, beta=1)
    assert oracle.rel_fro((Y - Y0).cpu().numpy(), oracle.gen_matmul(A, 2, 0, 0, 5)) <= 1e-5
    for dist in ("uniform", "rademacher"):
        Yd = sk.sketch_gen_matmul_cm(Ad, 2, 5, dist=dist).double().cpu().numpy()
        check(Yd, A, 2, 0, 0, 5, dist)
    # deterministic, and row blocks equal the rows of the whole
    for k in (5, 40):
        Yw = sk.sketch_gen_matmul_cm(Ad, 2, k)
        assert torch.equal(Yw, sk.sketch_gen_matmul_cm(Ad, 2, k))
        assert torch.equal(Yw[:100], sk.sketch_gen_matmul_cm(Ad[:100], 2, k))


@pytest.mark.parametrize("n,p,k,row0", [(9000, 5, 5, 0), (5000, 64, 64, 3), (1500, 16, 20, 1)])
def test_second_nystrom_product(n, p, k, row0):
    B = normal_matrix(n, p, seed=n + p)
    ld = (p + 3) // 4 * 4
    Bd = torch.zeros((n, ld), device=DEV)
    Bd[:, :p] = torch.from_numpy(B).to(DEV)
    C = sk.sketch_gen_tmatmul(Bd[:, :p], 6, k, omega_row0=row0).double().cpu().numpy()
    ref = oracle.gen_tmatmul(B, 6, row0, 0, k)
    Om = oracle.omega_block(6, row0, n, 0, k)
    mag = np.abs(Om).astype(np.float64).T @ np.abs(B).astype(np.float64)
    assert (np.abs(C - ref) <= 260 * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(C, ref) <= 1e-5


def test_nystrom_chain_against_oracle_chain():
    """B = A Omega (row-major sketch) then C = Omega^T B on the device, against the same
    two steps in the oracle (B rounded to FP32 between them, as on the device)."""
    n, k = 3000, 12
    X = normal_matrix(n, 40, seed=5)
    A = (X @ X.T / 40).astype(np.float32)          # symmetric PSD, rank 40
    Ad = torch.from_numpy(A).to(DEV)
    Bd = sk.sketch_gen_matmul(Ad, 8, k)
    C = sk.sketch_gen_tmatmul(Bd, 8, k).double().cpu().numpy()
    Bref = oracle.gen_matmul(A, 8, 0, 0, k).astype(np.float32)
    Cref = oracle.gen_tmatmul(Bref, 8, 0, 0, k)
    assert oracle.rel_fro(C, Cref) <= 1e-5
    assert oracle.rel_fro(C, C.T) <= 1e-5          # Omega^T A Omega is symmetric


@pytest.mark.parametrize("p,k", [(1, 5), (5, 5), (16, 16), (7, 9), (17, 20), (64, 64), (40, 256),
                                 (64, 17)])
def test_few_row_kernels_equal_tall_rows(p, k):
    """Few rows (m <= 16 on the VALU path, m <= 64 on the matrix cores; the shape of B^T in
    the second Nystrom product) run on kernels that spread a strip's chains over a whole
    workgroup; each chain is the tile kernel's, so a few-row call equals the matching rows
    of a tall call bit for bit."""
    n, P, r0 = 9000, 300, 100
    A = normal_matrix(P, n, seed=p + k)
    Ad = cm_dev(A)
    Yt = sk.sketch_gen_matmul_cm(Ad, 9, k, omega_row0=2)          # 300 rows: tile kernels
    Ys = sk.sketch_gen_matmul_cm(Ad[:p], 9, k, omega_row0=2)
    assert torch.equal(Ys, Yt[:p])
    Ys2 = sk.sketch_gen_matmul_cm(Ad[r0:r0 + p], 9, k, omega_row0=2, y_trans=True)
    assert torch.equal(Ys2.t(), Yt[r0:r0 + p])
    check(Ys.double().cpu().numpy(), A[:p], 9, 2, 0, k)
