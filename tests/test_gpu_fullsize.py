"""Full-size parity of the matrix-core paths and wide sketches (k up to 1024).

* A 65536 x 16384 FP32 N(0,1) (the k-sweep workload; byte offsets pass 2^32
  and the grid reaches (8 strips, 128 row tiles, 8 column blocks)), k = 64, 256
  and 1000 (the paper's r = 1000, Sec. 6.4): sampled rows, including tile,
  strip and matrix edges, against the FP64 oracle within the element bound of
  a 2048-product FP32 chain, 2052 u sum_j |a w| + u |y| (u = 2^-24), and the
  relative Frobenius error <= 1e-5.  The stored-operand product (Omega
  materialised, Sec. 6.3) equals the generated one bitwise, and so does the
  column layout (Alg. 1 on a (1, P, 1) grid: 8 blocks of 2048 columns, FP64
  device sum) against the row call.
* Column-major 32768 x 32768 FP32 A at k = 64: sampled rows against the oracle,
  and bitwise equal to the row-major call on the same matrix.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk
from sketch_inputs import normal_matrix, normal_matrix_device

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
DEV = "cuda:0"


def sample_rows(m, edges, count=24, seed=0):
    rng = np.random.default_rng(seed)
    rows = np.concatenate([np.array(edges), rng.choice(m, size=count, replace=False)])
    return np.unique(rows[(rows >= 0) & (rows < m)])


def check_rows(Y, Ah, rows, seed, k, c=2052):
    got = Y[torch.from_numpy(rows).to(DEV)].double().cpu().numpy()
    ref = oracle.gen_matmul(Ah, seed, 0, 0, k)
    Om = oracle.omega_block(seed, 0, Ah.shape[1], 0, k)
    mag = oracle.matmul(np.abs(Ah), np.abs(Om))
    err = np.abs(got - ref)
    bound = c * U * mag + U * np.abs(ref)
    assert (err <= bound).all(), (int((err > bound).sum()), float((err - bound).max()))
    rel = oracle.rel_fro(got, ref)
    assert rel <= 1e-5, rel
    return rel


@pytest.fixture(scope="module")
def tall():
    A = normal_matrix_device(65536, 16384, seed=0, device=DEV)
    yield A
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [64, 256, 1000])
def test_tall_matrix_cores_sampled_rows(tall, k):
    m, n = tall.shape
    rows = sample_rows(m, [0, 1, 511, 512, 513, 32767, 32768, 65024, m - 2, m - 1], seed=k)
    Ah = tall[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    Y = sk.sketch_gen_matmul(tall, 1, k)
    torch.cuda.synchronize()
    rel = check_rows(Y, Ah, rows, 1, k)
    print(f"65536x16384 k={k}: sampled-row relative Frobenius error {rel:.2e}")


@pytest.mark.parametrize("k", [64, 256])
def test_tall_stored_and_column_layout_bitwise(tall, k):
    m, n = tall.shape
    Y = sk.sketch_gen_matmul(tall, 1, k)
    Om = sk.sketch_gen_omega(1, 0, n, 0, k, device=DEV)
    assert torch.equal(sk.sketch_matmul_omega(tall, Om), Y)
    del Om
    P, w = 8, n // 8
    Yred = sk.sketch_gen_matmul_reduce([tall[:, b * w:(b + 1) * w] for b in range(P)],
                                       [b * w for b in range(P)], 1, k)
    assert torch.equal(Yred, Y)


def test_column_major_full_size_k64():
    N, k = 32768, 64
    T = normal_matrix_device(N, N, seed=3, device=DEV)     # A = T^T: column-major storage
    Acm = T.t()
    Y = sk.sketch_gen_matmul_cm(Acm, 2, k, omega_row0=5)
    rows = sample_rows(N, [0, 255, 256, 511, 512, 4095, 4096, N - 1], seed=1)
    Ah = T[:, torch.from_numpy(rows).to(DEV)].t().contiguous().cpu().numpy()
    got = Y[torch.from_numpy(rows).to(DEV)].double().cpu().numpy()
    ref = oracle.gen_matmul(Ah, 2, 5, 0, k)
    Om = oracle.omega_block(2, 5, N, 0, k)
    mag = oracle.matmul(np.abs(Ah), np.abs(Om))
    assert (np.abs(got - ref) <= 2052 * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(got, ref) <= 1e-5
    Arm = Acm.contiguous()
    del T
    assert torch.equal(sk.sketch_gen_matmul(Arm, 2, k, omega_row0=5), Y)
    del Arm, Acm
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------
# Sketch widths above 256 (the paper's r = 500, Sec. 6.3; r = 1000, Sec. 6.4)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k,row0,col0", [
    (300, 5000, 300, 0, 0),       # three 128-column blocks, the last of 44
    (130, 2100, 500, 3, 1),       # four blocks, ragged strips and rows
    (70, 4100, 1000, 0, 0),       # eight blocks, the last of 104
    (40, 1000, 1024, 5, 7),       # the widest sketch, one strip
    (513, 2049, 777, 1, 0),       # a row past a 512-row tile, a column past a strip
])
def test_wide_sketch_f32(m, n, k, row0, col0):
    A = normal_matrix(m, n, seed=m + k)
    ld = (n + 3) // 4 * 4
    Ad = torch.zeros((m, ld), device=DEV)
    Ad[:, :n] = torch.from_numpy(A).to(DEV)
    Y = sk.sketch_gen_matmul(Ad[:, :n], 4, k, omega_row0=row0, omega_col0=col0)
    got = Y.double().cpu().numpy()
    ref = oracle.gen_matmul(A, 4, row0, col0, k)
    Om = oracle.omega_block(4, row0, n, col0, k)
    mag = oracle.matmul(np.abs(A), np.abs(Om))
    assert (np.abs(got - ref) <= 2052 * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(got, ref) <= 1e-5
    # columns of a wide sketch are the same sketch columns as a narrower one
    Y64 = sk.sketch_gen_matmul(Ad[:, :n], 4, 64, omega_row0=row0, omega_col0=col0)
    assert torch.equal(Y[:, :64], Y64)


@pytest.mark.parametrize("kind,k", [("bf16", 500), ("fp8", 1000), ("fp8", 300)])
def test_wide_sketch_low_precision(kind, k):
    m, n = 200, 4500
    A = normal_matrix(m, n, seed=k)
    A[128:] *= np.float32(0.05)
    Ad = torch.zeros((m, (n + 3) // 4 * 4), device=DEV)
    Ad[:, :n] = torch.from_numpy(A).to(DEV)
    Aq, sc = sk.sketch_quantize(Ad[:, :n], kind)
    Y = sk.sketch_gen_matmul(Aq, 6, k, omega_row0=2, a_scales=sc).double().cpu().numpy()
    if kind == "bf16":
        codes = Aq.cpu().view(torch.int16).numpy().view(np.uint16)
        Adeq = oracle.bf16_decode(codes)
    else:
        Q = Aq.cpu().numpy()
        Adeq = oracle.fp8_decode_table()[Q] * np.repeat(sc.cpu().numpy().astype(np.float64),
                                                        128)[:m, None]
    Adeq = Adeq.astype(np.float32)
    ref = oracle.gen_matmul(Adeq, 6, 2, 0, k)
    Om = oracle.omega_block(6, 2, n, 0, k)
    mag = oracle.matmul(np.abs(Adeq), np.abs(Om))
    assert (np.abs(Y - ref) <= (4096 + 4 + 256) * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(Y, ref) <= 1e-5


@pytest.mark.parametrize("m,n,k", [(300, 5000, 1000), (5, 3000, 700), (600, 2100, 1024)])
def test_wide_sketch_column_major(m, n, k):
    A = normal_matrix(m, n, seed=k + 1)
    ld = (m + 3) // 4 * 4
    buf = torch.full((n, ld), float("nan"), device=DEV)
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).to(DEV)
    Acm = buf[:, :m].t()
    Y = sk.sketch_gen_matmul_cm(Acm, 8, k, omega_row0=1)
    got = Y.double().cpu().numpy()
    ref = oracle.gen_matmul(A, 8, 1, 0, k)
    Om = oracle.omega_block(8, 1, n, 0, k)
    mag = oracle.matmul(np.abs(A), np.abs(Om))
    assert (np.abs(got - ref) <= 2052 * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(got, ref) <= 1e-5
    Yt = sk.sketch_gen_matmul_cm(Acm, 8, k, omega_row0=1, y_trans=True)
    assert torch.equal(Yt.t(), Y)
