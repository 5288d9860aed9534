"""GPU parity of the precision form: A stored in BF16 or FP8-E4M3 (per-128-row
power-of-two scales), products accumulated in FP32, strips summed in FP64.

* quantised codes and scales: bit-exact against the oracle's codecs;
* Y against the oracle on the dequantised A: within the FP32 summation bound
  (the quantisation is exact input data, so this isolates the arithmetic).  On
  the VALU path (BF16, k <= 6) chains are 16 products per lane plus lane
  levels and chunk sums (bound 80u); on the BF16 matrix-core path (FP8 at every k, BF16 for
  k > 6) a chain runs over a 4096-column strip and Omega enters as hi + lo BF16
  terms whose sum is within 2^-16 = 256u of Omega (bound (4096 + 4 + 256)u);
* Y against the oracle on the original FP32 A (end-to-end error): relative
  Frobenius <= 1e-2 for BF16 (the stated target); for FP8 the error is reported
  and held to the model's order (3 mantissa bits: <= 5e-2).
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


def dev_f32(x):
    ld = (x.shape[1] + 3) // 4 * 4
    buf = torch.zeros((x.shape[0], max(ld, 4)), dtype=torch.float32, device=DEV)
    buf[:, :x.shape[1]] = torch.from_numpy(x).to(DEV)
    return buf[:, :x.shape[1]]


@pytest.mark.parametrize("m,n", [(300, 5000), (128, 1024), (1, 7), (257, 2049)])
def test_bf16_codes_bit_exact(m, n):
    A = normal_matrix(m, n, seed=m + n) * np.float32(3.0)
    Aq, sc = sk.sketch_quantize(dev_f32(A), "bf16")
    assert sc is None
    got = Aq.cpu().view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, oracle.bf16_encode(A))


@pytest.mark.parametrize("m,n", [(300, 5000), (128, 1024), (1, 7), (257, 2049)])
def test_fp8_codes_and_scales_bit_exact(m, n):
    A = normal_matrix(m, n, seed=2 * m + n) * np.float32(5.0)
    if m > 128:
        A[128:256] *= np.float32(1e-4)       # a block with a much smaller scale
    Aq, sc = sk.sketch_quantize(dev_f32(A), "fp8")
    Q, s = oracle.quantize_fp8_rows128(A)
    assert np.array_equal(sc.cpu().numpy(), s)
    assert np.array_equal(Aq.cpu().numpy(), Q)


def test_fp8_tiny_huge_and_subnormal_blocks_bit_exact():
    """Scales far from 1: a block near FP32's smallest normal (scale 2^-133, whose
    reciprocal is not an FP32 number), a block of FP32 subnormals only (scale at
    the FP32 floor 2^-149), a block near 1e30, and an ordinary block."""
    A = normal_matrix(512, 300, seed=4)
    A[0:128] *= np.float32(1e-38)
    A[128:256] *= np.float32(1e-43)
    A[256:384] *= np.float32(1e30)
    assert 0 < np.abs(A[128:256]).max() < np.float32(2.0 ** -126)
    Aq, sc = sk.sketch_quantize(dev_f32(A), "fp8")
    Q, s = oracle.quantize_fp8_rows128(A)
    assert s[1] == np.float32(2.0 ** -149) and s[0] < np.float32(2.0 ** -126)
    assert np.array_equal(sc.cpu().numpy().view(np.uint32), s.view(np.uint32))
    assert np.array_equal(Aq.cpu().numpy(), Q)
    assert Q[0:128].any() and Q[128:256].any()


def test_fp8_zero_block_scale_is_one():
    A = np.zeros((200, 64), dtype=np.float32)
    A[:128] = normal_matrix(128, 64, seed=1)
    Aq, sc = sk.sketch_quantize(dev_f32(A), "fp8")
    assert sc.cpu().numpy()[1] == 1.0
    assert not Aq.cpu().numpy()[128:].any()


def chain(kind, k):
    """FP32 summation-bound constant of the kernel that serves (storage, k)."""
    on_matrix_cores = kind == "fp8" or (kind == "bf16" and k > 6)
    return 4096 + 4 + 256 if on_matrix_cores else 80


def _deq_bound(Adeq, Y, seed, row0, k, ref, kind, col0=0):
    Om = oracle.omega_block(seed, row0, Adeq.shape[1], col0, k)
    mag = oracle.matmul(np.abs(Adeq).astype(np.float32), np.abs(Om))
    err = np.abs(Y - ref)
    c = chain(kind, k)
    assert (err <= c * U * mag + U * np.abs(ref)).all(), float((err - c * U * mag).max())


@pytest.mark.parametrize("m,n,k,row0", [(300, 5000, 5, 0), (200, 3000, 16, 7), (130, 2100, 40, 4),
                                        (600, 9000, 64, 1), (257, 4097, 17, 0), (90, 5000, 130, 2)])
def test_bf16_product(m, n, k, row0):
    A = normal_matrix(m, n, seed=3 * m + k)
    Aq, _ = sk.sketch_quantize(dev_f32(A), "bf16")
    Y = sk.sketch_gen_matmul(Aq, 11, k, omega_row0=row0).double().cpu().numpy()
    codes = Aq.cpu().view(torch.int16).numpy().view(np.uint16)
    ref_q = oracle.gen_matmul_q(codes, "bf16", None, 11, row0, 0, k)
    Adeq = oracle.bf16_decode(codes)
    _deq_bound(Adeq, Y, 11, row0, k, ref_q, "bf16")
    e2e = oracle.rel_fro(Y, oracle.gen_matmul(A, 11, row0, 0, k))
    assert e2e <= 1e-2, e2e
    assert e2e >= 1e-4          # BF16 storage does lose precision: the test sees it


@pytest.mark.parametrize("m,n,k,row0", [(300, 5000, 5, 0), (260, 3000, 16, 9), (600, 9000, 64, 3),
                                        (70, 4100, 100, 0), (1100, 800, 1, 5)])
def test_fp8_product(m, n, k, row0):
    A = normal_matrix(m, n, seed=5 * m + k)
    A[128:256] *= np.float32(0.01)
    Aq, sc = sk.sketch_quantize(dev_f32(A), "fp8")
    Y = sk.sketch_gen_matmul(Aq, 12, k, omega_row0=row0, a_scales=sc).double().cpu().numpy()
    Q = Aq.cpu().numpy()
    s = sc.cpu().numpy()
    ref_q = oracle.gen_matmul_q(Q, "fp8", s, 12, row0, 0, k)
    Adeq = oracle.fp8_decode_table()[Q] * np.repeat(s.astype(np.float64), 128)[:m, None]
    _deq_bound(Adeq, Y, 12, row0, k, ref_q, "fp8")
    e2e = oracle.rel_fro(Y, oracle.gen_matmul(A, 12, row0, 0, k))
    assert e2e <= 5e-2, e2e


def test_low_precision_reduce_layout_matches_row_layout():
    """1Dred over BF16 / FP8 column blocks equals the row layout bitwise when the
    blocks are whole strips (sketch_strip_width)."""
    P = 4
    for kind, code in (("bf16", 1), ("fp8", 2)):
        w = sk.sketch_strip_width(code, 5)
        m, n = 256, P * w
        A = normal_matrix(m, n, seed=77)
        Aq, sc = sk.sketch_quantize(dev_f32(A), kind)
        Yrow = sk.sketch_gen_matmul(Aq, 3, 5, a_scales=sc)
        blocks = [Aq[:, b * w:(b + 1) * w] for b in range(P)]
        Yred = sk.sketch_gen_matmul_reduce(blocks, [b * w for b in range(P)], 3, 5,
                                           scales=None if sc is None else [sc] * P)
        assert torch.equal(Yrow, Yred), kind


def test_full_size_errors_sampled_rows():
    """A 32768 x 32768 N(0,1) stored as BF16 and FP8 (per-128-row scales), k = 5 and 64:
    relative Frobenius error of sampled rows against the FP64 oracle on the original FP32
    rows.  BF16 target <= 1e-2; FP8 has no target and is reported (held <= 5e-2)."""
    from sketch_inputs import normal_matrix_device

    N = 32768
    A = normal_matrix_device(N, N, seed=0, device=DEV)
    rows = torch.from_numpy(np.random.default_rng(1).choice(N, size=16, replace=False)).to(DEV)
    Ah = A[rows].cpu().numpy()
    report = {}
    for kind in ("bf16", "fp8"):
        Aq, sc = sk.sketch_quantize(A, kind)
        for k in (5, 64):
            Y = sk.sketch_gen_matmul(Aq, 1, k, a_scales=sc)
            err = oracle.rel_fro(Y[rows].double().cpu().numpy(), oracle.gen_matmul(Ah, 1, 0, 0, k))
            report[(kind, k)] = err
            assert err <= (1e-2 if kind == "bf16" else 5e-2), (kind, k, err)
        del Aq
    Y = sk.sketch_gen_matmul(A, 1, 5)
    report[("f32", 5)] = oracle.rel_fro(Y[rows].double().cpu().numpy(),
                                        oracle.gen_matmul(Ah, 1, 0, 0, 5))
    assert report[("f32", 5)] <= 1e-5
    print("relative Frobenius errors vs FP64 oracle:",
          {f"{a}/k={k}": f"{e:.3e}" for (a, k), e in report.items()})
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,k", [("bf16", 64), ("fp8", 5), ("fp8", 64)])
def test_matrix_core_layouts_and_stored_omega_bitwise(kind, k):
    """BF16 matrix-core path: 1Dred over whole 4096-column strips equals the row
    layout bitwise, row blocks equal rows of the whole, and the stored-Omega
    product equals the generated one bitwise."""
    m, P = 700, 3
    w = sk.sketch_strip_width(1 if kind == "bf16" else 2, k)
    assert w == 4096
    n = P * w
    A = normal_matrix(m, n, seed=91)
    Aq, sc = sk.sketch_quantize(dev_f32(A), kind)
    Yrow = sk.sketch_gen_matmul(Aq, 6, k, a_scales=sc)
    Yred = sk.sketch_gen_matmul_reduce([Aq[:, b * w:(b + 1) * w] for b in range(P)],
                                       [b * w for b in range(P)], 6, k,
                                       scales=None if sc is None else [sc] * P)
    assert torch.equal(Yrow, Yred)
    parts = []
    for r in range(0, m, 256):      # row blocks on 128-row boundaries keep the FP8 scales aligned
        parts.append(sk.sketch_gen_matmul(Aq[r:r + 256], 6, k,
                                          a_scales=None if sc is None else sc[r // 128:]))
    assert torch.equal(torch.cat(parts), Yrow)
    Om = sk.sketch_gen_omega(6, 0, n, 0, k, device=DEV)
    assert torch.equal(sk.sketch_matmul_omega(Aq, Om, a_scales=sc), Yrow)
