"""The stored-operand product (the "communicate Omega" alternative of Sec. 6.3):
sketch_matmul_omega against the FP64 oracle on an explicit Omega.

Omega here is NOT the generated one: an arbitrary FP32 matrix held in a strided
device buffer (ldo > k, a column offset), so a wrong ldo, column base or row
index in the kernels' stored-operand branches shows.  Every kernel family runs:
FP32 A on the VALU path (k <= 8) and the FP32 matrix cores (k > 8, one and
several column blocks), BF16 A (VALU for k <= 6, BF16 matrix cores above),
FP8 A with per-128-row scales (BF16 matrix cores).

Bars (u = 2^-24): the reference is oracle.matmul on the exactly dequantised A
(FP32 A itself; BF16 and FP8 codes times the power-of-two scale are exact in
FP32), FP64 products and sums; each element within c u sum_j |a_ij w_jc| +
u |y_ic| with c the chain constant of the kernel (80 on the VALU paths, 2052
on the FP32 matrix cores, 4096 + 4 + 256 on the BF16 matrix cores, whose
Omega enters as hi + lo BF16 terms within 2^-16 of it), and the relative
Frobenius error <= 1e-5.  The stored generated Omega gives the generated
product bit for bit, and the oracle's generated product within the same bound.
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
    ld = max(4, (x.shape[1] + 3) // 4 * 4)
    buf = torch.zeros((x.shape[0], ld), dtype=torch.float32, device=DEV)
    buf[:, :x.shape[1]] = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return buf[:, :x.shape[1]]


def chain(kind, k):
    if kind == "f32":
        return 80 if k <= 8 else 2052
    if kind == "bf16" and k <= 6:
        return 80
    return 4096 + 4 + 256


def strided_omega(Om: np.ndarray, pad_left=3, pad_right=6):
    """Omega in a device buffer of width pad_left + k + pad_right (ldo > k), NaN around it:
    a read outside the k columns poisons the result."""
    n, k = Om.shape
    buf = torch.full((n, pad_left + k + pad_right), float("nan"), device=DEV)
    buf[:, pad_left:pad_left + k] = torch.from_numpy(Om).to(DEV)
    return buf[:, pad_left:pad_left + k]


def quantised(A, kind):
    """(device A in storage `kind`, scales or None, exactly dequantised FP32 host copy)."""
    Ad = dev_f32(A)
    if kind == "f32":
        return Ad, None, A
    Aq, sc = sk.sketch_quantize(Ad, kind)
    if kind == "bf16":
        codes = Aq.cpu().view(torch.int16).numpy().view(np.uint16)
        return Aq, None, oracle.bf16_decode(codes).astype(np.float32)
    Q = Aq.cpu().numpy()
    s = sc.cpu().numpy()
    deq = oracle.fp8_decode_table()[Q] * np.repeat(s.astype(np.float64), 128)[:A.shape[0], None]
    return Aq, sc, deq.astype(np.float32)


def check(Y, Adeq, Om, kind, k):
    Yg = Y.double().cpu().numpy()
    ref = oracle.matmul(Adeq, Om)
    mag = oracle.matmul(np.abs(Adeq), np.abs(Om))
    bound = chain(kind, k) * U * mag + U * np.abs(ref)
    err = np.abs(Yg - ref)
    assert np.isfinite(Yg).all()
    assert (err <= bound).all(), (int((err > bound).sum()), float((err - bound).max()))
    assert oracle.rel_fro(Yg, ref) <= 1e-5


@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("m,n,k", [(300, 5000, 5), (257, 4100, 16), (130, 4500, 40),
                                   (90, 2600, 130), (70, 2100, 300)])
def test_arbitrary_strided_omega(kind, m, n, k):
    A = normal_matrix(m, n, seed=m + 7 * k)
    if kind == "fp8" and m > 128:
        A[128:256] *= np.float32(0.03)          # a block with its own scale
    Om = normal_matrix(n, k, seed=n + k) * np.float32(0.7)
    Om[::97] = 0.0                              # some exact zeros
    Ad, sc, Adeq = quantised(A, kind)
    Y = sk.sketch_matmul_omega(Ad, strided_omega(Om), a_scales=sc)
    torch.cuda.synchronize()
    check(Y, Adeq, Om, kind, k)


@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8"])
def test_stored_generated_omega_equals_oracle_and_generated(kind):
    m, n = 200, 6000
    A = normal_matrix(m, n, seed=5)
    Ad, sc, Adeq = quantised(A, kind)
    for k, row0, col0 in [(5, 0, 0), (16, 3, 2), (64, 9, 0), (200, 1, 5)]:
        Om = oracle.omega_block(33, row0, n, col0, k)
        Ys = sk.sketch_matmul_omega(Ad, strided_omega(Om), a_scales=sc)
        Yg = sk.sketch_gen_matmul(Ad, 33, k, omega_row0=row0, omega_col0=col0, a_scales=sc)
        assert torch.equal(Ys, Yg), (kind, k)
        check(Ys, Adeq, Om, kind, k)


def test_stored_omega_beta_and_f64():
    m, n, k = 150, 3000, 24
    A = normal_matrix(m, n, seed=8)
    Om = normal_matrix(n, k, seed=9)
    Ad = dev_f32(A)
    Y0 = torch.from_numpy(normal_matrix(m, k, seed=10)).double().to(DEV)
    Y = Y0.clone()
    sk.sketch_matmul_omega(Ad, strided_omega(Om), Y=Y, beta=1)
    ref = oracle.matmul(A, Om)
    assert oracle.rel_fro((Y - Y0).cpu().numpy(), ref) <= 1e-5
    Y64 = sk.sketch_matmul_omega(Ad, strided_omega(Om), y_dtype=torch.float64)
    check(Y64, A, Om, "f32", k)
    assert torch.equal(sk.sketch_matmul_omega(Ad, strided_omega(Om)), Y64.float())
