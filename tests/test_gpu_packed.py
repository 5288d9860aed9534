"""GPU parity of the packed-Omega routes against the FP64 oracle.

On the FP32 matrix cores from four N-tiles (k > 32) and on the BF16 matrix cores from two
(k > 16) a call first writes its block of Omega (Sec. 4, the generated operand) once into
the workspace in the order the tiles consume it, and the tiles copy it instead of running
Philox themselves.  These cases put the packing on every boundary it has: Omega row offsets
that are not multiples of the four values one Philox call yields, column offsets, widths
that end inside a chunk or a strip, one-column blocks, contraction splits (1Dred) over
blocks of unequal width, and the three entry distributions.

Bars as for the other matrix-core tests: element by element within the FP32 chain bound
(2048-product strips for FP32 A: 2052 u; 4096-product strips with the hi + lo split of
Omega for BF16 / FP8 A: (4096 + 4 + 256) u), plus u |Y_ref| for the final rounding, and a
relative Frobenius error <= 1e-5 on the dequantised operand.
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
CHAIN = {"f32": 2052, "bf16": 4096 + 4 + 256, "fp8": 4096 + 4 + 256}


def dev_f32(x):
    """Device FP32 copy with its row pitch padded to 16 bytes; the (m, n) view."""
    ld = max(4, (x.shape[1] + 3) // 4 * 4)
    buf = torch.zeros((x.shape[0], ld), dtype=torch.float32, device=DEV)
    buf[:, :x.shape[1]] = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return buf[:, :x.shape[1]]


def dequantised(Aq, sc, kind):
    """FP64 values the kernel multiplies: the decoded codes times their row-block scales."""
    if kind == "bf16":
        return oracle.bf16_decode(Aq.cpu().view(torch.int16).numpy().view(np.uint16))
    s = np.repeat(sc.cpu().numpy().astype(np.float64), 128)[:Aq.shape[0], None]
    return oracle.fp8_decode_table()[Aq.cpu().numpy()] * s


def within_bound(Y, ref, mag, kind):
    Yg = Y.double().cpu().numpy()
    err = np.abs(Yg - ref)
    bound = CHAIN[kind] * U * mag + U * np.abs(ref)
    assert (err <= bound).all(), f"{int((err > bound).sum())} outside; " \
                                 f"max excess {float((err - bound).max())}"
    assert oracle.rel_fro(Yg, ref) <= 1e-5, oracle.rel_fro(Yg, ref)


@pytest.mark.parametrize("m,n,k,row0,col0,dist", [
    (150, 4100, 40, 3, 0, "normal"),        # ragged last strip, row offset inside a quad
    (70, 2049, 130, 1, 7, "normal"),        # one column past a strip, k ends inside a tile
    (33, 5000, 64, 6, 100, "uniform"),
    (64, 3000, 300, 2, 5, "rademacher"),    # two column blocks of 256 + 44
    (1, 4097, 33, 9, 0, "normal"),          # one row, k one past the N-tile count boundary
])
def test_f32_packed_generated(m, n, k, row0, col0, dist):
    A = normal_matrix(m, n, seed=m + n + k)
    Y = sk.sketch_gen_matmul(dev_f32(A), 17, k, omega_row0=row0, omega_col0=col0, dist=dist)
    ref = oracle.gen_matmul(A, 17, row0, col0, k, dist=dist)
    Om = oracle.omega_block(17, row0, n, col0, k, dist=dist)
    within_bound(Y, ref, oracle.matmul(np.abs(A), np.abs(Om)), "f32")


@pytest.mark.parametrize("k", [40, 130])
def test_f32_packed_reduce_ragged_blocks(k):
    """1Dred over blocks of 1000, 2048, 1, 777 and 4100 columns at Omega rows 3 + offset:
    each block packs its own rows of Omega into its own strips of the plane."""
    m, widths, base, col0 = 90, [1000, 2048, 1, 777, 4100], 3, 5
    A = normal_matrix(m, sum(widths), seed=41 + k)
    offs = np.cumsum([0] + widths)
    parts = [A[:, offs[b]:offs[b + 1]] for b in range(len(widths))]
    row0s = [int(o) + base for o in offs[:-1]]
    Y = sk.sketch_gen_matmul_reduce([dev_f32(p) for p in parts], row0s, 23, k, omega_col0=col0)
    ref = oracle.gen_matmul_reduce(parts, row0s, 23, col0, k)
    assert oracle.rel_fro(ref, oracle.gen_matmul(A, 23, base, col0, k)) <= 1e-12
    Om = oracle.omega_block(23, base, A.shape[1], col0, k)
    within_bound(Y, ref, oracle.matmul(np.abs(A), np.abs(Om)), "f32")


@pytest.mark.parametrize("kind,m,n,k,row0,col0", [
    ("bf16", 130, 4100, 20, 3, 0),
    ("bf16", 64, 2049, 70, 1, 9),
    ("fp8", 257, 4100, 20, 3, 0),
    ("fp8", 100, 5000, 70, 6, 33),
    ("fp8", 129, 1000, 130, 2, 0),          # two column blocks of 128 + 2
])
def test_low_precision_packed_generated(kind, m, n, k, row0, col0):
    A = normal_matrix(m, n, seed=7 * m + k)
    if kind == "fp8" and m > 128:
        A[128:256] *= np.float32(1e-3)      # a second row block with its own scale
    Aq, sc = sk.sketch_quantize(dev_f32(A), kind)
    Y = sk.sketch_gen_matmul(Aq, 19, k, omega_row0=row0, omega_col0=col0, a_scales=sc)
    Adeq = dequantised(Aq, sc, kind)
    codes = Aq.cpu().view(torch.int16).numpy().view(np.uint16) if kind == "bf16" \
        else Aq.cpu().numpy()
    ref = oracle.gen_matmul_q(codes, kind, None if sc is None else sc.cpu().numpy(), 19, row0,
                              col0, k)
    Om = oracle.omega_block(19, row0, n, col0, k)
    within_bound(Y, ref, oracle.matmul(np.abs(Adeq).astype(np.float32), np.abs(Om)), kind)


@pytest.mark.parametrize("kind,k,dist", [("bf16", 40, "uniform"), ("fp8", 64, "rademacher")])
def test_low_precision_packed_distributions(kind, k, dist):
    m, n, row0 = 96, 4500, 5
    A = normal_matrix(m, n, seed=k)
    Aq, sc = sk.sketch_quantize(dev_f32(A), kind)
    Y = sk.sketch_gen_matmul(Aq, 29, k, omega_row0=row0, a_scales=sc, dist=dist)
    Adeq = dequantised(Aq, sc, kind)
    Om = oracle.omega_block(29, row0, n, 0, k, dist=dist)
    ref = Adeq @ Om.astype(np.float64)
    within_bound(Y, ref, np.abs(Adeq) @ np.abs(Om).astype(np.float64), kind)


@pytest.mark.parametrize("kind,k", [("bf16", 20), ("fp8", 70)])
def test_low_precision_packed_reduce_ragged_blocks(kind, k):
    """1Dred over separately quantised blocks of 1000, 4096, 1 and 777 columns (each with
    its own FP8 scales) at Omega rows 5 + offset."""
    m, widths, base = 140, [1000, 4096, 1, 777], 5
    A = normal_matrix(m, sum(widths), seed=53 + k)
    offs = np.cumsum([0] + widths)
    row0s = [int(o) + base for o in offs[:-1]]
    qs = [sk.sketch_quantize(dev_f32(A[:, offs[b]:offs[b + 1]]), kind)
          for b in range(len(widths))]
    Y = sk.sketch_gen_matmul_reduce([q for q, _ in qs], row0s, 31, k,
                                    scales=None if kind == "bf16" else [s for _, s in qs])
    ref = np.zeros((m, k))
    mag = np.zeros((m, k))
    for (q, s), r0, w in zip(qs, row0s, widths):
        Adeq = dequantised(q, s, kind)
        Om = oracle.omega_block(31, r0, w, 0, k)
        codes = q.cpu().view(torch.int16).numpy().view(np.uint16) if kind == "bf16" \
            else q.cpu().numpy()
        ref += oracle.gen_matmul_q(codes, kind, None if s is None else s.cpu().numpy(), 31, r0,
                                   0, k)
        mag += oracle.matmul(np.abs(Adeq).astype(np.float32), np.abs(Om))
    within_bound(Y, ref, mag, kind)
