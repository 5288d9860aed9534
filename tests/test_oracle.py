"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* Philox4x32-10 integer stream: two independent open-source library
  implementations (PyTorch ATen's header-only engine and rocRAND's engine),
  run on the host.
* FP32 Box-Muller: exhaustively over all 2^23 uniforms against FP64 libm
  log / cos / sin, plus distribution statistics of a large sample.
* Product: special cases with exact answers (identity, selection matrices,
  zero, power-of-two scaling, zero padding of the offset), numpy's FP64
  matmul as a library routine, exactly rounded sums on tiny inputs, and the
  contraction-split identity of Alg. 1.
* Storage formats: torch's CPU casts to bfloat16 / float8_e4m3fn.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from sketch_inputs import normal_matrix, selection_matrix

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Philox integer stream
# --------------------------------------------------------------------------
def _counter_cases():
    rng = np.random.default_rng(12345)
    cases = []
    seeds = [0, 1, 2, 0xFFFFFFFF, 1 << 32, (1 << 63) + 5, 0xFFFFFFFFFFFFFFFF]
    qs = [0, 1, 2, 3, 0xFFFFFFFF, 1 << 32, (1 << 40) + 7, (1 << 62) - 1]
    cs = [0, 1, 5, 255, 1 << 31, 0xFFFFFFFF]
    for s in seeds:
        for q in qs:
            for c in cs:
                cases.append((s, q, c, 0))
    for _ in range(2000):
        cases.append((int(rng.integers(0, 1 << 63)), int(rng.integers(0, 1 << 62)),
                      int(rng.integers(0, 1 << 32)), int(rng.integers(0, 2))))
    return cases


def _run_pin(exe, cases):
    text = "".join(f"{s} {q} {c} {st}\n" for s, q, c, st in cases)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(w) for w in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64).astype(np.uint32)


def _oracle_words(cases):
    ctr = np.array([[q & 0xFFFFFFFF, q >> 32, c, st] for s, q, c, st in cases], dtype=np.uint64)
    out = []
    for (s, _, _, _), row in zip(cases, ctr.astype(np.uint32)):
        out.append(oracle.philox4x32_10(row[None, :], [s & 0xFFFFFFFF, s >> 32])[0])
    return np.array(out, dtype=np.uint32)


@pytest.fixture(scope="module")
def pin_exes(tmp_path_factory):
    d = tmp_path_factory.mktemp("pins")
    exes = {}
    import torch.utils.cpp_extension as ce

    inc = [f"-I{p}" for p in ce.include_paths()]
    aten = str(d / "pin_aten")
    subprocess.run(["g++", "-O1", "-std=c++17", *inc, os.path.join(HERE, "pins", "philox_aten.cpp"),
                    "-o", aten], check=True)
    exes["aten"] = aten
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if os.path.exists(hipcc):
        roc = str(d / "pin_rocrand")
        subprocess.run([hipcc, "-O1", "-std=c++17",
                        os.path.join(HERE, "pins", "philox_rocrand.cpp"), "-o", roc], check=True)
        exes["rocrand"] = roc
    return exes


@pytest.mark.parametrize("lib", ["aten", "rocrand"])
def test_philox_matches_library(pin_exes, lib):
    if lib not in pin_exes:
        pytest.skip(f"{lib} pin could not be built here")
    cases = _counter_cases()
    ref = _run_pin(pin_exes[lib], cases)
    got = _oracle_words(cases)
    assert ref.shape == got.shape
    assert np.array_equal(ref, got)


def test_philox_batch_equals_single():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 1 << 32, size=(257, 4), dtype=np.uint64).astype(np.uint32)
    key = [0x12345678, 0x9ABCDEF0]
    batch = oracle.philox4x32_10(ctr, key)
    single = np.stack([oracle.philox4x32_10(c[None], key)[0] for c in ctr])
    assert np.array_equal(batch, single)


# --------------------------------------------------------------------------
# FP32 Box-Muller
# --------------------------------------------------------------------------
ALL_ODD = (np.arange(1 << 23, dtype=np.uint64) * 2 + 1).astype(np.uint32)


def _ulps(got, ref):
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    return np.abs(got.astype(np.float64) - ref) / ulp


def test_spec_log_exhaustive_within_3ulp():
    u = ALL_ODD.astype(np.float64) * 2.0 ** -24
    L = oracle.spec_log(ALL_ODD)
    assert np.all(L < 0)
    assert _ulps(L, np.log(u)).max() <= 3.0
    # end points of the uniform range
    assert L[0] == np.float32(-24 * math.log(2)) or abs(L[0] + 24 * math.log(2)) < 2e-6
    assert abs(float(L[-1]) - math.log1p(-2.0 ** -24)) <= 2.0 ** -48


def test_spec_cossin_exhaustive_within_2ulp():
    th = 2 * np.pi * ALL_ODD.astype(np.float64) * 2.0 ** -24
    c, s = oracle.spec_cossin(ALL_ODD)
    assert _ulps(c, np.cos(th)).max() <= 2.0
    assert _ulps(s, np.sin(th)).max() <= 2.0


def test_normal_pair_matches_libm_box_muller():
    rng = np.random.default_rng(5)
    words = rng.integers(0, 1 << 32, size=(20000, 2), dtype=np.uint64)
    words = np.concatenate([words, np.array([[0, 0], [0xFFFFFFFF, 0xFFFFFFFF],
                                             [0, 0x40000000], [0xFFFFFFFF, 0x20000000]],
                                            dtype=np.uint64)])
    for re_, ro in words:
        zc, zs = oracle.normal_pair(int(re_), int(ro))
        ue = (2 * (int(re_) >> 9) + 1) * 2.0 ** -24
        uo = (2 * (int(ro) >> 9) + 1) * 2.0 ** -24
        rho = math.sqrt(-2 * math.log(ue))
        for got, ref in ((zc, rho * math.cos(2 * math.pi * uo)),
                         (zs, rho * math.sin(2 * math.pi * uo))):
            tol = 5 * float(np.spacing(np.float32(abs(ref)))) + 4 * rho * 2.0 ** -24 * 2e-6
            assert abs(got - ref) <= tol, (re_, ro, got, ref)
    # the batch form is the same function
    w32 = words.astype(np.uint32)
    zc, zs = oracle.normal_pairs(w32[:, 0], w32[:, 1])
    one = np.array([oracle.normal_pair(int(a), int(b)) for a, b in w32[:500]], dtype=np.float32)
    assert np.array_equal(zc[:500].view(np.uint32), one[:, 0].view(np.uint32))
    assert np.array_equal(zs[:500].view(np.uint32), one[:, 1].view(np.uint32))


def test_omega_matches_f64_reference_and_word_layout():
    seed = 0xDEADBEEF12345
    for j in list(range(0, 64)) + [4 * 10 ** 6 + 3, (1 << 34) + 1]:
        for c in (0, 1, 4, 1000):
            z = oracle.omega_value(seed, j, c)
            ref = oracle.omega_f64ref(seed, j, c)
            assert abs(z - ref) <= 5 * float(np.spacing(np.float32(abs(ref)))) + 1e-12
    # entry (j, c) uses word j mod 4 of counter (j div 4, c, 0): rows 4q..4q+3
    # of one column come from one Philox call, paired (0,1) and (2,3)
    q, c = 11, 3
    w = oracle.philox4x32_10(np.array([[q, 0, c, 0]], dtype=np.uint32),
                             [seed & 0xFFFFFFFF, seed >> 32])[0]
    z01 = oracle.normal_pair(int(w[0]), int(w[1]))
    z23 = oracle.normal_pair(int(w[2]), int(w[3]))
    got = [oracle.omega_value(seed, 4 * q + t, c) for t in range(4)]
    assert got == [z01[0], z01[1], z23[0], z23[1]]


def test_omega_statistics():
    from scipy import stats

    z = oracle.omega_block(1, 0, 1 << 18, 0, 4).ravel().astype(np.float64)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # columns are independent streams: sample correlation near zero
    Z = oracle.omega_block(1, 0, 1 << 16, 0, 4).astype(np.float64)
    C = np.corrcoef(Z.T)
    assert np.abs(C - np.eye(4)).max() < 5 / math.sqrt(Z.shape[0])
    # neighbouring seeds give unrelated matrices
    Z2 = oracle.omega_block(2, 0, 1 << 16, 0, 4).astype(np.float64)
    assert abs(np.corrcoef(Z[:, 0], Z2[:, 0])[0, 1]) < 5 / math.sqrt(Z.shape[0])


def test_uniform_entries_feed_the_normal_pairs():
    """Uniform Omega: entry (j, c) is the uniform of its own Philox word, so the
    uniforms of rows 4q and 4q+1 are exactly the Box-Muller inputs of the normal
    entries of those rows (checked against FP64 libm Box-Muller on the uniform
    values), and every value is an odd multiple of 2^-24 in (0, 1)."""
    seed = 987654321
    for q, c in ((0, 0), (7, 3), (12345, 1), ((1 << 33) + 5, 999)):
        u = [oracle.omega_value(seed, 4 * q + t, c, "uniform") for t in range(4)]
        for pair in (0, 1):
            ue, uo = u[2 * pair], u[2 * pair + 1]
            rho = math.sqrt(-2 * math.log(ue))
            for t, ref in ((0, rho * math.cos(2 * math.pi * uo)), (1, rho * math.sin(2 * math.pi * uo))):
                z = oracle.omega_value(seed, 4 * q + 2 * pair + t, c)
                assert abs(z - ref) <= 5 * float(np.spacing(np.float32(abs(ref)))) + 4 * rho * 2.0 ** -24 * 2e-6
    U = oracle.omega_block(seed, 0, 1 << 16, 0, 3, "uniform").astype(np.float64)
    m = U * 2.0 ** 24
    assert np.all(m == np.round(m)) and np.all(np.round(m) % 2 == 1)
    assert U.min() > 0 and U.max() < 1


def test_uniform_and_rademacher_statistics_and_signs():
    from scipy import stats

    U = oracle.omega_block(3, 0, 1 << 18, 0, 4, "uniform").ravel().astype(np.float64)
    assert abs(U.mean() - 0.5) < 5 * math.sqrt(1 / 12 / U.size)
    assert abs(U.var() - 1 / 12) < 5 * math.sqrt((1 / 80 - 1 / 144) / U.size)
    assert stats.kstest(U, "uniform").pvalue > 1e-4
    R = oracle.omega_block(3, 0, 1 << 18, 0, 4, "rademacher").ravel()
    # the sign is the word's top bit, i.e. the uniform of the same entry vs 1/2
    assert np.array_equal(R, np.where(U < 0.5, 1.0, -1.0).astype(np.float32))
    assert set(np.unique(R)) == {-1.0, 1.0}
    assert abs(R.astype(np.float64).mean()) < 5 / math.sqrt(R.size)


def test_rademacher_product_of_integer_matrix_is_exact():
    rng = np.random.default_rng(8)
    A = rng.integers(-100, 101, size=(37, 900)).astype(np.float32)
    R = oracle.omega_block(21, 50, 900, 4, 6, "rademacher")
    ref = A.astype(np.int64) @ R.astype(np.int64)
    Y = oracle.gen_matmul(A, 21, 50, 4, 6, "rademacher")
    assert np.array_equal(Y, ref.astype(np.float64))
    Yu = oracle.gen_matmul(A, 21, 50, 4, 6, "uniform")
    Uo = oracle.omega_block(21, 50, 900, 4, 6, "uniform").astype(np.float64)
    assert np.allclose(Yu, A.astype(np.float64) @ Uo, rtol=1e-13, atol=1e-9)
    Yr = oracle.gen_matmul_reduce([A[:, :400], A[:, 400:]], [50, 450], 21, 4, 6, "rademacher")
    assert np.array_equal(Yr, Y)


def test_column_major_equals_row_major_of_the_same_matrix():
    """A stored column-major (with NaN padding below each column that must never be
    read) gives bitwise the row-major product of the same matrix."""
    m, n, lda = 37, 500, 40
    A = normal_matrix(m, n, seed=12)
    Acm = np.full((n, lda), np.nan, dtype=np.float32)
    Acm[:, :m] = A.T
    for dist in ("normal", "uniform", "rademacher"):
        Y = oracle.gen_matmul_cm(Acm.ravel(), m, n, lda, 5, 9, 2, 7, dist)
        assert np.array_equal(Y, oracle.gen_matmul(A, 5, 9, 2, 7, dist)), dist


def test_second_nystrom_product_definition():
    """C = Omega^T B: against numpy on the oracle's Omega, against the column-major
    product of B^T (bitwise: same sums), a one-hot B picking one Omega row, and an
    exactly rounded sum on a tiny case."""
    n, p, k = 900, 6, 5
    B = normal_matrix(n, p, seed=13)
    C = oracle.gen_tmatmul(B, 3, 11, 4, k)
    Om = oracle.omega_block(3, 11, n, 4, k).astype(np.float64)
    assert np.allclose(C, Om.T @ B.astype(np.float64), rtol=1e-12, atol=1e-10)
    # B row-major n x p is B^T column-major p x n with lda = p
    Ct = oracle.gen_matmul_cm(B.ravel(), p, n, p, 3, 11, 4, k)
    assert np.array_equal(C, Ct.T)
    E = np.zeros((n, p), dtype=np.float32)
    E[123, 2] = 1.0
    Ce = oracle.gen_tmatmul(E, 3, 11, 4, k)
    assert np.array_equal(Ce[:, 2], Om[123])
    assert not np.delete(Ce, 2, axis=1).any()
    Bt = normal_matrix(9, 3, seed=14)
    Ct = oracle.gen_tmatmul(Bt, 8, 1, 0, 2)
    Omt = oracle.omega_block(8, 1, 9, 0, 2)
    for a in range(2):
        for b in range(3):
            ref = math.fsum(float(Omt[j, a]) * float(Bt[j, b]) for j in range(9))
            assert abs(Ct[a, b] - ref) <= 1e-15 * max(1.0, abs(ref))


def test_omega_block_is_slice_of_global():
    full = oracle.omega_block(9, 0, 300, 0, 40)
    for row0, n, col0, k in [(0, 300, 0, 40), (3, 101, 7, 5), (1, 1, 39, 1), (257, 43, 0, 16)]:
        assert np.array_equal(oracle.omega_block(9, row0, n, col0, k),
                              full[row0:row0 + n, col0:col0 + k])


# --------------------------------------------------------------------------
# Products
# --------------------------------------------------------------------------
def test_identity_gives_omega_block():
    n, k, row0, col0 = 77, 6, 13, 2
    Y = oracle.gen_matmul(np.eye(n, dtype=np.float32), 4, row0, col0, k)
    assert np.array_equal(Y, oracle.omega_block(4, row0, n, col0, k).astype(np.float64))


def test_selection_matrix_picks_global_rows():
    m, n, k, row0, col0 = 50, 300, 5, 4096 * 3 + 1, 0
    S, cols = selection_matrix(m, n, seed=2)
    Y = oracle.gen_matmul(S, 11, row0, col0, k)
    for i in range(m):
        expect = [oracle.omega_value(11, row0 + int(cols[i]), col0 + c) for c in range(k)]
        assert np.array_equal(Y[i], np.array(expect, dtype=np.float64))


def test_matches_numpy_matmul_nonsquare():
    m, n, k = 37, 203, 9
    A = normal_matrix(m, n, seed=6)
    Om = oracle.omega_block(21, 5, n, 3, k)
    Y = oracle.gen_matmul(A, 21, 5, 3, k)
    ref = A.astype(np.float64) @ Om.astype(np.float64)
    assert Y.shape == (m, k)
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(A).sum(1).max() * np.abs(Om).max()


def test_exactly_rounded_sum_tiny():
    m, n, k = 5, 17, 3
    A = normal_matrix(m, n, seed=8)
    Om = oracle.omega_block(1, 0, n, 0, k)
    Y = oracle.gen_matmul(A, 1, 0, 0, k)
    for i in range(m):
        for c in range(k):
            terms = [float(A[i, j]) * float(Om[j, c]) for j in range(n)]
            exact = math.fsum(terms)
            bound = n * 2.0 ** -53 * sum(abs(t) for t in terms)
            assert abs(Y[i, c] - exact) <= bound


def test_zero_scaling_and_padding():
    m, n, k = 9, 64, 4
    A = normal_matrix(m, n, seed=10)
    assert not oracle.gen_matmul(np.zeros((m, n), np.float32), 3, 0, 0, k).any()
    Y = oracle.gen_matmul(A, 3, 8, 1, k)
    assert np.array_equal(oracle.gen_matmul(A * np.float32(4.0), 3, 8, 1, k), 4.0 * Y)
    # an offset row0 equals zero columns of A in front of the block
    pad = np.zeros((m, 8 + n), np.float32)
    pad[:, 8:] = A
    assert np.array_equal(oracle.gen_matmul(pad, 3, 0, 1, k), Y)


def test_strided_view_equals_copy():
    A = normal_matrix(20, 100, seed=12)
    view = A[:, 30:70]
    assert np.array_equal(oracle.gen_matmul(view, 5, 30, 0, 3),
                          oracle.gen_matmul(np.ascontiguousarray(view), 5, 30, 0, 3))


def test_contraction_split_equals_single_product():
    """Alg. 1 with a (1, P, 1) grid: summing the P partial products over column
    blocks gives the product of the whole row (up to FP64 rounding)."""
    m, n, P, k = 33, 4 * 64 + 7, 4, 5
    A = normal_matrix(m, n, seed=14)
    bounds = [0, 64, 128, 192, n]
    blocks = [A[:, bounds[b]:bounds[b + 1]] for b in range(P)]
    Yred = oracle.gen_matmul_reduce(blocks, bounds[:P], 77, 0, k)
    Yfull = oracle.gen_matmul(A, 77, 0, 0, k)
    assert oracle.rel_fro(Yred, Yfull) <= 1e-13
    # row split (P, 1, 1): the row blocks of Y are the products of the row blocks of A
    Yrows = np.concatenate([oracle.gen_matmul(A[i:i + 11], 77, 0, 0, k) for i in range(0, m, 11)])
    assert np.array_equal(Yrows, Yfull)


def test_empty_shapes():
    assert oracle.gen_matmul(np.zeros((0, 5), np.float32), 1, 0, 0, 3).shape == (0, 3)
    Y = oracle.gen_matmul(np.zeros((4, 0), np.float32), 1, 0, 0, 3)
    assert Y.shape == (4, 3) and not Y.any()


# --------------------------------------------------------------------------
# Storage formats
# --------------------------------------------------------------------------
def test_bf16_matches_torch():
    import torch

    x = np.concatenate([normal_matrix(1, 5000, 3).ravel(),
                        np.array([0.0, -0.0, 1.0, 65504.0, 3.0e38, 1e-40, 1.00390625,
                                  1.01171875, -2.0 ** -130], dtype=np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.bf16_encode(x), ref)
    dec = oracle.bf16_decode(ref[:100])
    assert np.array_equal(dec, torch.from_numpy(ref[:100].view(np.int16)).view(torch.bfloat16)
                          .float().numpy().astype(np.float64))


def test_fp8_codec_matches_torch():
    import torch

    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    table = oracle.fp8_decode_table()
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(table))
    assert np.array_equal(ref[~nan], table[~nan])
    rng = np.random.default_rng(4)
    vals = np.concatenate([rng.standard_normal(4000) * 50, rng.standard_normal(1000) * 1e-3,
                           table[~nan], (table[~nan][1:] + table[~nan][:-1]) / 2])
    vals = vals[np.abs(vals) <= 448].astype(np.float32)
    tref = torch.from_numpy(vals).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = np.array([oracle.fp8_encode(float(v)) for v in vals], dtype=np.uint8)
    # +0 and -0 are distinct codes in both
    assert np.array_equal(got, tref)
    assert oracle.fp8_encode(1000.0) == 0x7E and oracle.fp8_encode(-1e9) == 0xFE


def test_fp8_rows128_scales_definition():
    A = normal_matrix(300, 40, seed=15) * np.float32(3.0)
    A[128:256] *= np.float32(1e-3)
    A[256:] = 0.0
    Q, s = oracle.quantize_fp8_rows128(A)
    assert s.shape == (3,)
    for b in range(2):
        amax = float(np.abs(A[128 * b:128 * (b + 1)]).max())
        E = math.log2(float(s[b]))
        assert E == int(E)
        assert amax <= 448 * s[b] and amax > 448 * s[b] / 2
    assert s[2] == 1.0 and not Q[256:].any()
    table = oracle.fp8_decode_table()
    deq = table[Q] * np.repeat(s.astype(np.float64), 128)[:300, None]
    rel = np.abs(deq - A) / np.maximum(np.abs(A), 1e-30)
    mask = np.abs(A) >= 2.0 ** -6 * np.repeat(s, 128)[:300, None]
    assert rel[mask].max() <= 2.0 ** -4 + 1e-12   # 3 mantissa bits, round to nearest


def test_fp8_scales_at_fp32_extremes():
    """Scales are FP32 powers of two: the smallest one with amax <= 448 s, but never
    below 2^-149 (FP32's smallest power of two).  Codes are torch's E4M3 cast of the
    exact quotient A / s."""
    import torch

    A = normal_matrix(512, 64, seed=17)
    A[0:128] *= np.float32(1e-38)           # scale 2^-133: its reciprocal overflows FP32
    A[128:256] *= np.float32(1e-43)         # subnormals only: amax < 448 * 2^-149
    A[256:384] *= np.float32(1e30)
    Q, s = oracle.quantize_fp8_rows128(A)
    assert s[1] == np.float32(2.0 ** -149)
    for b in range(4):
        blk = A[128 * b:128 * (b + 1)].astype(np.float64)
        amax = float(np.abs(blk).max())
        E = math.log2(float(s[b]))
        assert E == int(E) and E >= -149
        assert amax <= 448 * float(s[b])
        assert amax > 448 * float(s[b]) / 2 or E == -149
        q = torch.from_numpy((blk / float(s[b])).astype(np.float32))
        ref = q.to(torch.float8_e4m3fn).view(torch.uint8).numpy()
        assert np.array_equal(Q[128 * b:128 * (b + 1)], ref)


def test_quantized_product_equals_product_of_dequantized():
    m, n, k = 130, 96, 5
    A = normal_matrix(m, n, seed=16)
    Qb = oracle.bf16_encode(A)
    Ab = oracle.bf16_decode(Qb).astype(np.float32)
    assert np.array_equal(oracle.gen_matmul_q(Qb, "bf16", None, 2, 0, 0, k),
                          oracle.gen_matmul(Ab, 2, 0, 0, k))
    Q8, s = oracle.quantize_fp8_rows128(A)
    A8 = (oracle.fp8_decode_table()[Q8] * np.repeat(s.astype(np.float64), 128)[:m, None])
    assert np.array_equal(oracle.gen_matmul_q(Q8, "fp8", s, 2, 0, 0, k),
                          oracle.gen_matmul(A8.astype(np.float32), 2, 0, 0, k))


# --------------------------------------------------------------------------
# Golden fixtures (written by tests/golden/make_golden.py from the oracle)
# --------------------------------------------------------------------------
GOLDEN = os.path.join(HERE, "golden")


def _golden_rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if not line.startswith("#")]


def test_golden_omega_block():
    rows = _golden_rows("omega_seed1_r0-63_c0-4.txt")
    ref = np.array([[int(w, 16) for w in r] for r in rows], dtype=np.uint32)
    assert np.array_equal(oracle.omega_block(1, 0, 64, 0, 5).view(np.uint32), ref)


def test_golden_omega_offsets():
    for r, c, bits in _golden_rows("omega_seed2026_offsets.txt"):
        got = np.float32(oracle.omega_value(2026, int(r), int(c))).view(np.uint32)
        assert int(got) == int(bits, 16)


def _rbf(X, sigma):
    sq = (X * X).sum(1)
    D = np.maximum(sq[:, None] + sq[None, :] - 2 * X @ X.T, 0.0)
    return np.exp(-D / (2 * sigma ** 2))


def test_nystrom_oracle_closed_forms():
    """Nystrom approximation (Sec. 5): an exactly rank-q PSD A with q <= r is reproduced;
    A - A~ is positive semidefinite; with Omega's first r columns contained in the next
    sketch (column prefix) the error cannot grow."""
    from oracle.nystrom import nystrom

    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 10))
    A = X @ X.T
    _, _, At, err = nystrom(A, 20, 7)
    assert err <= 1e-10
    Xr = rng.standard_normal((300, 5))
    K = _rbf(Xr, np.linalg.norm(Xr) / math.sqrt(300))
    errs = []
    for r in (8, 16, 32, 64):
        _, C, At, e = nystrom(K, r, 3)
        assert np.allclose(C, C.T, rtol=1e-10, atol=1e-10 * np.abs(C).max())
        assert np.linalg.eigvalsh(K - At).min() >= -1e-9 * np.linalg.norm(K)
        errs.append(e)
    assert all(b <= a + 1e-12 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.5 * errs[0]


def test_core_pinv_oracle_known_spectrum():
    """The oracle's core pseudo-inverse (Sec. 5; eigenvalue cut of Sec. 6.2) on matrices
    built from a known spectrum: C = U diag(lambda) U^T gives U diag(mu) U^T with
    mu = 1/lambda above tol * max|lambda| and 0 below; the Moore-Penrose identities
    hold for the kept part; a planted eigenvalue just below the cut is dropped and one
    just above is kept; the symmetric part of a non-symmetric input is what is inverted."""
    from oracle.nystrom import core_pinv

    rng = np.random.default_rng(12)
    r = 40
    U, _ = np.linalg.qr(rng.standard_normal((r, r)))
    lam = np.logspace(0, -6, r)
    lam[5] = -0.25                 # indefinite: kept, inverted with its sign
    lam[-3:] = [0.0, 0.5e-12, 2e-12]
    C = (U * lam) @ U.T
    mu = np.where(np.abs(lam) > 1e-12, 1.0 / np.where(lam == 0, 1, lam), 0.0)
    want = (U * mu) @ U.T
    got = core_pinv(C, 1e-12)
    kappa = 1.0 / 2e-12
    assert np.linalg.norm(got - want) <= 64 * r * 2.0 ** -53 * kappa * np.linalg.norm(want)
    # dropping the two small planted eigenvalues: a clean projector identity on the rest
    got6 = core_pinv(C, 1e-9)
    P = got6 @ C
    keep = np.abs(lam) > 1e-9
    Pk = (U[:, keep]) @ U[:, keep].T
    assert np.abs(P - Pk).max() <= 1e-8
    kappa_kept = 1.0 / np.abs(lam[keep]).min()
    assert np.abs(C @ got6 @ C - (U[:, keep] * lam[keep]) @ U[:, keep].T).max() <= \
        64 * r * 2.0 ** -53 * kappa_kept
    # only the symmetric part counts: M and M^T give the same result, and an antisymmetric
    # addition leaves the (well-conditioned) kept part unchanged up to rounding
    Sk = rng.standard_normal((r, r))
    M = C + 1e-3 * (Sk - Sk.T)
    assert np.array_equal(core_pinv(M, 1e-12), core_pinv(M.T, 1e-12))
    assert np.linalg.norm(core_pinv(M, 1e-9) - got6) <= 1e-6 * np.linalg.norm(got6)
