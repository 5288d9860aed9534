"""GPU parity of the uniform and Rademacher Omega (paper's experiments draw uniform
entries, Sec. 6.3): entries bitwise equal to the oracle's; products against the
FP64 oracle on every kernel path (VALU k <= 8, FP32 matrix cores, BF16 matrix
cores for low-precision A); Rademacher products of small-integer A are exact and
so bitwise equal to the oracle; layouts and the server keep results bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk
from paper_2603_20966_amd import serve as sv
from sketch_inputs import normal_matrix

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
DEV = "cuda:0"
DISTS = ("uniform", "rademacher")


def to_dev(x):
    ld = max(4, (x.shape[1] + 3) // 4 * 4)
    buf = torch.zeros((x.shape[0], ld), dtype=torch.float32, device=DEV)
    buf[:, :x.shape[1]] = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return buf[:, :x.shape[1]]


def chain(k):
    return 80 if k <= 8 else 2052


@pytest.mark.parametrize("dist", DISTS)
def test_omega_entries_bit_exact(dist):
    for row0, n, col0, k in ((0, 1000, 0, 5), (3, 777, 2, 9), ((1 << 33) + 1, 130, 1000, 3)):
        got = sk.sketch_gen_omega(11, row0, n, col0, k, device=DEV, dist=dist).cpu().numpy()
        ref = oracle.omega_block(11, row0, n, col0, k, dist)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (dist, row0)


@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("m,n,k,row0,col0", [(300, 5000, 5, 0, 0), (129, 3001, 16, 7, 3),
                                             (257, 4100, 64, 1, 0), (70, 2100, 130, 0, 5)])
def test_fp32_products(dist, m, n, k, row0, col0):
    A = normal_matrix(m, n, seed=m + k)
    Y = sk.sketch_gen_matmul(to_dev(A), 5, k, omega_row0=row0, omega_col0=col0,
                             dist=dist).double().cpu().numpy()
    ref = oracle.gen_matmul(A, 5, row0, col0, k, dist)
    Om = oracle.omega_block(5, row0, n, col0, k, dist)
    mag = oracle.matmul(np.abs(A).astype(np.float32), np.abs(Om))
    assert (np.abs(Y - ref) <= chain(k) * U * mag + U * np.abs(ref)).all()
    assert oracle.rel_fro(Y, ref) <= 1e-5


@pytest.mark.parametrize("k", [5, 40])
def test_rademacher_integer_products_exact(k):
    rng = np.random.default_rng(k)
    A = rng.integers(-100, 101, size=(200, 5003)).astype(np.float32)
    Y = sk.sketch_gen_matmul(to_dev(A), 9, k, omega_row0=2, dist="rademacher").cpu().numpy()
    ref = oracle.gen_matmul(A, 9, 2, 0, k, "rademacher")
    assert np.array_equal(Y.astype(np.float64), ref)
    # BF16 storage holds these integers exactly, so the BF16 matrix-core path is exact too
    Aq, _ = sk.sketch_quantize(to_dev(A), "bf16")
    Yq = sk.sketch_gen_matmul(Aq, 9, 64, omega_row0=2, dist="rademacher").cpu().numpy()
    assert np.array_equal(Yq.astype(np.float64), oracle.gen_matmul(A, 9, 2, 0, 64, "rademacher"))


@pytest.mark.parametrize("kind,k", [("bf16", 64), ("fp8", 5)])
def test_low_precision_products(kind, k):
    m, n = 300, 5000
    A = normal_matrix(m, n, seed=31)
    Aq, sc = sk.sketch_quantize(to_dev(A), kind)
    Y = sk.sketch_gen_matmul(Aq, 4, k, a_scales=sc, dist="uniform").double().cpu().numpy()
    if kind == "bf16":
        Adq = oracle.bf16_decode(Aq.cpu().view(torch.int16).numpy().view(np.uint16))
    else:
        Adq = oracle.fp8_decode_table()[Aq.cpu().numpy()] * \
            np.repeat(sc.cpu().numpy().astype(np.float64), 128)[:m, None]
    Om = oracle.omega_block(4, 0, n, 0, k, "uniform")
    ref = Adq @ Om.astype(np.float64)
    mag = np.abs(Adq) @ np.abs(Om).astype(np.float64)
    assert (np.abs(Y - ref) <= (4096 + 4 + 256) * U * mag + U * np.abs(ref)).all()


def test_layouts_and_served_requests_bitwise():
    m, n, k, P = 256, 4 * 4096, 5, 4
    Ad = to_dev(normal_matrix(m, n, seed=44))
    w = n // P
    for dist in DISTS:
        Yrow = sk.sketch_gen_matmul(Ad, 3, k, dist=dist)
        Yred = sk.sketch_gen_matmul_reduce([Ad[:, b * w:(b + 1) * w] for b in range(P)],
                                           [b * w for b in range(P)], 3, k, dist=dist)
        assert torch.equal(Yrow, Yred), dist
        Om = sk.sketch_gen_omega(3, 0, n, 0, k, device=DEV, dist=dist)
        assert torch.equal(sk.sketch_matmul_omega(Ad, Om), Yrow), dist
    # the server carries the distribution per request, mixed in one batch
    Ys = {d: torch.empty((m, k), device=DEV) for d in ("normal",) + DISTS}
    torch.cuda.synchronize()
    with sk.SketchServer(1 << 28, max_slots=8, max_batch=8) as srv:
        ts = {d: srv.submit(sv.make_request(A=Ad, k=k, seed=3, Y=Y, dist=d), Ad, Y)
              for d, Y in Ys.items()}
        for t in ts.values():
            assert srv.wait(t, 60.0)["state"] == sv.SK_REQ_DONE
    for d, Y in Ys.items():
        assert torch.equal(Y, sk.sketch_gen_matmul(Ad, 3, k, dist=d)), d
    assert not torch.equal(Ys["uniform"], Ys["normal"])
