"""GPU tests of the request server (continuous batching of uneven sketches).

* Each request's Y is bitwise the same served alone (one request per launch,
  one in flight), in a mixed batch, and as a direct sketch_gen_matmul call:
  the server runs the same tiles, strip boundaries and FP64 summation order.
* Served results match the FP64 oracle (relative Frobenius <= 1e-5).
* Admission never holds more than the memory budget; oversized requests are
  refused; queued requests can be cancelled; requests that arrive while others
  run are admitted before those finish.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk
from paper_2603_20966_amd import serve as sv
from sketch_inputs import normal_matrix

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev_matrix(m, n, seed):
    """N(0,1) FP32 m x n on the device, row pitch padded to 16 bytes."""
    A = normal_matrix(m, n, seed=seed)
    ld = (n + 3) // 4 * 4
    buf = torch.zeros((m, ld), dtype=torch.float32, device=DEV)
    buf[:, :n] = torch.from_numpy(A).to(DEV)
    return A, buf[:, :n]


# (m, n, k, row0, col0): uneven shapes over every kernel class the server batches
MIX = [(300, 5000, 5, 0, 0), (1000, 700, 5, 3, 0), (129, 9000, 16, 7, 2), (64, 1500, 16, 0, 0),
       (513, 4100, 64, 0, 0), (200, 2049, 64, 5, 1), (77, 3000, 3, 1, 0), (450, 2500, 40, 0, 9),
       (31, 100, 5, 0, 0), (256, 8192, 5, 4096, 0), (600, 6000, 128, 0, 0), (90, 333, 12, 2, 0)]


def run_direct(As):
    out = []
    for (m, n, k, r0, c0), (_, Ad) in zip(MIX, As):
        out.append(sk.sketch_gen_matmul(Ad, 100 + k, k, omega_row0=r0, omega_col0=c0))
    torch.cuda.synchronize()
    return out


def run_served(As, max_slots, max_batch, budget=1 << 30):
    Ys = [torch.full((m, k), float("nan"), device=DEV) for (m, n, k, _, _) in MIX]
    torch.cuda.synchronize()
    infos = []
    with sk.SketchServer(budget, max_slots=max_slots, max_batch=max_batch) as srv:
        tickets = []
        for (m, n, k, r0, c0), (_, Ad), Y in zip(MIX, As, Ys):
            req = sv.make_request(A=Ad, k=k, seed=100 + k, Y=Y, omega_row0=r0, omega_col0=c0)
            tickets.append(srv.submit(req, Ad, Y))
            if max_slots == 1:
                infos.append(srv.wait(tickets[-1], 60.0))
        if max_slots > 1:
            infos = [srv.wait(t, 60.0) for t in tickets]
        stats = srv.stats()
    assert all(i["state"] == sv.SK_REQ_DONE and i["status"] == 0 for i in infos), infos
    return Ys, infos, stats


def test_alone_mix_and_direct_bitwise():
    As = [dev_matrix(m, n, seed=i) for i, (m, n, _, _, _) in enumerate(MIX)]
    Yd = run_direct(As)
    Ya, ia, sa = run_served(As, max_slots=1, max_batch=1)
    Ym, im, sm = run_served(As, max_slots=16, max_batch=16)
    assert max(i["batch_size"] for i in ia) == 1
    assert max(i["batch_size"] for i in im) > 1          # really batched
    assert sm["batches"] < len(MIX)
    for q, (d, a, x) in enumerate(zip(Yd, Ya, Ym)):
        assert torch.equal(d, a), (q, MIX[q])
        assert torch.equal(d, x), (q, MIX[q])
    # and the served values are the sketch: against the FP64 oracle
    for q in (0, 2, 4, 10):
        m, n, k, r0, c0 = MIX[q]
        ref = oracle.gen_matmul(As[q][0], 100 + k, r0, c0, k)
        assert oracle.rel_fro(Ym[q].double().cpu().numpy(), ref) <= 1e-5


def test_sixty_served_requests_against_oracle():
    """60 requests of the serving workload's mix (Poisson arrivals, m and n
    log-uniform, k uniform over {5, 16, 64}, distinct Omega seeds), scaled to
    m, n in [256, 4096] so the FP64 oracle checks every element: each served Y
    within the element bound of its kernel (80 u on the VALU path, 2052 u on the
    matrix cores; u = 2^-24) and within 1e-5 relative Frobenius."""
    from sketch_inputs import request_stream

    U = 2.0 ** -24
    reqs = request_stream(60, seed=7, rate_per_s=1.0, mn_lo=256, mn_hi=4096)
    As = [dev_matrix(r["m"], r["n"], seed=r["seed_a"]) for r in reqs]
    Ys = [torch.full((r["m"], r["k"]), float("nan"), device=DEV) for r in reqs]
    torch.cuda.synchronize()
    with sk.SketchServer(1 << 30, max_slots=16, max_batch=16) as srv:
        ts = [srv.submit(sv.make_request(A=Ad, k=r["k"], seed=r["seed_omega"], Y=Y,
                                         omega_row0=r["id"] % 5), Ad, Y)
              for r, (_, Ad), Y in zip(reqs, As, Ys)]
        infos = [srv.wait(t, 60.0) for t in ts]
        st = srv.stats()
    assert all(i["state"] == sv.SK_REQ_DONE and i["status"] == 0 for i in infos)
    assert st["batches"] < len(reqs)
    classes = set()
    for r, (A, _), Y in zip(reqs, As, Ys):
        k, row0 = r["k"], r["id"] % 5
        got = Y.double().cpu().numpy()
        ref = oracle.gen_matmul(A, r["seed_omega"], row0, 0, k)
        Om = oracle.omega_block(r["seed_omega"], row0, r["n"], 0, k)
        mag = oracle.matmul(np.abs(A), np.abs(Om))
        c = 80 if k <= 8 else 2052
        assert (np.abs(got - ref) <= c * U * mag + U * np.abs(ref)).all(), r
        assert oracle.rel_fro(got, ref) <= 1e-5, r
        classes.add(k)
    assert classes == {5, 16, 64}


def test_host_and_synthetic_sources():
    m, n, k = 700, 3000, 16
    A = normal_matrix(m, n, seed=5)
    Ah = torch.from_numpy(A).pin_memory()
    Ad = dev_matrix(m, n, seed=5)[1]
    Ydirect = sk.sketch_gen_matmul(Ad, 9, k)
    Yh = torch.empty((m, k), device=DEV)
    Ys1 = torch.empty((m, 64), device=DEV)
    Ys2 = torch.empty((m, 64), device=DEV)
    torch.cuda.synchronize()
    with sk.SketchServer(1 << 28, max_slots=4, max_batch=4) as srv:
        t1 = srv.submit(sv.make_request(A=Ah, k=k, seed=9, Y=Yh, source=sv.SK_SRC_HOST), Ah, Yh)
        syn = dict(m=m, n=n, source=sv.SK_SRC_SYNTH, a_seed=77, k=64, seed=3)
        t2 = srv.submit(sv.make_request(Y=Ys1, **syn), Ys1)
        i1, i2 = srv.wait(t1, 60.0), srv.wait(t2, 60.0)
        t3 = srv.submit(sv.make_request(Y=Ys2, **syn), Ys2)   # alone this time
        i3 = srv.wait(t3, 60.0)
    assert i1["state"] == i2["state"] == i3["state"] == sv.SK_REQ_DONE
    assert torch.equal(Yh, Ydirect)                     # staged copy: same bits as device A
    assert torch.equal(Ys1, Ys2)                        # synthetic A: same alone and mixed
    # a sketch of an N(0,1) matrix: entries ~ N(0, n)
    v = Ys1.double().var().item() / n
    assert 0.9 < v < 1.1, v
    assert i2["stage_us"] > 0 and i3["footprint"] >= m * n * 4


def test_budget_admission_and_rejection():
    m, n, k = 512, 16384, 5
    As = [dev_matrix(m, n, seed=40 + i)[1] for i in range(8)]
    req0 = sv.make_request(A=As[0], k=k, seed=1, Y=torch.empty((m, k), device=DEV))
    fp = sv.sk_request_footprint(req0)
    assert fp == 4 * m * k * 4                   # 4 strips of 4096 columns, FP32 partials
    budget = 2 * fp + fp // 2                    # room for two at a time
    Ys = [torch.empty((m, k), device=DEV) for _ in As]
    torch.cuda.synchronize()
    with sk.SketchServer(budget, max_slots=8, max_batch=8) as srv:
        ts = [srv.submit(sv.make_request(A=A, k=k, seed=1, Y=Y), A, Y) for A, Y in zip(As, Ys)]
        infos = [srv.wait(t, 60.0) for t in ts]
        st = srv.stats()
        big = sv.make_request(source=sv.SK_SRC_SYNTH, m=4096, n=4096, k=5, seed=1,
                              Y=torch.empty((4096, 5), device=DEV))
        with pytest.raises(sk.SketchError) as e:
            srv.submit(big)
        assert e.value.status == -8                 # SK_EBUDGET
    assert all(i["state"] == sv.SK_REQ_DONE for i in infos)
    assert st["peak_bytes_in_use"] <= budget
    assert st["max_running"] <= 2
    assert st["completed"] == 8 and st["rejected"] == 0
    for A, Y in zip(As, Ys):
        assert torch.equal(Y, sk.sketch_gen_matmul(A, 1, k))


def test_overlap_of_late_arrivals():
    """Requests submitted while a long one runs are admitted (and launched on
    another stream) before it finishes."""
    Ybig = torch.empty((32768, 5), device=DEV)
    small = [torch.empty((256, 5), device=DEV) for _ in range(3)]
    torch.cuda.synchronize()
    with sk.SketchServer(5 << 30, max_slots=4, max_batch=4) as srv:
        tb = srv.submit(sv.make_request(source=sv.SK_SRC_SYNTH, m=32768, n=32768, k=5, seed=2,
                                        Y=Ybig), Ybig)
        t_end = time.monotonic() + 30.0
        while srv.poll(tb)["state"] == sv.SK_REQ_QUEUED and time.monotonic() < t_end:
            pass
        ts = [srv.submit(sv.make_request(source=sv.SK_SRC_SYNTH, m=256, n=2048, k=5, seed=3 + i,
                                         Y=Y), Y) for i, Y in enumerate(small)]
        ib = srv.wait(tb, 60.0)
        infos = [srv.wait(t, 60.0) for t in ts]
    assert ib["state"] == sv.SK_REQ_DONE
    assert all(i["state"] == sv.SK_REQ_DONE for i in infos)
    assert all(i["batch"] != ib["batch"] for i in infos)
    assert all(i["t_admit_us"] < ib["t_done_us"] for i in infos), (ib, infos)
    assert min(i["t_done_us"] for i in infos) < ib["t_done_us"]   # they finished first


def test_cancel_queued_request():
    """One slot: while a long request runs, the requests behind it wait in the
    queue, and a cancelled one is never run."""
    Ybig = torch.empty((32768, 5), device=DEV)
    small = [torch.full((256, 5), -7.0, device=DEV) for _ in range(2)]
    torch.cuda.synchronize()
    with sk.SketchServer(5 << 30, max_slots=1, max_batch=1) as srv:
        tb = srv.submit(sv.make_request(source=sv.SK_SRC_SYNTH, m=32768, n=32768, k=5, seed=2,
                                        Y=Ybig), Ybig)
        t_end = time.monotonic() + 30.0
        while srv.poll(tb)["state"] == sv.SK_REQ_QUEUED and time.monotonic() < t_end:
            pass                                    # the worker admits it (about 1.5 ms of work)
        ts = [srv.submit(sv.make_request(source=sv.SK_SRC_SYNTH, m=256, n=2048, k=5, seed=3 + i,
                                         Y=Y), Y) for i, Y in enumerate(small)]
        cancelled = srv.cancel(ts[1])
        assert not srv.cancel(tb)                   # running: cannot be cancelled
        ib = srv.wait(tb, 60.0)
        i0, i1 = srv.wait(ts[0], 60.0), srv.wait(ts[1], 60.0)
        st = srv.stats()
    assert cancelled and i1["state"] == sv.SK_REQ_CANCELLED
    assert (small[1] == -7.0).all()                 # never touched
    assert ib["state"] == i0["state"] == sv.SK_REQ_DONE
    assert i0["t_admit_us"] >= ib["t_done_us"] - 1.0   # one slot: strictly after
    assert st["cancelled"] == 1 and st["completed"] == 2 and st["max_running"] == 1


def test_low_precision_requests_bitwise():
    """BF16 and FP8 requests (matrix-core and VALU classes) served in one mix equal
    direct calls bitwise."""
    cases = [("bf16", 700, 9000, 64), ("bf16", 300, 5000, 5), ("fp8", 600, 9000, 5),
             ("fp8", 257, 4100, 64), ("bf16", 129, 3000, 20)]
    reqs = []
    for i, (kind, m, n, k) in enumerate(cases):
        Aq, sc = sk.sketch_quantize(dev_matrix(m, n, seed=60 + i)[1], kind)
        reqs.append((Aq, sc, k, sk.sketch_gen_matmul(Aq, 70 + i, k, a_scales=sc)))
    Ys = [torch.empty((A.shape[0], k), device=DEV) for A, _, k, _ in reqs]
    torch.cuda.synchronize()
    with sk.SketchServer(1 << 30, max_slots=8, max_batch=8) as srv:
        ts = [srv.submit(sv.make_request(A=A, k=k, seed=70 + i, Y=Y, a_scales=sc), A, sc, Y)
              for i, ((A, sc, k, _), Y) in enumerate(zip(reqs, Ys))]
        infos = [srv.wait(t, 60.0) for t in ts]
    assert all(x["state"] == sv.SK_REQ_DONE for x in infos)
    for (A, sc, k, Yd), Y in zip(reqs, Ys):
        assert torch.equal(Y, Yd), (A.dtype, A.shape, k)


def test_request_validation():
    Y = torch.empty((10, 5), device=DEV)
    A = torch.empty((10, 64), device=DEV)
    with sk.SketchServer(1 << 20, max_slots=2, max_batch=2) as srv:
        for bad in (dict(k=0), dict(k=1025)):
            with pytest.raises(sk.SketchError):
                srv.submit(sv.make_request(A=A, seed=1, Y=Y, **bad))
        r = sv.make_request(A=A, k=5, seed=1, Y=Y)
        r.a_source = 7
        with pytest.raises(sk.SketchError):
            srv.submit(r)
        with pytest.raises(sk.SketchError):
            srv.poll(12345)


def test_packed_omega_route_equals_in_tile_generation():
    """Direct calls with k > 32 (FP32) or k > 16 (BF16/FP8) first pack the call's Omega
    and copy it into the tiles; the server's batched kernels generate each chunk inside
    the tile.  Whole-chunk widths (the unconditional-load kernels) and ragged rows: both
    routes give the same bits."""
    f32 = [(520, 4096, 40), (1030, 8192, 64), (600, 6144, 128), (300, 4096, 300)]
    lp = [("bf16", 700, 8192, 64), ("fp8", 513, 8192, 64), ("bf16", 129, 4096, 20),
          ("fp8", 1024, 4096, 100)]
    reqs = []
    for i, (m, n, k) in enumerate(f32):
        A = dev_matrix(m, n, seed=80 + i)[1]
        reqs.append((A, None, k, sk.sketch_gen_matmul(A, 90 + i, k)))
    for i, (kind, m, n, k) in enumerate(lp):
        Aq, sc = sk.sketch_quantize(dev_matrix(m, n, seed=85 + i)[1], kind)
        reqs.append((Aq, sc, k, sk.sketch_gen_matmul(Aq, 95 + i, k, a_scales=sc)))
    seeds = [90 + i for i in range(len(f32))] + [95 + i for i in range(len(lp))]
    Ys = [torch.full((A.shape[0], k), float("nan"), device=DEV) for A, _, k, _ in reqs]
    torch.cuda.synchronize()
    with sk.SketchServer(1 << 30, max_slots=8, max_batch=8) as srv:
        ts = [srv.submit(sv.make_request(A=A, k=k, seed=s, Y=Y, a_scales=sc), A, sc, Y)
              for (A, sc, k, _), Y, s in zip(reqs, Ys, seeds)]
        infos = [srv.wait(t, 60.0) for t in ts]
    assert all(x["state"] == sv.SK_REQ_DONE and x["status"] == 0 for x in infos), infos
    for (A, sc, k, Yd), Y in zip(reqs, Ys):
        assert torch.equal(Y, Yd), (A.dtype, A.shape, k)
