"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before enqueuing work.

Only invalid argument combinations are passed here (with placeholder
addresses that are never dereferenced): every such call returns before any
HIP call is made.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("sketch.h", "sketch_serve.h")]

import paper_2603_20966_amd as sk  # noqa: E402

F32, BF16, FP8 = 0, 1, 2
YF32, YF64 = 0, 1
OK, EINVAL, EDTYPE, EALIGN, EWS, EHIP, ENOMEM, EUNSUP = 0, -1, -2, -3, -4, -5, -6, -7
PA = 0x10000      # 16-byte aligned placeholder addresses (never dereferenced)
PB = 0x20000
PW = 0x30000


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:sketch|sk)_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_symbols_exported():
    L = sk.lib()
    names = declared_functions()
    assert len(names) >= 18
    assert {"sketch_gen_matmul", "sketch_gen_matmul_reduce", "sk_server_create",
            "sk_server_submit", "sk_server_poll", "sk_server_cancel",
            "sk_server_destroy"} <= set(names)
    for name in names:
        assert hasattr(L, name), name
    # and nothing exported under the ABI prefix that the header does not declare
    out = os.popen(f"nm -D --defined-only {sk.LIB_PATH}").read()
    exported = set(re.findall(r" T ((?:sketch|sk)_[a-z_0-9]+)$", out, flags=re.M))
    assert exported == set(names)


def test_version_and_status_strings():
    assert sk.sketch_abi_version() == 7
    for st in range(-11, 1):
        assert sk.sketch_status_string(st) != "unknown status"
    assert sk.sketch_status_string(-100) == "unknown status"


def gm(A=PA, adt=F32, m=64, n=1024, lda=1024, scales=None, seed=1, row0=0, col0=0, k=5, Y=PB,
       ydt=YF32, ldy=5, beta=0, ws=PW, wsb=1 << 30, stream=None):
    return sk.lib().sketch_gen_matmul(A, adt, m, n, lda, scales, seed, row0, col0, k, Y, ydt, ldy,
                                      beta, ws, wsb, stream)


@pytest.mark.parametrize("kw,expect", [
    (dict(adt=3), EDTYPE), (dict(adt=-1), EDTYPE), (dict(ydt=2), EDTYPE),
    (dict(m=-1), EINVAL), (dict(n=-1), EINVAL), (dict(k=-1), EINVAL), (dict(k=1025), EINVAL),
    (dict(beta=2), EINVAL), (dict(Y=None), EINVAL), (dict(ldy=4), EINVAL),
    (dict(A=None), EINVAL), (dict(lda=1000), EINVAL), (dict(row0=-1), EINVAL),
    (dict(row0=(1 << 62) - 100), EINVAL), (dict(col0=-1), EINVAL),
    (dict(col0=(1 << 32) - 4), EINVAL),
    (dict(A=PA + 4), EALIGN), (dict(lda=1025, n=1025), EALIGN), (dict(Y=PB + 2), EALIGN),
    (dict(ydt=YF64, Y=PB + 4, ldy=5), EALIGN),
    (dict(adt=FP8, lda=1024), EINVAL),                  # fp8 needs scales
    (dict(adt=BF16, lda=1028, n=1028), EALIGN),          # 1028*2 % 16 != 0
    (dict(ws=None), EWS), (dict(wsb=16), EWS), (dict(ws=PW + 8), EALIGN),
    (dict(m=70_000_000), EUNSUP),
    (dict(m=40_000_000, k=64, ldy=64), EUNSUP),           # matrix-core grid limit (65535 x 512 rows)
])
def test_gen_matmul_rejects(kw, expect):
    args = dict(n=8192, lda=8192)      # two 4096-column strips: a workspace is needed
    args.update(kw)
    assert gm(**args) == expect


NOALLOC_BYTES = 32 << 20    # SKETCH_NOALLOC_SCRATCH_BYTES


def gm_noalloc(A=PA, adt=F32, m=64, n=4096, lda=4096, scales=None, seed=1, row0=0, col0=0, k=5,
               Y=PB, ydt=YF32, ldy=5, beta=0, stream=None):
    return sk.lib().sketch_gen_matmul_noalloc(A, adt, m, n, lda, scales, seed, row0, col0, k, Y,
                                              ydt, ldy, beta, stream)


def test_noalloc_scratch_size_matches_header():
    text = open(HEADERS[0]).read()
    assert "#define SKETCH_NOALLOC_SCRATCH_BYTES (32u << 20)" in text


@pytest.mark.parametrize("kw,expect", [
    (dict(adt=3), EDTYPE), (dict(ydt=2), EDTYPE), (dict(m=-1), EINVAL), (dict(k=1025), EINVAL),
    (dict(beta=2), EINVAL), (dict(Y=None), EINVAL), (dict(ldy=4), EINVAL), (dict(A=None), EINVAL),
    (dict(lda=1000), EINVAL), (dict(row0=-1), EINVAL), (dict(A=PA + 4), EALIGN),
    (dict(adt=FP8), EINVAL), (dict(m=70_000_000), EUNSUP),
])
def test_noalloc_rejects(kw, expect):
    assert gm_noalloc(**kw) == expect


def test_noalloc_rejects_calls_beyond_its_scratch():
    # the largest m whose workspace fits, and one row more (checked on the host)
    ws = sk.sketch_workspace_size
    per_row = ws(0, F32, 2, 32768, 5, 1) - ws(0, F32, 1, 32768, 5, 1)
    base = ws(0, F32, 1, 32768, 5, 1) - per_row
    m_max = (NOALLOC_BYTES - base) // per_row
    assert ws(0, F32, m_max, 32768, 5, 1) <= NOALLOC_BYTES < ws(0, F32, m_max + 1, 32768, 5, 1)
    assert gm_noalloc(m=m_max + 1, n=32768, lda=32768) == -11
    assert gm_noalloc(m=1 << 20, n=1 << 15, lda=1 << 15, k=64, ldy=64) == -11
    assert sk.sketch_status_string(-11) != "unknown status"
    # m == 0 / k == 0 are no-ops that never touch the device
    assert gm_noalloc(m=0, Y=None, A=None) == OK
    assert gm_noalloc(k=0, Y=None, ldy=0) == OK


def test_noop_shapes_return_ok_without_launch():
    # m == 0 or k == 0 is a no-op: nothing is enqueued, pointers are not used
    assert gm(m=0, Y=None, A=None) == OK
    assert gm(k=0, Y=None, ldy=0) == OK


def test_reduce_rejects():
    L = sk.lib()
    P = 2
    A = (ctypes.c_void_p * P)(PA, PA + 4096 * 4)
    nb = (ctypes.c_int64 * P)(4096, 4096)
    ld = (ctypes.c_int64 * P)(8192, 8192)
    r0 = (ctypes.c_int64 * P)(0, 4096)

    def call(P=P, A=A, adt=F32, m=64, nb=nb, ld=ld, r0=r0, sc=None, k=5, Y=PB, ldy=5, ws=PW,
             wsb=1 << 30):
        return L.sketch_gen_matmul_reduce(A, P, adt, m, nb, ld, r0, sc, 1, 0, k, Y, YF32, ldy, 0,
                                          ws, wsb, None)

    assert call(P=0) == EINVAL
    assert call(P=65) == EINVAL
    assert call(A=None) == EINVAL
    assert call(nb=None) == EINVAL
    bad_ld = (ctypes.c_int64 * P)(8192, 4000)
    assert call(ld=bad_ld) == EINVAL
    bad_al = (ctypes.c_void_p * P)(PA, PA + 4)
    assert call(A=bad_al) == EALIGN
    assert call(ws=None) == EWS
    assert call(adt=FP8) == EINVAL       # fp8 without scales
    bad_r0 = (ctypes.c_int64 * P)(0, -5)
    assert call(r0=bad_r0) == EINVAL


def test_other_entry_points_reject():
    L = sk.lib()
    assert L.sketch_gen_omega(1, 0, 10, 0, 5, None, 5, None) == EINVAL
    assert L.sketch_gen_omega(1, 0, 10, 0, 5, PA, 4, None) == EINVAL
    assert L.sketch_gen_omega(1, -1, 10, 0, 5, PA, 5, None) == EINVAL
    assert L.sketch_gen_omega(1, 0, 10, 0, 5, PA + 2, 5, None) == EALIGN
    assert L.sketch_gen_omega(1, 0, 0, 0, 5, None, 5, None) == OK
    assert L.sketch_philox_raw(PA, 1, PB, -1, None) == EINVAL
    assert L.sketch_philox_raw(PA + 4, 1, PB, 8, None) == EALIGN
    assert L.sketch_philox_raw(None, 1, PB, 8, None) == EINVAL
    assert L.sketch_philox_raw(PA, 1, PB, 0, None) == OK
    assert L.sketch_quantize(PA, 10, 10, 10, 0, PB, 16, PW, None) == EDTYPE
    assert L.sketch_quantize(PA, 10, 10, 10, FP8, PB, 16, None, None) == EINVAL
    assert L.sketch_quantize(PA, 10, 10, 10, BF16, PB, 12, None, None) == EALIGN
    assert L.sketch_quantize(PA, 10, 10, 9, BF16, PB, 16, None, None) == EINVAL
    assert L.sketch_matmul_omega(PA, F32, 64, 1024, 1024, None, None, 5, 5, PB, YF32, 5, 0, PW,
                                 1 << 30, None) == EINVAL
    assert L.sketch_matmul_omega(PA, F32, 64, 1024, 1024, None, PW, 4, 5, PB, YF32, 5, 0, PW,
                                 1 << 30, None) == EINVAL


def test_distribution_argument_rejected_on_host():
    L = sk.lib()
    for d in (-1, 3):
        assert L.sketch_gen_matmul_dist(PA, F32, 64, 1024, 1024, None, 1, d, 0, 0, 5, PB, YF32, 5,
                                        0, PW, 1 << 30, None) == EINVAL
        assert L.sketch_gen_omega_dist(1, d, 0, 10, 0, 5, PA, 5, None) == EINVAL
        A = (ctypes.c_void_p * 1)(PA)
        nb = (ctypes.c_int64 * 1)(1024)
        r0 = (ctypes.c_int64 * 1)(0)
        assert L.sketch_gen_matmul_reduce_dist(A, 1, F32, 64, nb, nb, r0, None, 1, d, 0, 5, PB,
                                               YF32, 5, 0, PW, 1 << 30, None) == EINVAL
    # valid distributions reach the ordinary argument checks
    for d in (0, 1, 2):
        assert L.sketch_gen_matmul_dist(PA, F32, 64, 1024, 1000, None, 1, d, 0, 0, 5, PB, YF32, 5,
                                        0, PW, 1 << 30, None) == EINVAL      # lda < n
        assert L.sketch_gen_omega_dist(1, d, 0, 0, 0, 5, None, 5, None) == OK


def test_column_major_and_second_product_reject_on_host():
    L = sk.lib()

    def cm(A=PA, m=300, n=5000, lda=300, dist=0, k=5, Y=PB, ydt=YF32, ldy=5, yt=0, beta=0, ws=PW,
           wsb=1 << 30):
        return L.sketch_gen_matmul_cm(A, m, n, lda, 1, dist, 0, 0, k, Y, ydt, ldy, yt, beta, ws,
                                      wsb, None)

    assert cm(lda=299) == EINVAL                 # lda < m
    assert cm(lda=302) == EALIGN                 # lda * 4 not a multiple of 16
    assert cm(A=PA + 4) == EALIGN
    assert cm(dist=5) == EINVAL and cm(yt=2) == EINVAL and cm(beta=3) == EINVAL
    assert cm(k=1025, ldy=1100) == EINVAL
    assert cm(ldy=4) == EINVAL                   # row-major Y needs ldy >= k
    assert cm(yt=1, ldy=299) == EINVAL           # transposed Y needs ldy >= m
    assert cm(ydt=3) == EDTYPE
    assert cm(ws=None) == EWS
    assert cm(m=0, A=None, Y=None) == OK and cm(k=0, Y=None) == OK
    assert L.sketch_gen_tmatmul(PA, 5000, 6, 6, 1, 0, 0, 0, 5, PB, YF32, 5, 0, PW, 1 << 30,
                                None) == EINVAL                  # ldc < p
    assert L.sketch_gen_tmatmul(PA, 5000, 6, 6, 1, 0, 0, 0, 5, PB, YF32, 6, 0, PW, 1 << 30,
                                None) == EALIGN                  # ldb * 4 % 16 != 0
    ws = sk.sketch_workspace_size
    assert ws(2, F32, 300, 5000, 5, 1) == 5 * 300 * 5 * 4        # 5 strips of 1024 columns
    assert ws(2, F32, 300, 1024, 5, 1) == 0 and ws(2, BF16, 300, 5000, 5, 1) == 0
    assert ws(2, F32, 300, 5000, 16, 1) == 5 * 300 * 16 * 4      # 1024-column strips at every k <= 16


def test_workspace_size_rules():
    ws = sk.sketch_workspace_size
    assert ws(0, F32, 4096, 4096, 5, 1) == 0          # one strip: Y written directly, no partials
    a = ws(0, F32, 4096, 32768, 5, 1)
    assert a == 8 * 4096 * 5 * 4                        # 8 strips of 4096 columns
    b = ws(1, F32, 32768, 32768, 5, 8)
    assert b >= (8 + 8) * 32768 * 5 * 4                 # bound valid for any 8-way split
    assert ws(2, F32, 1, 1, 1, 1) == 0 and ws(0, 5, 1, 1, 1, 1) == 0 and ws(1, F32, 1, 1, 1, 0) == 0
    assert ws(0, F32, 100, 5000, 1025, 1) == 0          # k > 1024 is invalid
    # 2048-column strips; k > 32 on the FP32 matrix cores adds the call's packed
    # Omega (S * 2048 * kpad floats) after the 256-byte aligned partials
    assert ws(0, F32, 100, 5000, 1024, 1) == 3 * 100 * 1024 * 4 + 3 * 2048 * 1024 * 4
    # FP32 on the VALU path (k <= 8): 4096-column strips at every k; the matrix-core
    # path (FP32, k > 8) uses 2048-column strips
    assert ws(0, F32, 4096, 32768, 8, 1) == 8 * 4096 * 8 * 4
    assert ws(0, F32, 4096, 32768, 9, 1) == 16 * 4096 * 9 * 4
    assert ws(0, F32, 4096, 32768, 17, 1) == 16 * 4096 * 17 * 4
    assert ws(0, F32, 4096, 32768, 32, 1) == 16 * 4096 * 32 * 4        # two N-tiles: no packing
    assert ws(0, F32, 4096, 32768, 33, 1) == 16 * 4096 * 33 * 4 + 16 * 2048 * 64 * 4
    assert ws(0, F32, 100, 2048, 64, 1) == 2048 * 64 * 4                # one strip: packing only
    assert ws(0, F32, 7, 32768, 65, 1) == -(-16 * 7 * 65 * 4 // 256) * 256 + 16 * 2048 * 128 * 4
    assert sk.sketch_strip_width(F32, 5) == 4096 and sk.sketch_strip_width(F32, 8) == 4096
    assert sk.sketch_strip_width(F32, 9) == 2048 and sk.sketch_strip_width(F32, 17) == 2048
    # FP8 at every k and BF16 past 8 columns: BF16 matrix cores, 4096-column strips
    assert sk.sketch_strip_width(BF16, 5) == 4096 and sk.sketch_strip_width(FP8, 4) == 4096
    assert sk.sketch_strip_width(BF16, 9) == 4096 and sk.sketch_strip_width(FP8, 256) == 4096
    # column-major A (op 2): 1024-column strips on the VALU path (k <= 16), the
    # matrix-core strips of 2048 columns past 16, as the row-major matrix-core call
    assert ws(2, F32, 300, 5000, 5, 1) == 5 * 300 * 5 * 4
    assert ws(2, F32, 300, 5000, 16, 1) == 5 * 300 * 16 * 4
    assert ws(2, F32, 300, 5000, 17, 1) == 3 * 300 * 17 * 4
    # few rows (m <= 64) past k = 16: the few-row kernel copies the call's packed
    # Omega (one 2048 strip: no partials, Y written directly)
    assert ws(2, F32, 64, 2048, 64, 1) == 2048 * 64 * 4
    assert ws(2, F32, 5, 4096, 17, 1) == 768 + 2 * 2048 * 32 * 4     # 680 B of partials, aligned
    assert ws(2, F32, 64, 32768, 256, 1) == 16 * 64 * 256 * 4 + 16 * 2048 * 256 * 4
    # more than 64 rows and k > 32: the tile kernel's packed Omega after the partials
    assert ws(2, F32, 300, 32768, 64, 1) == 16 * 300 * 64 * 4 + 16 * 2048 * 64 * 4
    assert ws(2, F32, 65, 2048, 33, 1) == 2048 * 64 * 4


def test_python_binding_requires_library(monkeypatch, tmp_path):
    import importlib

    mod = importlib.import_module("paper_2603_20966_amd")
    monkeypatch.setattr(mod, "_lib", None)
    monkeypatch.setattr(mod, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        mod.lib()


def test_request_footprint_rule():
    """Serving admission charges FP32 strip partials (S > 1 strips) plus any staged A,
    each rounded up to 256 bytes; invalid requests have footprint 0.  Host-only."""
    from paper_2603_20966_amd import serve as sv

    def req(**kw):
        r = sv.SkRequest()
        r.a_source, r.a_dtype, r.A, r.m, r.n, r.lda = sv.SK_SRC_DEVICE, F32, PA, 512, 4096, 4096
        r.seed, r.k, r.Y, r.y_dtype, r.ldy = 1, 5, PB, YF32, 5
        for key, v in kw.items():
            setattr(r, key, v)
        return r

    fp = sv.sk_request_footprint
    assert fp(req(n=16384, lda=16384)) == 4 * 512 * 5 * 4     # 4 strips of 4096 columns
    assert fp(req()) == 0                                     # one strip: no partials
    assert fp(req(n=1000, lda=1000, m=3, k=1, ldy=1)) == 0
    assert fp(req(k=64, ldy=64)) == 2 * 512 * 64 * 4          # matrix core: 2048-column strips
    assert fp(req(a_source=sv.SK_SRC_SYNTH, A=None, n=16384, lda=16384)) == (
        512 * 16384 * 4 + 4 * 512 * 5 * 4)
    # staged rows padded to 16 bytes, each part rounded to 256 bytes
    assert fp(req(a_source=sv.SK_SRC_HOST, n=1001, lda=1001, m=3, k=1, ldy=1)) == 12288 + 0
    assert fp(req(a_source=sv.SK_SRC_HOST, n=1001, lda=1001, m=1, k=1, ldy=1)) == 4096
    for bad in (dict(k=0), dict(m=0), dict(n=0), dict(a_source=3), dict(ldy=4), dict(Y=None),
                dict(omega_dist=3), dict(omega_dist=-1),
                dict(a_source=sv.SK_SRC_SYNTH), dict(a_source=sv.SK_SRC_SYNTH, A=None, a_dtype=BF16),
                dict(a_source=sv.SK_SRC_HOST, lda=100), dict(A=PA + 4), dict(a_dtype=FP8)):
        assert fp(req(**bad)) == 0, bad


def test_server_entry_points_reject_without_a_server():
    L = sk.lib()
    from paper_2603_20966_amd import serve as sv

    sv._bind()
    t = ctypes.c_int64(5)
    r = sv.SkRequest()
    assert L.sk_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == EINVAL and t.value == 5
    info = sv.SkTicketInfo()
    assert L.sk_server_poll(None, 1, ctypes.byref(info)) == EINVAL
    assert L.sk_server_wait(None, 1, 0.0, ctypes.byref(info)) == EINVAL
    assert L.sk_server_cancel(None, 1) == EINVAL
    assert L.sk_server_destroy(None) == EINVAL
    h = ctypes.c_void_p()
    for bad in ((1 << 20, 0, 4, 2), (1 << 20, 4, 0, 2), (1 << 20, 4, 17, 2), (1 << 20, 4, 4, 0),
                (1 << 20, 4, 4, 9)):
        assert L.sk_server_create(*bad, ctypes.byref(h)) == EINVAL and not h.value
    assert L.sk_server_create(1 << 20, 4, 4, 2, None) == EINVAL


def test_nystrom_entry_points_reject_on_host():
    """Argument checks of the Nystrom core pseudo-inverse and reconstruction (Sec. 5, Alg. 2),
    all found before anything is enqueued (no GPU needed)."""
    L = sk.lib()
    need = L.sketch_core_pinv_workspace(256)
    assert need > 2 * 256 * 256 * 8 and L.sketch_core_pinv_workspace(1025) == 0
    assert L.sketch_core_pinv_workspace(0) == 0

    def pinv(C=PA, cdt=YF32, r=256, ldc=256, tol=1e-12, sw=16, Cp=PB, ldcp=256, eig=None,
             info=None, ws=PW, wsb=1 << 30):
        return L.sketch_core_pinv(C, cdt, r, ldc, tol, sw, Cp, ldcp, eig, info, ws, wsb, None)

    assert pinv(cdt=2) == EDTYPE
    assert pinv(r=1025) == EINVAL and pinv(r=-1) == EINVAL
    assert pinv(tol=-1.0) == EINVAL and pinv(tol=float("nan")) == EINVAL and pinv(tol=2.0) == EINVAL
    assert pinv(sw=0) == EINVAL and pinv(sw=101) == EINVAL
    assert pinv(C=None) == EINVAL and pinv(Cp=None) == EINVAL
    assert pinv(ldc=255) == EINVAL and pinv(ldcp=255) == EINVAL
    assert pinv(C=PA + 2) == EALIGN and pinv(cdt=YF64, C=PA + 4) == EALIGN
    assert pinv(Cp=PB + 4) == EALIGN and pinv(eig=PB + 4) == EALIGN and pinv(info=PB + 2) == EALIGN
    assert pinv(ws=None) == EWS and pinv(wsb=need - 1) == EWS
    assert pinv(r=0, C=None, Cp=None, ws=None) == OK
    nneed = L.sketch_nystrom_workspace(2000, 64)
    assert nneed >= 2000 * 64 * 8

    def err(A=PA, n=2000, lda=2000, B=PB, r=64, ldb=64, Cp=PW, ldcp=64, sums=PB, ws=PW,
            wsb=1 << 30):
        return L.sketch_nystrom_error(A, n, lda, B, r, ldb, Cp, ldcp, sums, ws, wsb, None)

    assert err(r=0) == EINVAL and err(r=1025) == EINVAL and err(n=-1) == EINVAL
    assert err(A=None) == EINVAL and err(sums=None) == EINVAL and err(B=None) == EINVAL
    assert err(lda=1999) == EINVAL and err(ldb=63) == EINVAL and err(ldcp=63) == EINVAL
    assert err(A=PA + 2) == EALIGN and err(sums=PB + 4) == EALIGN and err(Cp=PW + 4) == EALIGN
    assert err(ws=None) == EWS and err(wsb=nneed - 1) == EWS
    assert err(n=64 * 65536, lda=64 * 65536) == EUNSUP
    assert err(n=0, A=None, B=None, sums=None, ws=None) == OK

    def rows(B=PB, n=2000, r=64, ldb=64, Cp=PW, ldcp=64, row0=0, mr=10, out=PA, ldo=2000, ws=PW,
             wsb=1 << 30):
        return L.sketch_nystrom_rows(B, n, r, ldb, Cp, ldcp, row0, mr, out, ldo, ws, wsb, None)

    assert rows(row0=-1) == EINVAL and rows(row0=1995) == EINVAL and rows(mr=-1) == EINVAL
    assert rows(out=None) == EINVAL and rows(ldo=1999) == EINVAL and rows(out=PA + 4) == EALIGN
    assert rows(mr=0, out=None) == OK


def test_low_precision_workspace_holds_packed_omega():
    # BF16 / FP8 A with k > 16: the strip partials, then (256-byte aligned) the
    # call's Omega as hi and lo BF16 planes of S * 4096 * kpad values each
    ws = sk.sketch_workspace_size

    def packed(m, n, k, P=1, op=0):
        S = (n + 4095) // 4096 if op == 0 else n // 4096 + P
        part = S * m * k * 4 if S > 1 else 0
        kpad = -(-k // (32 if k <= 32 else 64)) * (32 if k <= 32 else 64)
        return -(-part // 256) * 256 + 2 * S * 4096 * kpad * 2

    for adt in (BF16, FP8):
        for (m, n, k) in ((32768, 32768, 64), (100, 4096, 17), (300, 5000, 33), (7, 12288, 1000)):
            assert ws(0, adt, m, n, k, 1) == packed(m, n, k)
        assert ws(1, adt, 32768, 32768, 64, 8) == packed(32768, 32768, 64, 8, op=1)
    # one N-tile (k <= 16) forms its Omega inside the tiles: partials only
    assert ws(0, FP8, 32768, 32768, 5, 1) == 8 * 32768 * 5 * 4
    assert ws(0, FP8, 100, 4096, 16, 1) == 0
    assert ws(0, BF16, 100, 4096, 16, 1) == 0
