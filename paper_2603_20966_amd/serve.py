"""Python binding of the request server in ``include/sketch_serve.h``.

Argument marshalling only: requests are copied into ``sk_request`` structs and
handed to the library's server, whose worker thread batches and launches them.
The binding keeps the tensors a request points to alive until it finishes.
"""
from __future__ import annotations

import ctypes

import torch

from . import SK_A_F32, SketchError, _adtype, _dist, _ld, _ydtype, lib

SK_SRC_DEVICE, SK_SRC_HOST, SK_SRC_SYNTH = 0, 1, 2
SK_REQ_QUEUED, SK_REQ_RUNNING, SK_REQ_DONE, SK_REQ_FAILED, SK_REQ_CANCELLED = range(5)
SK_ETIMEOUT = -10

_i64, _u64, _int, _vp, _sz, _dbl = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double)


class SkRequest(ctypes.Structure):
    _fields_ = [("a_source", _int), ("a_dtype", _int), ("A", _vp), ("m", _i64), ("n", _i64),
                ("lda", _i64), ("a_scales", _vp), ("a_seed", _u64), ("seed", _u64),
                ("omega_row0", _i64), ("omega_col0", _i64), ("k", _i64), ("Y", _vp),
                ("y_dtype", _int), ("ldy", _i64), ("beta", _int), ("omega_dist", _int)]


class SkTicketInfo(ctypes.Structure):
    _fields_ = [("state", _int), ("status", _int), ("batch", _i64), ("batch_size", _int),
                ("footprint", _sz), ("t_submit_us", _dbl), ("t_admit_us", _dbl),
                ("t_done_us", _dbl), ("stage_us", _dbl), ("sketch_us", _dbl)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class SkServeStats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("admitted", _i64), ("completed", _i64), ("failed", _i64),
                ("cancelled", _i64), ("rejected", _i64), ("batches", _i64), ("queued", _i64),
                ("running", _i64), ("max_running", _i64), ("budget_bytes", _sz),
                ("bytes_in_use", _sz), ("peak_bytes_in_use", _sz)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_bound = False


def _bind():
    global _bound
    L = lib()
    if _bound:
        return L
    P = ctypes.POINTER
    L.sk_request_footprint.argtypes = [P(SkRequest)]
    L.sk_request_footprint.restype = _sz
    L.sk_server_create.argtypes = [_sz, _int, _int, _int, P(_vp)]
    L.sk_server_submit.argtypes = [_vp, P(SkRequest), P(_i64)]
    L.sk_server_poll.argtypes = [_vp, _i64, P(SkTicketInfo)]
    L.sk_server_wait.argtypes = [_vp, _i64, _dbl, P(SkTicketInfo)]
    L.sk_server_cancel.argtypes = [_vp, _i64]
    L.sk_server_stats.argtypes = [_vp, P(SkServeStats)]
    L.sk_server_now_us.argtypes = [_vp]
    L.sk_server_now_us.restype = _dbl
    L.sk_server_destroy.argtypes = [_vp]
    for f in ("sk_server_create", "sk_server_submit", "sk_server_poll", "sk_server_wait",
              "sk_server_cancel", "sk_server_stats", "sk_server_destroy"):
        getattr(L, f).restype = _int
    _bound = True
    return L


def make_request(*, k: int, seed: int, Y: torch.Tensor, A: torch.Tensor | None = None,
                 m: int | None = None, n: int | None = None, source: int = SK_SRC_DEVICE,
                 a_seed: int = 0, omega_row0: int = 0, omega_col0: int = 0, beta: int = 0,
                 a_scales: torch.Tensor | None = None, dist="normal") -> SkRequest:
    """An sk_request: A a device tensor (SK_SRC_DEVICE), a host tensor (SK_SRC_HOST), or None
    with (m, n) for SK_SRC_SYNTH (A ~ N(0,1) from a_seed, filled by the server)."""
    r = SkRequest()
    r.a_source = source
    if source == SK_SRC_SYNTH:
        if A is not None or m is None or n is None:
            raise ValueError("a synthetic request takes m and n, not A")
        r.a_dtype, r.A, r.m, r.n, r.lda = SK_A_F32, None, m, n, n
    else:
        if A is None:
            raise ValueError("A is required")
        r.a_dtype = _adtype(A)
        r.A = A.data_ptr()
        r.m, r.n = A.shape
        r.lda = _ld(A, "A")
    r.a_scales = None if a_scales is None else a_scales.data_ptr()
    r.a_seed = a_seed
    r.seed = seed
    r.omega_row0 = omega_row0
    r.omega_col0 = omega_col0
    r.k = k
    r.Y = Y.data_ptr()
    r.y_dtype = _ydtype(Y.dtype)
    r.ldy = _ld(Y, "Y")
    r.beta = beta
    r.omega_dist = _dist(dist)
    return r


def sk_request_footprint(req: SkRequest) -> int:
    """Arena bytes a request holds while admitted (0 if it is invalid)."""
    return int(_bind().sk_request_footprint(ctypes.byref(req)))


class SketchServer:
    """Continuous-batching server of sketch requests on the current device."""

    def __init__(self, budget_bytes: int, max_slots: int = 32, max_batch: int = 16,
                 n_streams: int = 4):
        L = _bind()
        h = _vp()
        st = L.sk_server_create(budget_bytes, max_slots, max_batch, n_streams, ctypes.byref(h))
        if st != 0:
            raise SketchError(st, "sk_server_create")
        self._h = h
        self._L = L
        self._keep: dict[int, tuple] = {}

    def submit(self, req: SkRequest, *keep) -> int:
        """Queue a request; `keep` holds the tensors it points to until it finishes."""
        t = _i64()
        st = self._L.sk_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st != 0:
            raise SketchError(st, "sk_server_submit")
        self._keep[t.value] = keep
        return t.value

    def _info(self, ticket: int, info: SkTicketInfo) -> dict:
        d = info.as_dict()
        if d["state"] >= SK_REQ_DONE:
            self._keep.pop(ticket, None)
        return d

    def poll(self, ticket: int) -> dict:
        info = SkTicketInfo()
        st = self._L.sk_server_poll(self._h, ticket, ctypes.byref(info))
        if st != 0:
            raise SketchError(st, "sk_server_poll")
        return self._info(ticket, info)

    def wait(self, ticket: int, timeout_s: float = -1.0) -> dict:
        info = SkTicketInfo()
        st = self._L.sk_server_wait(self._h, ticket, timeout_s, ctypes.byref(info))
        if st != 0:
            raise SketchError(st, "sk_server_wait")
        return self._info(ticket, info)

    def cancel(self, ticket: int) -> bool:
        ok = self._L.sk_server_cancel(self._h, ticket) == 0
        if ok:
            self._keep.pop(ticket, None)
        return ok

    def stats(self) -> dict:
        s = SkServeStats()
        st = self._L.sk_server_stats(self._h, ctypes.byref(s))
        if st != 0:
            raise SketchError(st, "sk_server_stats")
        return s.as_dict()

    def now_us(self) -> float:
        return float(self._L.sk_server_now_us(self._h))

    def close(self) -> None:
        if self._h is not None:
            st = self._L.sk_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            if st != 0:
                raise SketchError(st, "sk_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["SketchServer", "SkRequest", "make_request", "sk_request_footprint",
           "SK_SRC_DEVICE", "SK_SRC_HOST", "SK_SRC_SYNTH", "SK_REQ_QUEUED", "SK_REQ_RUNNING",
           "SK_REQ_DONE", "SK_REQ_FAILED", "SK_REQ_CANCELLED", "SK_ETIMEOUT"]
