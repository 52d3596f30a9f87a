"""Python binding of the photon server (include/pp_server.h): argument
marshalling only. Queueing, admission, batching and launches run in the
library's scheduler thread; submit and wait release the GIL, so Python
client threads submit concurrently."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import pp
from . import workloads as W

_vp, _u64, _u32 = C.c_void_p, C.c_uint64, C.c_uint32


class ServerConfig(C.Structure):
    _fields_ = [("max_inflight", _u32), ("max_batch_events", _u32), ("hbm_budget_bytes", _u64),
                ("max_batch_photons", _u64)]


class RequestInfo(C.Structure):
    _fields_ = [("t_submit_s", C.c_double), ("t_launch_s", C.c_double), ("t_done_s", C.c_double),
                ("photons", _u64), ("n_hits", _u64), ("batch_events", _u32), ("reserved", _u32)]


class ServerStats(C.Structure):
    _fields_ = [(n, _u64) for n in ("submitted", "completed", "launches", "deferred", "bytes_in_use",
                                    "peak_bytes_in_use", "photons_completed", "arena_bytes",
                                    "overflow_bytes_peak", "shared_requests", "overlapped_launches")] + \
               [("gpu_busy_s", C.c_double), ("gpu_span_s", C.c_double)]


_dp = C.POINTER(C.c_double)
SIGNATURES = {
    "pp_server_request_bytes": (_u64, [_u32, _u64]),
    "pp_server_create": (C.c_int, [_vp, C.POINTER(ServerConfig), _vp, C.POINTER(_vp)]),
    "pp_server_destroy": (None, [_vp]),
    "pp_server_submit": (C.c_int, [_vp, _vp, _u32, C.POINTER(_u64)]),
    "pp_server_wait": (C.c_int, [_vp, _u64, _vp, _u64, _vp, C.POINTER(RequestInfo)]),
    "pp_server_get_stats": (C.c_int, [_vp, C.POINTER(ServerStats)]),
    "pp_server_last_error": (C.c_char_p, [_vp]),
    "pp_server_run_clients": (C.c_int, [_vp, _vp, _u64, _u32, C.c_double, _u32, C.c_double, _u64, _vp, _u64,
                                        C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64), _dp]),
}
for _name, (_res, _args) in SIGNATURES.items():
    _fn = getattr(pp._lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
_lib = pp._lib


def request_bytes(n_sources: int, n_photons: int) -> int:
    return int(_lib.pp_server_request_bytes(n_sources, n_photons))


class Server:
    """A photon server owning ctx until close()."""

    _close_order = 0

    def __init__(self, ctx: "pp.Context", max_inflight=0, max_batch_events=0, hbm_budget_bytes=0,
                 max_batch_photons=0, surrogate=None):
        cfg = ServerConfig(max_inflight, max_batch_events, hbm_budget_bytes, max_batch_photons)
        h = C.c_void_p()
        st = _lib.pp_server_create(ctx._h, C.byref(cfg), surrogate._h if surrogate else None, C.byref(h))
        ctx._check(st)
        self._h = h
        self.ctx = ctx
        self.surrogate = surrogate  # kept alive while the server may use it
        ctx._add_dependent(self)
        self.n_doms = ctx.n_doms
        self.has_surrogate = surrogate is not None

    def close(self):
        if self._h:
            _lib.pp_server_destroy(self._h)
            self._h = None
            self.ctx._release_dependent()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=(pp.PP_OK,)):
        if st not in allow:
            raise pp.PPError(st, _lib.pp_server_last_error(self._h).decode())
        return st

    def submit(self, sources: np.ndarray) -> int:
        sources = np.ascontiguousarray(sources, dtype=W.SOURCE_DTYPE)
        t = C.c_uint64()
        self._check(_lib.pp_server_submit(self._h, sources.ctypes.data, len(sources), C.byref(t)))
        return t.value

    def wait(self, ticket: int, cap: int = 256, expected: bool = False):
        """Blocks until the request is done; returns (hits, info dict,
        per-module expected hits or None). A request with more than cap hits
        is fetched again with a buffer of its exact size."""
        while True:
            out = np.empty(cap, pp.HIT_DTYPE)
            info = RequestInfo()
            dom = np.empty(self.n_doms, np.float32) if expected and self.has_surrogate else None
            st = _lib.pp_server_wait(self._h, ticket, out.ctypes.data, cap,
                                     dom.ctypes.data if dom is not None else None, C.byref(info))
            if st == pp.PP_ETRUNC:
                cap = int(info.n_hits)
                continue
            self._check(st)
            d = {k: getattr(info, k) for k, _ in RequestInfo._fields_ if k != "reserved"}
            return out[: info.n_hits], d, dom

    def run_clients(self, events: np.ndarray, n_clients: int, rate_per_s: float = 0.0, outstanding: int = 32,
                    duration_s: float = 5.0, seed: int = 0) -> dict:
        """pp_server_run_clients: native client threads submit events (one
        source each) open loop at rate_per_s, or closed loop with
        `outstanding` requests each; returns latencies (s) and totals."""
        events = np.ascontiguousarray(events, dtype=W.SOURCE_DTYPE)
        lat = np.zeros(len(events), np.float64)
        n, ph, hits, wall = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_double()
        self._check(_lib.pp_server_run_clients(self._h, events.ctypes.data, len(events), n_clients, rate_per_s,
                                               outstanding, duration_s, seed, lat.ctypes.data, len(lat),
                                               C.byref(n), C.byref(ph), C.byref(hits), C.byref(wall)))
        return {"latency_s": lat[: min(n.value, len(lat))], "done": n.value, "photons": ph.value,
                "hits": hits.value, "wall_s": wall.value}

    def stats(self) -> dict:
        s = ServerStats()
        self._check(_lib.pp_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}
