"""ctypes wrapper around the FP64 CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark. The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

FATE_ABSORBED, FATE_HIT, FATE_CAPPED, FATE_ESCAPED = 0, 1, 2, 3
NO_DOM = 0xFFFFFFFF
COUNTER_NAMES = ("photons", "iterations", "crossings", "dom_tests", "hits", "absorbed",
                 "capped", "escaped")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-pthread",
                               "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


class _Inputs(C.Structure):
    _fields_ = [
        ("z_lo", C.c_double), ("dz", C.c_double), ("n_layers", C.c_int32),
        ("n_group", C.c_double),
        ("abs_len", C.c_void_p), ("eff_scat_len", C.c_void_p), ("g", C.c_void_p),
        ("n_dom", C.c_uint32), ("dom_xyz", C.c_void_p), ("dom_string", C.c_void_p),
        ("dom_radius", C.c_double),
        ("n_src", C.c_uint32), ("src_type", C.c_void_p), ("src_event", C.c_void_p),
        ("src_particle", C.c_void_p), ("src_f", C.c_void_p), ("src_n", C.c_void_p),
        ("src_first", C.c_void_p),
        ("lambda_ref", C.c_double), ("kappa_abs", C.c_double), ("kappa_scat", C.c_double),
        ("n_acc", C.c_uint32), ("n_poly", C.c_uint32), ("acc_l0", C.c_double), ("acc_dl", C.c_double),
        ("acc", C.c_void_p), ("poly", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("PP_ORACLE_LIB")  # a mutated build, for mutation checks
        if not path:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            path = LIB
        L = C.CDLL(path)
        vp, u64 = C.c_void_p, C.c_uint64
        L.orc_philox.argtypes = [u64, vp, vp, vp]
        L.orc_uniform.argtypes = [u64, vp, vp]
        L.orc_hg_one_minus_mu.argtypes = [u64, C.c_double, vp, vp]
        L.orc_rotate.argtypes = [u64, vp, vp, vp, vp]
        L.orc_basis.argtypes = [u64, vp, vp, vp]
        L.orc_first_hit.argtypes = [u64, vp, vp, vp, C.c_uint32, vp, C.c_double, vp, vp]
        L.orc_emit.argtypes = [C.POINTER(_Inputs), u64, u64, vp, vp, vp, vp]
        L.orc_emit.restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(_Inputs), u64, u64, C.c_int32, C.c_int32, u64, vp, vp,
                              vp, vp, vp, vp]
        L.orc_run.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(np.broadcast_to(np.asarray(key, np.uint32), (ctr.shape[0], 2)))
    out = np.empty_like(ctr)
    lib().orc_philox(ctr.shape[0], _p(ctr), _p(key), _p(out))
    return out


def uniform(w: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.uint32).ravel()
    out = np.empty(w.shape[0], np.float64)
    lib().orc_uniform(w.shape[0], _p(w), _p(out))
    return out


def hg_one_minus_mu(g: float, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    out = np.empty_like(u)
    lib().orc_hg_one_minus_mu(u.shape[0], float(g), _p(u), _p(out))
    return out


def rotate(v: np.ndarray, om: np.ndarray, phi_turns: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    om = np.ascontiguousarray(om, dtype=np.float64).ravel()
    ph = np.ascontiguousarray(phi_turns, dtype=np.float64).ravel()
    out = np.empty_like(v)
    lib().orc_rotate(v.shape[0], _p(v), _p(om), _p(ph), _p(out))
    return out


def basis(v: np.ndarray):
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    e1, e2 = np.empty_like(v), np.empty_like(v)
    lib().orc_basis(v.shape[0], _p(v), _p(e1), _p(e2))
    return e1, e2


def first_hit(p, v, length, dom_xyz, radius):
    p = np.ascontiguousarray(p, np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    length = np.ascontiguousarray(np.broadcast_to(length, (p.shape[0],)), np.float64)
    d = np.ascontiguousarray(dom_xyz, np.float64).reshape(-1, 3)
    ids = np.empty(p.shape[0], np.uint32)
    ts = np.empty(p.shape[0], np.float64)
    lib().orc_first_hit(p.shape[0], _p(p), _p(v), _p(length), d.shape[0], _p(d), float(radius),
                        _p(ids), _p(ts))
    return ids, ts


class _Packed:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, w):
        L = w.layers
        self.abs_len = np.ascontiguousarray(L["abs_len_m"], np.float64)
        self.eff = np.ascontiguousarray(L["eff_scat_len_m"], np.float64)
        self.g = np.ascontiguousarray(L["g"], np.float64)
        d = w.doms
        self.dom_xyz = np.ascontiguousarray(np.stack([d["x"], d["y"], d["z"]], 1), np.float64)
        self.dom_string = np.ascontiguousarray(d["string_id"], np.int32)
        s = w.sources
        self.src_type = np.ascontiguousarray(s["type"], np.int32)
        self.src_event = np.ascontiguousarray(s["event_id"], np.uint32)
        self.src_particle = np.ascontiguousarray(s["particle_id"], np.uint32)
        names = ("x", "y", "z", "dx", "dy", "dz", "t0_ns", "length_m", "cherenkov_deg",
                 "lambda_min_nm", "lambda_max_nm")
        self.src_f = np.ascontiguousarray(np.stack([s[n] for n in names], 1), np.float64)
        self.src_n = np.ascontiguousarray(s["n_photons"], np.uint64)
        self.src_first = np.ascontiguousarray(s["first_photon_index"], np.uint64)
        ch = w.chromatic or (0.0, 0.0, 0.0)
        acc = w.acceptance
        self.acc = np.ascontiguousarray(acc["table"], np.float64) if acc else None
        self.poly = np.ascontiguousarray(acc["poly"], np.float64) if acc else None
        self.struct = _Inputs(
            float(w.z_lo_m), float(w.dz_m), len(L), float(w.n_group),
            _p(self.abs_len), _p(self.eff), _p(self.g),
            len(d), _p(self.dom_xyz), _p(self.dom_string), float(w.dom_radius_m),
            len(s), _p(self.src_type), _p(self.src_event), _p(self.src_particle),
            _p(self.src_f), _p(self.src_n), _p(self.src_first),
            float(ch[0]), float(ch[1]), float(ch[2]),
            len(self.acc) if acc else 0, len(self.poly) if acc else 0,
            float(acc["l0"]) if acc else 0.0, float(acc["dl"]) if acc else 1.0,
            _p(self.acc), _p(self.poly))


def emit(w, seed: int, sel_src, sel_local):
    """Emission state (x y z vx vy vz t tau_a lambda) and layer of photons."""
    pk = _Packed(w)
    ss = np.ascontiguousarray(sel_src, np.uint64)
    sl = np.ascontiguousarray(sel_local, np.uint64)
    out = np.empty((ss.shape[0], 9), np.float64)
    layer = np.empty(ss.shape[0], np.int32)
    rc = lib().orc_emit(C.byref(pk.struct), seed, ss.shape[0], _p(ss), _p(sl), _p(out), _p(layer))
    if rc != 0:
        raise ValueError("bad photon selection")
    return out, layer


class Result:
    def __init__(self, rec_u, rec_f, dom_counts, counters):
        self.rec_u = rec_u
        self.rec_f = rec_f
        self.dom_counts = dom_counts
        self.counters = dict(zip(COUNTER_NAMES, (int(c) for c in counters)))

    @property
    def fate(self):
        return self.rec_u[:, 0]

    @property
    def dom(self):
        return self.rec_u[:, 1]

    @property
    def n_iter(self):
        return self.rec_u[:, 2]

    @property
    def n_cross(self):
        return self.rec_u[:, 3]

    @property
    def t(self):
        return self.rec_f[:, 0]

    @property
    def pos(self):
        return self.rec_f[:, 1:4]

    @property
    def dir(self):
        return self.rec_f[:, 4:7]

    @property
    def wavelength(self):
        return self.rec_f[:, 7]

    @property
    def weight(self):
        return self.rec_f[:, 8]


def run(w, seed: int = 0, step_cap: int = 100_000, dom_mode: int = 0, threads: int | None = None,
        sel_src=None, sel_local=None, records: bool = True, dom_counts: bool = True) -> Result:
    """Propagate every photon of workload w (or a selection of
    (source index, local photon number) pairs) in FP64."""
    pk = _Packed(w)
    if sel_src is None:
        n_sel, ss, sl = 0, None, None
        n = int(pk.src_n.sum())
    else:
        ss = np.ascontiguousarray(sel_src, np.uint64)
        sl = np.ascontiguousarray(sel_local, np.uint64)
        n_sel = n = ss.shape[0]
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    rec_u = np.empty((n, 4), np.uint32) if records else None
    rec_f = np.empty((n, 9), np.float64) if records else None
    counts = np.zeros(len(w.doms), np.uint64) if dom_counts else None
    counters = np.zeros(8, np.uint64)
    rc = lib().orc_run(C.byref(pk.struct), seed, step_cap, dom_mode, threads, n_sel, _p(ss), _p(sl),
                       _p(rec_u), _p(rec_f), _p(counts), _p(counters))
    if rc != 0:
        raise ValueError("oracle rejected its inputs (bad selection or dom_mode)")
    return Result(rec_u, rec_f, counts, counters)
