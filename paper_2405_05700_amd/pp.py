"""Python binding of libpp (include/pp.h): argument marshalling only.

Every step of the propagation runs in the library's HIP kernels. PyTorch is
used only for device memory (hit and count tensors) and streams. If the
built library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

from . import workloads as W

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpp.so")

HIT_DTYPE = np.dtype([("photon_index", "<u8"), ("event_id", "<u4"), ("particle_id", "<u4"),
                      ("dom_id", "<u4"), ("time_ns", "<f4"), ("weight", "<f4"),
                      ("reserved", "<u4")], align=True)
RECORD_DTYPE = np.dtype([("fate", "<u4"), ("dom_id", "<u4"), ("n_iter", "<u4"), ("n_cross", "<u4"),
                         ("time_ns", "<f4"), ("x", "<f4"), ("y", "<f4"), ("z", "<f4"),
                         ("vx", "<f4"), ("vy", "<f4"), ("vz", "<f4"), ("wavelength_nm", "<f4")],
                        align=True)
assert HIT_DTYPE.itemsize == 32 and RECORD_DTYPE.itemsize == 48

PP_OK, PP_EINVAL, PP_ENOMEM, PP_EDEVICE, PP_ESTATE, PP_ETRUNC, PP_EBUDGET = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "PP_OK", -1: "PP_EINVAL", -2: "PP_ENOMEM", -3: "PP_EDEVICE",
                -4: "PP_ESTATE", -5: "PP_ETRUNC", -6: "PP_EBUDGET"}
FATE_ABSORBED, FATE_HIT, FATE_CAPPED, FATE_ESCAPED = 0, 1, 2, 3
RECORDS_OFF, RECORDS_ON, RECORDS_PRODUCTION = 0, 1, 2
NO_DOM = 0xFFFFFFFF


class PPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _IceHeader(C.Structure):
    _fields_ = [("z_lo_m", C.c_float), ("dz_m", C.c_float), ("n_layers", C.c_uint32),
                ("n_group", C.c_float)]


class _Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("photons", "iterations", "layer_crossings", "dom_tests",
                                          "hits", "absorbed", "capped", "escaped")] + \
               [("kernel_ms", C.c_float), ("block_size", C.c_uint32), ("grid_blocks", C.c_uint32),
                ("chunk_size", C.c_uint32), ("refill_interval", C.c_uint32)]


class _LaunchConfig(C.Structure):
    _fields_ = [("block_size", C.c_uint32), ("chunk_size", C.c_uint32),
                ("grid_blocks", C.c_uint32), ("refill_interval", C.c_uint32),
                ("hit_capacity", C.c_uint64)]


class _GeometryInfo(C.Structure):
    _fields_ = [("n_doms", C.c_uint32), ("n_strings", C.c_uint32), ("grid_nx", C.c_uint32),
                ("grid_ny", C.c_uint32), ("grid_x0_m", C.c_float), ("grid_y0_m", C.c_float),
                ("cell_m", C.c_float), ("max_reach_m", C.c_float)]


class _Chromatic(C.Structure):
    _fields_ = [("lambda_ref_nm", C.c_float), ("kappa_abs", C.c_float), ("kappa_scat", C.c_float),
                ("reserved", C.c_float)]


class _Acceptance(C.Structure):
    _fields_ = [("lambda0_nm", C.c_float), ("dlambda_nm", C.c_float), ("n_table", C.c_uint32),
                ("n_poly", C.c_uint32), ("table", C.c_void_p), ("poly", C.c_void_p)]


# name -> (restype, argtypes); every symbol declared in include/pp.h
_vp, _u64, _u32 = C.c_void_p, C.c_uint64, C.c_uint32
SIGNATURES = {
    "pp_create": (C.c_int, [C.c_int, _u64, C.POINTER(_vp)]),
    "pp_destroy": (None, [_vp]),
    "pp_last_error": (C.c_char_p, [_vp]),
    "pp_set_launch_config": (C.c_int, [_vp, C.POINTER(_LaunchConfig)]),
    "pp_get_launch_config": (C.c_int, [_vp, C.POINTER(_LaunchConfig)]),
    "pp_set_step_cap": (C.c_int, [_vp, _u64]),
    "pp_load_ice": (C.c_int, [_vp, C.POINTER(_IceHeader), _vp]),
    "pp_load_geometry": (C.c_int, [_vp, _vp, _u32, C.c_float]),
    "pp_get_geometry_info": (C.c_int, [_vp, C.POINTER(_GeometryInfo)]),
    "pp_geometry_cell": (C.c_int, [_vp, C.c_float, C.c_float, C.POINTER(_u32),
                                   C.POINTER(C.c_float)]),
    "pp_submit": (C.c_int, [_vp, _vp, _u32, C.POINTER(_u64)]),
    "pp_release": (C.c_int, [_vp, _u64]),
    "pp_set_debug_records": (C.c_int, [_vp, C.c_int]),
    "pp_propagate": (C.c_int, [_vp, _u64, _vp]),
    "pp_hit_count": (C.c_int, [_vp, _u64, C.POINTER(_u64)]),
    "pp_fetch_hits": (C.c_int, [_vp, _u64, _vp, _u64, C.POINTER(_u64)]),
    "pp_fetch_hits_device": (C.c_int, [_vp, _u64, _vp, _u64, C.POINTER(_u64), _vp]),
    "pp_dom_counts": (C.c_int, [_vp, _u64, _vp, _vp]),
    "pp_dom_weights": (C.c_int, [_vp, _u64, _vp, _vp]),
    "pp_sort_hits": (C.c_int, [_vp, _u64]),
    "pp_fetch_records": (C.c_int, [_vp, _u64, _vp, _u64, _u64]),
    "pp_get_stats": (C.c_int, [_vp, _u64, C.POINTER(_Stats)]),
    "pp_autotune": (C.c_int, [_vp, _u64, _vp, C.POINTER(_LaunchConfig)]),
    "pp_graph_capture": (C.c_int, [_vp, _u64, _vp]),
    "pp_graph_launch": (C.c_int, [_vp, _u64, _vp]),
    "pp_set_chromatic": (C.c_int, [_vp, C.POINTER(_Chromatic)]),
    "pp_set_acceptance": (C.c_int, [_vp, C.POINTER(_Acceptance)]),
    "pp_propagate_static": (C.c_int, [_vp, _vp, _u32, _vp, _u64, C.POINTER(_u64), C.POINTER(_Stats), _vp]),
}
STATIC_MAX_SOURCES = 32768


def load_library(path: str = _LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2405_05700_amd.build` "
                          "(the HIP library is required: there is no fallback path)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def sort_hits(hits: np.ndarray) -> np.ndarray:
    """Sorts a HIT_DTYPE array in place by (event_id, photon_index) with
    pp_sort_hits; returns it."""
    if hits.dtype != HIT_DTYPE or not hits.flags["C_CONTIGUOUS"] or not hits.flags["WRITEABLE"]:
        raise ValueError("sort_hits needs a writable contiguous HIT_DTYPE array")
    st = _lib.pp_sort_hits(_ptr(hits) if len(hits) else None, len(hits))
    if st != PP_OK:
        raise PPError(st, "pp_sort_hits failed")
    return hits


def _stream_handle(stream):
    """hipStream_t as an integer: None -> torch's current stream."""
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """One library context: ice, geometry and submitted batches on one GPU
    (device=-1: host-only, for validation and geometry indexing)."""

    def __init__(self, device: int = 0, seed: int = 0):
        h = C.c_void_p()
        st = _lib.pp_create(int(device), int(seed), C.byref(h))
        if st != PP_OK:
            raise PPError(st, _lib.pp_last_error(None).decode())
        self._h = h
        self.device = device
        self.n_doms = 0
        # surrogates and servers bound to this context: closed before it, and
        # counted, so that one that outlives it (objects of a reference cycle
        # are finalised in any order) defers the context's destruction
        self._dependents = weakref.WeakSet()
        self._n_dependents = 0
        self._close_pending = False

    # -- lifetime
    def _add_dependent(self, d):
        self._dependents.add(d)
        self._n_dependents += 1

    def _release_dependent(self):
        self._n_dependents -= 1
        if self._close_pending and self._n_dependents == 0:
            self._close_pending = False
            self.close()

    def close(self):
        if self._h:
            # servers first: one may use a surrogate of this context
            for d in sorted(self._dependents, key=lambda d: d._close_order):
                d.close()
            if self._n_dependents > 0:
                self._close_pending = True
                return
            _lib.pp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int, allow=(PP_OK,)):
        if st not in allow:
            raise PPError(st, _lib.pp_last_error(self._h).decode())
        return st

    # -- configuration
    def set_launch_config(self, block_size=0, chunk_size=0, grid_blocks=0, hit_capacity=0,
                          refill_interval=0):
        cfg = _LaunchConfig(block_size, chunk_size, grid_blocks, refill_interval, hit_capacity)
        self._check(_lib.pp_set_launch_config(self._h, C.byref(cfg)))

    def launch_config(self) -> dict:
        cfg = _LaunchConfig()
        self._check(_lib.pp_get_launch_config(self._h, C.byref(cfg)))
        return {k: getattr(cfg, k) for k, _ in _LaunchConfig._fields_}

    def set_step_cap(self, cap: int):
        self._check(_lib.pp_set_step_cap(self._h, int(cap)))

    def set_debug_records(self, on):
        """False: off; True or RECORDS_ON: records with each photon's drawn
        wavelength; RECORDS_PRODUCTION: records from the kernel variant that
        runs with records off (wavelength 0 unless that variant draws it)."""
        mode = RECORDS_OFF if on is False else (RECORDS_ON if on is True else int(on))
        self._check(_lib.pp_set_debug_records(self._h, mode))

    # -- inputs
    def load_ice(self, z_lo_m: float, dz_m: float, n_group: float, layers: np.ndarray):
        layers = np.ascontiguousarray(layers, dtype=W.ICE_LAYER_DTYPE)
        hdr = _IceHeader(z_lo_m, dz_m, len(layers), n_group)
        self._check(_lib.pp_load_ice(self._h, C.byref(hdr), _ptr(layers)))

    def load_geometry(self, doms: np.ndarray, dom_radius_m: float):
        doms = np.ascontiguousarray(doms, dtype=W.DOM_DTYPE)
        self._check(_lib.pp_load_geometry(self._h, _ptr(doms), len(doms), float(dom_radius_m)))
        self.n_doms = len(doms)

    def load_workload(self, w: "W.Workload"):
        self.load_ice(w.z_lo_m, w.dz_m, w.n_group, w.layers)
        self.load_geometry(w.doms, w.dom_radius_m)
        self.set_chromatic(*(w.chromatic or ()))
        a = w.acceptance
        if a:
            self.set_acceptance(a["l0"], a["dl"], a["table"], a["poly"])
        else:
            self.set_acceptance()

    def set_chromatic(self, lambda_ref_nm=None, kappa_abs=0.0, kappa_scat=0.0):
        """Coefficients scale as (lambda / lambda_ref)^-kappa; no argument:
        wavelength-independent optics."""
        if lambda_ref_nm is None:
            self._check(_lib.pp_set_chromatic(self._h, None))
            return
        c = _Chromatic(lambda_ref_nm, kappa_abs, kappa_scat, 0.0)
        self._check(_lib.pp_set_chromatic(self._h, C.byref(c)))

    def set_acceptance(self, lambda0_nm=None, dlambda_nm=1.0, table=(), poly=(1.0,)):
        """Hit weight = table(lambda) x poly(cos incidence); no argument:
        weight 1."""
        if lambda0_nm is None:
            self._check(_lib.pp_set_acceptance(self._h, None))
            return
        t = np.ascontiguousarray(table, np.float32)
        p = np.ascontiguousarray(poly, np.float32)
        a = _Acceptance(lambda0_nm, dlambda_nm, len(t), len(p), t.ctypes.data, p.ctypes.data)
        self._check(_lib.pp_set_acceptance(self._h, C.byref(a)))

    def geometry_info(self) -> dict:
        gi = _GeometryInfo()
        self._check(_lib.pp_get_geometry_info(self._h, C.byref(gi)))
        return {k: getattr(gi, k) for k, _ in _GeometryInfo._fields_}

    def geometry_cell(self, x: float, y: float):
        s, c = C.c_uint32(), C.c_float()
        self._check(_lib.pp_geometry_cell(self._h, x, y, C.byref(s), C.byref(c)))
        return s.value, c.value

    def submit(self, sources: np.ndarray) -> int:
        sources = np.ascontiguousarray(sources, dtype=W.SOURCE_DTYPE)
        b = C.c_uint64()
        self._check(_lib.pp_submit(self._h, _ptr(sources), len(sources), C.byref(b)))
        return b.value

    def release(self, batch: int):
        self._check(_lib.pp_release(self._h, batch))

    # -- run
    def propagate(self, batch: int, stream=None):
        self._check(_lib.pp_propagate(self._h, batch, _stream_handle(stream)))

    def hit_count(self, batch: int) -> int:
        n = C.c_uint64()
        self._check(_lib.pp_hit_count(self._h, batch, C.byref(n)))
        return n.value

    def fetch_hits(self, batch: int, sort: bool = False) -> np.ndarray:
        """All hits in host memory; sort=True orders them by (event_id,
        photon_index) (pp_sort_hits), else the order is unspecified."""
        n = self.hit_count(batch)
        out = np.zeros(n, HIT_DTYPE)
        tot = C.c_uint64()
        self._check(_lib.pp_fetch_hits(self._h, batch, _ptr(out), n, C.byref(tot)))
        assert tot.value == n
        if sort:
            sort_hits(out)
        return out

    def fetch_hits_into(self, batch: int, out: np.ndarray) -> int:
        """Copies at most len(out) hits; returns the total (may exceed it)."""
        tot = C.c_uint64()
        self._check(_lib.pp_fetch_hits(self._h, batch, _ptr(out), len(out), C.byref(tot)),
                    allow=(PP_OK, PP_ETRUNC))
        return tot.value

    def fetch_hits_device(self, batch: int, out, stream=None) -> int:
        """Copies hits into a uint8 (or any) CUDA tensor of >= 32 * n bytes."""
        cap = out.numel() * out.element_size() // HIT_DTYPE.itemsize
        tot = C.c_uint64()
        self._check(_lib.pp_fetch_hits_device(self._h, batch, C.c_void_p(out.data_ptr()), cap,
                                              C.byref(tot), _stream_handle(stream)),
                    allow=(PP_OK, PP_ETRUNC))
        return tot.value

    def dom_counts(self, batch: int, out=None, stream=None):
        """Per-module hit counts as an int32 CUDA tensor (computed on the
        device, asynchronously on the stream)."""
        import torch
        if out is None:
            out = torch.empty(max(self.n_doms, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(_lib.pp_dom_counts(self._h, batch, C.c_void_p(out.data_ptr()),
                                       _stream_handle(stream)))
        return out[: self.n_doms]

    def dom_weights(self, batch: int, out=None, stream=None):
        """Per-module sums of hit weights as a float64 CUDA tensor (computed
        on the device, asynchronously on the stream)."""
        import torch
        if out is None:
            out = torch.empty(max(self.n_doms, 1), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(_lib.pp_dom_weights(self._h, batch, C.c_void_p(out.data_ptr()),
                                        _stream_handle(stream)))
        return out[: self.n_doms]

    def fetch_records(self, batch: int, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = self._n_photons_hint(batch) - first
        out = np.zeros(count, RECORD_DTYPE)
        self._check(_lib.pp_fetch_records(self._h, batch, _ptr(out), first, count))
        return out

    def _n_photons_hint(self, batch: int) -> int:
        return self.stats(batch)["photons"]

    def autotune(self, batch: int, stream=None) -> dict:
        """Times the batch under a set of launch configurations and keeps the
        fastest; returns it."""
        cfg = _LaunchConfig()
        self._check(_lib.pp_autotune(self._h, batch, _stream_handle(stream), C.byref(cfg)))
        return {k: getattr(cfg, k) for k, _ in _LaunchConfig._fields_}

    def graph_capture(self, batch: int, stream):
        self._check(_lib.pp_graph_capture(self._h, batch, _stream_handle(stream)))

    def graph_launch(self, batch: int, stream=None):
        self._check(_lib.pp_graph_launch(self._h, batch, _stream_handle(stream)))

    def propagate_static(self, sources: np.ndarray, dev_hits, stream=None):
        """pp_propagate_static: propagates the sources with no device
        allocation into dev_hits (a CUDA tensor of >= 32 bytes per hit);
        returns (n_total, stats). n_total may exceed the buffer's capacity
        (then only that many hits were written)."""
        sources = np.ascontiguousarray(sources, dtype=W.SOURCE_DTYPE)
        cap = dev_hits.numel() * dev_hits.element_size() // HIT_DTYPE.itemsize
        tot = C.c_uint64()
        s = _Stats()
        self._check(_lib.pp_propagate_static(self._h, _ptr(sources) if len(sources) else None, len(sources),
                                             C.c_void_p(dev_hits.data_ptr()) if cap else None, cap,
                                             C.byref(tot), C.byref(s), _stream_handle(stream)),
                    allow=(PP_OK, PP_ETRUNC))
        return tot.value, {k: getattr(s, k) for k, _ in _Stats._fields_}

    def stats(self, batch: int) -> dict:
        s = _Stats()
        self._check(_lib.pp_get_stats(self._h, batch, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}
