"""Host-side tests of the C-ABI library: exported symbols, struct layouts,
input validation, call-order errors and the search grid's conservativeness.
No device compute: contexts here are host-only (device -1)."""
import glob
import math
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pp.h")


@pytest.fixture(scope="module")
def pp():
    from paper_2405_05700_amd import pp as mod
    return mod


def declared_functions(header=None):
    headers = [header] if header else sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
    names = set()
    for h in headers:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(pp_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(pp):
    from paper_2405_05700_amd import server, surrogate
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(pp._lib, n), n
    assert set(declared_functions(HEADER)) == set(pp.SIGNATURES)
    assert set(names) == set(pp.SIGNATURES) | set(surrogate.SIGNATURES) | set(server.SIGNATURES)
    out = subprocess.check_output(["nm", "-D", "--defined-only", pp._LIB_PATH], text=True)
    exported = set(re.findall(r" T (pp_[a-z_]+)", out))
    assert set(names) <= exported


def test_struct_layouts_match_bindings(tmp_path, pp):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "pp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(pp_source), sizeof(pp_hit),
         sizeof(pp_photon_record), sizeof(pp_dom), sizeof(pp_ice_layer), sizeof(pp_ice_header),
         offsetof(pp_source, n_photons), offsetof(pp_hit, time_ns), sizeof(pp_chromatic),
         sizeof(pp_acceptance), offsetof(pp_acceptance, poly), sizeof(pp_stats));
  return 0;
}''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)], text=True).split()]
    assert got == [W.SOURCE_DTYPE.itemsize, pp.HIT_DTYPE.itemsize, pp.RECORD_DTYPE.itemsize,
                   W.DOM_DTYPE.itemsize, W.ICE_LAYER_DTYPE.itemsize, 16,
                   W.SOURCE_DTYPE.fields["n_photons"][1], pp.HIT_DTYPE.fields["time_ns"][1],
                   C.sizeof(pp._Chromatic), C.sizeof(pp._Acceptance), pp._Acceptance.poly.offset,
                   C.sizeof(pp._Stats)]


def test_chromatic_and_acceptance_validation(pp):
    ctx = host_ctx(pp)
    for bad in ((0.0, 1.0, 1.0), (-400.0, 0.0, 0.0), (400.0, 11.0, 0.0), (400.0, 0.0, float("nan"))):
        expect(pp, pp.PP_EINVAL, ctx.set_chromatic, *bad)
    ctx.set_chromatic(400.0, 1.0, 0.5)
    ctx.set_chromatic()
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 10.0, [], [1.0])
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 10.0, [1.0] * 257, [1.0])
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 10.0, [1.0, -0.5], [1.0])
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 0.0, [1.0, 2.0], [1.0])
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 10.0, [1.0], [])
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 10.0, [1.0], [1.0] * 9)
    expect(pp, pp.PP_EINVAL, ctx.set_acceptance, 300.0, 10.0, [1.0], [float("inf")])
    ctx.set_acceptance(300.0, 0.0, [0.8], [0.0, 1.0])  # one point: dlambda unused
    ctx.set_acceptance()
    ctx.close()


def host_ctx(pp, w=None):
    ctx = pp.Context(-1, seed=0)
    if w is not None:
        ctx.load_workload(w)
    return ctx


def expect(pp, status, fn, *args):
    with pytest.raises(pp.PPError) as e:
        fn(*args)
    assert e.value.status == status, str(e.value)


def test_call_order_and_device_errors(pp):
    w = W.tiny_point_source(100)
    ctx = host_ctx(pp)
    expect(pp, pp.PP_ESTATE, ctx.submit, w.sources)
    ctx.load_workload(w)
    b = ctx.submit(w.sources)
    expect(pp, pp.PP_EDEVICE, ctx.propagate, b, 0)
    expect(pp, pp.PP_EINVAL, ctx.release, b + 100)
    ctx.release(b)
    ctx.close()
    with pytest.raises(pp.PPError):
        pp.Context(-2)


def test_static_propagation_argument_checks(pp):
    """pp_propagate_static checks its arguments and the call order before it
    touches a device: on a host-only context it reports the first problem."""
    import ctypes as C
    w = W.tiny_point_source(100)
    ctx = host_ctx(pp)
    src = np.ascontiguousarray(w.sources, dtype=W.SOURCE_DTYPE)
    tot = C.c_uint64(123)
    f = pp._lib.pp_propagate_static
    assert f(None, None, 0, None, 0, C.byref(tot), None, None) == pp.PP_EINVAL
    assert f(ctx._h, None, 0, None, 0, None, None, None) == pp.PP_EINVAL      # n_total missing
    assert f(ctx._h, None, 1, None, 0, C.byref(tot), None, None) == pp.PP_EINVAL  # sources missing
    assert f(ctx._h, src.ctypes.data, 1, None, 5, C.byref(tot), None, None) == pp.PP_EINVAL  # hits missing
    assert f(ctx._h, src.ctypes.data, 1, None, 0, C.byref(tot), None, None) == pp.PP_ESTATE  # no ice yet
    assert tot.value == 0
    ctx.load_workload(w)
    ctx.set_debug_records(True)
    assert f(ctx._h, src.ctypes.data, 1, None, 0, C.byref(tot), None, None) == pp.PP_ESTATE
    assert b"records" in pp._lib.pp_last_error(ctx._h)
    ctx.set_debug_records(False)
    many = np.repeat(src, pp.STATIC_MAX_SOURCES + 1)
    assert f(ctx._h, many.ctypes.data, len(many), None, 0, C.byref(tot), None, None) == pp.PP_EINVAL
    assert b"at most 32768" in pp._lib.pp_last_error(ctx._h)
    assert f(ctx._h, src.ctypes.data, 1, None, 0, C.byref(tot), None, None) == pp.PP_EDEVICE
    ctx.close()


def test_ice_validation(pp):
    w = W.tiny_point_source(10)
    ctx = host_ctx(pp)
    good = w.layers.copy()
    ctx.load_ice(w.z_lo_m, w.dz_m, w.n_group, good)
    for field, bad in [("abs_len_m", 0.0), ("abs_len_m", np.nan), ("eff_scat_len_m", -1.0),
                       ("g", 1.0), ("g", -1.0), ("g", np.nan)]:
        L = good.copy()
        L[field][3] = bad
        expect(pp, pp.PP_EINVAL, ctx.load_ice, w.z_lo_m, w.dz_m, w.n_group, L)
    inf_ok = good.copy()
    inf_ok["abs_len_m"][:] = np.inf
    inf_ok["eff_scat_len_m"][:] = np.inf
    ctx.load_ice(w.z_lo_m, w.dz_m, w.n_group, inf_ok)  # no absorption, no scattering: allowed
    expect(pp, pp.PP_EINVAL, ctx.load_ice, w.z_lo_m, 0.0, w.n_group, good)
    expect(pp, pp.PP_EINVAL, ctx.load_ice, np.inf, w.dz_m, w.n_group, good)
    expect(pp, pp.PP_EINVAL, ctx.load_ice, w.z_lo_m, w.dz_m, 0.0, good)
    expect(pp, pp.PP_EINVAL, ctx.load_ice, w.z_lo_m, w.dz_m, w.n_group, good[:0])
    big = np.repeat(good[:1], 1025)
    expect(pp, pp.PP_EINVAL, ctx.load_ice, w.z_lo_m, w.dz_m, w.n_group, big)


def test_geometry_validation(pp):
    w = W.tiny_point_source(10)
    ctx = host_ctx(pp)
    d = w.doms.copy()
    d["om_index"][5] = d["om_index"][6]
    expect(pp, pp.PP_EINVAL, ctx.load_geometry, d, 0.2)
    d = w.doms.copy()
    d["z"][0] = np.nan
    expect(pp, pp.PP_EINVAL, ctx.load_geometry, d, 0.2)
    expect(pp, pp.PP_EINVAL, ctx.load_geometry, w.doms, 0.0)
    expect(pp, pp.PP_EINVAL, ctx.load_geometry, w.doms, np.inf)
    many = np.zeros(513, W.DOM_DTYPE)
    many["string_id"] = np.arange(513)
    expect(pp, pp.PP_EINVAL, ctx.load_geometry, many, 0.2)
    ctx.load_geometry(w.doms[:0], 0.2)  # no modules at all is allowed
    assert ctx.geometry_info()["n_strings"] == 0


def test_source_validation(pp):
    w = W.full_detector(n_sources=4, photons_per_source=10)
    ctx = host_ctx(pp, w)
    ctx.submit(w.sources)
    ctx.submit(w.sources[:0])  # empty batch
    zero = w.sources.copy()
    zero["n_photons"] = 0
    ctx.submit(zero)
    cases = [("type", 7), ("x", np.nan), ("t0_ns", np.inf), ("dx", 0.5), ("length_m", -1.0),
             ("cherenkov_deg", 0.0), ("cherenkov_deg", 180.0), ("lambda_min_nm", 700.0),
             ("lambda_min_nm", 0.0)]
    for field, bad in cases:
        s = w.sources.copy()
        s[field][1] = bad
        expect(pp, pp.PP_EINVAL, ctx.submit, s)
    s = w.sources.copy()
    s["first_photon_index"][2] = np.uint64(2**64 - 5)
    expect(pp, pp.PP_EINVAL, ctx.submit, s)
    # overlapping photon-index ranges in one event are rejected, disjoint ones accepted
    s = w.sources.copy()
    s["event_id"] = 9
    s["first_photon_index"] = [0, 10, 20, 25]
    expect(pp, pp.PP_EINVAL, ctx.submit, s)
    s["first_photon_index"] = [0, 10, 20, 30]
    ctx.submit(s)
    # a point source ignores its direction fields
    p = W.point_source(n_photons=5)
    p["dx"] = p["dy"] = p["dz"] = np.nan
    ctx.submit(p)


def test_launch_config_validation(pp):
    ctx = host_ctx(pp)
    expect(pp, pp.PP_EINVAL, ctx.set_launch_config, 100)
    expect(pp, pp.PP_EINVAL, ctx.set_launch_config, 2048)
    ctx.set_launch_config(512, 77, 3, 10, 6)
    assert ctx.launch_config() == {"block_size": 512, "chunk_size": 77, "grid_blocks": 3,
                                   "hit_capacity": 10, "refill_interval": 6}
    ctx.set_launch_config()
    assert ctx.launch_config()["refill_interval"] == 4
    expect(pp, pp.PP_EINVAL, ctx.set_step_cap, 2**31 + 1)
    ctx.set_step_cap(0)


def string_table(w):
    """Independent string centres and reaches from the module array."""
    d = w.doms
    out = []
    for s in np.unique(d["string_id"]):
        m = d[d["string_id"] == s]
        cx, cy = m["x"].astype(float).mean(), m["y"].astype(float).mean()
        reach = np.hypot(m["x"] - cx, m["y"] - cy).max() + w.dom_radius_m
        out.append((cx, cy, reach))
    return np.array(out)


@pytest.mark.parametrize("make", [lambda: W.full_detector(n_sources=1, photons_per_source=1),
                                  lambda: W.tiny_point_source(1),
                                  lambda: W.random_tiny(3),
                                  lambda: W.random_tiny(4, n_strings=9)])
def test_search_grid_is_conservative(pp, make):
    """For every sampled point, every string other than the cell's listed one
    is at least the cell's clearance away (horizontal distance to its reach
    cylinder); so a step shorter than the clearance can only reach the listed
    string. Points far outside the grid are included."""
    w = make()
    ctx = host_ctx(pp, w)
    info = ctx.geometry_info()
    tab = string_table(w)
    assert info["n_strings"] == len(tab)
    rng = np.random.default_rng(0)
    span = max(info["grid_nx"], info["grid_ny"]) * info["cell_m"]
    cx = info["grid_x0_m"] + info["grid_nx"] * info["cell_m"] / 2
    cy = info["grid_y0_m"] + info["grid_ny"] * info["cell_m"] / 2
    # strings are indexed by ascending string_id, as np.unique orders them
    pts = np.concatenate([rng.uniform(-0.6, 0.6, (3000, 2)) * span,
                          rng.uniform(-3, 3, (500, 2)) * span]) + [cx, cy]
    for x, y in pts.astype(np.float32):
        s1, clr = ctx.geometry_cell(float(x), float(y))
        d = np.hypot(tab[:, 0] - x, tab[:, 1] - y) - tab[:, 2]
        others = np.ones(len(tab), bool)
        if s1 != pp.NO_DOM:
            others[s1] = False
        if others.any():
            assert np.maximum(d[others], 0).min() >= clr - 1e-4, (x, y, s1, clr, d[others].min())
        if len(tab) == 1:
            assert s1 == 0 and math.isinf(clr)


def test_full_detector_geometry_shape(pp):
    w = W.full_detector(n_sources=1, photons_per_source=1)
    ctx = host_ctx(pp, w)
    info = ctx.geometry_info()
    assert info["n_doms"] == 5160 and info["n_strings"] == 86
    assert info["grid_nx"] <= 64 and info["grid_ny"] <= 64
    assert abs(info["max_reach_m"] - W.DOM_RADIUS_M) < 1e-3


def test_server_request_bytes(pp):
    """The serving queue's admission cost (host logic): 80-byte source
    records plus 16-byte work-queue entries of at most 256 photon ids."""
    from paper_2405_05700_amd import server
    assert server.request_bytes(1, 0) == 80 + 16
    assert server.request_bytes(1, 1000) == 80 + 16 * (1 + 1000 // 256)
    assert server.request_bytes(3, 10**8) == 3 * 80 + 16 * (3 + 10**8 // 256)


def test_sort_hits_orders_by_event_then_photon(pp):
    """pp_sort_hits (host only) against numpy's sort of the same records."""
    rng = np.random.default_rng(8)
    n = 5000
    hits = np.zeros(n, pp.HIT_DTYPE)
    ev = rng.integers(0, 40, n).astype(np.uint32)
    ph = rng.permutation(10 * n)[:n].astype(np.uint64) + np.uint64(2**40)  # distinct, above 32 bits
    hits["event_id"], hits["photon_index"] = ev, ph
    hits["dom_id"] = rng.integers(0, 5160, n)
    hits["time_ns"] = rng.random(n).astype(np.float32)
    want = np.sort(hits.copy(), order=["event_id", "photon_index"])
    got = pp.sort_hits(hits)
    assert got is hits and (hits == want).all()
    assert len(pp.sort_hits(np.zeros(0, pp.HIT_DTYPE))) == 0
    with pytest.raises(ValueError):
        pp.sort_hits(np.zeros(3, np.float64))
