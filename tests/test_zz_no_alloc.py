"""pp_propagate_static (the entry point that allocates no device memory)
against the allocating path pp_submit + pp_propagate + pp_fetch_hits_device
on the same sources: the same hit set, bit for bit, on two calls in a row,
the second with a smaller input. Both calls share the library's fixed
scratch array, so the second call also shows that nothing of the first one
is left over (counters, queue entries or sources)."""
import sys

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pp():
    import torch
    assert torch.cuda.is_available()
    from paper_2405_05700_amd import pp as mod
    return mod


def _key(h):
    return np.sort(h[["event_id", "photon_index", "dom_id", "particle_id"]].copy(),
                   order=["event_id", "photon_index"])


def allocating(pp, ctx, sources):
    import torch
    b = ctx.submit(sources)
    ctx.propagate(b)
    n = ctx.hit_count(b)
    out = torch.empty(max(n, 1) * 32, dtype=torch.uint8, device="cuda:0")
    assert ctx.fetch_hits_device(b, out) == n
    torch.cuda.synchronize()
    hits = out.cpu().numpy()[: 32 * n].view(pp.HIT_DTYPE).copy()
    st = ctx.stats(b)
    ctx.release(b)
    return pp.sort_hits(hits), st


def static(pp, ctx, sources, cap):
    import torch
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda:0")
    n, st = ctx.propagate_static(sources, out)
    torch.cuda.synchronize()
    hits = out.cpu().numpy()[: 32 * min(n, cap)].view(pp.HIT_DTYPE).copy()
    return n, pp.sort_hits(hits), st


def check_same(pp, ctx, sources, cap):
    ref, st_ref = allocating(pp, ctx, sources)
    n, got, st = static(pp, ctx, sources, cap)
    say(f"  {len(sources)} sources, {int(sources['n_photons'].sum())} photons: "
        f"allocating path {len(ref)} hits, static path {n} hits")
    assert n == len(ref) == len(got)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))  # every field, every bit
    for k in ("photons", "iterations", "layer_crossings", "dom_tests", "hits", "absorbed", "capped",
              "escaped"):
        assert st[k] == st_ref[k], k


def test_static_equals_allocating_twice_second_smaller(pp):
    w = W.full_detector(n_sources=200, photons_per_source=20_000)
    with pp.Context(0, seed=7) as ctx:
        ctx.load_workload(w)
        say("call 1: 200 full-detector segments")
        check_same(pp, ctx, w.sources, cap=1 << 16)
        say("call 2: 37 segments, fewer photons each")
        small = w.sources[50:87].copy()
        small["n_photons"] = 3_000 + 97 * np.arange(len(small))
        check_same(pp, ctx, small, cap=1 << 14)


def test_static_tiny_point_source_and_edge_cases(pp):
    import torch
    w = W.tiny_point_source(50_000, dom_radius_m=2.0)
    with pp.Context(0, seed=0) as ctx:
        ctx.load_workload(w)
        check_same(pp, ctx, w.sources, cap=4096)
        # no sources, and a source with no photons: nothing propagates
        out = torch.empty(32 * 16, dtype=torch.uint8, device="cuda:0")
        n, st = ctx.propagate_static(w.sources[:0], out)
        assert n == 0 and st["photons"] == 0
        z = w.sources.copy()
        z["n_photons"] = 0
        n, st = ctx.propagate_static(z, out)
        assert n == 0 and st["photons"] == 0
        # a buffer too small: the true total comes back with PP_ETRUNC and
        # the hits written are a subset of the full set
        ref, _ = allocating(pp, ctx, w.sources)
        n, got, _ = static(pp, ctx, w.sources, cap=7)
        assert n == len(ref) and len(got) == 7
        assert set(map(tuple, _key(got).tolist())) <= set(map(tuple, _key(ref).tolist()))
        # too many sources is refused before anything runs
        many = np.repeat(w.sources, pp.STATIC_MAX_SOURCES + 1)
        many["first_photon_index"] = np.arange(len(many))
        many["n_photons"] = 1
        with pytest.raises(pp.PPError, match="at most"):
            ctx.propagate_static(many, out)
        # debug records need per-photon memory: refused
        ctx.set_debug_records(True)
        with pytest.raises(pp.PPError, match="records"):
            ctx.propagate_static(w.sources, out)
