"""Parity at the size the throughput is measured on: the full detector (86 x
60 modules, 171 layers with the dust bump, 1000 Cherenkov segments x 1e5
photons = 1e8 photons, Philox seed 0) in the default launch configuration
with debug records off, exactly as the benchmark times it.

The hot path's outputs at this size are the hit list and the batch
counters. The oracle checks them three ways:
* photon by photon for every GPU hit (the oracle propagates exactly those
  photons);
* both ways, every photon, for the 50 segments with the most hits: the set
  of photons that hit, and their modules and times, are the same on both
  sides;
* in total over all 1e8 photons (the oracle run without per-photon
  records): steps, layer crossings, hits and per-module counts.
The oracle runs with its per-string module pre-filter, which its own pins
show equal to the brute-force search (about 35 s for 1e8 photons on 16
cores).
"""
import os
import sys

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

pytestmark = pytest.mark.gpu

TIME_RTOL = 1e-4
MIN_AGREE = 0.999
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def full_run():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_05700_amd import pp
    from oracle import pyoracle
    pyoracle.lib()
    w = W.full_detector()
    assert w.n_photons == 100_000_000
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    b = ctx.submit(w.sources)
    ctx.propagate(b)
    st = ctx.stats(b)
    hits = ctx.fetch_hits(b)
    say("full detector:", st["hits"], "hits,", st["iterations"], "steps, launch", st["block_size"], "x",
        st["grid_blocks"], "chunk", st["chunk_size"], "refill", st["refill_interval"])
    # hit -> (source index, local photon number); each segment is its own event
    src = hits["event_id"].astype(np.int64)
    assert (w.sources["event_id"][src] == hits["event_id"]).all()
    local = hits["photon_index"].astype(np.int64) - w.sources["first_photon_index"][src].astype(np.int64)
    return w, st, hits, src, local, pyoracle


def test_every_gpu_hit_is_the_oracle_hit(full_run):
    w, st, hits, src, local, orc = full_run
    assert st["hits"] == len(hits) > 1000
    ref = orc.run(w, sel_src=src.astype(np.uint64), sel_local=local.astype(np.uint64), dom_mode=1,
                  threads=THREADS)
    ok = (ref.fate == 1) & (ref.dom == hits["dom_id"]) & \
         (np.abs(hits["time_ns"] - ref.t) <= TIME_RTOL * np.abs(ref.t) + 1e-6)
    say("GPU hits confirmed by the oracle:", int(ok.sum()), "of", len(ok))
    assert ok.mean() >= MIN_AGREE


def test_brightest_segments_photon_by_photon(full_run):
    w, st, hits, src, local, orc = full_run
    top = np.argsort(-np.bincount(src, minlength=len(w.sources)), kind="stable")[:50]
    n = w.sources["n_photons"][top].astype(np.int64)
    sel_src = np.repeat(top, n).astype(np.uint64)
    sel_local = np.concatenate([np.arange(k) for k in n]).astype(np.uint64)
    ref = orc.run(w, sel_src=sel_src, sel_local=sel_local, dom_mode=1, threads=THREADS)
    base = np.concatenate([[0], np.cumsum(n)])
    pos_of = {int(s): int(base[i]) for i, s in enumerate(top)}
    mine = np.isin(src, top)
    gpu = {pos_of[int(s)] + int(l): (int(d), float(t))
           for s, l, d, t in zip(src[mine], local[mine], hits["dom_id"][mine], hits["time_ns"][mine])}
    ref_hit = np.nonzero(ref.fate == 1)[0]
    orc_hits = {int(k): (int(ref.dom[k]), float(ref.t[k])) for k in ref_hit}
    union = set(gpu) | set(orc_hits)
    good = sum(1 for k in union if k in gpu and k in orc_hits and gpu[k][0] == orc_hits[k][0] and
               abs(gpu[k][1] - orc_hits[k][1]) <= TIME_RTOL * abs(orc_hits[k][1]) + 1e-6)
    say("brightest 50 segments:", int(n.sum()), "photons,", len(gpu), "GPU hits,", len(orc_hits),
        "oracle hits,", good, "agree")
    assert len(union) > 500
    assert good >= MIN_AGREE * len(union)


def test_full_totals_match_the_oracle(full_run):
    """Oracle over all 1e8 photons without per-photon records."""
    w, st, hits, src, local, orc = full_run
    ref = orc.run(w, threads=THREADS, records=False, dom_mode=1)
    c = ref.counters
    say("totals gpu/oracle: steps", st["iterations"], c["iterations"], "crossings", st["layer_crossings"],
        c["crossings"], "hits", st["hits"], c["hits"])
    assert c["photons"] == st["photons"] == w.n_photons
    assert abs(st["iterations"] - c["iterations"]) <= 1e-4 * c["iterations"]
    assert abs(st["layer_crossings"] - c["crossings"]) <= 1e-4 * c["crossings"]
    assert abs(st["hits"] - c["hits"]) <= 0.002 * c["hits"] + 2
    gpu_counts = np.bincount(hits["dom_id"], minlength=len(w.doms))
    diff = np.abs(gpu_counts.astype(np.int64) - ref.dom_counts.astype(np.int64)).sum()
    assert diff <= 0.002 * c["hits"] + 4
    assert st["capped"] == 0 and st["escaped"] == c.get("escaped", 0)
