"""The photon server on the GPU: continuous batching of events from many
client threads out of a device-resident photon queue, HBM-budget admission,
and results that are the same for a request alone, in the mix, and in the
FP64 oracle (exactly alone vs mixed: randomness is keyed by photon)."""
import os
import sys
import threading
import time

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

pytestmark = pytest.mark.gpu
TIME_RTOL = 1e-4
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2405_05700_amd import pp, server, surrogate
    return pp, server, surrogate


def events(n, seed, cap=50_000):
    w = W.uneven_events(n, seed=seed)
    src = w.sources.copy()
    src["n_photons"] = np.minimum(src["n_photons"], cap)
    src["event_id"] = 1000 + np.arange(n)
    return w.with_sources(src)


def key(h):
    return np.sort(h, order=["event_id", "photon_index"])


def alone_hits(pp, w, i):
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    b = ctx.submit(w.sources[i:i + 1])
    ctx.propagate(b)
    return key(ctx.fetch_hits(b))


def run_clients(srv, w, n_clients, jitter_s=0.002, seed=0, expected=True):
    """n_clients threads submit the events round-robin with random pauses,
    then wait for their own tickets."""
    results = {}
    lock = threading.Lock()

    def client(c):
        rng = np.random.default_rng(seed + c)
        mine = []
        for i in range(c, len(w.sources), n_clients):
            time.sleep(rng.uniform(0, jitter_s))
            mine.append((i, srv.submit(w.sources[i:i + 1])))
        for i, t in mine:
            hits, info, dom = srv.wait(t, expected=expected)
            with lock:
                results[i] = (key(hits), info, dom)

    th = [threading.Thread(target=client, args=(c,)) for c in range(n_clients)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    return results


def test_each_request_same_alone_and_in_the_mix(mods):
    """48 events from 16 threads, at most 6 per launch, 4 launch slots: the
    work overlaps on the device (launches enqueued while others run,
    requests sharing launches) and every request's hits equal those of the
    event propagated alone."""
    pp, server, surrogate = mods
    w = events(48, seed=9)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, max_inflight=4, max_batch_events=6)
    res = run_clients(srv, w, n_clients=16, jitter_s=0.0005)
    st = srv.stats()
    srv.close()
    say("server stats", st)
    assert st["completed"] == 48 and st["bytes_in_use"] == 0
    assert st["shared_requests"] > 0 and st["launches"] < st["completed"]
    assert st["overlapped_launches"] > 0
    assert 0 < st["gpu_busy_s"] <= st["gpu_span_s"] + 1e-9
    shared = sum(1 for r in res.values() if r[1]["batch_events"] > 1)
    assert shared == st["shared_requests"]
    for i in [0, 5, 17, 31, 47] + list(np.argsort(w.sources["n_photons"])[-3:]):
        ref = alone_hits(pp, w, i)
        got = res[int(i)][0]
        assert len(got) == len(ref) and (got == ref).all(), i
    for i, (hits, info, _) in res.items():
        assert info["photons"] == w.sources["n_photons"][i]
        assert info["t_submit_s"] <= info["t_launch_s"] <= info["t_done_s"]
        assert (hits["event_id"] == w.sources["event_id"][i]).all()


def test_served_events_match_the_oracle(mods):
    """Events served from 8 threads against the FP64 oracle photon by
    photon: 24 segments 3-8 m from modules, 6e4 photons each (about 600
    hits). Every served hit is the oracle's hit of that photon (module
    exact, time within 1e-4), and the oracle's hits are served, for >= 99.9%
    of the union."""
    pp, server, surrogate = mods
    from oracle import pyoracle
    det = W.full_detector(n_sources=1, photons_per_source=1)
    src = W.near_module_segments(det, 24, 60_000, seed=31, r_min=3.0, r_max=8.0, first_event_id=500)
    w = det.with_sources(src, "served_near_modules")
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, max_inflight=3, max_batch_events=5)
    res = run_clients(srv, w, n_clients=8, jitter_s=0.001, expected=False)
    st = srv.stats()
    srv.close()
    ref = pyoracle.run(w, seed=0, threads=THREADS, dom_mode=1)
    base = np.concatenate([[0], np.cumsum(src["n_photons"].astype(np.int64))])
    served = {}
    for i, (hits, info, _) in res.items():
        for h in hits:
            served[int(base[i] + h["photon_index"] - src["first_photon_index"][i])] = (int(h["dom_id"]),
                                                                                     float(h["time_ns"]))
    orc = {int(k): (int(ref.dom[k]), float(ref.t[k])) for k in np.nonzero(ref.fate == 1)[0]}
    union = set(served) | set(orc)
    good = sum(1 for k in union if k in served and k in orc and served[k][0] == orc[k][0] and
               abs(served[k][1] - orc[k][1]) <= TIME_RTOL * abs(orc[k][1]) + 1e-6)
    say(f"served vs oracle: {len(served)} served hits, {len(orc)} oracle hits, {good} agree; {st['launches']} launches")
    assert len(union) > 500 and st["shared_requests"] > 0
    assert good >= 0.999 * len(union)


def test_small_queue_defers_and_bounds_memory(mods):
    """A 16 KiB budget: the device queue holds 256 work-queue entries and 24
    events of 40 000 photons need 157 each, so no two fit at once: each
    admission waits for the launch before it to free ring space. The queue
    bytes held never exceed the rings, the arena and any overflow buffer fit
    the budget, and results stay those of solo runs."""
    pp, server, surrogate = mods
    base = events(1, seed=10)
    src = W.cherenkov_segments(24, 40_000, seed=10, first_event_id=2000)
    w = base.with_sources(src)
    budget = 16 * 1024
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, max_inflight=2, hbm_budget_bytes=budget)
    st0 = srv.stats()
    assert st0["arena_bytes"] <= budget
    assert 2 * int(np.ceil(40_000 / 256)) > 256
    res = run_clients(srv, w, n_clients=8, jitter_s=0.0)
    st = srv.stats()
    srv.close()
    say("small queue", budget, st)
    assert st["completed"] == 24 and st["deferred"] > 0 and st["launches"] == 24
    assert st["peak_bytes_in_use"] <= 256 * 16 + 64 * 80
    assert st["arena_bytes"] + st["overflow_bytes_peak"] <= budget
    for i in (0, 11, 23):
        assert (res[i][0] == alone_hits(pp, w, i)).all()


def test_device_memory_within_budget(mods):
    """The device memory the server holds, measured by the runtime's free
    memory before creation and while serving, stays within a 64 MiB
    budget."""
    pp, server, surrogate = mods
    import torch
    w = events(32, seed=13, cap=200_000)
    budget = 64 << 20
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(0)
    srv = server.Server(ctx, max_inflight=4, hbm_budget_bytes=budget)
    res = run_clients(srv, w, n_clients=8, jitter_s=0.0, expected=False)
    free1, _ = torch.cuda.mem_get_info(0)
    st = srv.stats()
    srv.close()
    say(f"budget {budget}, arena {st['arena_bytes']}, measured {free0 - free1}")
    assert len(res) == 32
    assert st["arena_bytes"] <= budget and free0 - free1 <= budget


def test_request_too_large_is_refused(mods):
    pp, server, surrogate = mods
    w = events(2, seed=11)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, hbm_budget_bytes=1 << 20)  # a ring of 16384 entries: 4.2e6 photons
    big = w.sources[:1].copy()
    big["n_photons"] = 10_000_000
    with pytest.raises(pp.PPError) as e:
        srv.submit(big)
    assert e.value.status == pp.PP_EBUDGET
    bad = w.sources[:1].copy()
    bad["x"] = np.nan
    with pytest.raises(pp.PPError) as e:
        srv.submit(bad)
    assert e.value.status == pp.PP_EINVAL
    t = srv.submit(w.sources[1:2])  # a valid one still goes through
    hits, info, _ = srv.wait(t)
    assert info["photons"] == w.sources["n_photons"][1]
    srv.close()
    with pytest.raises(pp.PPError) as e:
        server.Server(ctx, hbm_budget_bytes=1024)
    assert e.value.status == pp.PP_EBUDGET


def test_native_clients_open_and_closed_loop(mods):
    """The native load generator: 16 threads, an open loop at 400 events/s
    and a closed loop with 8 requests outstanding per thread; every request
    completes, photons add up, latencies are positive."""
    pp, server, surrogate = mods
    w = events(4000, seed=14, cap=100_000)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, max_inflight=4)
    o = srv.run_clients(w.sources, n_clients=16, rate_per_s=400.0, duration_s=1.0, seed=5)
    c = srv.run_clients(w.sources, n_clients=16, rate_per_s=0.0, outstanding=8, duration_s=0.5)
    st = srv.stats()
    srv.close()
    say(f"open loop: {o['done']} events in {o['wall_s']:.2f} s, p50 {1e3 * np.median(o['latency_s']):.2f} ms; "
        f"closed loop: {c['done']} events in {c['wall_s']:.2f} s; launches {st['launches']}")
    assert 200 <= o["done"] <= 800 and c["done"] > 0
    assert (o["latency_s"] > 0).all() and (c["latency_s"] > 0).all()
    assert st["completed"] == o["done"] + c["done"]
    assert st["photons_completed"] == o["photons"] + c["photons"]
    assert c["done"] / c["wall_s"] > o["done"] / o["wall_s"]


def test_surrogate_expectations_ride_along(mods):
    """With a surrogate attached every request also returns expected hits
    per module for its sources, equal to the surrogate run on that event
    alone."""
    pp, server, surrogate = mods
    w = events(12, seed=12, cap=10_000)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    sur = surrogate.Surrogate(ctx, seed=4)
    srv = server.Server(ctx, max_inflight=2, surrogate=sur)
    res = run_clients(srv, w, n_clients=4)
    srv.close()
    ctx2 = pp.Context(0, seed=0)
    ctx2.load_workload(w)
    sur2 = surrogate.Surrogate(ctx2, seed=4)
    for i in (0, 6, 11):
        b = ctx2.submit(w.sources[i:i + 1])
        ref = sur2.predict_pairs(b, 1)[0]
        got = res[i][2]
        assert got is not None and np.allclose(got, ref, rtol=1e-4, atol=1e-12), i
