"""The photon server on the GPU: continuous batching of events from many
client threads, HBM-budget admission, and results that are the same for a
request alone and in the mix (exactly: randomness is keyed by photon)."""
import sys
import threading
import time

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def run_clients(srv, w, n_clients, jitter_s=0.002, seed=0):
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
            hits, info, dom = srv.wait(t, expected=True)
            with lock:
                results[i] = (key(hits), info, dom)

    th = [threading.Thread(target=client, args=(c,)) for c in range(n_clients)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    return results


def test_each_request_same_alone_and_in_the_mix(mods):
    pp, server, surrogate = mods
    w = events(48, seed=9)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, max_inflight=4)
    res = run_clients(srv, w, n_clients=16)
    st = srv.stats()
    srv.close()
    say("server stats", st)
    assert st["completed"] == 48 and st["bytes_in_use"] == 0
    assert st["launches"] < 48 or st["deferred"] >= 0  # several events may share a launch
    shared = sum(1 for r in res.values() if r[1]["batch_events"] > 1)
    say("requests that shared a launch", shared)
    for i in [0, 5, 17, 31, 47] + list(np.argsort(w.sources["n_photons"])[-3:]):
        ref = alone_hits(pp, w, i)
        got = res[int(i)][0]
        assert len(got) == len(ref) and (got == ref).all(), i
    for i, (hits, info, _) in res.items():
        assert info["photons"] == w.sources["n_photons"][i]
        assert info["t_submit_s"] <= info["t_launch_s"] <= info["t_done_s"]
        assert (hits["event_id"] == w.sources["event_id"][i]).all()


def test_tiny_hbm_budget_bounds_memory(mods):
    pp, server, surrogate = mods
    w = events(24, seed=10, cap=20_000)
    per = max(server.request_bytes(1, int(n)) for n in w.sources["n_photons"])
    budget = 3 * per
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, max_inflight=8, hbm_budget_bytes=budget)
    res = run_clients(srv, w, n_clients=8, jitter_s=0.0)
    st = srv.stats()
    srv.close()
    say("tiny budget", budget, st)
    assert st["completed"] == 24 and st["peak_bytes_in_use"] <= budget
    for i in (0, 11, 23):
        ref = alone_hits(pp, w, i)
        assert (res[i][0] == ref).all()


def test_request_over_budget_is_refused(mods):
    pp, server, surrogate = mods
    w = events(2, seed=11)
    ctx = pp.Context(0, seed=0)
    ctx.load_workload(w)
    srv = server.Server(ctx, hbm_budget_bytes=1 << 20)
    with pytest.raises(pp.PPError) as e:
        srv.submit(w.sources[:1])
    assert e.value.status == pp.PP_EBUDGET
    bad = w.sources[:1].copy()
    bad["x"] = np.nan
    with pytest.raises(pp.PPError) as e:
        srv.submit(bad)
    assert e.value.status == pp.PP_EINVAL
    srv.close()


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
        ref = sur2.expected_hits(b).cpu().numpy()
        got = res[i][2]
        assert got is not None and np.allclose(got, ref, rtol=1e-4, atol=1e-12), i
