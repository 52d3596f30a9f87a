"""Host logic of the surrogate+MC path (paper_2405_05700_amd/hybrid.py):
the fallback threshold, the Monte Carlo plan, and the merge, on small
hand-made arrays whose answers follow from the definitions."""
import numpy as np

from paper_2405_05700_amd import hybrid as H
from paper_2405_05700_amd import workloads as W


def test_threshold_keeps_the_largest_prefix_that_matches_monte_carlo():
    # spreads in order; the first three are within 2%, the last two far off
    spread = np.array([0.05, 0.01, 0.03, 0.02, 0.04])
    rel = np.array([0.10, 0.001, 0.015, 0.01, 0.10])
    # sorted: 0.01 ok, 0.02 ok, 0.03 ok, 0.04 bad, 0.05 bad; four of them are
    # 75% within 2% but only 75% within 4% (< 95.4%): three pass
    assert H.calibrate_threshold(spread, rel) == 0.04
    # everything good: no threshold
    assert H.calibrate_threshold(spread, np.zeros(5)) == np.inf
    # the smallest spread fails and no larger prefix recovers: nothing is accepted
    assert H.calibrate_threshold(np.array([0.01, 0.02]), np.array([0.5, 0.0])) == 0.0
    assert H.calibrate_threshold(np.array([0.01]), np.array([0.5])) == 0.0
    # 2 of 3 within 2% is below 68.3%, but all within 4%: only the first passes
    assert H.calibrate_threshold(np.array([0.1, 0.2, 0.3]), np.array([0.0, 0.03, 0.03])) == 0.2
    # coverage alone would accept all 40, but one of them is 12% off: the
    # threshold stops below it
    sp = np.arange(40) / 40.0
    rel = np.zeros(40)
    rel[30] = 0.12
    assert H.calibrate_threshold(sp, rel) == sp[30]


def test_spread_is_the_members_relative_standard_deviation():
    L = np.zeros((3, 2, 4))
    L[:, 0, 1] = [9.0, 10.0, 11.0]      # one cluster lights module 1
    L[:, 1, 1] = [1.0, 1.0, 1.0]        # and a second one adds a constant
    L[:, 0, 2] = [5.0, 5.0, 5.0]
    mean, spread = H.ensemble_spread(L)
    assert np.allclose(mean, [0.0, 11.0, 5.0, 0.0])
    assert np.isclose(spread[1], 1.0 / 11.0) and spread[2] == 0.0


def test_plan_sizes_each_cluster_for_its_dimmest_module():
    L = np.zeros((3, 6))
    L[0, [1, 2]] = [100.0, 50.0]   # cluster 0 lights modules 1 and 2
    L[1, 2] = 20.0                 # cluster 1 lights module 2 less than cluster 0 does
    L[2, [3, 4]] = [10.0, 1000.0]
    p = H.plan_mc(L, np.array([1, 2, 3, 4]), photons_ref=1e6, cap=1e12)
    # module 2 belongs to cluster 0 (50 > 20): photons for 2500 hits at 50 per 1e6
    assert p.photons[0] == 2500 * 1e6 / 50 and p.photons[1] == 0
    assert p.photons[2] == 2500 * 1e6 / 10
    assert sorted(p.modules) == [0, 2]
    assert H.plan_mc(L, np.array([3]), 1e6, cap=1e8).photons[2] == 1e8  # capped
    assert (H.plan_mc(L, np.array([], np.int64), 1e6, 1e9).photons == 0).all()


def test_plan_sources_and_merge():
    segs = np.zeros(6, W.SOURCE_DTYPE)
    segs["event_id"] = np.arange(6)
    segs["n_photons"] = 777
    cluster = np.arange(6) % 3
    plan = H.Plan(np.array([1000.0, 0.0, 4000.0]), {})
    src = H.plan_sources(segs, cluster, plan, first_index=10**9)
    assert src["event_id"].tolist() == [0, 2, 3, 5]
    assert src["n_photons"].tolist() == [1000, 4000, 1000, 4000]
    assert (src["first_photon_index"] == 10**9).all()
    # merge: cluster 0 and 2 ran (counts scaled to 1e6 photons per segment),
    # cluster 1 contributes the surrogate's expectation
    L = np.array([[5.0, 0.0], [7.0, 3.0], [0.0, 11.0]])
    counts = np.array([[20.0, 0.0], [999.0, 999.0], [0.0, 8.0]])
    est = H.merge(L, counts, plan, photons_ref=1e6, modules=np.array([0, 1]))
    assert np.allclose(est, [20.0 * 1e3 + 7.0, 3.0 + 8.0 * 250.0])
