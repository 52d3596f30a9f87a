"""Surrogate+MC against plain Monte Carlo on the GPU, both executed
(paper_2405_05700_amd.hybrid.evaluate), at test scale: an ensemble of three
networks trained on 24 000 segments near modules (1e6 photons each, 60
epochs), one calibration set and one graded set of 40 clusters of four
segments, truth at 1e8 photons per segment.

What the trained network gains over the method without it: the merged
per-module answers reach the accuracy of plain Monte Carlo at its 2% target
(68.3% of modules within 2% of the truth, 95.4% within 4%, up to the
finite-sample slack below) in less device time than plain Monte Carlo takes.
The fallback decision reads only the ensemble; the truth only grades."""
import sys

import numpy as np
import pytest

from paper_2405_05700_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    from paper_2405_05700_amd import pp, surrogate
    det = W.full_detector(n_sources=1, photons_per_source=1)
    ctx = pp.Context(0, seed=7)
    ctx.load_workload(det)
    ctx.set_launch_config(hit_capacity=40_000_000)
    targets = W.training_targets(det, 24_000, 0.4, seed=77)
    tr = W.near_module_segments(det, 24_000, 1_000_000, seed=101, r_min=3.0, r_max=25.0, targets=targets)
    b = ctx.submit(tr)
    ctx.propagate(b)
    members = []
    for seed in (1, 2, 3):
        m = surrogate.Surrogate(ctx, seed=seed)
        m.set_sampling(150.0, 64)
        m.set_training_set(b)
        losses = m.train(epochs=60, batch_size=8192, lr=1e-3, lr_final=1e-5)
        say(f"network {seed}: epoch losses {losses[0]:.3f} -> {losses[-1]:.3f}")
        members.append(m)
    ctx.release(b)
    yield ctx, det, members
    for m in members:
        m.close()
    ctx.close()


def test_surrogate_plus_mc_beats_plain_mc_at_its_accuracy(trained):
    from paper_2405_05700_amd import hybrid
    ctx, det, members = trained
    r = hybrid.evaluate(ctx, det, members, n_sets=2, truth_photons=100_000_000, cut_m=300.0, log=say)
    acc = r["accuracy"]
    say(f"graded {r['graded_modules']}, threshold {r['fallback_spread_threshold']:.4f}, fallback "
        f"{r['fallback_modules']} modules in {r['clusters_with_mc']} clusters; times: surrogate "
        f"{r['t_surrogate_s']:.4f} s + fallback {r['t_fallback_mc_s']:.4f} s vs plain {r['t_plain_mc_s']:.4f} s "
        f"-> speed-up {r['speedup_at_2pct']:.2f}")
    say("accuracy", acc)
    assert r["graded_modules"] >= 40
    # the merged answers are as accurate as Monte Carlo at 2% (finite-sample slack: 0.1 and 0.05)
    assert acc["surrogate_plus_mc"]["within_2pct"] >= hybrid.WITHIN_2PCT - 0.1
    assert acc["surrogate_plus_mc"]["within_4pct"] >= hybrid.WITHIN_4PCT - 0.05
    # and plain Monte Carlo at its 2% target behaves as the statistics say
    assert acc["plain_mc"]["within_4pct"] >= hybrid.WITHIN_4PCT - 0.05
    assert r["speedup_at_2pct"] > 2.0
    assert r["plain_mc_photons"] > r["fallback_mc_photons"]
