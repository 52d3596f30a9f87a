"""Host-side input generators: the training-target selection of the
surrogate recipe."""
import dataclasses

import numpy as np

from paper_2405_05700_amd import workloads as W


def test_structured_modules_follow_the_optics():
    det = W.full_detector(n_sources=1, photons_per_source=1)
    # homogeneous ice: nothing is structured
    flat = det.layers.copy()
    flat["abs_len_m"], flat["eff_scat_len_m"] = 100.0, 25.0
    assert len(W.structured_modules(dataclasses.replace(det, layers=flat))) == 0
    # one layer with twice the absorption: exactly the modules whose
    # +-30 m window reaches into it (sampled every half layer)
    one = flat.copy()
    k = 90
    one["abs_len_m"][k] = 50.0
    lo, hi = det.z_lo_m + det.dz_m * k, det.z_lo_m + det.dz_m * (k + 1)
    got = W.structured_modules(dataclasses.replace(det, layers=one))
    z = det.doms["z"].astype(float)
    offs = np.arange(-30.0, 30.0 + 1e-9, 5.0)
    reach = ((z[:, None] + offs[None, :] >= lo) & (z[:, None] + offs[None, :] < hi)).any(1)
    assert np.array_equal(np.sort(got), np.nonzero(reach)[0])
    # the full-detector ice: the modules in and around the dust layer
    hard = W.structured_modules(det)
    assert 500 < len(hard) < 1500
    dust_z = 1950.0 - 2000.0
    assert np.abs(z[hard] - dust_z).max() < 100.0


def test_training_targets_mix():
    det = W.full_detector(n_sources=1, photons_per_source=1)
    hard = W.structured_modules(det)
    t = W.training_targets(det, 20000, 0.4, seed=3)
    assert len(t) == 20000 and t.min() >= 0 and t.max() < len(det.doms)
    # 40% drawn from the structured set plus their share of the uniform 60%
    expect = 0.4 + 0.6 * len(hard) / len(det.doms)
    assert abs(np.isin(t, hard).mean() - expect) < 0.02
    assert np.array_equal(t, W.training_targets(det, 20000, 0.4, seed=3))
    assert np.isin(W.training_targets(det, 1000, 0.0, seed=1), hard).mean() < 0.3
