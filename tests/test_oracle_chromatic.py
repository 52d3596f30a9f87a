"""Pins of the oracle's wavelength-dependent optics and hit acceptance
against closed forms.

Reading: the layer table holds the coefficients at a reference wavelength;
a photon of wavelength l sees a (l / l_ref)^-kappa_abs and
b (l / l_ref)^-kappa_scat (g unchanged). A hit's weight is a tabulated
acceptance at l (linear between table points) times a polynomial in the
cosine of incidence on the module surface. With no scattering the path to
absorption is exponential with mean 1 / a(l); with no absorption the first
step is exponential with mean 1 / b(l). A sphere lit by a distant point
source is hit uniformly over its cross-section, so the cosine of incidence
c = sqrt(1 - rho^2) (rho^2 uniform on [0, 1]) has mean 2/3.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import pyoracle
from paper_2405_05700_amd import workloads as W


def homogeneous(n, abs_len, eff_scat_len, wavelength, radius=W.DOM_RADIUS_M):
    w = W.tiny_point_source(n, dom_radius_m=radius, abs_len_m=abs_len, eff_scat_len_m=eff_scat_len)
    src = w.sources.copy()
    src["lambda_min_nm"] = src["lambda_max_nm"] = wavelength
    return w.with_sources(src)


def test_absorption_length_scales_with_wavelength():
    w = homogeneous(20_000, 50.0, np.inf, 600.0)
    w = W.dataclasses.replace(w, chromatic=(400.0, 1.5, 0.0))
    r = pyoracle.run(w, dom_mode=1)
    mean = 50.0 * (600.0 / 400.0) ** 1.5  # 1 / a(l)
    ab = r.fate == pyoracle.FATE_ABSORBED
    d = np.linalg.norm(r.pos[ab], axis=1)
    assert ab.mean() > 0.99
    assert abs(d.mean() / mean - 1) < 0.03
    assert stats.kstest(d / mean, "expon").pvalue > 1e-3


def test_scattering_length_scales_with_wavelength():
    w = homogeneous(20_000, np.inf, 25.0, 300.0)
    w = W.dataclasses.replace(w, chromatic=(400.0, 0.0, 2.0))
    r = pyoracle.run(w, step_cap=1, dom_mode=1)
    mean = 25.0 * (1 - 0.9) * (300.0 / 400.0) ** 2.0  # 1 / b(l), b = 1 / (lambda_e (1 - g))
    first = r.fate == pyoracle.FATE_CAPPED
    d = np.linalg.norm(r.pos[first], axis=1)
    assert abs(d.mean() / mean - 1) < 0.03
    assert stats.kstest(d / mean, "expon").pvalue > 1e-3


def test_zero_exponents_change_nothing():
    w = W.tiny_point_source(5_000)
    src = w.sources.copy()
    src["lambda_min_nm"], src["lambda_max_nm"] = 300.0, 600.0
    w = w.with_sources(src)
    a = pyoracle.run(w, dom_mode=1)
    b = pyoracle.run(W.dataclasses.replace(w, chromatic=(400.0, 0.0, 0.0)), dom_mode=1)
    assert (a.rec_u == b.rec_u).all() and (a.rec_f == b.rec_f).all()


@pytest.fixture(scope="module")
def beam():
    """Clear ice (no absorption, no scattering), 405 nm, r = 1 m modules 30 m
    and more from the source: every module sees a nearly parallel beam."""
    return homogeneous(3_000_000, np.inf, np.inf, 405.0, radius=1.0)


def test_cosine_acceptance_of_a_lit_sphere(beam):
    w = W.dataclasses.replace(beam, acceptance={"l0": 300.0, "dl": 300.0, "table": [1.0], "poly": [0.0, 1.0]})
    r = pyoracle.run(w, dom_mode=1, threads=8)
    hit = r.fate == pyoracle.FATE_HIT
    c = r.weight[hit]
    assert hit.sum() > 1500
    assert ((c >= 0) & (c <= 1)).all()
    sem = c.std() / math.sqrt(len(c))
    assert abs(c.mean() - 2.0 / 3.0) < 4 * sem + 1e-3
    # c^2 = 1 - rho^2 is uniform on [0, 1]
    assert stats.kstest(c ** 2, "uniform").pvalue > 1e-3
    assert (r.weight[~hit] == 1.0).all()


def test_acceptance_table_interpolates_in_wavelength(beam):
    w = W.dataclasses.replace(beam, acceptance={"l0": 300.0, "dl": 150.0, "table": [1.0, 3.0, 0.5],
                                                "poly": [1.0]})
    r = pyoracle.run(w, sel_src=np.zeros(200_000, np.uint64), sel_local=np.arange(200_000, dtype=np.uint64),
                     dom_mode=1)
    hit = r.fate == pyoracle.FATE_HIT
    assert hit.any()
    # 405 nm lies 0.7 of the way from the first table point to the second
    assert np.allclose(r.weight[hit], 1.0 * 0.3 + 3.0 * 0.7, rtol=1e-12)
