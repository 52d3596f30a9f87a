"""The oracle's pins must catch plausible mistakes: each mutant below is the
oracle with one planted error (a dropped term, a flipped sign, a wrong
index or operand), built to its own library and run against the pin suites
on the CPU. Every mutant must fail at least one pin.

One mistake is knowingly absent: drawing the wavelength from 1 - u instead
of u leaves every distribution unchanged, so only the GPU's photon-by-photon
parity can see it."""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

MUTANTS = [
    ("dropped scattering-budget decrement at a crossing",
     "tau_s = std::max(0.0, tau_s - b * d_bnd);", "tau_s = std::max(0.0, tau_s);"),
    ("dropped absorption-budget decrement at a crossing",
     "ph.tau_a = std::max(0.0, ph.tau_a - a * d_bnd);", "ph.tau_a = std::max(0.0, ph.tau_a);"),
    ("dropped absorption-budget decrement at a scatter",
     "ph.tau_a = std::max(0.0, ph.tau_a - a * d_sca);", "ph.tau_a = std::max(0.0, ph.tau_a);"),
    ("Henyey-Greenstein sign",
     "return (1.0 - g) * (1.0 - u) * (s + 1.0 - g) / w;", "return (1.0 + g) * (1.0 - u) * (s + 1.0 - g) / w;"),
    ("basis vector sign", "*e2 = {b, sign + n.y * n.y * a, -n.y};", "*e2 = {b, sign + n.y * n.y * a, n.y};"),
    ("upper boundary off by one layer",
     "(ice.z_lo + (i + 1) * ice.dz - zc) / ph.v.z", "(ice.z_lo + (i + 2) * ice.dz - zc) / ph.v.z"),
    ("exit root of the sphere instead of the entry",
     "const double t = -b - std::sqrt(disc);", "const double t = -b + std::sqrt(disc);"),
    ("group index missing from the time",
     "const double time_per_m = ice.n_group / kLightSpeed;", "const double time_per_m = 1.0 / kLightSpeed;"),
    ("tie goes to the higher module id",
     "(t == h->best_t && id < h->best_id)", "(t == h->best_t && id > h->best_id)"),
    ("Philox key words swapped", "uint32_t k0 = key[0], k1 = key[1];", "uint32_t k0 = key[1], k1 = key[0];"),
    ("travel time along the track dropped", "ph.t = s.t0 + sdist / kLightSpeed;", "ph.t = s.t0;"),
    ("scattering angle from the azimuth's word",
     "hg_one_minus_mu(ice.g[ph.layer], uniform(w[1]))", "hg_one_minus_mu(ice.g[ph.layer], uniform(w[2]))"),
    ("wavelength exponent of absorption with the wrong sign",
     "std::pow(ph.lambda / ice.lambda_ref, -ice.kappa_abs)", "std::pow(ph.lambda / ice.lambda_ref, ice.kappa_abs)"),
    ("absorption exponent used for scattering",
     "std::pow(ph.lambda / ice.lambda_ref, -ice.kappa_scat)", "std::pow(ph.lambda / ice.lambda_ref, -ice.kappa_abs)"),
    ("outward normal in the cosine of incidence",
     "std::max(-dot(ph.v, n), 0.0)", "std::max(dot(ph.v, n), 0.0)"),
    ("acceptance interpolation weights swapped",
     "A = acc.table[k] * (1.0 - f) + acc.table[k + 1] * f;", "A = acc.table[k] * f + acc.table[k + 1] * (1.0 - f);"),
]


def run_mutant(tmp, i, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    path = os.path.join(tmp, f"mutant{i}.cpp")
    lib = os.path.join(tmp, f"mutant{i}.so")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread", path,
                           "-o", lib])
    env = dict(os.environ, PP_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-k", "not rocrand",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_chromatic.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin(tmp_path):
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(lambda a: run_mutant(str(tmp_path), *a),
                                [(i, *m) for i, m in enumerate(MUTANTS)]))
    missed = [name for name, rc in results if rc == 0]
    assert not missed, f"mutants no pin caught: {missed}"
