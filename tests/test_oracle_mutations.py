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


# Mistakes planted in the surrogate's oracle (oracle/mlp_oracle.py). Where a
# mistake would be made the same way in a value and its derivative, both are
# planted, so the finite-difference pins alone cannot see it.
MLP_MUTANTS = [
    ("sign of (kappa - 1) sum log delay, in the loss and its gradient",
     [("- (kappa - 1.0) * s2 + s1 / theta", "+ (kappa - 1.0) * s2 + s1 / theta"),
      ("np.log(theta)) - s2) / P", "np.log(theta)) + s2) / P")]),
    ("gamma scale used as a rate, in the loss and its gradient",
     [("n_t * (special.gammaln(kappa) + kappa * np.log(theta)) - (kappa - 1.0) * s2 + s1 / theta",
       "n_t * (special.gammaln(kappa) - kappa * np.log(theta)) - (kappa - 1.0) * s2 + s1 * theta"),
      ("(n_t * (special.digamma(kappa) + np.log(theta)) - s2)", "(n_t * (special.digamma(kappa) - np.log(theta)) - s2)"),
      ("(n_t * kappa - s1 / theta)", "(-n_t * kappa + s1 * theta)")]),
    ("sign of k log mu, in the loss and its gradient",
     [("poisson = mu - k * np.log(mu)", "poisson = mu + k * np.log(mu)"), ("w * (mu - k) / P", "w * (mu + k) / P")]),
    ("lgamma(kappa) dropped, in the loss and its gradient",
     [("special.gammaln(kappa) + kappa * np.log(theta)", "kappa * np.log(theta)"),
      ("special.digamma(kappa) + np.log(theta)", "np.log(theta)")]),
    ("diffusion constant lambda_e instead of lambda_e / 3", [("D = lam_e / 3.0", "D = lam_e")]),
    ("diffusion length without D", [("dl = np.sqrt(D * lam_a)", "dl = np.sqrt(lam_e * lam_a)")]),
    ("module radius instead of its square in the baseline",
     [("mu_base = r * r * np.exp(-R / dl)", "mu_base = r * np.exp(-R / dl)")]),
    ("GELU with erf(z / 2), and its derivative",
     [("special.erf(z / math.sqrt(2.0))", "special.erf(z / 2.0)"),
      ("z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)", "z * np.exp(-0.25 * z * z) / (2.0 * math.sqrt(math.pi))")]),
    ("Adam bias correction of v with beta1", [("c2 = 1.0 - self.b2 ** self.t", "c2 = 1.0 - self.b1 ** self.t")]),
    ("neighbouring scattering feature without (1 - g)",
     [("X[:, 22 + 2 * q] = 10.0 / (le_all[li] * (1.0 - g_all[li]))", "X[:, 22 + 2 * q] = 10.0 / le_all[li]")]),
    ("Cherenkov emission point with tan instead of 1/tan",
     [("(along - b / TAN_CHERENKOV) / L", "(along - b * TAN_CHERENKOV) / L")]),
    ("GELU derivative dropped from the backward pass", [("g = (g @ W) * gelu_grad(pre[li - 1])", "g = (g @ W)")]),
    ("weighted loss normalised by the weight sum",
     [("loss = (w * (poisson + TIME_WEIGHT * gam)).sum() / P", "loss = (w * (poisson + TIME_WEIGHT * gam)).sum() / w.sum()")]),
    ("far pairs kept with weight 1", [("np.where(near, 1.0, float(far_stride))", "np.where(near, 1.0, 1.0)")]),
]
MLP_SRC = os.path.join(ROOT, "oracle", "mlp_oracle.py")


def run_mlp_mutant(tmp, i, name, edits):
    src = open(MLP_SRC).read()
    for old, new in edits:
        assert old in src, f"mutation site missing: {name}: {old}"
        src = src.replace(old, new)
    path = os.path.join(tmp, f"mlp_mutant{i}.py")
    with open(path, "w") as f:
        f.write(src)
    env = dict(os.environ, PP_MLP_ORACLE=path)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_mlp_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_surrogate_oracle_mistake_fails_a_pin(tmp_path):
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(lambda a: run_mlp_mutant(str(tmp_path), *a),
                                [(i, *m) for i, m in enumerate(MLP_MUTANTS)]))
    missed = [name for name, rc in results if rc == 0]
    assert not missed, f"surrogate-oracle mutants no pin caught: {missed}"


def test_every_planted_mistake_fails_a_pin(tmp_path):
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(lambda a: run_mutant(str(tmp_path), *a),
                                [(i, *m) for i, m in enumerate(MUTANTS)]))
    missed = [name for name, rc in results if rc == 0]
    assert not missed, f"mutants no pin caught: {missed}"
