"""The table GELU of the surrogate kernels: the tables compiled into
sur_kernels.hip (gelu_cdf_table.h) are the ones gelu_table.py derives, their
nodes hold the standard normal CDF and the GELU derivative to float32
rounding, the training kernel's FP32 interpolation stays within 5.3e-6 of
GELU(z) = z Phi(z) (scipy's erf) for every z, and within 2^-12 relative
where |GELU| > 0.01 (an eighth of the bf16 rounding the stored activation
then takes), the inference kernel's float16 copy within 5.0e-4 relative
there (a quarter of it), and the derivative's within 1.4e-5 of
Phi(z) + z phi(z) (a seventeenth of the FP16 rounding it is then stored
with)."""
import importlib.util
import os
import re

import numpy as np
from scipy import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_05700_amd", "csrc")


def load_generator():
    spec = importlib.util.spec_from_file_location("gelu_table", os.path.join(CSRC, "gelu_table.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def compiled_tables():
    src = open(os.path.join(CSRC, "gelu_cdf_table.h")).read()
    cdf_src, grad_src = src.split("kGeluGradTable")
    pat = r"\{(-?[0-9.e+-]+)f, (-?[0-9.e+-]+)f\}"
    a = float(re.search(r"kCdfA = ([0-9.e+-]+)f", src).group(1))
    b = float(re.search(r"kCdfB = ([0-9.e+-]+)f", src).group(1))
    return (np.array(re.findall(pat, cdf_src), np.float64).astype(np.float32),
            np.array(re.findall(pat, grad_src), np.float64).astype(np.float32), np.float32(a), np.float32(b))


def compiled_table():
    tab, _, a, b = compiled_tables()
    return tab, a, b


def test_compiled_table_is_the_generated_one():
    g = load_generator()
    tab, grad, a, b = compiled_tables()
    assert tab.shape == (g.N + 1, 2) and grad.shape == (g.N + 1, 2)
    assert np.array_equal(tab, g.table())
    assert np.array_equal(grad, g.grad_table())
    assert (a, b) == g.mapping()


def test_nodes_hold_the_normal_cdf():
    g = load_generator()
    tab, a, b = compiled_table()
    z = (np.arange(g.N + 1) - np.float64(b)) / np.float64(a)
    phi = 0.5 * special.erfc(-z / np.sqrt(2.0))
    assert np.allclose(tab[:, 0], phi, rtol=2 ** -23, atol=1e-30)
    assert abs(z[0] + g.Z) < 1e-6 and abs(z[-1] - g.Z) < 1e-6
    assert tab[-1, 1] == 0.0 and (tab[:-1, 1] >= 0).all()


def test_fp32_interpolation_error_bound():
    g = load_generator()
    tab, _, _ = compiled_table()
    z = np.concatenate([np.linspace(-12.0, 12.0, 2_400_001), [-6.0, 6.0, 0.0, -1e-3, 1e-3]])
    exact = 0.5 * z * (1.0 + special.erf(z / np.sqrt(2.0)))
    err = np.abs(g.gelu_f32(z, tab).astype(np.float64) - exact)
    assert err.max() <= 5.3e-6
    big = np.abs(exact) > 1e-2
    assert (err[big] / np.abs(exact[big])).max() < 2.0 ** -12


def test_derivative_table():
    g = load_generator()
    _, grad, a, b = compiled_tables()
    zn = (np.arange(g.N + 1) - np.float64(b)) / np.float64(a)
    exact_n = 0.5 * special.erfc(-zn / np.sqrt(2.0)) + zn * np.exp(-0.5 * zn * zn) / np.sqrt(2.0 * np.pi)
    assert np.allclose(grad[:, 0], exact_n, rtol=2 ** -23, atol=1e-30)
    assert grad[-1, 1] == 0.0
    z = np.concatenate([np.linspace(-12.0, 12.0, 2_400_001), [-6.0, 6.0, 0.0, -0.7518, 0.8025]])
    zd = z.astype(np.float32).astype(np.float64)
    exact = 0.5 * special.erfc(-zd / np.sqrt(2.0)) + zd * np.exp(-0.5 * zd * zd) / np.sqrt(2.0 * np.pi)
    err = np.abs(g.interp_f32(z, grad).astype(np.float64) - exact)
    assert err.max() <= 1.4e-5


def compiled_half_table():
    src = open(os.path.join(CSRC, "gelu_cdf_table.h")).read()
    body = src[src.index("kCdfTableHalf"):src.index("kGeluGradTable")]
    return np.array([int(w, 16) for w in re.findall(r"0x([0-9a-f]{8})u", body)], np.uint32)


def test_half_table():
    g = load_generator()
    bits = compiled_half_table()
    t16 = g.half_table()
    assert bits.shape == (g.N + 1,)
    assert np.array_equal(bits, g.half_bits(t16))
    # the packed halves are the float64 values rounded once to float16
    lo = (bits & 0xFFFF).astype(np.uint16).view(np.float16)
    hi = (bits >> 16).astype(np.uint16).view(np.float16)
    a, b = g.mapping()
    zn = (np.arange(g.N + 1) - np.float64(b)) / np.float64(a)
    assert np.array_equal(lo, (0.5 * special.erfc(-zn / np.sqrt(2.0))).astype(np.float16))
    assert hi[-1] == 0
    z = np.concatenate([np.linspace(-12.0, 12.0, 2_400_001), [-6.0, 6.0, 0.0, -1e-3, 1e-3]])
    exact = 0.5 * z * (1.0 + special.erf(z / np.sqrt(2.0)))
    err = np.abs(g.gelu_half_f32(z, np.stack([lo, hi], 1)).astype(np.float64) - exact)
    assert err.max() <= 8.5e-4
    big = np.abs(exact) > 1e-2
    assert (err[big] / np.abs(exact[big])).max() < 5.0e-4
