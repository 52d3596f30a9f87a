"""The polynomial GELU of the surrogate kernels: the coefficients written in
sur_kernels.hip are the ones gelu_poly.py derives, and their FP32 evaluation
stays within 3.4e-6 of GELU(z) = z Phi(z) (scipy's erf) for every z,
including the switch to the linear tail at |z| = 5 (there the polynomial's
value at the clamp and FP32 rounding at |z| up to 12 set the bound)."""
import importlib.util
import os
import re

import numpy as np
from scipy import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_05700_amd", "csrc")


def load_generator():
    spec = importlib.util.spec_from_file_location("gelu_poly", os.path.join(CSRC, "gelu_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def kernel_coefficients():
    src = open(os.path.join(CSRC, "sur_kernels.hip")).read()
    body = src[src.index("__device__ __forceinline__ float gelu(float z) {"):]
    body = body[:body.index("h = __builtin_fmaf(0.5f, fmaxf(")]
    first = re.search(r"float h = (-?[0-9.e-]+)f;", body).group(1)
    rest = re.findall(r"h = __builtin_fmaf\(h, x, (-?[0-9.e-]+)f\);", body)
    return np.array([float(first)] + [float(v) for v in rest], np.float32)  # highest degree first


def test_kernel_coefficients_are_the_generated_ones():
    g = load_generator()
    want = np.asarray(g.coefficients(), np.float64)[::-1].astype(np.float32)
    got = kernel_coefficients()
    assert len(got) == g.DEGREE + 1
    assert np.array_equal(got, want)


def test_fp32_gelu_error_bound():
    g = load_generator()
    coef = kernel_coefficients()[::-1].astype(np.float64)
    z = np.concatenate([np.linspace(-12.0, 12.0, 2_400_001), [-5.0, 5.0, np.nextafter(5.0, 9), -np.nextafter(5.0, 9)]])
    exact = 0.5 * z * (1.0 + special.erf(z / np.sqrt(2.0)))
    err = np.abs(g.gelu_f32(z, coef).astype(np.float64) - exact)
    assert err.max() <= 3.4e-6
    # relative accuracy where the activation is not tiny: 2^-12, an eighth of
    # the bf16 rounding (2^-9) the stored activation then takes
    big = np.abs(exact) > 1e-2
    assert (err[big] / np.abs(exact[big])).max() < 2.0 ** -12
