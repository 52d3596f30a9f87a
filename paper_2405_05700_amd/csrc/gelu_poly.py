"""Coefficients of the polynomial GELU used by the surrogate kernels
(sur_kernels.hip, gelu()). Run: python paper_2405_05700_amd/csrc/gelu_poly.py

GELU(z) = z Phi(z) = z / 2 + H(z^2) / 2 with H(u) = sqrt(u) erf(sqrt(u / 2)).
z erf(z / sqrt 2) is an even entire function of z, so H is an entire function
of u and a polynomial in u approximates it well on a bounded range; beyond
|z| = C, erf(|z| / sqrt 2) = 1 to within 6e-7 and H(u) = |z|: the kernel
clamps the polynomial's argument at u = C^2 and adds (|z| - C) / 2.

The fit is a least-squares Chebyshev fit of H(u) / 2 at 4 (degree + 1)
Chebyshev nodes of u in [0, C^2], written as
a power series in the centred variable x = u (2 / C^2) - 1, so the Horner
evaluation in FP32 is well conditioned (coefficients below 2). The script
prints the coefficients (highest degree first) and the maximum absolute error
of the FP32 evaluation against float64 GELU.
"""
from __future__ import annotations

import numpy as np
from scipy import special

C = 5.0
DEGREE = 12


def coefficients(c: float = C, degree: int = DEGREE) -> np.ndarray:
    """Power-series coefficients in x (lowest degree first)."""
    U = c * c
    x = np.cos(np.pi * (np.arange(4 * degree + 4) + 0.5) / (4 * degree + 4))
    u = (x + 1.0) * 0.5 * U
    h = np.sqrt(u) * special.erf(np.sqrt(u / 2.0))
    cheb = np.polynomial.chebyshev.Chebyshev.fit(x, 0.5 * h, degree, domain=[-1, 1])
    return cheb.convert(kind=np.polynomial.Polynomial).coef


def gelu_f32(z: np.ndarray, coef: np.ndarray, c: float = C) -> np.ndarray:
    """The kernel's evaluation order in float32, each fused multiply-add
    rounded once: x = min(fma(z z, 2 / C^2, -1), 1), Horner in x, then
    h += max(|z| - C, 0) / 2 and GELU = fma(1/2, z, h)."""
    z = np.asarray(z, np.float32)
    u = (z * z).astype(np.float32)
    x = np.minimum((u.astype(np.float64) * np.float32(2.0 / (c * c)) - 1.0).astype(np.float32), np.float32(1.0))
    acc = np.full_like(x, np.float32(coef[-1]))
    for k in coef[-2::-1]:
        acc = (acc.astype(np.float64) * x + np.float64(np.float32(k))).astype(np.float32)
    tail = np.maximum((np.abs(z) - np.float32(c)).astype(np.float32), np.float32(0.0))
    h = (0.5 * tail.astype(np.float64) + acc).astype(np.float32)
    return (z.astype(np.float64) * 0.5 + h).astype(np.float32)


def main():
    coef = coefficients()
    z = np.linspace(-10.0, 10.0, 2_000_001)
    exact = 0.5 * z * (1.0 + special.erf(z / np.sqrt(2.0)))
    err = np.abs(gelu_f32(z, coef).astype(np.float64) - exact)
    print(f"// degree {DEGREE}, |z| <= {C}: max |error| {err.max():.2e} (FP32 evaluation)")
    for k in coef[::-1]:
        print(f"    {np.float32(k)!r:>16}f,".replace("np.float32(", "").replace(")", ""))


if __name__ == "__main__":
    main()
