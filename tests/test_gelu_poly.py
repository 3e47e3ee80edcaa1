"""The polynomial normal CDF that the matrix-core MLP inference uses for
GELU: its coefficients in the kernel source, evaluated in FP32 exactly as
the kernel does (Phi(x) = 1/2 + x P(x^2), |x| clamped to 4, Horner in x^2),
stay within 6e-5 of Phi(x) = (1 + erf(x / sqrt 2)) / 2, GELU within 5e-4 of
x Phi(x) for |x| <= 8, and within 2^-10 relative wherever |GELU| >= 0.05
(half the bf16 half-unit that rounds the activation next)."""
import os
import re

import numpy as np
from scipy.special import erf

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2006_11851_amd", "csrc", "k_mlp.hip")


def _coefficients():
    s = open(SRC).read()
    body = s[s.index("float gelu_poly_f(float x)"):]
    body = body[: body.index("return")]
    first = float(re.search(r"float p = ([-0-9.e]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fmaf\(p, u, ([-0-9.e]+)f\);", body)]
    c = float(re.search(r"constexpr float c = ([0-9.]+)f;", body).group(1))
    return [first] + rest, c  # highest degree first


def test_phi_polynomial_error_bound():
    coef, c = _coefficients()
    coef = [np.float32(v) for v in coef]
    assert len(coef) == 8 and c == 4.0
    xs = np.linspace(-9, 9, 900001).astype(np.float32)
    xc = np.clip(xs, -np.float32(c), np.float32(c))
    u = (xc * xc).astype(np.float32)
    p = np.full_like(xs, coef[0])
    for v in coef[1:]:
        p = (p * u + v).astype(np.float32)
    phi = (xc * p + np.float32(0.5)).astype(np.float32)
    ref = 0.5 * (1.0 + erf(xs.astype(np.float64) / np.sqrt(2.0)))
    assert np.abs(phi - ref).max() <= 6e-5
    # GELU itself: x Phi(x) against x Phi_exact(x), absolute, on the range activations take
    g = xs.astype(np.float64) * phi
    assert np.abs(g - xs * ref)[np.abs(xs) <= 8].max() <= 5e-4
    # and, where the activation is not tiny, below half the bf16 half-unit
    # (2^-9 relative) that rounds it next
    big = np.abs(xs * ref) >= 0.05
    rel = np.abs(g - xs * ref)[big] / np.abs(xs * ref)[big]
    assert rel.max() <= 2.0 ** -10
