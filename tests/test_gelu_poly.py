"""The polynomial normal CDF that the matrix-core MLP inference uses for
GELU: its coefficients in the kernel source, evaluated in FP32 exactly as
the kernel does, stay within 5e-6 of Phi(x) = (1 + erf(x / sqrt 2)) / 2."""
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
    rest = [float(v) for v in re.findall(r"p = fmaf\(p, t, ([-0-9.e]+)f\);", body)]
    return [first] + rest  # highest degree first


def test_phi_polynomial_error_bound():
    coef = [np.float32(v) for v in _coefficients()]
    assert len(coef) == 11
    c = np.float32(4.5)
    a = np.float32(2.0) / (c * c)
    xs = np.linspace(-9, 9, 900001).astype(np.float32)
    xc = np.clip(xs, -c, c)
    t = (xc * xc * a - np.float32(1)).astype(np.float32)
    p = np.full_like(xs, coef[0])
    for v in coef[1:]:
        p = (p * t + v).astype(np.float32)
    phi = (xc * p + np.float32(0.5)).astype(np.float32)
    ref = 0.5 * (1.0 + erf(xs.astype(np.float64) / np.sqrt(2.0)))
    assert np.abs(phi - ref).max() <= 5e-6
    # GELU itself: x Phi(x) against x Phi_exact(x), absolute, on the range activations take
    g = xs.astype(np.float64) * phi
    assert np.abs(g - xs * ref)[np.abs(xs) <= 8].max() <= 4e-5
