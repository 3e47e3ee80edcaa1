"""Coefficients of the normal-CDF polynomial used by the matrix-core MLP
inference (GELU(x) = x Phi(x)).

Phi(x) = 1/2 + x P(t) for |x| <= c, with t = 2 x^2 / c^2 - 1 in [-1, 1] and
P of degree 10 in t, fitted to (Phi(x) - 1/2) / x by iteratively reweighted
least squares (Lawson's algorithm, which converges to the minimax fit) on
Chebyshev nodes; |x| > c is clamped to c.  With c = 4.5 the FP32 evaluation
(Horner in t) stays within 3e-6 of Phi everywhere - far below the bf16
rounding of the activations it feeds.  Run to print the coefficients.
"""
import numpy as np
from numpy.polynomial import chebyshev as C
from scipy.special import erf


def fit(c=4.5, deg=10, iters=80):
    x = np.cos(np.pi * (np.arange(8000) + 0.5) / 8000) * c
    x = x[x > 1e-6]
    x = np.concatenate([x, np.linspace(1e-4, c, 40000)])
    t = 2 * x * x / (c * c) - 1
    V = C.chebvander(t, deg) * x[:, None]
    y = 0.5 * erf(x / np.sqrt(2))
    w = np.ones_like(x)
    for _ in range(iters):
        cc, *_ = np.linalg.lstsq(V * np.sqrt(w)[:, None], y * np.sqrt(w), rcond=None)
        e = np.abs(V @ cc - y)
        w = np.maximum(w * e / (w * e).mean(), 1e-12)
    return C.cheb2poly(cc)


def max_error_fp32(pt, c=4.5):
    xs = np.linspace(-8, 8, 1600001).astype(np.float32)
    xc = np.clip(xs, -c, c).astype(np.float32)
    tt = (xc * xc * np.float32(2 / (c * c)) - np.float32(1)).astype(np.float32)
    p = np.full_like(xs, np.float32(pt[-1]))
    for k in range(len(pt) - 2, -1, -1):
        p = (p * tt + np.float32(pt[k])).astype(np.float32)
    phi = (np.float32(0.5) + xc * p).astype(np.float32)
    return float(np.abs(phi - 0.5 * (1 + erf(xs.astype(np.float64) / np.sqrt(2)))).max())


if __name__ == "__main__":
    pt = fit()
    print("coefficients (t^0 .. t^10):", ", ".join("%.9ef" % v for v in pt.astype(np.float32)))
    print("max |error| of the FP32 evaluation: %.2e" % max_error_fp32(pt))
