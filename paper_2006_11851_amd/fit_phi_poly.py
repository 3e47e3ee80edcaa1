"""Coefficients of the normal-CDF polynomial used by the matrix-core MLP
inference (GELU(x) = x Phi(x)).

Phi(x) = 1/2 + x P(x^2) for |x| <= c, |x| > c clamped to c.  P is fitted in
t = 2 x^2 / c^2 - 1 (Chebyshev basis, well conditioned) to (Phi(x) - 1/2) / x
by iteratively reweighted least squares (Lawson's algorithm, which converges
to the minimax fit) on Chebyshev nodes, then rewritten as a polynomial in
u = x^2, which the kernel evaluates by Horner's rule (one operation fewer
than going through t).  With c = 4 and degree 7 the FP32 evaluation stays
within 5.3e-5 of Phi and GELU within 4.2e-4 for |x| <= 8; wherever
|GELU| >= 0.05 its relative error is below a quarter of the bf16 half-unit
that rounds the activations it feeds.  Run to print the coefficients.
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


def to_u(pt, c):
    """P(t) with t = 2 u / c^2 - 1 as a polynomial in u (coefficients u^0 ..)."""
    a = 2.0 / (c * c)
    res, powk = np.zeros(1), np.array([1.0])
    for ck in pt:
        res = np.polynomial.polynomial.polyadd(res, ck * powk)
        powk = np.polynomial.polynomial.polymul(powk, np.array([-1.0, a]))
    return res


def max_error_fp32_u(pu, c):
    """(max |Phi error|, max |GELU error| for |x| <= 8) of the FP32 u-form evaluation."""
    cu = np.asarray(pu, dtype=np.float32)
    xs = np.linspace(-9, 9, 1800001).astype(np.float32)
    xc = np.clip(xs, -np.float32(c), np.float32(c))
    u = (xc * xc).astype(np.float32)
    p = np.full_like(xs, cu[-1])
    for v in cu[-2::-1]:
        p = (p * u + v).astype(np.float32)
    phi = (xc * p + np.float32(0.5)).astype(np.float32)
    ref = 0.5 * (1 + erf(xs.astype(np.float64) / np.sqrt(2)))
    g = np.abs(xs.astype(np.float64) * phi - xs * ref)[np.abs(xs) <= 8]
    return float(np.abs(phi - ref).max()), float(g.max())


if __name__ == "__main__":
    C_CLAMP, DEG = 4.0, 7
    pu = to_u(fit(c=C_CLAMP, deg=DEG), C_CLAMP)
    print("coefficients (u^0 .. u^%d):" % DEG, ", ".join("%.9ef" % v for v in pu.astype(np.float32)))
    print("max |error| of the FP32 evaluation: Phi %.2e, GELU %.2e" % max_error_fp32_u(pu, C_CLAMP))
