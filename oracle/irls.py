"""Robust texture energy and IRLS weights (oracle, FP64).  Test infra only.

Methodology 2.1:
  Eq. 4   E_T = sum_p ||x_p - z_p||^2
  Eq. 5   E_T = sum_p ||x_p - z_p||^r with r = 0.8 (robust form)
  Eq. 6-8 IRLS: with W_p = ||x_p - z_p||^(r-2), E_T = sum_p W_p ||x_p - z_p||^2.

Reading where the paper is silent: at a zero distance W_p is undefined, so
the distance is floored at delta (1e-3 on the [0, 1] pixel scale),
W = max(d, delta)^(r-2), and the energy uses the matching smoothed penalty

  rho(d) = d^r                                          for d >= delta,
  rho(d) = (1 - r/2) delta^r + (r/2) delta^(r-2) d^2   for d <  delta,

which is continuous with a continuous first derivative at delta and is
concave in t = d^2; W equals (2/r) d rho / d t, so the IRLS step is a
majorise-minimise step of this energy.
"""
from __future__ import annotations

import numpy as np

R_DEFAULT = 0.8
DELTA_DEFAULT = 1e-3


def weights(d, r: float = R_DEFAULT, delta: float = DELTA_DEFAULT):
    d = np.asarray(d, dtype=np.float64)
    return np.maximum(d, delta) ** (r - 2.0)


def rho(d, r: float = R_DEFAULT, delta: float = DELTA_DEFAULT):
    d = np.asarray(d, dtype=np.float64)
    big = np.power(np.maximum(d, delta), r)
    small = (1.0 - r / 2.0) * delta**r + (r / 2.0) * delta ** (r - 2.0) * d * d
    return np.where(d >= delta, big, small)


def energy(d, r: float = R_DEFAULT, delta: float = DELTA_DEFAULT):
    """(E = sum rho(d_q), E2 = sum d_q^2), both float64."""
    d = np.asarray(d, dtype=np.float64)
    return float(rho(d, r, delta).sum()), float((d * d).sum())
