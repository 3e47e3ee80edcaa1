"""PCA of the exemplar neighbourhoods (oracle, FP64).  Test infra only.

Methodology 2.2: before the search tree is built, PCA reduces the dimension
of the neighbourhood vectors (the paper keeps 95 % of the variance; for 8x8
RGBS neighbourhoods 256 dimensions drop to about 20-45).

Definitions used:
  mu = mean of the N exemplar vectors,
  C  = (1/N) sum_e (z_e - mu)(z_e - mu)^T,
  eigenpairs of C sorted by descending eigenvalue (numpy.linalg.eigh),
  B  = the first d eigenvectors as columns, each with its largest-magnitude
       entry made positive (ties to the lowest index) - a sign convention,
       since an eigenvector's sign is free,
  z' = B^T (z - mu),  x' = B^T (x - mu),
  retained variance = sum_{k<d} lambda_k / trace C.
"""
from __future__ import annotations

import numpy as np


def covariance(Z: np.ndarray):
    Z = np.asarray(Z, dtype=np.float64)
    mu = Z.mean(axis=0)
    A = Z - mu
    return mu, (A.T @ A) / Z.shape[0]


def canonical_signs(B: np.ndarray) -> np.ndarray:
    B = B.copy()
    for j in range(B.shape[1]):
        i = int(np.argmax(np.abs(B[:, j])))
        if B[i, j] < 0:
            B[:, j] = -B[:, j]
    return B


def basis(Z: np.ndarray, d: int = 0, variance_target: float = 0.95):
    """Return (mu [D], B [D][d], eigenvalues [D] descending, retained).

    ``d = 0`` picks the smallest d whose retained variance reaches
    ``variance_target`` (the paper's 95 % rule).
    """
    mu, C = covariance(Z)
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    V = V[:, order]
    tr = np.trace(C)
    if d <= 0:
        frac = np.cumsum(lam) / tr if tr > 0 else np.ones_like(lam)
        d = int(np.searchsorted(frac, variance_target - 1e-12) + 1)
        d = min(d, lam.size)
    B = canonical_signs(V[:, :d])
    retained = float(lam[:d].sum() / tr) if tr > 0 else 1.0
    return mu, B, lam, retained


def project(V: np.ndarray, mu: np.ndarray, B: np.ndarray) -> np.ndarray:
    return (np.asarray(V, dtype=np.float64) - mu) @ B
