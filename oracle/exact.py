"""Exhaustive nearest-neighbourhood search (oracle, FP64).  Test infra only.

Methodology 2.1, Eq. 4: z_p is the exemplar neighbourhood most similar to
x_p under the Euclidean norm.  The plain definition is written out:
e*(q) = argmin_e ||x_q - z_e||^2 over every exemplar window, ties going to
the lowest e (the paper is silent on ties; this is the reading used).

``topk_direct`` evaluates sum_k (x_k - z_k)^2 literally.  ``topk`` gets the
same answer faster: it ranks with the expanded form
||x||^2 + ||z||^2 - 2 x.z (one BLAS product), then recomputes in the direct
form every candidate whose expanded value lies within the expansion's
rounding bound of the k-th smallest, so the returned set and order are those
of the direct form.
"""
from __future__ import annotations

import numpy as np

EPS64 = np.finfo(np.float64).eps


def _direct_d2(q: np.ndarray, Z: np.ndarray, idx: np.ndarray) -> np.ndarray:
    diff = Z[idx] - q[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def topk_direct(Q: np.ndarray, Z: np.ndarray, k: int = 1, block: int = 0, offset=None):
    """Exact k nearest (squared distance, id) per query by the direct form.

    ``offset`` (optional, [N]) is added to every exemplar's squared distance
    before ranking.  Returns (ids int64 [nq][k], d2 float64 [nq][k]) sorted by
    (d2, id).
    """
    Q = np.asarray(Q, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nq, D = Q.shape
    N = Z.shape[0]
    k = min(k, N)
    if block <= 0:
        block = max(1, int(2e7 // max(1, N)))
    ids = np.empty((nq, k), dtype=np.int64)
    d2s = np.empty((nq, k), dtype=np.float64)
    for b0 in range(0, nq, block):
        Qb = Q[b0 : b0 + block]
        acc = np.zeros((Qb.shape[0], N), dtype=np.float64)
        for c in range(D):
            t = Qb[:, c][:, None] - Z[:, c][None, :]
            acc += t * t
        if offset is not None:
            acc += np.asarray(offset, dtype=np.float64)[None, :]
        # lexicographic (d2, id): stable sort on d2 keeps ids ascending
        order = np.argsort(acc, axis=1, kind="stable")[:, :k]
        ids[b0 : b0 + block] = order
        d2s[b0 : b0 + block] = np.take_along_axis(acc, order, axis=1)
    return ids, d2s


def topk(Q: np.ndarray, Z: np.ndarray, k: int = 1, block: int = 0, offset=None):
    """Same result as :func:`topk_direct`, using a proven-safe BLAS prefilter."""
    Q = np.asarray(Q, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nq, D = Q.shape
    N = Z.shape[0]
    k = min(k, N)
    zn = np.einsum("ij,ij->i", Z, Z)
    zmax = zn.max() if N else 0.0
    off = np.zeros(N) if offset is None else np.asarray(offset, dtype=np.float64)
    if block <= 0:
        block = max(1, int(1.6e7 // max(1, N)))
    # |expanded - direct| <= gamma * (||q||^2 + ||z||^2), gamma = (D + 4) eps
    gamma = (D + 4) * EPS64
    ids = np.empty((nq, k), dtype=np.int64)
    d2s = np.empty((nq, k), dtype=np.float64)
    for b0 in range(0, nq, block):
        Qb = Q[b0 : b0 + block]
        qn = np.einsum("ij,ij->i", Qb, Qb)
        dexp = qn[:, None] + zn[None, :] - 2.0 * (Qb @ Z.T) + off[None, :]
        kth = np.partition(dexp, k - 1, axis=1)[:, k - 1]
        for r in range(Qb.shape[0]):
            bound = 2.0 * gamma * (qn[r] + zmax)
            cand = np.nonzero(dexp[r] <= kth[r] + 2.0 * bound)[0]
            d = _direct_d2(Qb[r], Z, cand) + off[cand]
            o = np.lexsort((cand, d))[:k]
            ids[b0 + r] = cand[o]
            d2s[b0 + r] = d[o]
    return ids, d2s


def exact_nn(Q: np.ndarray, Z: np.ndarray):
    """e*(q) and ||x_q - z_e*||^2 plus the runner-up squared distance."""
    ids, d2 = topk(Q, Z, k=2)
    runner = d2[:, 1] if d2.shape[1] > 1 else np.full(Q.shape[0], np.inf)
    return ids[:, 0], d2[:, 0], runner
