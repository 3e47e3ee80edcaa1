"""Hierarchical k-means search tree (oracle, FP64).  Test infra only.

Methodology 2.2: starting at the root, k-means with k = 4 splits the
neighbourhoods held by a node into k children, and each child is split again
recursively; the paper stops when a node holds fewer than k neighbourhoods
(replacing the 1 % rule of the method it builds on).  The search runs in the
PCA-reduced space.  Here k is the ``branching`` argument; the recursion may
also stop at ``depth`` levels (``depth=None``: no cap, the paper's rule
alone), so that a node is a leaf at depth ``depth`` or when it holds fewer
than ``branching`` members.

Readings where the paper is silent:
* k-means++ seeding from one seeded PCG64 stream, drawn in breadth-first
  node order; Lloyd iterations until the assignment no longer changes or 50
  iterations; a cluster that becomes empty is dropped; the final centroids
  are the means of the final assignment; children are ordered by cluster
  index; assignment ties go to the lowest cluster index; a node whose
  k-means keeps a single cluster (its points are identical, so no split
  separates them) stays a leaf, which the uncapped recursion needs to end;
* search = greedy descent (nearest child centroid at every level, ties to the
  lowest child), then exhaustive search of that one leaf, ties to the lowest
  exemplar id.

Tree layout (shared with the GPU library through its host export format):
nodes in breadth-first order; ``first_child``/``n_children`` per node
(children contiguous); ``leaf_of_node`` (-1 for internal nodes); leaves
numbered in node order; ``perm`` lists exemplar ids leaf by leaf, ascending
within a leaf; ``leaf_off`` [n_leaves + 1] indexes ``perm``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Tree:
    centroids: np.ndarray  # float64 [n_nodes][d]; row 0 (root) unused
    first_child: np.ndarray  # int64 [n_nodes]
    n_children: np.ndarray  # int64 [n_nodes]
    leaf_of_node: np.ndarray  # int64 [n_nodes]
    node_depth: np.ndarray  # int64 [n_nodes]
    leaf_off: np.ndarray  # int64 [n_leaves + 1]
    perm: np.ndarray  # int64 [N]

    @property
    def n_nodes(self) -> int:
        return int(self.first_child.size)

    @property
    def n_leaves(self) -> int:
        return int(self.leaf_off.size - 1)

    def leaf_members(self, leaf: int) -> np.ndarray:
        return self.perm[self.leaf_off[leaf] : self.leaf_off[leaf + 1]]

    def leaf_of_exemplar(self) -> np.ndarray:
        out = np.empty(self.perm.size, dtype=np.int64)
        for l in range(self.n_leaves):
            out[self.leaf_members(l)] = l
        return out


def _sqdist(P: np.ndarray, C: np.ndarray) -> np.ndarray:
    """[m][k] squared distances, direct form."""
    out = np.zeros((P.shape[0], C.shape[0]), dtype=np.float64)
    for c in range(P.shape[1]):
        t = P[:, c][:, None] - C[:, c][None, :]
        out += t * t
    return out


def kmeanspp(P: np.ndarray, k: int, rng: np.random.Generator) -> np.ndarray:
    m = P.shape[0]
    idx = [int(rng.integers(m))]
    D2 = _sqdist(P, P[idx[0]][None, :])[:, 0]
    for _ in range(1, k):
        tot = D2.sum()
        if tot > 0.0:
            u = rng.random() * tot
            j = int(np.searchsorted(np.cumsum(D2), u, side="right"))
            j = min(j, m - 1)
        else:
            j = int(rng.integers(m))
        idx.append(j)
        D2 = np.minimum(D2, _sqdist(P, P[j][None, :])[:, 0])
    return P[idx].copy()


def lloyd(P: np.ndarray, C: np.ndarray, max_iter: int = 50):
    """Lloyd iterations; returns (centroids [k'][d], assignment [m])."""
    prev = None
    a = None
    for _ in range(max_iter):
        a = np.argmin(_sqdist(P, C), axis=1)  # first minimum: lowest index
        used = np.unique(a)
        if used.size < C.shape[0]:  # drop empty clusters, keep order
            remap = -np.ones(C.shape[0], dtype=np.int64)
            remap[used] = np.arange(used.size)
            a = remap[a]
        C = np.stack([P[a == j].mean(axis=0) for j in range(used.size)])
        if prev is not None and np.array_equal(a, prev):
            break
        prev = a
    return C, a


def build(Zp: np.ndarray, branching: int, depth, seed: int = 0, max_iter: int = 50) -> Tree:
    """Build the tree over PCA-projected exemplar vectors Zp [N][d]
    (depth None or negative: no depth cap)."""
    Zp = np.asarray(Zp, dtype=np.float64)
    N, d = Zp.shape
    rng = np.random.default_rng(seed)
    cents = [np.zeros(d)]
    first = [0]
    nch = [0]
    ndepth = [0]
    members = [np.arange(N)]
    head = 0
    while head < len(members):
        mem = members[head]
        dep = ndepth[head]
        if (depth is None or depth < 0 or dep < depth) and mem.size >= branching:
            P = Zp[mem]
            C, a = lloyd(P, kmeanspp(P, branching, rng), max_iter)
            if C.shape[0] < 2:  # one cluster: the points cannot be separated
                head += 1
                continue
            first[head] = len(members)
            nch[head] = C.shape[0]
            for j in range(C.shape[0]):
                cents.append(C[j])
                first.append(0)
                nch.append(0)
                ndepth.append(dep + 1)
                members.append(mem[a == j])
        head += 1
    n = len(members)
    leaf_of = -np.ones(n, dtype=np.int64)
    offs = [0]
    perm = []
    for i in range(n):
        if nch[i] == 0:
            leaf_of[i] = len(offs) - 1
            perm.append(np.sort(members[i]))
            offs.append(offs[-1] + members[i].size)
    return Tree(
        centroids=np.stack(cents),
        first_child=np.asarray(first, dtype=np.int64),
        n_children=np.asarray(nch, dtype=np.int64),
        leaf_of_node=leaf_of,
        node_depth=np.asarray(ndepth, dtype=np.int64),
        leaf_off=np.asarray(offs, dtype=np.int64),
        perm=np.concatenate(perm).astype(np.int64) if perm else np.zeros(0, np.int64),
    )


def descend(tree: Tree, Qp: np.ndarray):
    """Greedy descent; returns (leaf [nq], smallest relative decision gap [nq]).

    The gap at a decision is (second-nearest - nearest) / nearest child
    distance (inf when a node has one child); parity uses it to excuse a
    descent that a different rounding could flip.
    """
    Qp = np.asarray(Qp, dtype=np.float64)
    nq = Qp.shape[0]
    leaves = np.empty(nq, dtype=np.int64)
    gaps = np.full(nq, np.inf)
    for q in range(nq):
        node = 0
        while tree.n_children[node] > 0:
            f, n = tree.first_child[node], tree.n_children[node]
            diff = tree.centroids[f : f + n] - Qp[q][None, :]
            dd = np.einsum("ij,ij->i", diff, diff)
            j = int(np.argmin(dd))
            if n > 1:
                srt = np.sort(dd)
                g = (srt[1] - srt[0]) / srt[0] if srt[0] > 0 else np.inf
                gaps[q] = min(gaps[q], g)
            node = f + j
        leaves[q] = tree.leaf_of_node[node]
    return leaves, gaps


def search_leaves(Qp: np.ndarray, Zp: np.ndarray, tree: Tree, leaves_per_query):
    """Exhaustive search of the given leaves (a list of leaf ids per query).

    Returns (nn original exemplar id [nq], squared PCA distance [nq]).
    """
    Qp = np.asarray(Qp, dtype=np.float64)
    nq = Qp.shape[0]
    nn = np.empty(nq, dtype=np.int64)
    dd = np.empty(nq, dtype=np.float64)
    for q in range(nq):
        cand = np.concatenate([tree.leaf_members(int(l)) for l in np.atleast_1d(leaves_per_query[q])])
        diff = Zp[cand] - Qp[q][None, :]
        d2 = np.einsum("ij,ij->i", diff, diff)
        o = np.lexsort((cand, d2))[0]
        nn[q] = cand[o]
        dd[q] = d2[o]
    return nn, dd


def search_leaves_topk(Qp: np.ndarray, Zp: np.ndarray, tree: Tree, leaves_per_query, k: int = 8, offset=None):
    """The k best members of the given leaves (a list of leaf ids per query;
    a repeated leaf counts once) by squared PCA distance plus the optional
    per-exemplar offset, ties to the lowest id: the candidates the learned
    form re-ranks in full dimension.  Returns (list of id arrays, list of
    distance arrays)."""
    Qp = np.asarray(Qp, dtype=np.float64)
    off = None if offset is None else np.asarray(offset, dtype=np.float64)
    ids_out, d_out = [], []
    for q in range(Qp.shape[0]):
        cand = np.unique(np.concatenate([tree.leaf_members(int(l)) for l in np.atleast_1d(leaves_per_query[q])]))
        diff = Zp[cand] - Qp[q][None, :]
        d2 = np.einsum("ij,ij->i", diff, diff)
        if off is not None:
            d2 = d2 + off[cand]
        o = np.lexsort((cand, d2))[:k]
        ids_out.append(cand[o])
        d_out.append(d2[o])
    return ids_out, d_out


def tree_nn(Qp: np.ndarray, Zp: np.ndarray, tree: Tree):
    """Tree search: greedy descent to one leaf, then exhaustive leaf scan."""
    leaves, gaps = descend(tree, Qp)
    nn, d2 = search_leaves(Qp, Zp, tree, leaves)
    return nn, d2, leaves, gaps
