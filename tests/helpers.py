"""Test helpers: workload inputs and index format conversions."""
from __future__ import annotations

import numpy as np

from oracle import solve as osolve
from oracle import tree as otree
from oracle import vectors
from paper_2006_11851_amd import synth


def workload_inputs(name: str):
    """(exemplar u8, init u8 at the coarsest level, workload)."""
    wl = synth.workload(name)
    ex = wl.exemplar()
    return ex, wl.initial_output(ex), wl


def oracle_index_to_dict(ix: osolve.Index, Zshape) -> dict:
    t = ix.tree
    return {
        "w": ix.w,
        "N": ix.Zp.shape[0],
        "mu": ix.mu,
        "basis": ix.B,
        "eigenvalues": np.zeros(ix.B.shape[1]),
        "centroids": t.centroids,
        "first_child": t.first_child.astype(np.int32),
        "n_children": t.n_children.astype(np.int32),
        "leaf_of_node": t.leaf_of_node.astype(np.int32),
        "leaf_off": t.leaf_off.astype(np.int64),
        "perm": t.perm.astype(np.int32),
    }


def dict_to_oracle_tree(a: dict) -> otree.Tree:
    nn = a["first_child"].size
    depth = np.zeros(nn, np.int64)
    for i in range(nn):
        for j in range(a["n_children"][i]):
            depth[a["first_child"][i] + j] = depth[i] + 1
    return otree.Tree(
        centroids=np.asarray(a["centroids"], np.float64),
        first_child=np.asarray(a["first_child"], np.int64),
        n_children=np.asarray(a["n_children"], np.int64),
        leaf_of_node=np.asarray(a["leaf_of_node"], np.int64),
        node_depth=depth,
        leaf_off=np.asarray(a["leaf_off"], np.int64),
        perm=np.asarray(a["perm"], np.int64),
    )


def node_members(t: otree.Tree) -> list:
    """Exemplar ids under every node (children before parents are not
    assumed: nodes are visited from the last, which is breadth-first safe)."""
    mem = [None] * t.n_nodes
    for i in range(t.n_nodes - 1, -1, -1):
        if t.n_children[i] == 0:
            l = t.leaf_of_node[i]
            mem[i] = np.asarray(t.perm[t.leaf_off[l]:t.leaf_off[l + 1]], np.int64)
        else:
            f = t.first_child[i]
            mem[i] = np.concatenate([mem[f + j] for j in range(t.n_children[i])])
    return mem


def check_tree_rules(t: otree.Tree, Zp: np.ndarray, branching: int, depth=None, atol: float = 0.0):
    """The tree's structural rules (Methodology 2.2's stop rule): the leaves
    partition the N ids; a node is split only if it holds >= branching
    members and has >= 2 children (up to the depth cap, if any); a leaf with
    >= branching members is allowed only at the cap or when its points are
    identical (within atol, per coordinate); every child's centroid is the
    mean of its members.  Returns (depth reached, leaf sizes)."""
    N = Zp.shape[0]
    assert np.array_equal(np.sort(np.asarray(t.perm, np.int64)), np.arange(N))
    assert t.leaf_off[0] == 0 and t.leaf_off[-1] == N and np.all(np.diff(t.leaf_off) >= 0)
    mem = node_members(t)
    dep = np.zeros(t.n_nodes, np.int64)
    for i in range(t.n_nodes):
        nc = t.n_children[i]
        if nc > 0:
            assert nc >= 2 and mem[i].size >= branching, (i, nc, mem[i].size)
            assert depth is None or dep[i] < depth
            for j in range(nc):
                c = t.first_child[i] + j
                assert c > i
                dep[c] = dep[i] + 1
                assert mem[c].size > 0
                cen = Zp[mem[c]].mean(axis=0)
                assert np.abs(t.centroids[c] - cen).max() <= 1e-6 + 1e-5 * np.abs(cen).max(), (c,)
        elif mem[i].size >= branching and not (depth is not None and dep[i] == depth):
            P = Zp[mem[i]]
            assert np.abs(P - P[0]).max() <= atol, (i, mem[i].size)
    sizes = np.diff(t.leaf_off)
    return int(dep.max()), sizes


def projector_gap(B1, B2) -> float:
    return float(np.abs(B1 @ B1.T - B2 @ B2.T).max())


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def query_and_exemplar(X, Z, w, s):
    return vectors.query_matrix(X, w, s), vectors.exemplar_matrix(Z, w)


def scanned_members(t, leaves) -> np.ndarray:
    """Exemplar ids of the members of the listed leaves (each once)."""
    return np.unique(np.concatenate([t.leaf_members(int(l)) for l in leaves]))


def topk_rerank_validity(Qp, Zp, t, lists, got, k=8, offset=None, Q_full=None, Zm=None, mu=None, bf16=True):
    """Per query: is ``got`` a valid outcome of the exact BF16 top-k over the
    members of the leaves in ``lists[i]`` (with t None: lists[i] holds the
    exemplar ids themselves) followed by the FP32 re-rank (full
    dimension when Q_full/Zm are given, else PCA space with the offset)?
    The scores are the oracle's exact values; two scores closer than the
    bound of their FP32 evaluation (or 1e-4 of the k-th) may be ordered
    either way (oracle.parity.topk_rerank_valid).  bf16=False: the scores are
    the unrounded PCA-space distances the FP32 scan ranks by (evaluated in
    the direct form, whose FP32 error is relative).  Returns a bool array."""
    from oracle import bf16 as obf16
    from oracle import parity

    d = Zp.shape[1]
    ok = np.zeros(len(lists), dtype=bool)
    for i, ls in enumerate(lists):
        m = scanned_members(t, ls) if t is not None else np.unique(np.asarray(ls, dtype=np.int64))
        off = None if offset is None else offset[m]
        if bf16:
            sc = obf16.scan_scores(Qp[i], Zp[m], off)
            sk = np.sort(sc)[min(k, sc.size) - 1]
            tol = max(1e-4 * abs(sk), obf16.fp32_score_tolerance(
                Qp[i], Zp[m], d, off, None if (offset is None or Zm is None) else Zm[m], mu))
        else:
            df = Zp[m] - Qp[i][None, :]
            sc = np.einsum("ij,ij->i", df, df) + (0.0 if off is None else off)
            sk = np.sort(sc)[min(k, sc.size) - 1]
            tol = max(1e-4, 2 * (d + 4) * 2.0 ** -24) * abs(sk)
        if Q_full is not None:
            diff = Zm[m] - Q_full[i][None, :]
        else:
            diff = Zp[m] - Qp[i][None, :]
        rd = np.einsum("ij,ij->i", diff, diff)
        if Q_full is None and offset is not None:
            rd = rd + off
        ok[i] = parity.topk_rerank_valid(m, sc, rd, int(got[i]), k, tol_score=tol)
    return ok
