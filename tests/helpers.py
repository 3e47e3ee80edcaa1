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


def projector_gap(B1, B2) -> float:
    return float(np.abs(B1 @ B1.T - B2 @ B2.T).max())


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def query_and_exemplar(X, Z, w, s):
    return vectors.query_matrix(X, w, s), vectors.exemplar_matrix(Z, w)
