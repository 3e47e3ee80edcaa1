"""Pins of the uncapped k-means tree (Methodology 2.2: recursion stops when
a node holds fewer than k members): structural rules on random points,
identical points, and the degenerate sizes."""
import numpy as np

from oracle import tree
from tests import helpers


def test_uncapped_tree_splits_until_every_leaf_is_below_k():
    rng = np.random.default_rng(0)
    Zp = rng.normal(size=(700, 5))
    t = tree.build(Zp, 4, None, seed=1)
    depth, sizes = helpers.check_tree_rules(t, Zp, 4)
    assert sizes.max() < 4 and depth >= 4  # 700 points need at least log4(700/3) levels
    # the capped tree is a prefix of the same rule
    t2 = tree.build(Zp, 4, 2, seed=1)
    d2, s2 = helpers.check_tree_rules(t2, Zp, 4, depth=2)
    assert d2 == 2 and s2.max() >= 4


def test_identical_points_end_in_one_leaf():
    rng = np.random.default_rng(2)
    Zp = np.concatenate([np.tile(rng.normal(size=(1, 3)), (11, 1)), rng.normal(size=(30, 3))])
    t = tree.build(Zp, 4, None, seed=0)
    _, sizes = helpers.check_tree_rules(t, Zp, 4)
    mem = helpers.node_members(t)
    leaves = [m for i, m in enumerate(mem) if t.n_children[i] == 0]
    dup = [m for m in leaves if 0 in m][0]
    assert set(range(11)) <= set(dup.tolist())  # the 11 copies stay together
    assert sizes.max() >= 11


def test_fewer_points_than_k_is_a_single_leaf():
    Zp = np.random.default_rng(3).normal(size=(3, 4))
    t = tree.build(Zp, 4, None)
    assert t.n_nodes == 1 and t.n_leaves == 1 and np.array_equal(np.sort(t.perm), np.arange(3))
    Zp = np.random.default_rng(4).normal(size=(4, 4))
    t = tree.build(Zp, 4, None)
    helpers.check_tree_rules(t, Zp, 4)
    assert t.n_nodes > 1  # four distinct points must split


def test_rule_checker_rejects_planted_mistakes():
    """The checker fails on a leaf left unsplit, a node split below k, and a
    wrong centroid (mistakes planted in an oracle tree, on the CPU)."""
    import dataclasses

    import pytest

    rng = np.random.default_rng(5)
    Zp = rng.normal(size=(60, 3))
    good = tree.build(Zp, 4, None, seed=0)
    helpers.check_tree_rules(good, Zp, 4)
    capped = tree.build(Zp, 4, 1, seed=0)  # leaves of >= 4 distinct points, checked as uncapped
    with pytest.raises(AssertionError):
        helpers.check_tree_rules(capped, Zp, 4)
    bad = dataclasses.replace(good, centroids=good.centroids.copy())
    bad.centroids[1] += 0.01
    with pytest.raises(AssertionError):
        helpers.check_tree_rules(bad, Zp, 4)
    with pytest.raises(AssertionError):
        helpers.check_tree_rules(good, Zp, 64)  # the root splits below k = 64
