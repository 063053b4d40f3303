"""Pins of the oracle's friends-of-friends groups: brute force over all
pairs on small sets, chains just inside and just outside the linking
length, links across the periodic boundary, and the label convention (the
smallest index of each group)."""
import numpy as np
import pytest


@pytest.mark.parametrize("seed,n,b", [(1, 300, 0.05), (2, 500, 0.03),
                                      (3, 200, 0.12)])
def test_tree_equals_brute_force(orc, seed, n, b):
    rng = np.random.default_rng(seed)
    P = 1.0 + rng.random((3, n)).astype(np.float32)
    a = orc.fof_labels(*P, b)
    c = orc.fof_labels(*P, b, brute=True)
    assert np.array_equal(a, c)
    assert 1 < len(np.unique(a)) < n  # groups of several sizes


def test_chain_links_inside_the_length():
    import oracle as orc
    b = 0.01
    n = 40
    x = 1.2 + 0.9 * b * np.arange(n)
    lab = orc.fof_labels(x, np.full(n, 1.5), np.full(n, 1.5), b)
    assert np.all(lab == 0)
    x = 1.2 + 1.1 * b * np.arange(n)
    lab = orc.fof_labels(x, np.full(n, 1.5), np.full(n, 1.5), b)
    assert np.array_equal(lab, np.arange(n))


def test_links_across_the_periodic_boundary():
    import oracle as orc
    b = 0.02
    x = np.array([1.995, 1.005, 1.5, 1.0 + 0.5 * b])
    lab = orc.fof_labels(x, np.full(4, 1.3), np.full(4, 1.7), b)
    # 1.995 and 1.005 are 0.01 apart through the boundary; 1.005 and 1.01
    # are 0.005 apart: one group of three, labelled by its smallest index
    assert lab.tolist() == [0, 0, 2, 0]


def test_labels_are_group_minima(orc):
    rng = np.random.default_rng(9)
    P = 1.0 + rng.random((3, 400))
    lab = orc.fof_labels(*P, 0.06)
    for g in np.unique(lab):
        members = np.nonzero(lab == g)[0]
        assert members.min() == g
