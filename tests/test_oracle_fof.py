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


# ---------------------------------------------------------------------------
# group properties
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("xa,xb,centre", [(1.995, 1.003, 1.999),
                                         (1.998, 1.004, 1.001)])
def test_properties_of_a_group_across_the_boundary(orc, xa, xb, centre):
    """Two equal masses linked through the periodic boundary: the centre is
    the midpoint of the minimum-image pair, wrapped into [1, 2)."""
    x = np.array([xa, xb])
    y = np.array([1.5, 1.5])
    z = np.array([1.25, 1.25])
    m = np.array([2.0, 2.0])
    lab = orc.fof_labels(x, y, z, 0.02, brute=True)
    assert lab.tolist() == [0, 0]
    count, mass, com = orc.fof_properties(x, y, z, m, lab)
    assert count.tolist() == [2, 0] and mass.tolist() == [4.0, 0.0]
    assert abs(com[0, 0] - centre) < 1e-12
    assert com[1, 0] == 1.5 and com[2, 0] == 1.25
    assert np.all(com[:, 1] == 0.0)


def test_properties_totals_singletons_and_translation(orc):
    rng = np.random.default_rng(17)
    n = 3000
    P = 1.0 + rng.random((3, n))
    # a few tight clumps, one of them across a corner of the box
    for k, c in enumerate(([1.02, 1.97, 1.5], [1.5, 1.5, 1.5],
                           [1.999, 1.001, 1.998])):
        P[:, k * 40:(k + 1) * 40] = (np.asarray(c)[:, None] - 1.0 + 0.004
                                     * rng.standard_normal((3, 40))) % 1.0 + 1.0
    m = rng.uniform(0.5, 1.5, n)
    lab = orc.fof_labels(*P, 0.005)
    count, mass, com = orc.fof_properties(*P, m, lab)
    assert count.sum() == n and abs(mass.sum() - m.sum()) < 1e-9
    roots = np.unique(lab)
    assert np.all(count[roots] > 0)
    others = np.setdiff1d(np.arange(n), roots)
    assert np.all(count[others] == 0) and np.all(mass[others] == 0)
    assert count.max() >= 30
    single = roots[count[roots] == 1]
    assert np.array_equal(com[:, single], P[:, single])
    # a periodic translation moves every centre by the same amount
    s = np.array([0.3125, 0.625, 0.875])[:, None]
    Q = (P - 1.0 + s) % 1.0 + 1.0
    count2, mass2, com2 = orc.fof_properties(*Q, m, lab)
    assert np.array_equal(count2, count)
    d = (com2[:, roots] - com[:, roots] - s[:, :]) % 1.0
    d = np.minimum(d, 1.0 - d)
    assert d.max() < 1e-12
