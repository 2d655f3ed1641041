"""The oracle's overlap-signature clustering (oracle.cluster) against what the mathematics fixes: the
cosine distance's special values, average linkage as the library routine scipy.cluster.hierarchy
computes it, the dendrogram invariant of a leaf order and the orientation rule checked by brute force."""
import numpy as np
import pytest
from scipy.cluster import hierarchy
from scipy.spatial.distance import squareform

import synth
from oracle import cluster


def test_cosine_distance_special_values():
    S = np.array([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 3.0, 0.0], [-1.0, 0.0, 0.0], [1.0, 1.0, 0.0]])
    d = cluster.cosine_distance(S)
    assert abs(d[0, 1]) < 1e-15 and abs(d[0, 2] - 1.0) < 1e-15 and abs(d[0, 3] - 2.0) < 1e-15
    assert abs(d[0, 4] - (1 - 1 / np.sqrt(2))) < 1e-15
    assert np.allclose(d, d.T, atol=0, rtol=0) and np.allclose(np.diag(d), 0, atol=1e-15)


def test_hand_example_line():
    # four points on a line at 0, 1, 10, 11 in the order (10, 0, 11, 1): the tie between {10, 11} and
    # {0, 1} goes to the pair of smaller ids (0, 2), and the orientation joins 1 and 10
    x = np.array([10.0, 0.0, 11.0, 1.0])
    d = np.abs(x[:, None] - x[None, :])
    order, merges = cluster.average_linkage_order(d)
    assert [tuple(sorted(m[:2])) for m in merges] == [(0, 2), (1, 3), (4, 5)]
    assert list(x[order]) in ([0.0, 1.0, 10.0, 11.0], [11.0, 10.0, 1.0, 0.0])
    assert merges[2][2] == pytest.approx(10.0)


def _check_tree(d, order, merges):
    n = d.shape[0]
    pos = np.empty(n, int)
    pos[order] = np.arange(n)
    members = {i: [i] for i in range(n)}
    for k, (a, b, dist, size) in enumerate(merges):
        m = members[a] + members[b]
        members[n + k] = m
        p = np.sort(pos[m])
        assert p[-1] - p[0] == len(m) - 1          # every cluster is a contiguous range of the leaf order
        assert size == len(m)
        assert dist == pytest.approx(float(np.mean(d[np.ix_(members[a], members[b])])), rel=1e-12)


def test_average_linkage_equals_scipy_and_tree_invariants():
    rng = np.random.default_rng(0)
    for n in (2, 3, 7, 25, 60):
        X = rng.normal(size=(n, 3))
        d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
        order, merges = cluster.average_linkage_order(d)
        Z = hierarchy.linkage(squareform(d, checks=False), method="average")
        assert len(merges) == n - 1
        for (a, b, dist, size), z in zip(merges, Z):
            assert {a, b} == {int(z[0]), int(z[1])}
            assert dist == pytest.approx(z[2], rel=1e-12) and size == int(z[3])
        _check_tree(d, order, merges)


def test_orientation_brute_force():
    """Rebuild the leaf order from the merge list: at every merge, of the four ways to join the two leaf
    sequences the chosen one has the smallest junction distance (first in the stated order on ties)."""
    rng = np.random.default_rng(1)
    X = rng.normal(size=(30, 2))
    d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    order, merges = cluster.average_linkage_order(d)
    seq = {i: [i] for i in range(30)}
    for k, (a, b, dist, size) in enumerate(merges):
        A, B = seq.pop(a), seq.pop(b)
        best = None
        for x, y in ((A, B), (A[::-1], B), (A, B[::-1]), (A[::-1], B[::-1])):
            j = d[x[-1], y[0]]
            if best is None or j < best[0]:
                best = (j, list(x) + list(y))
        seq[30 + k] = best[1]
        assert best[0] == min(d[A[0], B[0]], d[A[0], B[-1]], d[A[-1], B[0]], d[A[-1], B[-1]])
    assert list(seq[58]) == list(order)


def test_overlap_order_hand_example():
    """Four s functions with S = [[1, .9, 0, 0], [.9, 1, 0, 0], [0, 0, 1, .5], [0, 0, .5, 1]]: cosine
    distances d01 = 1 - 1.8/1.81, d23 = 1 - 1/1.25 = 0.2, every cross pair 1; average linkage merges
    {0,1}, then {2,3}, then the two at 1; all junctions tie at 1, so the first way (A, B) is taken."""
    S = np.array([[1, .9, 0, 0], [.9, 1, 0, 0], [0, 0, 1, .5], [0, 0, .5, 1]], float)

    class B:
        shell_l = np.zeros(4, np.int32)
        shell_atom = np.arange(4, dtype=np.int32)

    d = cluster.cosine_distance(S)
    assert d[0, 1] == pytest.approx(1 - 1.8 / 1.81, rel=1e-14) and d[2, 3] == pytest.approx(0.2, rel=1e-14)
    so, order = cluster.overlap_shell_order(S, B)
    assert list(order) == [0, 1, 2, 3] and list(so) == [0, 1, 2, 3]
    _, merges = cluster.average_linkage_order(d)
    assert [m[:2] for m in merges] == [(0, 1), (2, 3), (4, 5)] and merges[2][2] == pytest.approx(1.0)


def test_overlap_order_of_a_molecule_is_a_permutation_with_valid_tree():
    p = synth.tiny_problem(n_atoms=4, n_rad=8, n_ang=26, n_occ=2, seed=11)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    so, order = cluster.overlap_shell_order(S, p.basis)
    assert sorted(so) == list(range(p.basis.n_shells)) and sorted(order) == list(range(p.n_ao))
    d = cluster.cosine_distance(S)
    o2, merges = cluster.average_linkage_order(d)
    _check_tree(d, o2, merges)


def test_shell_order_from_leaves():
    # shells of sizes 1, 3, 1: AOs 0 | 1 2 3 | 4
    so = cluster.shell_order_from_leaves([4, 2, 0, 1, 3], [0, 1, 1, 1, 2])
    assert list(so) == [2, 1, 0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_scipy_merges_give_the_plain_leaf_order(seed):
    """The fast path (scipy's merges, the same orientation rule) gives the plain procedure's leaf order."""
    p = synth.tiny_problem(n_atoms=5, n_rad=8, n_ang=26, n_occ=1, seed=20 + seed, box_A=5.0)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    d = cluster.cosine_distance(S)
    assert np.array_equal(cluster.average_linkage_order(d)[0], cluster.average_linkage_order_lib(d))
    so, o = cluster.overlap_shell_order(S, p.basis)
    so2, o2 = cluster.overlap_shell_order(S, p.basis, lib=True)
    assert np.array_equal(so, so2) and np.array_equal(o, o2)
