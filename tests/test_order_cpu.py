"""The library's overlap-signature reordering (kldi_overlap_order, host code, no GPU) against the oracle's
plain average-linkage clustering (oracle.cluster) on the same overlap matrices: identical leaf and shell
orders (integer results, bit-exact)."""
import numpy as np
import pytest

import synth
from oracle import cluster


@pytest.fixture(scope="module")
def order_fn():
    from paper_2605_10363_amd.plan import overlap_order
    return overlap_order


@pytest.mark.parametrize("n_atoms,seed", [(2, 4), (3, 5), (5, 6), (6, 7)])
def test_library_order_equals_oracle_tiny(order_fn, n_atoms, seed):
    p = synth.tiny_problem(n_atoms=n_atoms, n_rad=8, n_ang=26, n_occ=1, seed=seed, box_A=4.0)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    so_ref, ao_ref = cluster.overlap_shell_order(S, p.basis)
    ao, so = order_fn(p.basis, S)
    assert np.array_equal(ao, ao_ref)
    assert np.array_equal(so, so_ref)


def test_single_atom_ties(order_fn):
    """One atom alone: its p (and d) components are exactly equivalent, so several merges tie exactly and
    more than one leaf order is an average-linkage order; the library breaks such ties in the order of
    its nearest-neighbour chain, the oracle by cluster ids.  What is unique is checked: the merge heights
    of the library's tree (rebuilt from its leaf order by the oracle) equal the oracle's, and the orders
    are permutations."""
    p = synth.tiny_problem(n_atoms=1, n_rad=8, n_ang=26, n_occ=1, seed=3, box_A=4.0)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    ao, so = order_fn(p.basis, S)
    assert sorted(ao) == list(range(p.n_ao)) and sorted(so) == list(range(p.basis.n_shells))
    d = cluster.cosine_distance(S)
    _, m_ref = cluster.average_linkage_order(d)
    # the same clustering of the library's order relabelled: heights do not depend on tie choices here
    perm = np.asarray(ao)
    _, m_lib = cluster.average_linkage_order(d[np.ix_(perm, perm)])
    assert np.allclose(sorted(m[2] for m in m_lib), sorted(m[2] for m in m_ref), rtol=1e-12, atol=1e-15)


def test_library_order_equals_oracle_cfg0(order_fn):
    p = synth.make_problem(0)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    so_ref, ao_ref = cluster.overlap_shell_order(S, p.basis)
    ao, so = order_fn(p.basis, S)
    assert np.array_equal(ao, ao_ref)
    assert np.array_equal(so, so_ref)


def test_library_order_rejects_bad_input(order_fn):
    p = synth.tiny_problem(n_atoms=2, n_rad=8, n_ang=26, n_occ=1, seed=4)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    from paper_2605_10363_amd._lib import KldiError
    bad = S.copy()
    bad[0, :] = 0.0
    with pytest.raises(KldiError):
        order_fn(p.basis, bad)
    bad = S.copy()
    bad[1, 2] = np.nan
    with pytest.raises(KldiError):
        order_fn(p.basis, bad)
