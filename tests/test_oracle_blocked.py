"""The oracle's block-filtered method against its definitions (no GPU)."""
import math

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
import synth
from oracle import addressing, reorder


# ---------------------------------------------------------------- Appendix D, parallel addressing
@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(0, 1), min_size=0, max_size=300))
def test_parallel_where_is_order_preserving_compaction(mask):
    S, I = addressing.parallel_where(np.array(mask, dtype=np.int64))
    ref = np.flatnonzero(np.array(mask, dtype=np.int64))
    assert S == len(ref)
    assert np.array_equal(I, ref)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 256, 1000])
def test_scan_is_logarithmic_and_exclusive(n):
    M = np.random.default_rng(n).integers(0, 2, n)
    P, steps = addressing.exclusive_scan_steps(M)
    assert P[0] == 0 and np.array_equal(P[1:], np.cumsum(M))
    assert steps == math.ceil(math.log2(n + 1))


# ---------------------------------------------------------------- Appendix B.1, Morton codes
def test_morton_matches_string_interleave():
    rng = np.random.default_rng(0)
    q = rng.integers(0, 1 << 20, size=(500, 3))
    m = reorder.morton_key(q[:, 0], q[:, 1], q[:, 2])
    for (x, y, z), key in zip(q, m):
        bx, by, bz = (format(int(v), "020b") for v in (x, y, z))
        s = "".join(bx[i] + by[i] + bz[i] for i in range(20))      # MSB first: x, y, z
        assert int(s, 2) == int(key)
    assert m.max() < (1 << 60)


def test_grid_and_ao_orders(cfg0):
    p = cfg0
    ao_perm, pt_perm, aperm = reorder.orders(p.atom_xyz, p.basis, p.grid.xyz, p.grid.point_atom)
    assert np.array_equal(np.sort(ao_perm), np.arange(p.n_ao))
    assert np.array_equal(np.sort(pt_perm), np.arange(p.n_points))
    rank = np.empty_like(aperm)
    rank[aperm] = np.arange(len(aperm))
    r = rank[p.grid.point_atom[pt_perm]]
    assert np.all(np.diff(r) >= 0)                       # grouped by atom, in atom order
    origin = reorder.origin_of(p.atom_xyz, p.grid.xyz)
    q = reorder.discretise(p.grid.xyz[pt_perm], origin)
    key = reorder.morton_key(q[:, 0], q[:, 1], q[:, 2])
    for a in range(p.n_atoms):
        k = key[r == a]
        assert np.all(np.diff(k) >= 0)                   # Morton-sorted within the atom
    # AOs: each atom's AOs contiguous, atoms in Morton order of their centres
    ao_atom = np.repeat(p.basis.shell_atom, [(l + 1) * (l + 2) // 2 for l in p.basis.shell_l])
    seq = ao_atom[ao_perm]
    changes = seq[np.r_[True, seq[1:] != seq[:-1]]]
    assert np.array_equal(changes, aperm)


# ---------------------------------------------------------------- Sec. III-B/C, blocked = dense at t=0
@pytest.mark.parametrize("xc,seed,d_ao,G", [("lda", 3, 32, 128), ("pbe", 4, 32, 128), ("pbe", 5, 16, 64),
                                            ("lda", 6, 8, 64)])
def test_blocked_equals_dense_without_screening(xc, seed, d_ao, G):
    p = synth.tiny_problem(n_atoms=4, n_rad=14, n_ang=26, xc=xc, seed=seed)
    d = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    b = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc,
                            t_b=0.0, t_d=0.0, d_ao=d_ao, G=G)
    assert abs(b["E"] - d["E"]) <= 1e-13 * abs(d["E"])
    assert np.abs(b["V"] - d["V"]).max() <= 1e-13 * np.abs(d["V"]).max()
    assert np.abs(b["rho"] - d["rho"]).max() <= 1e-13 * np.abs(d["rho"]).max()
    assert np.array_equal(b["V"], b["V"].T)


def test_blocked_cfg0_screening_error_and_structure(cfg0):
    p = cfg0
    d = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "lda")
    b = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, "lda",
                            t_b=1e-10, t_d=1e-10)
    # the thresholds' effect is far below the accuracy targets (1e-6 Eh, 1e-7 in V)
    assert abs(b["E"] - d["E"]) < 1e-9
    assert np.abs(b["V"] - d["V"]).max() < 1e-7
    assert np.array_equal(b["V"], b["V"].T)
    assert b["n_tiles"] == 4 and b["n_blocks"] == math.ceil(p.n_points / 128)
    assert 0 < b["S_phi"].mean() < 1


def test_error_grows_with_pair_threshold():
    # Sec. IV-A: fewer executed pairs as t_d grows, error not decreasing (Fig. td_sensitivity)
    p = synth.tiny_problem(n_atoms=5, n_rad=20, n_ang=50, xc="lda", seed=31, box_A=6.0)
    d = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "lda")
    errs, pairs = [], []
    for td in (1e-12, 1e-8, 1e-5, 1e-3, 1e-2):
        b = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, "lda",
                                t_b=1e-12, t_d=td, d_ao=8, G=64)
        errs.append(abs(b["E"] - d["E"]))
        pairs.append(b["nP_X"] + b["nP_M"])
    assert all(x >= y for x, y in zip(pairs, pairs[1:]))
    assert pairs[-1] < pairs[0]
    assert errs[-1] > errs[0]


# ---------------------------------------------------------------- block-at-a-time evaluation
@pytest.mark.parametrize("xc", ["lda", "pbe"])
@pytest.mark.parametrize("t", [1e-10, 1e-6])
def test_stream_evaluation_equals_blocked(xc, t):
    """eval_blocked_stream visits the grid blocks one at a time; it must reproduce eval_blocked (the
    same executed pairs, the same E, rho and V up to rounding) and its sampled V entries must be the
    entries of its full V."""
    p = synth.tiny_problem(n_atoms=5, n_rad=16, n_ang=38, n_occ=5, xc=xc, seed=71, box_A=5.0)
    args = (p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc)
    ref = oracle.eval_blocked(*args, t_b=t, t_d=t)
    s = oracle.blocked.eval_blocked_stream(*args, t_b=t, t_d=t, blocks_per_chunk=3)
    assert (s["nP_X"], s["nP_M"], s["nP_M_diag"]) == (ref["nP_X"], ref["nP_M"], ref["nP_M_diag"])
    assert 0 < ref["nP_M_diag"] < ref["nP_M"]
    assert abs(s["E"] - ref["E"]) <= 1e-13 * abs(ref["E"])
    assert np.abs(s["rho"] - ref["rho"]).max() <= 1e-13 * np.abs(ref["rho"]).max()
    assert np.abs(s["V"] - ref["V"]).max() <= 1e-13 * np.abs(ref["V"]).max()
    ij = np.random.default_rng(1).integers(0, p.n_ao, size=(300, 2))
    ij = np.concatenate([ij, np.stack([np.arange(p.n_ao)] * 2, 1)])
    v = oracle.blocked.eval_blocked_stream(*args, t_b=t, t_d=t, blocks_per_chunk=2, v_entries=ij)["v"]
    assert np.abs(v - s["V"][ij[:, 0], ij[:, 1]]).max() <= 1e-13 * np.abs(ref["V"]).max()
