"""Seeded input generator: determinism, recipe shapes, quadrature building blocks."""
import math

import numpy as np
import pytest

import synth


def test_seeded_determinism():
    a = synth.tiny_problem(seed=11)
    b = synth.tiny_problem(seed=11)
    assert np.array_equal(a.atom_xyz, b.atom_xyz)
    assert np.array_equal(a.basis.prim_exp, b.basis.prim_exp)
    assert np.array_equal(a.grid.weight, b.grid.weight)
    assert np.array_equal(a.D, b.D)


def test_cfg0_shapes(cfg0):
    p = cfg0
    assert p.n_atoms == 12 and int(p.atom_heavy.sum()) == 4
    assert p.n_ao == 4 * 15 + 8 * 5 == 100
    assert p.basis.n_shells == 4 * 6 + 8 * 3
    assert p.n_points == 12 * 40 * 110
    d = np.linalg.norm(p.atom_xyz[:, None] - p.atom_xyz[None], axis=2) + np.eye(12) * 1e9
    assert d.min() >= 1.0 * synth.BOHR_PER_ANGSTROM - 1e-12
    assert np.all(p.basis.prim_exp >= 0.1) and np.all(p.basis.prim_exp <= 50.0)
    nprim = np.diff(p.basis.prim_ptr)
    assert nprim.min() >= 1 and nprim.max() <= 3


@pytest.mark.parametrize("n,alpha", [(0, 0.1), (2, 1.0), (4, 50.0), (1, 3.0)])
def test_radial_quadrature_closed_form(n, alpha):
    # int_0^inf r^n exp(-a r^2) r^2 dr = Gamma((n+3)/2) / (2 a^((n+3)/2))
    r, w = synth.radial_grid(75)
    exact = math.gamma((n + 3) / 2) / (2 * alpha ** ((n + 3) / 2))
    got = np.sum(w * r ** n * np.exp(-alpha * r * r))
    assert abs(got - exact) <= 1e-9 * exact


def test_fibonacci_weights_and_low_moments():
    u, w = synth.fibonacci_sphere(302)
    assert abs(w.sum() - 4 * math.pi) < 1e-12
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0)
    # first moments vanish to the accuracy of an equal-weight spiral
    assert np.all(np.abs(w @ u) < 1e-2)


def test_becke_partition_of_unity():
    rng = np.random.default_rng(5)
    atoms = rng.uniform(0, 6, size=(5, 3))
    pts = rng.uniform(-2, 8, size=(40, 3))
    tot = np.zeros(len(pts))
    for a in range(5):
        tot += synth.becke_fractions(atoms, pts, np.full(len(pts), a, np.int32), 0.0)
    assert np.allclose(tot, 1.0, atol=1e-14)


def test_overlap_and_density_normalisation(cfg0):
    p = cfg0
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    assert np.allclose(np.diag(S), 1.0, atol=1e-13)
    assert np.allclose(S, S.T)
    assert abs(np.trace(p.D @ S) - p.n_occ) < 1e-10
    assert np.allclose(p.D, p.D.T)


def test_two_s_gaussians_overlap_closed_form():
    # <g_a(A)|g_b(B)> for normalised s Gaussians = (2 sqrt(ab)/(a+b))^{3/2} exp(-ab R^2/(a+b))
    a, b, R = 0.7, 2.3, 1.3
    basis = synth.Basis(np.array([0, 1], np.int32), np.array([0, 0], np.int32), np.array([0, 1, 2], np.int32),
                        np.array([a, b]), np.array([(2 * a / math.pi) ** 0.75, (2 * b / math.pi) ** 0.75]))
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    S = synth.overlap_matrix(basis, xyz)
    exact = (2 * math.sqrt(a * b) / (a + b)) ** 1.5 * math.exp(-a * b * R * R / (a + b))
    assert abs(S[0, 1] - exact) < 1e-14
