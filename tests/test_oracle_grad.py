"""The oracle's fixed-grid EXC nuclear gradient (oracle.grad) against what the calculus fixes: central
finite differences of the basis derivatives and of E_xc itself in the atom positions (basis functions
moved, grid and D held fixed), and the block-filtered form reducing to the dense one without screening."""
import numpy as np
import pytest

import oracle
import synth
from oracle import basis as ob
from oracle import grad as og


def test_basis_second_derivatives_match_central_differences():
    p = synth.tiny_problem(n_atoms=3, n_rad=6, n_ang=14, n_occ=1, seed=5, box_A=3.0)
    pts = p.grid.xyz[::7][:60]
    phi, dphi, hphi = ob.eval_ao_hess(p.atom_xyz, p.basis, pts)
    phi1, dphi1 = ob.eval_ao(p.atom_xyz, p.basis, pts, deriv=1)
    assert np.array_equal(phi, phi1) and np.allclose(dphi, dphi1, rtol=1e-14, atol=1e-300)
    h = 1e-5
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        _, dp = ob.eval_ao(p.atom_xyz, p.basis, pts + e, deriv=1)
        _, dm = ob.eval_ao(p.atom_xyz, p.basis, pts - e, deriv=1)
        fd = (dp - dm) / (2 * h)                       # [a, mu, i] = d_b d_a chi
        scale = np.abs(hphi).max()
        assert np.abs(fd - hphi[:, b]).max() <= 1e-6 * scale
    assert np.allclose(hphi, np.swapaxes(hphi, 0, 1), rtol=0, atol=1e-14 * np.abs(hphi).max())


@pytest.mark.parametrize("xc", ["lda", "pbe", "pbe_x"])
def test_gradient_matches_finite_differences_of_energy(xc):
    p = synth.tiny_problem(n_atoms=3, n_rad=14, n_ang=38, n_occ=3, xc=xc, seed=9, box_A=3.0)
    g = og.exc_gradient(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    h = 1e-4
    fd = np.zeros_like(g)
    for A in range(p.n_atoms):
        for a in range(3):
            xp = p.atom_xyz.copy()
            xp[A, a] += h
            xm = p.atom_xyz.copy()
            xm[A, a] -= h
            Ep = oracle.eval_exc(xp, p.basis, p.grid.xyz, p.grid.weight, p.D, xc, want_v=False)["E"]
            Em = oracle.eval_exc(xm, p.basis, p.grid.xyz, p.grid.weight, p.D, xc, want_v=False)["E"]
            fd[A, a] = (Ep - Em) / (2 * h)
    print(xc, "max |g - fd| %.2e, max |g| %.2e" % (np.abs(g - fd).max(), np.abs(g).max()))
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(g).max())
    # with the grid fixed the sum over atoms is not zero (the grid does not move with the atoms): the
    # check is that it is not forced to zero by a dropped term
    assert np.abs(g).max() > 1e-4


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_blocked_gradient_without_screening_equals_dense(xc):
    p = synth.tiny_problem(n_atoms=4, n_rad=10, n_ang=26, n_occ=3, xc=xc, seed=12, box_A=4.0)
    g = og.exc_gradient(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    gb = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc, t_b=0.0)
    assert np.abs(gb - g).max() <= 1e-12 * np.abs(g).max()
    gs = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc,
                                 t_b=1e-10)
    print(xc, "screening at 1e-10 moves the gradient by %.2e" % np.abs(gs - g).max())
    assert np.abs(gs - g).max() <= 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_gradient_pair_filter_drops_only_bounded_triples(xc):
    """The gradient products' pair filter a_pq max|A_pr| max|B_qr| >= t: raising t drops triples, and each
    dropped triple moves the D-contracted sum by at most d^2 G times its bound (< t), so the gradient moves
    by at most 2 n_dropped d^2 G t (d = 32 AOs, G = 128 points); t = 0 keeps every triple."""
    p = synth.tiny_problem(n_atoms=4, n_rad=12, n_ang=26, n_occ=3, xc=xc, seed=12, box_A=4.0)
    args = (p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc)
    g0, n0 = og.exc_gradient_blocked(*args, t_b=1e-10, t_d=1e-10, t_grad=0.0, return_count=True)
    for t in (1e-8, 1e-6, 1e-4):
        g1, n1 = og.exc_gradient_blocked(*args, t_b=1e-10, t_d=1e-10, t_grad=t, return_count=True)
        bound = 2.0 * (n0 - n1) * 32 * 32 * 128 * t
        print(xc, "t %.0e: %d of %d triples, |dg| %.2e <= %.2e" % (t, n1, n0, np.abs(g1 - g0).max(), bound))
        assert n1 <= n0
        assert np.abs(g1 - g0).max() <= bound
    assert n1 < n0        # the largest t drops triples


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_gradient_magnitude_bounds_the_gradient(xc):
    """magnitude=True: the same sums over |D|, |A|, |B|.  Without screening it equals the dense sums over
    all points written out here (both products of each axis, summed over the AOs of each atom); with
    screening it bounds the gradient component by component (triangle inequality)."""
    p = synth.tiny_problem(n_atoms=4, n_rad=10, n_ang=26, n_occ=3, xc=xc, seed=12, box_A=4.0)
    args = (p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc)
    m0 = og.exc_gradient_blocked(*args, t_b=0.0, magnitude=True)
    phi, dphi, hphi = ob.eval_ao_hess(p.atom_xyz, p.basis, p.grid.xyz)
    X = p.D @ phi
    rho = np.einsum("mi,mi->i", phi, X)
    gga = xc == "pbe"
    grad = 2.0 * np.einsum("ami,mi->ai", dphi, X) if gga else None
    sigma = np.einsum("ai,ai->i", grad, grad) if gga else None
    c0, cb = og._coefs(xc, rho, grad, sigma, p.grid.weight, 1e-14)
    W = c0[None, :] * phi + (np.einsum("bi,bmi->mi", cb, dphi) if gga else 0.0)
    ncart = [(int(l) + 1) * (int(l) + 2) // 2 for l in p.basis.shell_l]
    atom_of_ao = np.repeat(np.asarray(p.basis.shell_atom, np.int64), ncart)
    ref = np.zeros_like(m0)
    for ax in range(3):
        K = np.abs(dphi[ax]) @ np.abs(W).T
        if gga:
            K += np.abs(np.einsum("bi,bmi->mi", cb, hphi[ax])) @ np.abs(phi).T
        row = np.sum(np.abs(p.D) * K, axis=1)
        for mu, at in enumerate(atom_of_ao):
            ref[at, ax] += 2.0 * row[mu]
    assert np.all(m0 >= 0)
    assert np.abs(m0 - ref).max() <= 1e-12 * ref.max()
    g = og.exc_gradient_blocked(*args, t_b=1e-10)
    m = og.exc_gradient_blocked(*args, t_b=1e-10, magnitude=True)
    print(xc, "max |g| %.3e, max magnitude %.3e" % (np.abs(g).max(), m.max()))
    assert np.all(np.abs(g) <= m * (1 + 1e-12))
