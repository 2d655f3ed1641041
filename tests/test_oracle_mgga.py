"""The oracle's meta-GGA path (MVS exchange + PBE correlation with the kinetic-energy density tau) against
what the mathematics fixes: derivative checks of the functional, its uniform-gas and single-orbital
limits and uniform-scaling homogeneity, tau by brute force and against the kinetic energy of one
Gaussian in closed form, and Vxc = dE_xc/dD through tau."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import basis as ob
from oracle import functionals as fx


def _pts(n=400, seed=0):
    rng = np.random.default_rng(seed)
    rho = 10 ** rng.uniform(-6, 1, n)
    sig = rho ** (8 / 3) * 10 ** rng.uniform(-3, 1, n)
    tw = sig / (8 * rho)
    tau = tw + fx.CTAU * rho ** (5 / 3) * 10 ** rng.uniform(-2, 0.7, n)
    return rho, sig, tau


@pytest.mark.parametrize("xc", ["mvs", "mvs_x"])
def test_mgga_potentials_match_central_differences(xc):
    rho, sig, tau = _pts()
    f, vr, vs, vt = fx.evaluate_mgga(xc, rho, sig, tau, 0.0)
    for k, v in ((0, vr), (1, vs), (2, vt)):
        args = [rho, sig, tau]
        h = 1e-6 * args[k]
        up = list(args)
        dn = list(args)
        up[k] = args[k] + h
        dn[k] = args[k] - h
        fd = (fx.evaluate_mgga(xc, *up, 0.0)[0] - fx.evaluate_mgga(xc, *dn, 0.0)[0]) / (2 * h)
        scale = np.abs(fd) + np.abs(f) / args[k] * 1e-3
        assert np.all(np.abs(v - fd) <= 1e-6 * scale), k


def test_mvs_limits_and_scaling():
    rho = np.array([1e-3, 0.1, 2.0])
    # uniform gas: sigma = 0, tau = tau_unif -> alpha = 1, F_x = 1: LDA exchange
    f, _, _, _ = fx.mvs_x(rho, 0 * rho, fx.CTAU * rho ** (5 / 3))
    assert np.allclose(f, fx.lda_x(rho)[0], rtol=1e-14, atol=0)
    # one orbital with no gradient weight: alpha = 0, s = 0 -> F_x = 1 + k0
    f0, _, _, _ = fx.mvs_x(rho, 0 * rho, 0 * rho)
    assert np.allclose(f0, (1 + fx.MVS_K0) * fx.lda_x(rho)[0], rtol=1e-14, atol=0)
    # uniform coordinate scaling rho(r) -> lam^3 rho(lam r): s and alpha invariant, f -> lam^4 f
    r, s, t = _pts(50, 3)
    for lam in (0.5, 3.0):
        a = fx.mvs_x(lam ** 3 * r, lam ** 8 * s, lam ** 5 * t)[0]
        assert np.allclose(a, lam ** 4 * fx.mvs_x(r, s, t)[0], rtol=1e-13, atol=0)


def test_tau_brute_force_and_gaussian_kinetic_energy():
    p = synth.tiny_problem(n_atoms=2, n_rad=8, n_ang=26, n_occ=2, xc="pbe", seed=5, box_A=3.0)
    pts = p.grid.xyz[::9][:50]
    _, dphi = ob.eval_ao(p.atom_xyz, p.basis, pts, deriv=1)
    t_ref = np.array([0.5 * sum(p.D[m, n] * np.dot(dphi[:, m, i], dphi[:, n, i])
                                for m in range(p.n_ao) for n in range(p.n_ao)) for i in range(len(pts))])
    r = oracle.eval_exc(p.atom_xyz, p.basis, pts, np.ones(len(pts)), p.D, "mvs", want_v=False)
    assert np.allclose(r["tau"], t_ref, rtol=1e-13, atol=1e-300)
    # one normalised s Gaussian (exponent a) occupied by N electrons: sum_i w_i tau_i = (3/2) a N
    a, N = 0.8, 2.0
    basis = synth.Basis(np.array([0], np.int32), np.array([0], np.int32), np.array([0, 1], np.int32),
                        np.array([a]), np.array([(2 * a / math.pi) ** 0.75]))
    g = synth.make_grid(np.zeros((1, 3)), 75, 302)
    r = oracle.eval_exc(np.zeros((1, 3)), basis, g.xyz, g.weight, np.array([[N]]), "mvs", want_v=False)
    assert abs(np.dot(g.weight, r["tau"]) - 1.5 * a * N) <= 1e-10 * 1.5 * a * N


@pytest.mark.parametrize("xc", ["mvs", "mvs_x"])
def test_mgga_vxc_is_energy_derivative(xc):
    p = synth.tiny_problem(n_atoms=3, n_rad=12, n_ang=26, n_occ=3, xc="pbe", seed=13, box_A=3.5)
    r = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    V = r["V"]
    assert np.abs(V - V.T).max() <= 1e-14 * np.abs(V).max()
    lam, U = np.linalg.eigh(p.D)
    C = U[:, -p.n_occ:] * np.sqrt(lam[-p.n_occ:])[None, :]
    R = np.random.default_rng(2).normal(size=(p.n_occ, p.n_occ))
    Dl = C @ (0.5 * (R + R.T)) @ C.T
    h = 1e-5
    Ep = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D + h * Dl, xc, want_v=False)["E"]
    Em = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D - h * Dl, xc, want_v=False)["E"]
    fd = (Ep - Em) / (2 * h)
    an = float(np.sum(V * Dl))
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_blocked_mgga_without_screening_equals_dense():
    p = synth.tiny_problem(n_atoms=4, n_rad=10, n_ang=26, n_occ=3, xc="pbe", seed=12, box_A=4.0)
    d = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "mvs")
    b = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, "mvs",
                            t_b=0.0, t_d=0.0)
    assert abs(b["E"] - d["E"]) <= 1e-13 * abs(d["E"])
    assert np.abs(b["V"] - d["V"]).max() <= 1e-13 * np.abs(d["V"]).max()
    s = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, "mvs",
                            t_b=1e-10, t_d=1e-10)
    assert abs(s["E"] - d["E"]) <= 1e-8 and np.abs(s["V"] - d["V"]).max() <= 1e-7
