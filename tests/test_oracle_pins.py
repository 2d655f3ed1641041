"""Pins of the FP64 oracle against what the paper and the mathematics fix (no GPU).

Each test pins the oracle to something other than itself: closed forms, limits, exact identities,
symbolic differentiation, independent quadrature, brute force and invariances.
"""
import math

import numpy as np
import pytest
import sympy as sp
from scipy import integrate

import oracle
import synth
from oracle import basis as obasis
from oracle import functionals as fx


def _one_shell_problem(l, alpha, n_rad=75, n_ang=302, coef=None):
    c = (2 * alpha / math.pi) ** 0.75 * (4 * alpha) ** (l / 2) / math.sqrt(obasis._dfact(2 * l - 1)) if coef is None else coef
    basis = synth.Basis(np.array([0], np.int32), np.array([l], np.int32), np.array([0, 1], np.int32),
                        np.array([alpha]), np.array([c]))
    xyz = np.zeros((1, 3))
    grid = synth.make_grid(xyz, n_rad, n_ang)
    return basis, xyz, grid


# ---------------------------------------------------------------- P3: LDA closed form on one Gaussian
@pytest.mark.parametrize("alpha,N", [(0.1, 2.0), (1.0, 2.0), (50.0, 1.0), (3.7, 0.6)])
def test_lda_exchange_single_gaussian_closed_form(alpha, N):
    basis, xyz, grid = _one_shell_problem(0, alpha)
    r = oracle.eval_exc(xyz, basis, grid.xyz, grid.weight, np.array([[N]]), "lda")
    exact = -0.6784095460107604 * N ** (4 / 3) * math.sqrt(alpha / math.pi)
    assert abs(r["E"] - exact) <= 1e-10 * abs(exact)
    # the closed form's constant: 4 (3/8)^{3/2} C_x
    assert abs(4 * 0.375 ** 1.5 * fx.CX - 0.6784095460107604) < 1e-15


def test_lda_worked_value():
    # N=2, alpha=1 -> -0.9644735935233615 Eh
    basis, xyz, grid = _one_shell_problem(0, 1.0)
    r = oracle.eval_exc(xyz, basis, grid.xyz, grid.weight, np.array([[2.0]]), "lda")
    assert abs(r["E"] - (-0.9644735935233615)) < 1e-10


# ---------------------------------------------------------------- P11: PBE-x on one Gaussian vs quad
def test_pbe_exchange_single_gaussian_vs_radial_quad():
    alpha, N = 0.8, 2.0
    basis, xyz, grid = _one_shell_problem(0, alpha)
    r = oracle.eval_exc(xyz, basis, grid.xyz, grid.weight, np.array([[N]]), "pbe_x")

    def integrand(x):
        rho = N * (2 * alpha / math.pi) ** 1.5 * math.exp(-2 * alpha * x * x)
        if rho <= 1e-14:          # the oracle's density floor
            return 0.0
        kf = (3 * math.pi ** 2 * rho) ** (1 / 3)
        s2 = (4 * alpha * x) ** 2 / (4 * kf * kf)     # |grad rho| = 4 alpha x rho
        F = 1.804 - 0.804 / (1 + 0.2195149727645171 * s2 / 0.804)
        return 4 * math.pi * x * x * (-0.75 * (3 / math.pi) ** (1 / 3) * rho ** (4 / 3) * F)

    xmax = math.sqrt(math.log(N * (2 * alpha / math.pi) ** 1.5 / 1e-14) / (2 * alpha))
    ref, _ = integrate.quad(integrand, 0, xmax, epsabs=1e-14, epsrel=1e-13, limit=400)
    assert abs(r["E"] - ref) <= 1e-9 * abs(ref)


# ---------------------------------------------------------------- P1: electron count identity
def test_electron_count_in_grid_metric(cfg0):
    p = cfg0
    phi = obasis.eval_ao(p.atom_xyz, p.basis, p.grid.xyz)
    Sg = (phi * p.grid.weight[None, :]) @ phi.T
    rng = np.random.default_rng(3)
    C = rng.normal(size=(p.n_ao, p.n_occ))
    L = np.linalg.cholesky(C.T @ Sg @ C)
    C = np.linalg.solve(L, C.T).T
    D = C @ C.T
    r = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, D, "lda", want_v=False)
    assert abs(p.grid.weight @ r["rho"] - p.n_occ) < 1e-8


def test_electron_count_analytic_metric_grid_quality(cfg0):
    # D is orthonormalised with the analytic (Obara-Saika) overlap: the grid integral of rho
    # reproduces n_occ to quadrature accuracy only
    p = cfg0
    r = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "lda", want_v=False)
    assert abs(p.grid.weight @ r["rho"] - p.n_occ) < 1e-3 * p.n_occ


# ---------------------------------------------------------------- P12: basis normalisation / overlap
@pytest.mark.parametrize("l", [0, 1, 2])
def test_ao_unit_norm_and_one_centre_overlap(l):
    basis, xyz, grid = _one_shell_problem(l, 1.3, n_rad=75, n_ang=2000)
    phi = obasis.eval_ao(xyz, basis, grid.xyz)
    Sg = (phi * grid.weight[None, :]) @ phi.T
    S = synth.overlap_matrix(basis, xyz)
    assert np.allclose(np.diag(S), 1.0, atol=1e-13)
    assert np.abs(Sg - S).max() < 2e-3


def test_two_centre_overlap_on_grid():
    b = synth.make_basis(np.random.default_rng(4), np.array([True, False]))
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.3, 2.1]])
    grid = synth.make_grid(xyz, 75, 1202)
    phi = obasis.eval_ao(xyz, b, grid.xyz)
    Sg = (phi * grid.weight[None, :]) @ phi.T
    S = synth.overlap_matrix(b, xyz)
    assert np.abs(Sg - S).max() < 5e-3


def test_gradient_matches_central_differences():
    p = synth.tiny_problem(n_atoms=2, xc="pbe", seed=21)
    pts = p.grid.xyz[::37][:50]
    phi, dphi = obasis.eval_ao(p.atom_xyz, p.basis, pts, deriv=1)
    h = 1e-5
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        fd = (obasis.eval_ao(p.atom_xyz, p.basis, pts + e) - obasis.eval_ao(p.atom_xyz, p.basis, pts - e)) / (2 * h)
        assert np.abs(fd - dphi[ax]).max() <= 1e-6 * max(1.0, np.abs(dphi[ax]).max())


# ---------------------------------------------------------------- P10: brute-force density
def test_density_brute_force_double_sum():
    p = synth.tiny_problem(n_atoms=3, seed=5)
    pts = p.grid.xyz[::53][:12]
    r = oracle.eval_exc(p.atom_xyz, p.basis, pts, np.ones(len(pts)), p.D, "lda", want_v=False)
    # chi_mu(r) from scratch, one point and one AO at a time
    sh, lx, ly, lz, _ = obasis.ao_table(p.basis)
    for i, x in enumerate(pts):
        chi = []
        for mu in range(p.n_ao):
            s = sh[mu]
            l = p.basis.shell_l[s]
            d = x - p.atom_xyz[p.basis.shell_atom[s]]
            rad = sum(p.basis.prim_coef[k] * math.exp(-p.basis.prim_exp[k] * (d @ d))
                      for k in range(p.basis.prim_ptr[s], p.basis.prim_ptr[s + 1]))
            nrel = math.sqrt(obasis._dfact(2 * l - 1) /
                             (obasis._dfact(2 * lx[mu] - 1) * obasis._dfact(2 * ly[mu] - 1) * obasis._dfact(2 * lz[mu] - 1)))
            chi.append(nrel * d[0] ** lx[mu] * d[1] ** ly[mu] * d[2] ** lz[mu] * rad)
        ref = 0.0
        for mu in range(p.n_ao):
            for nu in range(p.n_ao):
                ref += p.D[mu, nu] * chi[mu] * chi[nu]
        assert abs(r["rho"][i] - ref) <= 1e-13 * max(1.0, abs(ref))


# ---------------------------------------------------------------- P2 / P5: symmetry and V = dE/dD
@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_vxc_symmetric_and_is_energy_derivative(xc):
    p = synth.tiny_problem(n_atoms=3, n_rad=30, n_ang=50, xc=xc, seed=8)
    r = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    V = r["V"]
    assert np.abs(V - V.T).max() <= 1e-14 * np.abs(V).max()
    # direction inside the occupied space, D = C C^T -> Delta = C R C^T: |rho_Delta| <= |R| rho, so
    # rho +- h rho_Delta stays positive and the finite difference sees a smooth E
    lam, U = np.linalg.eigh(p.D)
    C = U[:, -p.n_occ:] * np.sqrt(lam[-p.n_occ:])[None, :]
    rng = np.random.default_rng(9)
    R = rng.normal(size=(p.n_occ, p.n_occ))
    Dl = C @ (0.5 * (R + R.T)) @ C.T
    h = 1e-4
    Ep = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D + h * Dl, xc, want_v=False)["E"]
    Em = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D - h * Dl, xc, want_v=False)["E"]
    fd = (Ep - Em) / (2 * h)
    an = float(np.sum(V * Dl))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


# ---------------------------------------------------------------- P6: scaling laws of exchange
def test_lda_exchange_homogeneity():
    p = synth.tiny_problem(n_atoms=3, n_rad=30, n_ang=50, xc="lda", seed=12)
    E1 = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "lda", want_v=False)["E"]
    lam = 1.7
    E2 = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, lam * p.D, "lda", want_v=False)["E"]
    assert abs(E2 - lam ** (4 / 3) * E1) <= 1e-13 * abs(E2)


@pytest.mark.parametrize("xc", ["lda", "pbe_x"])
def test_exchange_uniform_coordinate_scaling(xc):
    # rho_g(r) = g^3 rho(g r)  =>  E_x[rho_g] = g E_x[rho]  (exact for exchange)
    p = synth.tiny_problem(n_atoms=3, n_rad=30, n_ang=50, xc="pbe", seed=13)
    g = 1.9
    b = p.basis
    l_of_prim = np.repeat(b.shell_l, np.diff(b.prim_ptr))
    bs = synth.Basis(b.shell_atom, b.shell_l, b.prim_ptr, b.prim_exp * g * g,
                     b.prim_coef * g ** (1.5 + l_of_prim))
    E1 = oracle.eval_exc(p.atom_xyz, b, p.grid.xyz, p.grid.weight, p.D, xc, rho_cut=0, want_v=False)["E"]
    E2 = oracle.eval_exc(p.atom_xyz / g, bs, p.grid.xyz / g, p.grid.weight / g ** 3, p.D, xc, rho_cut=0,
                         want_v=False)["E"]
    assert abs(E2 - g * E1) <= 1e-12 * abs(E2)


# ---------------------------------------------------------------- P7 and limits of the PBE forms
def test_pbe_reduces_to_lda_plus_pw92_at_zero_gradient():
    rho = np.logspace(-8, 2, 50)
    f, vr, vs = fx.evaluate("pbe", rho, np.zeros_like(rho), 0.0)
    fl, vl = fx.lda_x(rho)
    rs = (3 / (4 * math.pi * rho)) ** (1 / 3)
    eps, deps = fx.pw92_eps(rs)
    assert np.allclose(f, fl + rho * eps, rtol=1e-14, atol=0)
    assert np.allclose(vr, vl + eps - rs / 3 * deps, rtol=1e-13, atol=0)


def test_pbe_exchange_enhancement_limits():
    rho = np.full(3, 0.3)
    fl, _ = fx.lda_x(rho)
    big = fx.pbe_x(rho, np.full(3, 1e12))[0] / fl
    assert np.allclose(big, 1.804, rtol=1e-9)
    # small s: F_x = 1 + mu s^2, mu = beta pi^2 / 3
    kf = (3 * math.pi ** 2 * 0.3) ** (1 / 3)
    s2 = 1e-6
    sig = s2 * 4 * kf * kf * 0.09
    F = fx.pbe_x(np.array([0.3]), np.array([sig]))[0] / fx.lda_x(np.array([0.3]))[0]
    assert abs(F[0] - 1 - 0.0667245506031492 * math.pi ** 2 / 3 * s2) < 1e-12
    assert abs(fx.MU - 0.2195149727645171) < 1e-15


def test_pbe_correlation_limits():
    rho = np.array([0.01, 0.1, 1.0, 10.0])
    rs = (3 / (4 * math.pi * rho)) ** (1 / 3)
    eps, _ = fx.pw92_eps(rs)
    kf = (3 * math.pi ** 2 * rho) ** (1 / 3)
    ks2 = 4 * kf / math.pi
    # t -> infinity: the gradient correction cancels the local correlation, eps + H -> 0
    t2 = 1e14
    f = fx.pbe_c(rho, t2 * 4 * ks2 * rho * rho)[0]
    assert np.all(np.abs(f / rho) < 1e-9 * np.abs(eps))
    # t -> 0: H = beta t^2 + O(t^4)
    t2 = 1e-8
    H = fx.pbe_c(rho, t2 * 4 * ks2 * rho * rho)[0] / rho - eps
    assert np.allclose(H / t2, 0.06672455060314922, rtol=1e-6)


def test_pw92_high_density_logarithm():
    # eps_c ~ c0 ln r_s + c1 as r_s -> 0, with the exact c0 = (1 - ln 2)/pi^2 (PW92's A = 0.031091)
    r1, r2 = 1e-10, 1e-9
    e1, _ = fx.pw92_eps(np.array([r1]))
    e2, _ = fx.pw92_eps(np.array([r2]))
    slope = (e2[0] - e1[0]) / math.log(r2 / r1)
    assert abs(slope - (1 - math.log(2)) / math.pi ** 2) < 1e-4 * slope


# ---------------------------------------------------------------- P8: derivatives (SymPy + FD)
def _sympy_pbe():
    rho, sig = sp.symbols("rho sigma", positive=True)
    Cx = sp.Rational(3, 4) * (3 / sp.pi) ** sp.Rational(1, 3)
    kappa, beta = sp.Float("0.804", 30), sp.Float("0.06672455060314922", 30)
    mu = beta * sp.pi ** 2 / 3
    kf = (3 * sp.pi ** 2 * rho) ** sp.Rational(1, 3)
    s2 = sig / (4 * kf ** 2 * rho ** 2)
    fxs = -Cx * rho ** sp.Rational(4, 3) * (1 + kappa - kappa / (1 + mu * s2 / kappa))
    A0, a1 = sp.Float("0.031091", 30), sp.Float("0.21370", 30)
    b1, b2, b3, b4 = (sp.Float(v, 30) for v in ("7.5957", "3.5876", "1.6382", "0.49294"))
    rs = (3 / (4 * sp.pi * rho)) ** sp.Rational(1, 3)
    eps = -2 * A0 * (1 + a1 * rs) * sp.log(1 + 1 / (2 * A0 * (b1 * sp.sqrt(rs) + b2 * rs + b3 * rs ** sp.Rational(3, 2) + b4 * rs ** 2)))
    gam = (1 - sp.log(2)) / sp.pi ** 2
    ks = sp.sqrt(4 * kf / sp.pi)
    t2 = sig / (4 * ks ** 2 * rho ** 2)
    A = (beta / gam) / (sp.exp(-eps / gam) - 1)
    H = gam * sp.log(1 + (beta / gam) * t2 * (1 + A * t2) / (1 + A * t2 + A ** 2 * t2 ** 2))
    fcs = rho * (eps + H)
    return rho, sig, fxs, fcs


def test_pbe_derivatives_vs_sympy():
    rho, sig, fxs, fcs = _sympy_pbe()
    ftot = fxs + fcs
    dr = sp.diff(ftot, rho)
    ds = sp.diff(ftot, sig)
    for (r0, s0) in [(1e-3, 1e-7), (0.05, 0.01), (0.7, 0.3), (5.0, 40.0), (2e-6, 1e-12)]:
        f, vr, vs = fx.evaluate("pbe", np.array([r0]), np.array([s0]), 0.0)
        subs = {rho: r0, sig: s0}
        ef = float(ftot.evalf(25, subs=subs))
        er = float(dr.evalf(25, subs=subs))
        es = float(ds.evalf(25, subs=subs))
        assert abs(f[0] - ef) <= 1e-12 * abs(ef)
        assert abs(vr[0] - er) <= 1e-10 * abs(er)
        assert abs(vs[0] - es) <= 1e-10 * abs(es)


def test_functional_derivatives_central_fd():
    rng = np.random.default_rng(1)
    rho = 10 ** rng.uniform(-4, 1, 20)
    sig = rho ** (8 / 3) * 10 ** rng.uniform(-2, 1, 20)
    for xc in ("lda", "pbe"):
        f, vr, vs = fx.evaluate(xc, rho, sig, 0.0)
        h = 1e-6 * rho
        fr = (fx.evaluate(xc, rho + h, sig, 0.0)[0] - fx.evaluate(xc, rho - h, sig, 0.0)[0]) / (2 * h)
        assert np.allclose(vr, fr, rtol=1e-7)
        if xc == "pbe":
            # 5-point stencil; f is dominated by its sigma-independent part, so the rounding floor of
            # the difference quotient is eps |f| / h -- compare on that scale
            hs = 1e-3 * sig
            e = lambda k: fx.evaluate(xc, rho, sig + k * hs, 0.0)[0]
            fs = (-e(2) + 8 * e(1) - 8 * e(-1) + e(-2)) / (12 * hs)
            assert np.all(np.abs(vs - fs) <= 1e-7 * np.abs(vs) + 1e-12 * np.abs(f) / hs)


def test_density_floor():
    f, vr, vs = fx.evaluate("pbe", np.array([1e-15, 0.0, 1e-3]), np.array([1e-20, 0.0, 1e-5]), 1e-14)
    assert f[0] == 0 and vr[0] == 0 and vs[0] == 0 and f[1] == 0
    assert f[2] != 0


# ---------------------------------------------------------------- P9: invariances
def test_translation_and_permutation_invariance():
    p = synth.tiny_problem(n_atoms=3, n_rad=20, n_ang=50, xc="pbe", seed=17)
    r0 = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "pbe")
    t = np.array([1.3, -2.2, 0.7])
    r1 = oracle.eval_exc(p.atom_xyz + t, p.basis, p.grid.xyz + t, p.grid.weight, p.D, "pbe")
    assert abs(r1["E"] - r0["E"]) <= 1e-13 * abs(r0["E"])
    assert np.abs(r1["V"] - r0["V"]).max() <= 1e-12 * np.abs(r0["V"]).max()
    # grid permutation: rho permutes, E and V unchanged
    perm = np.random.default_rng(2).permutation(p.n_points)
    r2 = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz[perm], p.grid.weight[perm], p.D, "pbe")
    assert np.allclose(r2["rho"], r0["rho"][perm], rtol=1e-13, atol=1e-300)
    assert abs(r2["E"] - r0["E"]) <= 1e-13 * abs(r0["E"])
    # shell permutation: V permutes with the AOs
    b = p.basis
    sp_ = np.random.default_rng(3).permutation(b.n_shells)
    nprim = np.diff(b.prim_ptr)
    new_ptr = np.concatenate([[0], np.cumsum(nprim[sp_])]).astype(np.int32)
    idx = np.concatenate([np.arange(b.prim_ptr[s], b.prim_ptr[s + 1]) for s in sp_])
    bp = synth.Basis(b.shell_atom[sp_], b.shell_l[sp_], new_ptr, b.prim_exp[idx], b.prim_coef[idx])
    off = b.ao_offsets()
    ncart = [(l + 1) * (l + 2) // 2 for l in b.shell_l]
    aop = np.concatenate([np.arange(off[s], off[s] + ncart[s]) for s in sp_])
    r3 = oracle.eval_exc(p.atom_xyz, bp, p.grid.xyz, p.grid.weight, p.D[np.ix_(aop, aop)], "pbe")
    assert abs(r3["E"] - r0["E"]) <= 1e-13 * abs(r0["E"])
    assert np.abs(r3["V"] - r0["V"][np.ix_(aop, aop)]).max() <= 1e-12 * np.abs(r0["V"]).max()
