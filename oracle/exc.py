"""Dense EXC evaluation -- oracle, FP64, no screening.

Follows Sec. II-A and Appendix A literally, chunked over grid points only to bound memory:

1. Phi_{mu i} = chi_mu(r_i) (eq. phi_def), and grad Phi for GGA.
2. X = D Phi (eq. r_equals_dphi); rho_i = sum_mu Phi_{mu i} X_{mu i}, which is
   sum_{mu nu} D_{mu nu} chi_mu(r_i) chi_nu(r_i) (Appendix A, "The density matrix").
   For GGA, grad rho_i = 2 sum_mu grad Phi_{mu i} X_{mu i} (D symmetric), sigma_i = |grad rho_i|^2.
3. f_i, v_rho,i, v_sigma,i from the functional (zero where rho_i <= rho_cut).
4. E_xc = sum_i w_i f_i, summed exactly (math.fsum over per-point terms).
5. Z_{mu i} = w_i (v_rho,i Phi_{mu i} / 2 + 2 v_sigma,i grad rho_i . grad Phi_{mu i}),
   M = Phi Z^T,  V = M + M^T.
   For LDA this is V = Phi diag(w v_rho) Phi^T, i.e. F^xc = b Phi W Phi^T with b = 1
   (eq. fxc_matrix_form, eq. w_def); the GGA terms are the standard extension (reading), chosen so
   that V = dE_xc/dD exactly.

Meta-GGA (xc "mvs", "mvs_x"): also tau_i = (1/2) sum_a sum_{mu nu} D_{mu nu} d_a chi_mu d_a chi_nu =
(1/2) sum_a sum_mu d_a Phi_{mu i} (D d_a Phi)_{mu i}, the functional's v_tau, and the Vxc term
(1/2) sum_i w_i v_tau,i grad chi_mu . grad chi_nu (= dE/dD through tau), added to M as
sum_a d_a Phi diag(w v_tau / 4) d_a Phi^T so that V = M + M^T carries it.

All outputs are in the caller's AO and grid order.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis as _basis
from . import functionals as _fx


def eval_exc(atom_xyz, basis, pts, weights, D, xc, rho_cut=1e-14, chunk=4096, want_v=True):
    """Dense FP64 EXC.  Returns dict(rho, grad (3 x P, GGA only), sigma, E, V, f, vrho, vsigma)."""
    pts = np.asarray(pts, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    P = pts.shape[0]
    nao = D.shape[0]
    gga = _fx.is_gga(xc)
    mgga = _fx.is_mgga(xc)
    tau_all = np.zeros(P) if mgga else None
    vt_all = np.zeros(P) if mgga else None
    rho = np.zeros(P)
    grad = np.zeros((3, P)) if gga else None
    sigma = np.zeros(P) if gga else None
    fpt = np.zeros(P)
    vr_all = np.zeros(P)
    vs_all = np.zeros(P)
    M = np.zeros((nao, nao)) if want_v else None
    for c0 in range(0, P, chunk):
        c1 = min(P, c0 + chunk)
        if gga:
            phi, dphi = _basis.eval_ao(atom_xyz, basis, pts[c0:c1], deriv=1)
        else:
            phi = _basis.eval_ao(atom_xyz, basis, pts[c0:c1], deriv=0)
        X = D @ phi
        r = np.einsum("mi,mi->i", phi, X)
        rho[c0:c1] = r
        if gga:
            g = 2.0 * np.einsum("ami,mi->ai", dphi, X)
            grad[:, c0:c1] = g
            s = np.einsum("ai,ai->i", g, g)
            sigma[c0:c1] = s
            if mgga:
                t = 0.5 * sum(np.einsum("mi,mi->i", dphi[a], D @ dphi[a]) for a in range(3))
                tau_all[c0:c1] = t
                f, vr, vs, vt = _fx.evaluate_mgga(xc, r, s, t, rho_cut)
                vt_all[c0:c1] = vt
            else:
                f, vr, vs = _fx.evaluate(xc, r, s, rho_cut)
        else:
            f, vr, vs = _fx.evaluate(xc, r, None, rho_cut)
        fpt[c0:c1] = f
        vr_all[c0:c1] = vr
        vs_all[c0:c1] = vs
        if want_v:
            Z = 0.5 * (w[c0:c1] * vr)[None, :] * phi
            if gga:
                gd = np.einsum("ai,ami->mi", g, dphi)
                Z += 2.0 * (w[c0:c1] * vs)[None, :] * gd
            M += phi @ Z.T
            if mgga:
                ct = 0.25 * w[c0:c1] * vt
                for a in range(3):
                    M += dphi[a] @ (ct[None, :] * dphi[a]).T
    E = math.fsum((w * fpt).tolist())
    out = dict(rho=rho, E=E, f=fpt, vrho=vr_all, vsigma=vs_all)
    if gga:
        out["grad"] = grad
        out["sigma"] = sigma
    if mgga:
        out["tau"] = tau_all
        out["vtau"] = vt_all
    if want_v:
        out["V"] = M + M.T
    return out


def rho_at_points(atom_xyz, basis, pts, D):
    """rho (and grad rho) at a few points, by the same definition; for sampled checks."""
    phi, dphi = _basis.eval_ao(atom_xyz, basis, pts, deriv=1)
    X = D @ phi
    return np.einsum("mi,mi->i", phi, X), 2.0 * np.einsum("ami,mi->ai", dphi, X)
