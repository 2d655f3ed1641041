"""Pointwise exchange-correlation functionals -- oracle, FP64, spin-unpolarised (total density).

The paper's experiments use M06-2X through Libxc (Sec. IV, "Numerical settings"); the workloads here
use the published LDA and PBE forms instead (reading).  Each routine returns the energy per unit
volume f(rho, sigma) (so E_xc = sum_i w_i f_i) and the partial derivatives v_rho = df/drho and
v_sigma = df/dsigma, with sigma = |grad rho|^2.

LDA (Slater/Dirac) exchange:
    f = -C_x rho^{4/3},  C_x = (3/4)(3/pi)^{1/3},  v_rho = -(3/pi)^{1/3} rho^{1/3}.

PBE exchange (Perdew, Burke, Ernzerhof, PRL 77, 3865 (1996)):
    k_F = (3 pi^2 rho)^{1/3},  s^2 = sigma / (4 k_F^2 rho^2),
    F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa),  kappa = 0.804,  mu = beta pi^2 / 3,
    f_x = -C_x rho^{4/3} F_x.

PW92 correlation (Perdew, Wang, PRB 45, 13244 (1992)), zeta = 0:
    r_s = (3 / (4 pi rho))^{1/3},
    eps_c = -2A (1 + a1 r_s) ln(1 + 1 / (2A (b1 r_s^{1/2} + b2 r_s + b3 r_s^{3/2} + b4 r_s^2))).

PBE correlation gradient correction (phi = 1):
    gamma = (1 - ln 2)/pi^2,  k_s = sqrt(4 k_F / pi),  t^2 = sigma / (4 k_s^2 rho^2),
    A = (beta/gamma) / (exp(-eps_c/gamma) - 1),
    H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
    f_c = rho (eps_c + H).

Meta-GGA (the tau path the paper's M06-2X needs; its parameters are not available, so a published
meta-GGA exchange of simple form stands in): MVS exchange (Sun, Perdew, Ruzsinszky, PNAS 112, 685 (2015))
with PBE correlation, tau = (1/2) sum_i |grad psi_i|^2 = (1/2) sum D_{mu nu} grad chi_mu . grad chi_nu,
    alpha = (tau - tau_W) / tau_unif,  tau_W = sigma / (8 rho),  tau_unif = (3/10)(3 pi^2)^{2/3} rho^{5/3},
    F_x = (1 + k0 f(alpha)) / (1 + b s^4)^{1/8},  f(alpha) = (1 - alpha) / ((1 + e1 alpha^2)^2 + c1 alpha^4)^{1/4},
    k0 = 0.174, e1 = -1.6665, c1 = 0.7672, b = 0.0233,   f_x = -C_x rho^{4/3} F_x,
returning also v_tau = df/dtau.

Points with rho <= rho_cut get f = v_rho = v_sigma = 0 (reading: the paper gives no density floor).
"""
from __future__ import annotations

import math

import numpy as np

CX = 0.75 * (3.0 / math.pi) ** (1.0 / 3.0)
KAPPA = 0.804
BETA = 0.06672455060314922
MU = BETA * math.pi ** 2 / 3.0
GAMMA = (1.0 - math.log(2.0)) / math.pi ** 2
PW_A, PW_A1 = 0.031091, 0.21370
PW_B1, PW_B2, PW_B3, PW_B4 = 7.5957, 3.5876, 1.6382, 0.49294


def lda_x(rho):
    rho = np.asarray(rho, dtype=np.float64)
    r13 = np.cbrt(rho)
    f = -CX * rho * r13
    v = -(4.0 / 3.0) * CX * r13
    return f, v


def pbe_x(rho, sigma):
    rho = np.asarray(rho, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    r13 = np.cbrt(rho)
    kf = np.cbrt(3.0 * math.pi ** 2 * rho)
    ds2_dsigma = 1.0 / (4.0 * kf * kf * rho * rho)
    s2 = sigma * ds2_dsigma
    den = 1.0 + MU * s2 / KAPPA
    F = 1.0 + KAPPA - KAPPA / den
    dF = MU / (den * den)                     # dF / d(s^2)
    e_lda = -CX * rho * r13
    f = e_lda * F
    # s^2 is proportional to sigma rho^{-8/3}
    vrho = -CX * r13 * ((4.0 / 3.0) * F - (8.0 / 3.0) * s2 * dF)
    vsigma = e_lda * dF * ds2_dsigma
    return f, vrho, vsigma


def pw92_eps(rs):
    """eps_c(r_s) and d eps_c / d r_s for the unpolarised PW92 fit."""
    rs = np.asarray(rs, dtype=np.float64)
    srs = np.sqrt(rs)
    q0 = -2.0 * PW_A * (1.0 + PW_A1 * rs)
    q1 = 2.0 * PW_A * (PW_B1 * srs + PW_B2 * rs + PW_B3 * rs * srs + PW_B4 * rs * rs)
    dq1 = 2.0 * PW_A * (0.5 * PW_B1 / srs + PW_B2 + 1.5 * PW_B3 * srs + 2.0 * PW_B4 * rs)
    lg = np.log1p(1.0 / q1)
    eps = q0 * lg
    deps = -2.0 * PW_A * PW_A1 * lg - q0 * dq1 / (q1 * q1 + q1)
    return eps, deps


def pbe_c(rho, sigma):
    rho = np.asarray(rho, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    rs = np.cbrt(3.0 / (4.0 * math.pi * rho))
    eps, deps_drs = pw92_eps(rs)
    deps = deps_drs * (-rs / (3.0 * rho))             # d eps / d rho
    kf = np.cbrt(3.0 * math.pi ** 2 * rho)
    ks2 = 4.0 * kf / math.pi
    dt2_dsigma = 1.0 / (4.0 * ks2 * rho * rho)
    t2 = sigma * dt2_dsigma
    em = np.expm1(-eps / GAMMA)
    A = (BETA / GAMMA) / em
    dA_deps = A * A * np.exp(-eps / GAMMA) / BETA
    u = A * t2
    Q = (1.0 + u) / (1.0 + u + u * u)
    dQ_du = -u * (2.0 + u) / (1.0 + u + u * u) ** 2
    y = (BETA / GAMMA) * t2 * Q
    H = GAMMA * np.log1p(y)
    dH_dy = GAMMA / (1.0 + y)
    dy_dt2 = (BETA / GAMMA) * (Q + t2 * dQ_du * A)
    dy_dA = (BETA / GAMMA) * t2 * dQ_du * t2
    # t^2 is proportional to sigma rho^{-7/3}
    dH_drho = dH_dy * (dy_dA * dA_deps * deps + dy_dt2 * (-7.0 / 3.0) * t2 / rho)
    f = rho * (eps + H)
    vrho = eps + H + rho * (deps + dH_drho)
    vsigma = rho * dH_dy * dy_dt2 * dt2_dsigma
    return f, vrho, vsigma


MVS_K0, MVS_E1, MVS_C1, MVS_B = 0.174, -1.6665, 0.7672, 0.0233
CTAU = 0.3 * (3.0 * math.pi ** 2) ** (2.0 / 3.0)


def mvs_x(rho, sigma, tau):
    """MVS exchange: f, v_rho, v_sigma, v_tau."""
    rho = np.asarray(rho, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    r13 = np.cbrt(rho)
    kf = np.cbrt(3.0 * math.pi ** 2 * rho)
    ds2_dsigma = 1.0 / (4.0 * kf * kf * rho * rho)
    s2 = sigma * ds2_dsigma
    tu = CTAU * rho * r13 * r13                      # tau_unif
    tw = sigma / (8.0 * rho)                         # tau_W
    alpha = (tau - tw) / tu
    g = (1.0 + MVS_E1 * alpha ** 2) ** 2 + MVS_C1 * alpha ** 4
    dg = 4.0 * MVS_E1 * alpha * (1.0 + MVS_E1 * alpha ** 2) + 4.0 * MVS_C1 * alpha ** 3
    fa = (1.0 - alpha) * g ** -0.25
    dfa = -g ** -0.25 - 0.25 * (1.0 - alpha) * g ** -1.25 * dg
    den = (1.0 + MVS_B * s2 * s2) ** 0.125
    F = (1.0 + MVS_K0 * fa) / den
    dF_ds2 = -(1.0 + MVS_K0 * fa) * 0.125 * (1.0 + MVS_B * s2 * s2) ** -1.125 * 2.0 * MVS_B * s2
    dF_da = MVS_K0 * dfa / den
    e_lda = -CX * rho * r13
    # d alpha / d rho, d sigma, d tau (tau_unif ~ rho^{5/3}, tau_W ~ sigma / rho)
    da_drho = (sigma / (8.0 * rho * rho)) / tu - (5.0 / 3.0) * alpha / rho
    da_dsigma = -1.0 / (8.0 * rho * tu)
    da_dtau = 1.0 / tu
    f = e_lda * F
    vrho = -(4.0 / 3.0) * CX * r13 * F + e_lda * (dF_ds2 * (-8.0 / 3.0) * s2 / rho + dF_da * da_drho)
    vsigma = e_lda * (dF_ds2 * ds2_dsigma + dF_da * da_dsigma)
    vtau = e_lda * dF_da * da_dtau
    return f, vrho, vsigma, vtau


def evaluate_mgga(xc, rho, sigma, tau, rho_cut=1e-14):
    """(f, v_rho, v_sigma, v_tau) for xc = "mvs" (MVS exchange + PBE correlation) or "mvs_x"; zero wherever
    rho <= rho_cut."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape[0]
    out = [np.zeros(n) for _ in range(4)]
    m = rho > rho_cut
    if not np.any(m):
        return tuple(out)
    r, s, t = rho[m], np.asarray(sigma, np.float64)[m], np.asarray(tau, np.float64)[m]
    fx, vrx, vsx, vtx = mvs_x(r, s, t)
    if xc == "mvs":
        fc, vrc, vsc = pbe_c(r, s)
        fx, vrx, vsx = fx + fc, vrx + vrc, vsx + vsc
    elif xc != "mvs_x":
        raise ValueError(xc)
    out[0][m], out[1][m], out[2][m], out[3][m] = fx, vrx, vsx, vtx
    return tuple(out)


def is_mgga(xc) -> bool:
    return xc in ("mvs", "mvs_x")


def evaluate(xc, rho, sigma=None, rho_cut=1e-14):
    """(f, v_rho, v_sigma) for xc in {"lda", "pbe", "pbe_x"}; zero wherever rho <= rho_cut."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape[0]
    f = np.zeros(n)
    vr = np.zeros(n)
    vs = np.zeros(n)
    m = rho > rho_cut
    if not np.any(m):
        return f, vr, vs
    r = rho[m]
    if xc == "lda":
        f[m], vr[m] = lda_x(r)
        return f, vr, vs
    s = np.asarray(sigma, dtype=np.float64)[m]
    if xc == "pbe":
        fx, vrx, vsx = pbe_x(r, s)
        fc, vrc, vsc = pbe_c(r, s)
        f[m], vr[m], vs[m] = fx + fc, vrx + vrc, vsx + vsc
    elif xc == "pbe_x":
        f[m], vr[m], vs[m] = pbe_x(r, s)
    else:
        raise ValueError(xc)
    return f, vr, vs


def is_gga(xc) -> bool:
    return xc in ("pbe", "pbe_x", "mvs", "mvs_x")
