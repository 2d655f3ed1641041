"""Nuclear gradient of E_xc with the grid held fixed -- oracle, FP64 (test infrastructure only).

The paper reports the EXC gradient beside the energy (Sec. IV-B, Fig. 5(b)).  Here E_xc depends on the
nuclear positions R_A only through the basis functions centred on atom A; the grid points and weights
are held fixed (no grid response, a reading: the paper does not say).  chi_mu depends on r - R_A(mu),
so d chi_mu / d R_A = - grad chi_mu for the functions mu on A.  With X = D Phi and Y^b = D d_b Phi
(rho = sum Phi X and d_b rho = 2 sum d_b Phi X, D symmetric),
    d rho_i / d R_Aa           = -2 sum_{mu on A} d_a chi_mu(r_i) X_{mu i}
    d (d_b rho_i) / d R_Aa     = -2 sum_{mu on A} [d_a d_b chi_mu(r_i) X_{mu i} + d_a chi_mu(r_i) Y^b_{mu i}]
    d E_xc / d R_Aa = sum_i w_i [v_rho,i d rho_i/dR_Aa + 2 v_sigma,i grad rho_i . d grad rho_i/dR_Aa].
Collecting the terms of each basis function mu (c0 = w v_rho, c_b = 2 w v_sigma d_b rho,
G = sum_b c_b d_b Phi, so that sum_b c_b Y^b = D G):
    d E_xc / d R_Aa = -2 sum_{mu on A} sum_i [(c0 d_a Phi + Q^a)_{mu i} X_{mu i} + d_a chi_mu (D G)_{mu i}],
    Q^a = sum_b c_b d_a d_b Phi   (Q = G = 0 for LDA).
Written as products of the Vxc shape,
    d E_xc / d R_Aa = -2 sum_{mu on A} sum_nu D_{mu nu} K^a_{mu nu},
    K^a = (d_a Phi) W^T + Q^a Phi^T,   W = c0 Phi + G,
the form the block-filtered evaluation uses.
"""
from __future__ import annotations

import numpy as np

from . import basis as _basis
from . import functionals as _fx
from . import reorder as _reorder


def _coefs(xc, rho, grad, sigma, w, rho_cut):
    f, vr, vs = _fx.evaluate(xc, rho, sigma, rho_cut)
    c0 = w * vr
    cb = 2.0 * (w * vs)[None, :] * grad if grad is not None else None
    return c0, cb


def exc_gradient(atom_xyz, basis, pts, weights, D, xc, rho_cut=1e-14, chunk=2048):
    """Dense dE_xc/dR (n_atoms x 3) by the definition above, chunked over grid points."""
    atom_xyz = np.asarray(atom_xyz, np.float64)
    pts = np.asarray(pts, np.float64)
    w = np.asarray(weights, np.float64)
    D = np.asarray(D, np.float64)
    gga = _fx.is_gga(xc)
    ncart = [(int(l) + 1) * (int(l) + 2) // 2 for l in basis.shell_l]
    atom_of_ao = np.repeat(np.asarray(basis.shell_atom, np.int64), ncart)
    g_ao = np.zeros((3, D.shape[0]))
    for c0_ in range(0, pts.shape[0], chunk):
        c1_ = min(pts.shape[0], c0_ + chunk)
        phi, dphi, hphi = _basis.eval_ao_hess(atom_xyz, basis, pts[c0_:c1_])
        X = D @ phi
        rho = np.einsum("mi,mi->i", phi, X)
        if gga:
            grad = 2.0 * np.einsum("ami,mi->ai", dphi, X)
            sigma = np.einsum("ai,ai->i", grad, grad)
        else:
            grad = sigma = None
        c0, cb = _coefs(xc, rho, grad, sigma, w[c0_:c1_], rho_cut)
        G = np.einsum("bi,bmi->mi", cb, dphi) if gga else 0.0
        DG = D @ G if gga else 0.0
        for a in range(3):
            H = c0[None, :] * dphi[a]
            if gga:
                H = H + np.einsum("bi,bmi->mi", cb, hphi[a])
                g_ao[a] += np.sum(H * X + dphi[a] * DG, axis=1)
            else:
                g_ao[a] += np.sum(H * X, axis=1)
    out = np.zeros((atom_xyz.shape[0], 3))
    for a in range(3):
        np.add.at(out[:, a], atom_of_ao, -2.0 * g_ao[a])
    return out


def exc_gradient_blocked(atom_xyz, basis, pts, weights, point_atom, D, xc, t_b=1e-10, t_d=None, d_ao=32, G=128,
                         rho_cut=1e-14, shell_order=None, return_count=False, t_grad=None, magnitude=False):
    """The gradient of the block-filtered evaluation: rho, grad rho and the functional exactly as
    oracle.blocked.eval_blocked computes them at thresholds (t_b, t_d; t_d = t_b when not given), then
        dE/dR_Aa = -2 sum_{mu on A} sum_nu D_{mu nu} K^a_{mu nu},
    K^a_{pq} = sum over executed (p, q, r) of (d_a Phi)_pr W_qr^T + Q^a_pr Phi_qr^T, each of the two products
    executing its own tile triples.  Reading (the paper states no filter for the gradient): a product
    A B^T contracted with D executes (p, q, r) when both operand tiles are retained at block r, the D block
    is retained (a_pq >= t_b), and the bound of the triple's contribution passes the pair threshold,
        a_pq * max|A_pr| * max|B_qr| >= t_d,
    the analogue of eq. block_pair_filter for a three-factor term (t_grad, the products' threshold, is t_d
    unless given: the library uses t_d).  return_count: also the number of executed triples over all axes
    and products.  magnitude: instead of the gradient, the same sums taken over absolute values,
        2 sum_{mu on A} sum_nu |D_{mu nu}| sum over executed (p, q, r) of (|A| |B|^T)_{mu nu},
    the scale against which the rounding of the products' operands and sums is bounded."""
    from . import blocked as _blocked
    if t_d is None:
        t_d = t_b
    if t_grad is None:
        t_grad = t_d
    atom_xyz = np.asarray(atom_xyz, np.float64)
    pts = np.asarray(pts, np.float64)
    w = np.asarray(weights, np.float64)
    gga = _fx.is_gga(xc)
    ref = _blocked.eval_blocked(atom_xyz, basis, pts, w, point_atom, D, xc, t_b=t_b, t_d=t_d, d_ao=d_ao, G=G,
                                rho_cut=rho_cut, shell_order=shell_order)
    ao_perm, pt_perm = ref["ao_perm"], ref["pt_perm"]
    nao = len(ao_perm)
    Dp = np.asarray(D, np.float64)[np.ix_(ao_perm, ao_perm)]
    T = _reorder.tiles(nao, d_ao)
    B = _reorder.tiles(len(pt_perm), G)
    S_phi = ref["S_phi"]                                          # [n_tiles, n_blocks]
    a = ref["a"]
    phi, dphi, hphi = _basis.eval_ao_hess(atom_xyz, basis, pts[pt_perm])
    phi, dphi, hphi = phi[ao_perm], dphi[:, ao_perm], hphi[:, :, ao_perm]
    rho = ref["rho"][pt_perm]
    if gga:
        grad = ref["grad"][:, pt_perm]
        sigma = np.einsum("ai,ai->i", grad, grad)
    else:
        grad = sigma = None
    c0, cb = _coefs(xc, rho, grad, sigma, w[pt_perm], rho_cut)
    g_ao = np.zeros((3, nao))
    W = c0[None, :] * phi
    if gga:
        W = W + np.einsum("bi,bmi->mi", cb, dphi)

    def tile_max(X):
        return np.array([[np.max(np.abs(X[t0:t1, r0:r1])) for (r0, r1) in B] for (t0, t1) in T])

    count = 0
    for ax in range(3):
        products = [(dphi[ax], W)]
        if gga:
            products.append((np.einsum("bi,bmi->mi", cb, hphi[ax]), phi))
        K = np.zeros((nao, nao))
        for (Aop, Bop) in products:
            mA, mB = tile_max(Aop), tile_max(Bop)
            for ip, (p0, p1) in enumerate(T):
                for iq, (q0, q1) in enumerate(T):
                    if not a[ip, iq] >= t_b:
                        continue
                    for ir, (r0, r1) in enumerate(B):
                        if S_phi[ip, ir] and S_phi[iq, ir] and a[ip, iq] * mA[ip, ir] * mB[iq, ir] >= t_grad:
                            if magnitude:
                                K[p0:p1, q0:q1] += np.abs(Aop[p0:p1, r0:r1]) @ np.abs(Bop[q0:q1, r0:r1]).T
                            else:
                                K[p0:p1, q0:q1] += Aop[p0:p1, r0:r1] @ Bop[q0:q1, r0:r1].T
                            count += 1
        g_ao[ax] = np.sum((np.abs(Dp) if magnitude else Dp) * K, axis=1)
    ncart = [(int(l) + 1) * (int(l) + 2) // 2 for l in basis.shell_l]
    atom_of_ao = np.repeat(np.asarray(basis.shell_atom, np.int64), ncart)[ao_perm]
    out = np.zeros((atom_xyz.shape[0], 3))
    for ax in range(3):
        np.add.at(out[:, ax], atom_of_ao, (2.0 if magnitude else -2.0) * g_ao[ax])
    return (out, count) if return_count else out
