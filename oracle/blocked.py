"""Block-filtered EXC evaluation -- oracle, FP64, literal transcription of Sec. III-B/III-C.

For tiny inputs only (dense Phi is formed).  Steps, in the paper's order and notation:

* Reorder grid points and AOs (Sec. III-B.2, ``reorder``), then cut AO tiles p of d_ao AOs and grid
  blocks r of G points (Sec. III-B.1; rectangular d_ao x G blocks instead of square d x d -- reading).
* Block summaries = max-abs entry of a block (eq. block_summary_A):
      b_pr = max |Phi_pr|,  a_pq = max |D_pq|,
  and for GGA the retention summary of a basis tile also covers its gradient blocks,
      s_pr = max(|Phi_pr|, |dPhi_pr/dx|, |dPhi_pr/dy|, |dPhi_pr/dz|)   (reading; LDA: s_pr = b_pr).
* Retained blocks (eqs. block_filter_A, retained_blocks_A/B):
      S_Phi = {(p,r) : s_pr >= t_b},  S_D = {(p,q) : a_pq >= t_b}.
  Blocks outside S_Phi are zero in Phi and in grad Phi.
* R = D Phi (eq. r_equals_dphi) on retained output blocks only (reading: rho needs X only where Phi
  is retained):  X_pr = sum_{q in E(p,r)} D_pq Phi_qr  (eq. executed_block_output) with
      E(p,r) = {q in I(p,r) : a_pq b_qr >= t_d},  I(p,r) = {q : (p,q) in S_D, (q,r) in S_Phi}
  (eqs. block_intersection, executed_block_pairs); the candidate q are compacted with the
  parallel-addressing prefix sum (Appendix D).
* rho_i = sum_{p:(p,r) in S_Phi} Phi_pi . X_pi;  grad rho_i = 2 sum grad Phi_pi . X_pi.
* functional, E_xc = sum_i w_i f_i.
* Z_qr = w (v_rho Phi_qr / 2 + 2 v_sigma grad rho . grad Phi_qr) on (q,r) in S_Phi, z_qr = max|Z_qr|.
* M = Phi Z^T as the block product C = A B with A = Phi (blocks p x r), B = Z^T (blocks r x q):
      M_pq = sum_{r in E_M(p,q)} Phi_pr Z_qr^T,
      E_M(p,q) = {r : (p,r) in S_Phi, (q,r) in S_Phi, z_qr >= t_b, b_pr z_qr >= t_d}.
* GGA: V = M + M^T.  LDA: M is formed on tiles p <= q only, V_pq = 2 M_pq and V_qp = V_pq^T for
  p < q, V_pp = M_pp + M_pp^T (Sec. III-C.2 exploits symmetry; symmetric by construction -- reading).
* Un-permute rho and V to the caller's order.
"""
from __future__ import annotations

import math

import numpy as np

from . import addressing
from . import basis as _basis
from . import functionals as _fx
from . import reorder as _reorder


def eval_blocked(atom_xyz, basis, pts, weights, point_atom, D, xc, t_b=1e-10, t_d=1e-10,
                 d_ao=32, G=128, rho_cut=1e-14):
    atom_xyz = np.asarray(atom_xyz, np.float64)
    pts = np.asarray(pts, np.float64)
    w = np.asarray(weights, np.float64)
    gga = _fx.is_gga(xc)
    ao_perm, pt_perm, _ = _reorder.orders(atom_xyz, basis, pts, point_atom)
    nao = len(ao_perm)
    npt = len(pt_perm)
    phi_c, dphi_c = _basis.eval_ao(atom_xyz, basis, pts, deriv=1)
    phi = phi_c[ao_perm][:, pt_perm]
    dphi = dphi_c[:, ao_perm][:, :, pt_perm]
    Dp = np.asarray(D, np.float64)[np.ix_(ao_perm, ao_perm)]
    wp = w[pt_perm]
    T = _reorder.tiles(nao, d_ao)
    B = _reorder.tiles(npt, G)
    nT, nB = len(T), len(B)

    # block summaries and retention
    b = np.zeros((nT, nB))
    s = np.zeros((nT, nB))
    for p, (a0, a1) in enumerate(T):
        for r, (g0, g1) in enumerate(B):
            b[p, r] = np.max(np.abs(phi[a0:a1, g0:g1]))
            s[p, r] = max(b[p, r], np.max(np.abs(dphi[:, a0:a1, g0:g1]))) if gga else b[p, r]
    a = np.zeros((nT, nT))
    for p, (a0, a1) in enumerate(T):
        for q, (c0, c1) in enumerate(T):
            a[p, q] = np.max(np.abs(Dp[a0:a1, c0:c1]))
    S_phi = s >= t_b
    S_D = a >= t_b

    # R = D Phi on retained output blocks, executable pairs only
    X = np.zeros((nao, npt))
    nP_X = 0
    for r, (g0, g1) in enumerate(B):
        for p, (a0, a1) in enumerate(T):
            if not S_phi[p, r]:
                continue
            mask = np.array([S_D[p, q] and S_phi[q, r] and a[p, q] * b[q, r] >= t_d for q in range(nT)])
            n_exec, E = addressing.parallel_where(mask)
            nP_X += n_exec
            acc = np.zeros((a1 - a0, g1 - g0))
            for q in E:
                c0, c1 = T[q]
                acc += Dp[a0:a1, c0:c1] @ phi[c0:c1, g0:g1]
            X[a0:a1, g0:g1] = acc

    # density and gradient from retained blocks
    keep = np.zeros((nao, npt), dtype=bool)
    for p, (a0, a1) in enumerate(T):
        for r, (g0, g1) in enumerate(B):
            keep[a0:a1, g0:g1] = S_phi[p, r]
    phik = np.where(keep, phi, 0.0)
    dphik = np.where(keep[None], dphi, 0.0)
    rho = np.einsum("mi,mi->i", phik, X)
    grad = 2.0 * np.einsum("ami,mi->ai", dphik, X)
    sigma = np.einsum("ai,ai->i", grad, grad)
    f, vr, vs = _fx.evaluate(xc, rho, sigma if gga else None, rho_cut)
    E = math.fsum((wp * f).tolist())

    # Z and its block summaries
    Z = 0.5 * (wp * vr)[None, :] * phik
    if gga:
        Z += 2.0 * (wp * vs)[None, :] * np.einsum("ai,ami->mi", grad, dphik)
    z = np.zeros((nT, nB))
    for q, (c0, c1) in enumerate(T):
        for r, (g0, g1) in enumerate(B):
            z[q, r] = np.max(np.abs(Z[c0:c1, g0:g1]))

    # M = Phi Z^T over executable grid blocks
    M = np.zeros((nao, nao))
    nP_M = 0
    for p, (a0, a1) in enumerate(T):
        for q, (c0, c1) in enumerate(T):
            if not gga and q < p:
                continue
            mask = np.array([S_phi[p, r] and S_phi[q, r] and z[q, r] >= t_b and b[p, r] * z[q, r] >= t_d
                             for r in range(nB)])
            n_exec, E_M = addressing.parallel_where(mask)
            nP_M += n_exec
            acc = np.zeros((a1 - a0, c1 - c0))
            for r in E_M:
                g0, g1 = B[r]
                acc += phik[a0:a1, g0:g1] @ Z[c0:c1, g0:g1].T
            M[a0:a1, c0:c1] = acc
    if gga:
        Vp = M + M.T
    else:
        Vp = np.zeros_like(M)
        for p, (a0, a1) in enumerate(T):
            for q, (c0, c1) in enumerate(T):
                if q >= p:
                    Vp[a0:a1, c0:c1] = 2.0 * M[a0:a1, c0:c1]
                    Vp[c0:c1, a0:a1] = 2.0 * M[a0:a1, c0:c1].T
        # a diagonal tile is M_pp + M_pp^T (equal to 2 M_pp up to rounding, and exactly symmetric)
        for p, (a0, a1) in enumerate(T):
            Vp[a0:a1, a0:a1] = M[a0:a1, a0:a1] + M[a0:a1, a0:a1].T

    # back to caller order
    rho_c = np.empty(npt)
    rho_c[pt_perm] = rho
    V = np.empty((nao, nao))
    V[np.ix_(ao_perm, ao_perm)] = Vp
    return dict(rho=rho_c, E=E, V=V, S_phi=S_phi, S_D=S_D, b=b, s=s, a=a, z=z, nP_X=nP_X, nP_M=nP_M,
                ao_perm=ao_perm, pt_perm=pt_perm, n_tiles=nT, n_blocks=nB)
