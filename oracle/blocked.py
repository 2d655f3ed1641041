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
                 d_ao=32, G=128, rho_cut=1e-14, shell_order=None, count_unit=None):
    atom_xyz = np.asarray(atom_xyz, np.float64)
    pts = np.asarray(pts, np.float64)
    w = np.asarray(weights, np.float64)
    gga = _fx.is_gga(xc)
    ao_perm, pt_perm, _ = _reorder.orders(atom_xyz, basis, pts, point_atom, shell_order)
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
    # executed pairs are counted per grid block, or per count_unit points of it (rounded up)
    wt = [1 if not count_unit else -(-(g1 - g0) // count_unit) for (g0, g1) in B]

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
            nP_X += n_exec * wt[r]
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
    mgga = _fx.is_mgga(xc)
    if mgga:
        # tau = (1/2) sum_a sum_p d_a Phi_pr (D d_a Phi)_pr on retained output blocks; the products run
        # over every retained operand tile q with a retained D block (reading: no t_d filter, whose
        # summaries are those of Phi)
        tau = np.zeros(npt)
        for ax in range(3):
            Xa = np.zeros((nao, npt))
            for r, (g0, g1) in enumerate(B):
                for p, (a0, a1) in enumerate(T):
                    if not S_phi[p, r]:
                        continue
                    for q, (c0, c1) in enumerate(T):
                        if S_D[p, q] and S_phi[q, r]:
                            Xa[a0:a1, g0:g1] += Dp[a0:a1, c0:c1] @ dphi[ax][c0:c1, g0:g1]
            tau += 0.5 * np.einsum("mi,mi->i", dphik[ax], Xa)
        f, vr, vs, vt = _fx.evaluate_mgga(xc, rho, sigma, tau, rho_cut)
    else:
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
    nP_M = nP_M_diag = 0
    for p, (a0, a1) in enumerate(T):
        for q, (c0, c1) in enumerate(T):
            if not gga and q < p:
                continue
            mask = np.array([S_phi[p, r] and S_phi[q, r] and z[q, r] >= t_b and b[p, r] * z[q, r] >= t_d
                             for r in range(nB)])
            n_exec, E_M = addressing.parallel_where(mask)
            nP_M += sum(wt[r] for r in E_M)
            if p == q:
                nP_M_diag += sum(wt[r] for r in E_M)
            acc = np.zeros((a1 - a0, c1 - c0))
            for r in E_M:
                g0, g1 = B[r]
                acc += phik[a0:a1, g0:g1] @ Z[c0:c1, g0:g1].T
            M[a0:a1, c0:c1] = acc
    if mgga:
        # the tau term of Vxc, sum_a d_a Phi diag(w v_tau / 4) d_a Phi^T, over every pair of retained
        # tiles of a block (reading: no t_d filter)
        ct = 0.25 * wp * vt
        for p, (a0, a1) in enumerate(T):
            for q, (c0, c1) in enumerate(T):
                for r, (g0, g1) in enumerate(B):
                    if S_phi[p, r] and S_phi[q, r]:
                        for ax in range(3):
                            M[a0:a1, c0:c1] += dphi[ax][a0:a1, g0:g1] @ (ct[g0:g1][None, :] * dphi[ax][c0:c1, g0:g1]).T
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
    grad_c = np.empty((3, npt))
    grad_c[:, pt_perm] = grad
    V = np.empty((nao, nao))
    V[np.ix_(ao_perm, ao_perm)] = Vp
    return dict(rho=rho_c, grad=grad_c, E=E, V=V, S_phi=S_phi, S_D=S_D, b=b, s=s, a=a, z=z, nP_X=nP_X, nP_M=nP_M, nP_M_diag=nP_M_diag,
                ao_perm=ao_perm, pt_perm=pt_perm, n_tiles=nT, n_blocks=nB)


def eval_blocked_stream(atom_xyz, basis, pts, weights, point_atom, D, xc, t_b=1e-10, t_d=1e-10, d_ao=32, G=128,
                        rho_cut=1e-14, blocks_per_chunk=32, v_entries=None, progress=None, shell_order=None,
                        count_unit=None):
    """The same block-filtered evaluation as eval_blocked, one grid block at a time, for inputs whose
    dense Phi does not fit in memory.

    Every quantity of a grid block r (b_pr, s_pr, the executed pairs of X_pr, rho, Z_qr, z_qr and the
    executed pairs of M at r) depends only on D and on the points of block r, so the blocks are
    visited in order and M is accumulated over them.  Within a block, X_r = D^(r) Phi_r with D^(r)
    the matrix D restricted to the retained tiles of r and zero on the tile pairs (p, q) outside
    E(p, r); M += (Phi_r Z_r^T) restricted to the executed tile pairs of E_M at r.  Zero tiles add
    exact zeros, so this is the sum over executed pairs of eq. executed_block_output.

    v_entries: None (full V returned) or an [n, 2] array of caller-order (mu, nu) pairs; then only
    those entries of V are formed (their M_{mu nu} and M_{nu mu} accumulated) and returned as "v".
    Returns rho (caller order), E, V or v, and the executed pair counts nP_X, nP_M.
    """
    atom_xyz = np.asarray(atom_xyz, np.float64)
    pts = np.asarray(pts, np.float64)
    w = np.asarray(weights, np.float64)
    gga = _fx.is_gga(xc)
    ao_perm, pt_perm, _ = _reorder.orders(atom_xyz, basis, pts, point_atom, shell_order)
    nao = len(ao_perm)
    npt = len(pt_perm)
    Dp = np.asarray(D, np.float64)[np.ix_(ao_perm, ao_perm)]
    T = _reorder.tiles(nao, d_ao)
    B = _reorder.tiles(npt, G)
    nT = len(T)
    tile_of = np.repeat(np.arange(nT), d_ao)[:nao]          # internal AO -> its tile

    a = np.zeros((nT, nT))
    for p, (a0, a1) in enumerate(T):
        for q, (c0, c1) in enumerate(T):
            a[p, q] = np.max(np.abs(Dp[a0:a1, c0:c1]))
    S_D = a >= t_b

    inv_ao = np.empty(nao, np.int64)
    inv_ao[ao_perm] = np.arange(nao)
    if v_entries is None:
        M = np.zeros((nao, nao))
    else:
        ve = np.asarray(v_entries, np.int64).reshape(-1, 2)
        vi, vj = inv_ao[ve[:, 0]], inv_ao[ve[:, 1]]               # internal indices
        m_ij = np.zeros(len(ve))
        m_ji = np.zeros(len(ve))
    rho = np.zeros(npt)
    ef = np.zeros(npt)
    nP_X = nP_M = nP_M_diag = 0
    for c0b in range(0, len(B), blocks_per_chunk):
        blocks = B[c0b:c0b + blocks_per_chunk]
        g0c, g1c = blocks[0][0], blocks[-1][1]
        ip = pt_perm[g0c:g1c]
        phi_c, dphi_c = _basis.eval_ao(atom_xyz, basis, pts[ip], deriv=1)
        phi_c = phi_c[ao_perm]
        dphi_c = dphi_c[:, ao_perm]
        for (g0, g1) in blocks:
            ph = phi_c[:, g0 - g0c:g1 - g0c]
            dph = dphi_c[:, :, g0 - g0c:g1 - g0c]
            wr = w[pt_perm[g0:g1]]
            # block summaries and retention at r
            b = np.array([np.max(np.abs(ph[a0:a1])) for (a0, a1) in T])
            if gga:
                s = np.array([max(b[p], np.max(np.abs(dph[:, a0:a1]))) for p, (a0, a1) in enumerate(T)])
            else:
                s = b
            ret = s >= t_b
            R = np.nonzero(ret)[0]
            if len(R) == 0:
                continue
            rows = np.concatenate([np.arange(*T[p]) for p in R])
            # executable pairs of X at r: (p, q) in S_D, q retained, a_pq b_qr >= t_d
            ex = S_D[np.ix_(R, R)] & (a[np.ix_(R, R)] * b[R][None, :] >= t_d)
            wt = 1 if not count_unit else -(-(g1 - g0) // count_unit)
            nP_X += int(ex.sum()) * wt
            tr = np.searchsorted(R, tile_of[rows])                # position of each row's tile in R
            Dm = np.where(ex[np.ix_(tr, tr)], Dp[np.ix_(rows, rows)], 0.0)
            phr = ph[rows]
            dphr = dph[:, rows]
            X = Dm @ phr
            rr = np.einsum("mi,mi->i", phr, X)
            grad = 2.0 * np.einsum("ami,mi->ai", dphr, X)
            sig = np.einsum("ai,ai->i", grad, grad)
            f, vr, vs = _fx.evaluate(xc, rr, sig if gga else None, rho_cut)
            rho[g0:g1] = rr
            ef[g0:g1] = wr * f
            Z = 0.5 * (wr * vr)[None, :] * phr
            if gga:
                Z += 2.0 * (wr * vs)[None, :] * np.einsum("ai,ami->mi", grad, dphr)
            z = np.array([np.max(np.abs(Z[tr == k])) for k in range(len(R))])
            # executable (p, q) of M at r: both retained, z_qr >= t_b, b_pr z_qr >= t_d (LDA: p <= q)
            exm = (z[None, :] >= t_b) & (b[R][:, None] * z[None, :] >= t_d)
            if not gga:
                exm &= R[:, None] <= R[None, :]
            nP_M += int(exm.sum()) * wt
            nP_M_diag += int(np.trace(exm)) * wt
            if v_entries is None:
                Mr = np.where(exm[np.ix_(tr, tr)], phr @ Z.T, 0.0)
                M[np.ix_(rows, rows)] += Mr
            else:
                pos = np.full(nao, -1, np.int64)
                pos[rows] = np.arange(len(rows))
                for (x, y, acc) in ((vi, vj, m_ij), (vj, vi, m_ji)):
                    px, py = pos[x], pos[y]
                    ok = (px >= 0) & (py >= 0)
                    ok[ok] &= exm[tr[px[ok]], tr[py[ok]]]
                    acc[ok] += np.einsum("ki,ki->k", phr[px[ok]], Z[py[ok]])
        if progress is not None:
            progress(c0b + len(blocks), len(B))
    E = math.fsum(ef.tolist())
    rho_c = np.empty(npt)
    rho_c[pt_perm] = rho
    out = dict(rho=rho_c, E=E, nP_X=nP_X, nP_M=nP_M, nP_M_diag=nP_M_diag, ao_perm=ao_perm, pt_perm=pt_perm)
    if v_entries is None:
        if gga:
            Vp = M + M.T
        else:
            Vp = np.zeros_like(M)
            for p, (a0, a1) in enumerate(T):
                for q, (c0, c1) in enumerate(T):
                    if q > p:
                        Vp[a0:a1, c0:c1] = 2.0 * M[a0:a1, c0:c1]
                        Vp[c0:c1, a0:a1] = 2.0 * M[a0:a1, c0:c1].T
                Vp[a0:a1, a0:a1] = M[a0:a1, a0:a1] + M[a0:a1, a0:a1].T
        V = np.empty((nao, nao))
        V[np.ix_(ao_perm, ao_perm)] = Vp
        out["V"] = V
    else:
        if gga:
            v = m_ij + m_ji
        else:
            pi, pj = tile_of[vi], tile_of[vj]
            v = np.where(pi < pj, 2.0 * m_ij, np.where(pi > pj, 2.0 * m_ji, m_ij + m_ji))
        out["v"] = v
    return out
