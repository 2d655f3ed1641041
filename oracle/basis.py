"""Basis-on-grid values Phi_{mu i} = chi_mu(r_i) (Sec. II-A, eq. phi_def) -- oracle, FP64.

A basis function is a contracted cartesian Gaussian (Appendix A, "Gaussian basis functions"):
    chi_mu(r) = N_rel(lx,ly,lz) * dx^lx dy^ly dz^lz * sum_k c_k exp(-alpha_k |r - R|^2),
with (dx,dy,dz) = r - R.  The contraction coefficients c_k are inputs that already carry the
normalisation of the x^l component; N_rel = sqrt((2l-1)!! / ((2lx-1)!!(2ly-1)!!(2lz-1)!!)) makes
every cartesian component unit-normalised (reading: the paper prints only x^l y^m z^n exp(-a r^2)).

AO order (caller order): shells in the given order, components within a shell lexicographic
(x, y, z for p; xx, xy, xz, yy, yz, zz for d).

The gradient follows by the product rule:
    d/dx chi = N_rel [lx dx^(lx-1) dy^ly dz^lz R(r^2) + dx^lx dy^ly dz^lz * dx * R1(r^2)],
    R = sum_k c_k e^{-a_k r^2},  R1 = sum_k (-2 a_k) c_k e^{-a_k r^2}.
"""
from __future__ import annotations

import math

import numpy as np

CART = {
    0: [(0, 0, 0)],
    1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def n_rel(lx, ly, lz):
    l = lx + ly + lz
    return math.sqrt(_dfact(2 * l - 1) / (_dfact(2 * lx - 1) * _dfact(2 * ly - 1) * _dfact(2 * lz - 1)))


def n_ao(basis) -> int:
    return int(sum(len(CART[int(l)]) for l in basis.shell_l))


def ao_table(basis):
    """Per-AO (caller order) arrays: shell index, lx, ly, lz, N_rel."""
    sh, lx, ly, lz, nr = [], [], [], [], []
    for s, l in enumerate(basis.shell_l):
        for (a, b, c) in CART[int(l)]:
            sh.append(s)
            lx.append(a)
            ly.append(b)
            lz.append(c)
            nr.append(n_rel(a, b, c))
    return (np.array(sh), np.array(lx), np.array(ly), np.array(lz), np.array(nr))


def eval_ao(atom_xyz, basis, pts, deriv=0):
    """Phi (n_ao x P), and with deriv=1 also dPhi (3 x n_ao x P), at points pts (P x 3, bohr)."""
    pts = np.asarray(pts, dtype=np.float64)
    P = pts.shape[0]
    nao = n_ao(basis)
    phi = np.zeros((nao, P))
    dphi = np.zeros((3, nao, P)) if deriv else None
    mu = 0
    for s in range(len(basis.shell_l)):
        l = int(basis.shell_l[s])
        A = atom_xyz[int(basis.shell_atom[s])]
        d = pts - A[None, :]
        r2 = np.einsum("pi,pi->p", d, d)
        k0, k1 = int(basis.prim_ptr[s]), int(basis.prim_ptr[s + 1])
        R = np.zeros(P)
        R1 = np.zeros(P)
        for k in range(k0, k1):
            e = basis.prim_coef[k] * np.exp(-basis.prim_exp[k] * r2)
            R += e
            R1 += -2.0 * basis.prim_exp[k] * e
        for (a, b, c) in CART[l]:
            nr = n_rel(a, b, c)
            ang = d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c
            phi[mu] = nr * ang * R
            if deriv:
                pw = (a, b, c)
                for ax in range(3):
                    if pw[ax] > 0:
                        q = list(pw)
                        q[ax] -= 1
                        dang = pw[ax] * d[:, 0] ** q[0] * d[:, 1] ** q[1] * d[:, 2] ** q[2]
                    else:
                        dang = 0.0
                    dphi[ax, mu] = nr * (dang * R + ang * d[:, ax] * R1)
            mu += 1
    return (phi, dphi) if deriv else phi


def eval_ao_hess(atom_xyz, basis, pts):
    """Phi (n_ao x P), grad Phi (3 x n_ao x P) and the second derivatives d_a d_b Phi (3 x 3 x n_ao x P).

    With A(d) = dx^lx dy^ly dz^lz and R(r^2) as above, R1 = sum_k (-2 a_k) c_k e^{-a_k r^2} and
    R2 = sum_k (2 a_k)^2 c_k e^{-a_k r^2} (so d_a R = d_a R1, d_b (d_a R1) = delta_ab R1 + d_a d_b R2):
        d_a d_b chi = N_rel [A_ab R + A_a d_b R1 + A_b d_a R1 + A (delta_ab R1 + d_a d_b R2)],
    A_a, A_ab the first and second derivatives of the monomial."""
    pts = np.asarray(pts, dtype=np.float64)
    P = pts.shape[0]
    nao = n_ao(basis)
    phi = np.zeros((nao, P))
    dphi = np.zeros((3, nao, P))
    hphi = np.zeros((3, 3, nao, P))
    mu = 0

    def mono(d, pw):
        return d[:, 0] ** pw[0] * d[:, 1] ** pw[1] * d[:, 2] ** pw[2]

    def dmono(d, pw, ax):
        if pw[ax] == 0:
            return np.zeros(d.shape[0])
        q = list(pw)
        q[ax] -= 1
        return pw[ax] * mono(d, q)

    def d2mono(d, pw, a, b):
        if pw[a] == 0:
            return np.zeros(d.shape[0])
        q = list(pw)
        c = q[a]
        q[a] -= 1
        return c * dmono(d, q, b)

    for s in range(len(basis.shell_l)):
        l = int(basis.shell_l[s])
        A0 = atom_xyz[int(basis.shell_atom[s])]
        d = pts - A0[None, :]
        r2 = np.einsum("pi,pi->p", d, d)
        R = np.zeros(P)
        R1 = np.zeros(P)
        R2 = np.zeros(P)
        for k in range(int(basis.prim_ptr[s]), int(basis.prim_ptr[s + 1])):
            al = float(basis.prim_exp[k])
            e = float(basis.prim_coef[k]) * np.exp(-al * r2)
            R += e
            R1 += -2.0 * al * e
            R2 += 4.0 * al * al * e
        for pw in CART[l]:
            nr = n_rel(*pw)
            A = mono(d, pw)
            Ad = [dmono(d, pw, a) for a in range(3)]
            phi[mu] = nr * A * R
            for a in range(3):
                dphi[a, mu] = nr * (Ad[a] * R + A * d[:, a] * R1)
                for b in range(3):
                    h = d2mono(d, pw, a, b) * R + Ad[a] * d[:, b] * R1 + Ad[b] * d[:, a] * R1
                    h = h + A * ((R1 if a == b else 0.0) + d[:, a] * d[:, b] * R2)
                    hphi[a, b, mu] = nr * h
            mu += 1
    return phi, dphi, hphi
