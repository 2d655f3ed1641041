"""Locality-preserving reordering (Sec. III-B.2; Appendix B.1, eq. morton_code) -- oracle.

Grid points: grouped by their associated atom, then ordered by a 60-bit Morton key within the
group, stable so that equal keys keep their input order.  A coordinate is discretised by
multiplying by 128 and truncating; the three 20-bit integers are bit-interleaved as
    m = sum_k z_k 2^{3k} + y_k 2^{3k+1} + x_k 2^{3k+2}.

Readings where the paper is silent:
* coordinates are in bohr, shifted by the per-axis minimum over all grid points and atom centres
  before scaling, and the scaled integers are clamped to [0, 2^20 - 1];
* the "associated atom" of a point is the atom whose atom-centred grid generated it;
* the groups follow one atom order, the atoms sorted (stably) by the Morton key of their centres;
* basis functions, by default: AOs ordered by the same atom order, each atom's shells kept in their
  input order and each shell's components contiguous; or, given a shell order (the paper's overlap-
  signature clustering, oracle.cluster), the shells in that order, components contiguous.

Also here: the cut into AO tiles of d_ao consecutive (internal) AOs and grid blocks of G
consecutive (internal) points, the last of each ragged (Sec. III-B.1: M_r = ceil(M/d) etc.).
"""
from __future__ import annotations

import numpy as np

SCALE = 128.0
BITS = 20


def discretise(xyz, origin):
    q = np.floor((np.asarray(xyz, np.float64) - origin[None, :]) * SCALE)
    q = np.clip(q, 0, (1 << BITS) - 1)
    return q.astype(np.int64)


def morton_key(ix, iy, iz):
    """Bit-interleave three 20-bit integers per eq. morton_code (bit by bit, no tricks)."""
    ix = np.asarray(ix, np.int64)
    iy = np.asarray(iy, np.int64)
    iz = np.asarray(iz, np.int64)
    m = np.zeros(ix.shape, np.int64)
    for k in range(BITS):
        zk = (iz >> k) & 1
        yk = (iy >> k) & 1
        xk = (ix >> k) & 1
        m |= (zk << (3 * k)) | (yk << (3 * k + 1)) | (xk << (3 * k + 2))
    return m


def origin_of(atom_xyz, pts):
    return np.minimum(np.min(pts, axis=0), np.min(atom_xyz, axis=0))


def atom_order(atom_xyz, origin):
    q = discretise(atom_xyz, origin)
    key = morton_key(q[:, 0], q[:, 1], q[:, 2])
    return np.argsort(key, kind="stable")


def orders(atom_xyz, basis, pts, point_atom, shell_order=None):
    """Returns (ao_perm, pt_perm, atom_perm): internal index -> caller index for AOs, points, atoms.
    shell_order: None (atom order) or the internal sequence of caller shell indices."""
    atom_xyz = np.asarray(atom_xyz, np.float64)
    pts = np.asarray(pts, np.float64)
    origin = origin_of(atom_xyz, pts)
    aperm = atom_order(atom_xyz, origin)
    rank = np.empty_like(aperm)
    rank[aperm] = np.arange(len(aperm))
    # AOs
    ncart = np.array([(l + 1) * (l + 2) // 2 for l in basis.shell_l], np.int64)
    off = np.concatenate([[0], np.cumsum(ncart)[:-1]])
    ao = []
    if shell_order is None:
        shell_order = [s for a in aperm for s in np.nonzero(np.asarray(basis.shell_atom) == a)[0]]
    for s in shell_order:
        ao.extend(range(off[s], off[s] + ncart[s]))
    ao_perm = np.asarray(ao, np.int64)
    # points: primary key atom rank, secondary Morton key, stable
    q = discretise(pts, origin)
    key = morton_key(q[:, 0], q[:, 1], q[:, 2])
    by_key = np.argsort(key, kind="stable")
    by_atom = np.argsort(rank[np.asarray(point_atom)[by_key]], kind="stable")
    pt_perm = by_key[by_atom]
    return ao_perm, pt_perm, aperm


def tiles(n, size):
    """[start, stop) ranges of consecutive chunks of `size` (last one ragged)."""
    return [(s, min(n, s + size)) for s in range(0, n, size)]
