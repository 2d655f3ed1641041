"""Basis-function reordering by overlap-signature clustering -- oracle (test infrastructure only).

Sec. III-B.2 ("Locality-Preserving Reordering") and the appendix on reordering details:

* the overlap signature of basis function i is row i of the overlap matrix S (eq. overlap_signature);
* two functions are compared by the cosine distance of their signatures,
      d(i, j) = 1 - s_i . s_j / (|s_i| |s_j|)                  (eqs. cosine_similarity, cosine_distance);
* agglomerative clustering with average linkage: start from singletons and repeatedly merge the two
  clusters whose average inter-cluster distance (the mean of d over all pairs with one function in each)
  is smallest, until one cluster remains;
* at each merge the two sub-trees are oriented so that their closest leaves meet, and the leaf order of
  the final tree is the basis permutation.

Readings where the paper is silent:
* orientation: the merged leaf sequence is A' + B', A the cluster formed earlier (a singleton counts as
  formed at its index), A' in {A, reversed A}, B' in {B, reversed B}; of the four ways the one whose
  junction pair (last of A', first of B') has the smallest d is taken, ties in the order (A, B),
  (rev A, B), (A, rev B), (rev A, rev B);
* ties between candidate merges go to the pair (a, b), a < b, that comes first in row-major order of the
  cluster ids (singletons 0 .. n-1, merged clusters n, n+1, ... in order of formation).  Exact ties
  arise only from symmetric inputs (one atom alone: its p and d components are equivalent); there
  several leaf orders are average-linkage orders and the library may pick another one;
* the library keeps each shell's cartesian components contiguous (its basis evaluation works per
  shell), so the permutation it applies is a shell order: shells sorted (stably) by the first position
  of any of their components in the leaf order.

average_linkage_order is the plain O(n^3) procedure, meant for small inputs; for a few thousand
functions, average_linkage_order_lib takes the merges from the library routine
scipy.cluster.hierarchy.linkage (method "average", pinned against the plain procedure in the tests) and
applies the same orientation rule to them.
"""
from __future__ import annotations

import numpy as np


def cosine_distance(S):
    """d(i, j) = 1 - s_i . s_j / (|s_i| |s_j|) for the rows s_i of S."""
    S = np.asarray(S, np.float64)
    nrm = np.sqrt(np.sum(S * S, axis=1))
    return 1.0 - (S @ S.T) / np.outer(nrm, nrm)


def average_linkage_order(d):
    """Leaf order and merge list of average-linkage clustering of the distance matrix d.

    Returns (order, merges): order is the leaf permutation; merges[k] = (a, b, dist, size) in the
    numbering of scipy.cluster.hierarchy (cluster n + k is formed by merge k)."""
    d = np.asarray(d, np.float64)
    n = d.shape[0]
    leaves = {i: [i] for i in range(n)}
    active = list(range(n))
    merges = []
    nxt = n
    while len(active) > 1:
        best = None
        for ia in range(len(active)):
            for ib in range(ia + 1, len(active)):
                a, b = active[ia], active[ib]
                dist = float(np.mean(d[np.ix_(leaves[a], leaves[b])]))
                if best is None or dist < best[2]:
                    best = (a, b, dist)
        a, b, dist = best
        A, B = leaves[a], leaves[b]
        cands = [(A, B), (A[::-1], B), (A, B[::-1]), (A[::-1], B[::-1])]
        junction = [d[x[-1], y[0]] for x, y in cands]
        x, y = cands[int(np.argmin(junction))]
        leaves[nxt] = list(x) + list(y)
        merges.append((a, b, dist, len(leaves[nxt])))
        del leaves[a], leaves[b]
        active = [c for c in active if c not in (a, b)] + [nxt]
        nxt += 1
    return np.asarray(leaves[active[0]], np.int64), merges


def _orient(d, merges, n):
    """Leaf order of a merge list (scipy numbering), joining sub-trees by the orientation rule."""
    leaves = {i: [i] for i in range(n)}
    for k, (a, b) in enumerate(merges):
        A, B = leaves.pop(a), leaves.pop(b)
        cands = [(A, B), (A[::-1], B), (A, B[::-1]), (A[::-1], B[::-1])]
        junction = [d[x[-1], y[0]] for x, y in cands]
        x, y = cands[int(np.argmin(junction))]
        leaves[n + k] = list(x) + list(y)
    return np.asarray(leaves[2 * n - 2] if n > 1 else [0], np.int64)


def average_linkage_order_lib(d):
    """The same leaf order from scipy's average-linkage merges (the earlier-formed cluster first)."""
    from scipy.cluster import hierarchy
    from scipy.spatial.distance import squareform
    d = np.asarray(d, np.float64)
    n = d.shape[0]
    if n == 1:
        return np.zeros(1, np.int64)
    dd = 0.5 * (d + d.T)
    np.fill_diagonal(dd, 0.0)
    Z = hierarchy.linkage(squareform(dd, checks=False), method="average")
    merges = [(min(int(z[0]), int(z[1])), max(int(z[0]), int(z[1]))) for z in Z]
    return _orient(d, merges, n)


def shell_order_from_leaves(order, shell_of_ao):
    """Shells sorted (stably) by the first position of any of their AOs in the leaf order."""
    shell_of_ao = np.asarray(shell_of_ao, np.int64)
    first = np.full(int(shell_of_ao.max()) + 1, np.iinfo(np.int64).max)
    for pos, ao in enumerate(np.asarray(order, np.int64)):
        s = shell_of_ao[ao]
        first[s] = min(first[s], pos)
    return np.argsort(first, kind="stable")


def overlap_shell_order(S, basis, lib=False):
    """The shell order the library applies for the overlap-signature reordering of `basis` (lib: take
    the merges from scipy, for large inputs)."""
    ncart = [(int(l) + 1) * (int(l) + 2) // 2 for l in basis.shell_l]
    shell_of_ao = np.repeat(np.arange(len(ncart)), ncart)
    d = cosine_distance(S)
    order = average_linkage_order_lib(d) if lib else average_linkage_order(d)[0]
    return shell_order_from_leaves(order, shell_of_ao), order
