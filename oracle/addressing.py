"""Parallel addressing (Appendix D, Alg. parallel_where) -- oracle.

Each of n "threads" holds a 0/1 flag M[tid] (did its block pair pass the filter).  An exclusive
prefix sum P of length n+1 gives, for every passing thread, its slot in a gap-free output list:
    P[0] = 0,  P[i] = M[0] + ... + M[i-1],  S = P[n],
    if P[tid] != P[tid+1]:  I[P[tid+1] - 1] = tid.
Reading of the "copy M to P, then prefix sum" step: M[tid] is written to P[tid+1] and an inclusive
scan of P follows, which yields the exclusive sum of M.  The scan is carried out as the
log2(n)-step data-parallel (Hillis-Steele) recurrence a thread block would run, so this module
also models the O(log n) step count the paper states.
"""
from __future__ import annotations

import numpy as np


def exclusive_scan_steps(M):
    """Exclusive prefix sum of M (length n+1) by the doubling recurrence; returns (P, steps)."""
    M = np.asarray(M, dtype=np.int64)
    n = M.shape[0]
    P = np.zeros(n + 1, dtype=np.int64)
    P[1:] = M
    steps = 0
    off = 1
    while off < n + 1:
        nxt = P.copy()
        nxt[off:] = P[off:] + P[:-off]
        P = nxt
        off *= 2
        steps += 1
    return P, steps


def parallel_where(M):
    """Order-preserving compaction of the set positions of a 0/1 mask: returns (S, I)."""
    M = np.asarray(M)
    n = M.shape[0]
    P, _ = exclusive_scan_steps(M)
    S = int(P[n])
    I = np.empty(S, dtype=np.int64)
    for tid in range(n):
        v = P[tid + 1]
        if P[tid] != v:
            I[v - 1] = tid
    return S, I
