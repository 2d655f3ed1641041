"""Writes the stored expected values of the full-size parity tests.

Calls only the seeded input generator and the FP64 oracle (never the HIP library).  Both files hold the
same seeded samples: 2000 random grid points and 4000 random (mu, nu) entries of Vxc (plus its
diagonal), drawn from numpy's default_rng(12345).
  cfg1_oracle.json   200-atom chain, PBE: dense (unscreened) evaluation, oracle.eval_exc
  cfg1_blocked.json  the same problem with the block filter at t_b = t_d = 1e-10, d = 32, G = 128,
                     oracle.blocked.eval_blocked_stream (the method's own result at those thresholds)
  cfg2sub_blocked.json  the 200 atoms of the 1000-atom cluster nearest its centroid (synth.subset_problem:
                     1970 AOs, 4.53M points, own grid and D), PBE, block-filtered at 1e-10, d = 32, G = 128
  member_blocked.json   the largest molecule of the 256-molecule batch (synth.make_batch), PBE,
                     block-filtered at 1e-10, d = 32, G = 128
  cfg1_overlap_blocked.json  the 200-atom chain block-filtered at 1e-10 with the basis functions ordered by
                     overlap-signature clustering (oracle.cluster, shell order from the analytic overlap
                     matrix of synth)
Run from the repository root:  python tests/golden/make_golden.py [dense|blocked|cfg2sub|member|overlap]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def samples(p):
    rng = np.random.default_rng(12345)
    pts = np.sort(rng.choice(p.n_points, 2000, replace=False))
    ij = rng.integers(0, p.n_ao, size=(4000, 2))
    return pts, ij


def dense(p):
    t0 = time.time()
    r = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, p.xc, chunk=4096)
    dt = time.time() - t0
    pts, ij = samples(p)
    V = r["V"]
    return {
        "workload": "cfg1: 200-atom chain, 2000 AOs, 4.53M points, PBE, dense (unscreened) FP64 oracle",
        "generator": synth.GENERATOR_VERSION, "seeds": p.meta["seeds"], "oracle_seconds": dt,
        "E": r["E"], "electrons": float(p.grid.weight @ r["rho"]), "n_occ": p.n_occ,
        "rho_idx": pts.tolist(), "rho": r["rho"][pts].tolist(), "grad": r["grad"][:, pts].T.tolist(),
        "v_ij": ij.tolist(), "v": V[ij[:, 0], ij[:, 1]].tolist(), "v_diag": np.diag(V).tolist(),
        "v_maxabs": float(np.abs(V).max()), "v_asym": float(np.abs(V - V.T).max()),
    }


def blocked(p, t=1e-10, label="cfg1: 200-atom chain, 2000 AOs, 4.53M points, PBE", shell_order=None):
    pts, ij = samples(p)
    diag = np.stack([np.arange(p.n_ao)] * 2, 1)
    t0 = time.time()

    def prog(done, tot):
        if done % (32 * 100) == 0 or done == tot:
            print("  %d / %d blocks, %.0f s" % (done, tot, time.time() - t0), flush=True)

    r = oracle.blocked.eval_blocked_stream(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom,
                                           p.D, p.xc, t_b=t, t_d=t, d_ao=32, G=128,
                                           v_entries=np.concatenate([ij, diag]), progress=prog,
                                           shell_order=shell_order)
    dt = time.time() - t0
    v = r["v"]
    return {
        "workload": label + ", block-filtered FP64 oracle (t_b = t_d = %g, d = 32, G = 128)" % t,
        "t_b": t, "t_d": t, "generator": synth.GENERATOR_VERSION, "seeds": p.meta["seeds"], "oracle_seconds": dt,
        "E": r["E"], "electrons": float(p.grid.weight @ r["rho"]), "n_occ": p.n_occ,
        "n_pairs_x": r["nP_X"], "n_pairs_v": r["nP_M"],
        "rho_idx": pts.tolist(), "rho": r["rho"][pts].tolist(),
        "v_ij": ij.tolist(), "v": v[:len(ij)].tolist(), "v_diag": v[len(ij):].tolist(),
    }


def largest_member():
    """Index and problem of the largest molecule of the batching workload, with the PBE functional."""
    sizes = synth.batch_sizes()
    j = int(np.argmax(sizes))
    mols = synth.make_batch(n_mol=j + 1, xc="pbe")
    return j, mols[j]


def main():
    which = sys.argv[1:] or ["dense", "blocked"]
    for w in which:
        if w in ("dense", "blocked"):
            p = synth.make_problem(1)
            out = dense(p) if w == "dense" else blocked(p)
            name = "cfg1_oracle.json" if w == "dense" else "cfg1_blocked.json"
        elif w == "cfg2sub":
            p = synth.subset_problem(2)
            out = blocked(p, label="cfg2 subset: the 200 atoms of the 1000-atom cluster nearest its centroid, "
                                   "%d AOs, %d points, PBE" % (p.n_ao, p.n_points))
            out["subset"] = p.meta["subset"]
            name = "cfg2sub_blocked.json"
        elif w == "overlap":
            from oracle import cluster
            p = synth.make_problem(1)
            so, _ = cluster.overlap_shell_order(synth.overlap_matrix(p.basis, p.atom_xyz), p.basis, lib=True)
            out = blocked(p, label="cfg1: 200-atom chain, 2000 AOs, 4.53M points, PBE, basis functions ordered by "
                                   "overlap-signature clustering", shell_order=so)
            out["shell_order"] = so.tolist()
            name = "cfg1_overlap_blocked.json"
        elif w == "member":
            j, p = largest_member()
            out = blocked(p, label="batch member %d (%d atoms, %d AOs, %d points), PBE" % (
                j, p.n_atoms, p.n_ao, p.n_points))
            out["member"] = j
            name = "member_blocked.json"
        else:
            raise SystemExit("unknown golden %r" % w)
        path = os.path.join(ROOT, "tests", "golden", name)
        with open(path, "w") as f:
            json.dump(out, f)
        print("wrote", path, "E =", out["E"], "in %.0f s" % out["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main()
