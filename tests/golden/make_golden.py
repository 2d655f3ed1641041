"""Writes the stored expected values of the full-size parity tests.

Calls only the seeded input generator and the FP64 oracle (never the HIP library):
  cfg1_oracle.json  200-atom chain, PBE: dense E_xc, the electron count, rho and grad rho at 2000
                    seeded random points, and 4000 seeded random entries of Vxc (plus its diagonal).
Run from the repository root:  python tests/golden/make_golden.py
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


def main():
    k = 1
    p = synth.make_problem(k)
    t0 = time.time()
    r = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, p.xc, chunk=4096)
    dt = time.time() - t0
    rng = np.random.default_rng(12345)
    pts = np.sort(rng.choice(p.n_points, 2000, replace=False))
    ij = rng.integers(0, p.n_ao, size=(4000, 2))
    V = r["V"]
    out = {
        "workload": "cfg1: 200-atom chain, 2000 AOs, 4.53M points, PBE, dense (unscreened) FP64 oracle",
        "generator": synth.GENERATOR_VERSION, "seeds": p.meta["seeds"], "oracle_seconds": dt,
        "E": r["E"], "electrons": float(p.grid.weight @ r["rho"]), "n_occ": p.n_occ,
        "rho_idx": pts.tolist(), "rho": r["rho"][pts].tolist(), "grad": r["grad"][:, pts].T.tolist(),
        "v_ij": ij.tolist(), "v": V[ij[:, 0], ij[:, 1]].tolist(), "v_diag": np.diag(V).tolist(),
        "v_maxabs": float(np.abs(V).max()), "v_asym": float(np.abs(V - V.T).max()),
    }
    path = os.path.join(ROOT, "tests", "golden", "cfg1_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "E =", r["E"], "in %.0f s" % dt)


if __name__ == "__main__":
    main()
