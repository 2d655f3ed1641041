"""GPU parity on the precision form's workload against stored FP64 oracle values: the 200 atoms of the
1000-atom cluster nearest its centroid (synth.subset_problem(2): 1970 AOs, 4.53M points, own grid and
D, PBE), and the largest molecule of the 256-molecule batch under PBE.  The values were written by
tests/golden/make_golden.py with the block-filtered oracle (oracle.blocked.eval_blocked_stream,
t_b = t_d = 1e-10, 32-AO tiles, 128-point blocks), i.e. the result the GPU path computes.

The cluster subset is compact (a 8 A ball at liquid density), so most grid blocks keep every one of its
62 AO tiles, the dense regime of the large clusters; it runs once with the Phi/Z workspaces of all
retained tiles resident (one grid chunk) and once with them limited so that the grid is processed in
several chunks.  Bars: the FP64 path to rounding (1e-9 Eh, 1e-11 in Vxc, 1e-10 relative in rho, executed
pair counts exact); the mixed path within its precision targets (1e-6 Eh in E_xc, 1e-7 max abs in Vxc,
1e-5 relative in rho where rho > 1e-8).
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def errors(g, E, V, r):
    ij = np.array(g["v_ij"])
    dE = abs(E - g["E"])
    dV = max(np.abs(V[ij[:, 0], ij[:, 1]] - np.array(g["v"])).max(), np.abs(np.diag(V) - np.array(g["v_diag"])).max())
    idx = np.array(g["rho_idx"])
    rr = np.array(g["rho"])
    m = rr > 1e-8
    drho = np.max(np.abs(r[idx][m] - rr[m]) / rr[m])
    return dE, dV, drho


def check(plan, p, g, prec, label):
    D = torch.from_numpy(p.D).cuda()
    rho, exc, vxc = plan.eval(D)
    st = plan.check()
    E = float(exc.item())
    V = vxc.cpu().numpy()
    r = rho.cpu().numpy()
    dE, dV, drho = errors(g, E, V, r)
    print("%s %s vs blocked oracle: dE %.3e  dV(sampled) %.3e  drho(rel) %.3e  pairs x %d/%d v %d/%d" % (
        label, prec, dE, dV, drho, st["n_pairs_x"], g["n_pairs_x"], st["n_pairs_v"], g["n_pairs_v"]), flush=True)
    assert np.array_equal(V, V.T)
    assert dE < 1e-6 and dV < 1e-7 and drho < 1e-5
    if prec == "fp64":
        assert (st["n_pairs_x"], st["n_pairs_v"]) == (g["n_pairs_x"], g["n_pairs_v"])
        assert dE < 1e-9 and dV < 1e-11 and drho < 1e-10
    else:
        assert st["n_pairs_x"] == g["n_pairs_x"]
        assert abs(st["n_pairs_v"] - g["n_pairs_v"]) <= 1e-5 * g["n_pairs_v"]


@pytest.fixture(scope="module")
def subset():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.subset_problem(2)
    g = json.load(open(os.path.join(HERE, "cfg2sub_blocked.json")))
    assert g["seeds"] == p.meta["seeds"] and g["generator"] == synth.GENERATOR_VERSION
    assert g["subset"] == p.meta["subset"]
    return p, g


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("chunked", [False, True])
def test_cluster_subset_against_stored_oracle(subset, prec, chunked):
    from paper_2605_10363_amd.plan import Plan
    p, g = subset
    print("case: cfg2 subset prec=%s chunked=%s" % (prec, chunked), flush=True)
    kw = {}
    if chunked:
        # about a third of the retained tiles per chunk: three or more chunks of whole Vxc segments
        probe = Plan.from_problem(p, prec=prec)
        n_ret = probe.info()["n_retained_tiles"]
        probe.close()
        kw = dict(chunk_tiles=n_ret // 3 + 1)
    plan = Plan.from_problem(p, prec=prec, **kw)
    inf = plan.info()
    print("  retained fraction %.4f, max tiles per block %d, %d grid chunks" % (
        inf["retained_fraction"], inf["max_tiles_per_block"], inf["n_grid_chunks"]), flush=True)
    assert inf["n_grid_chunks"] >= (3 if chunked else 1)
    if not chunked:
        assert inf["n_grid_chunks"] == 1
    check(plan, p, g, prec, "cfg2 subset (%d chunks)" % inf["n_grid_chunks"])
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_largest_batch_member_pbe_against_stored_oracle(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10363_amd.plan import Plan
    g = json.load(open(os.path.join(HERE, "member_blocked.json")))
    j = g["member"]
    p = synth.make_batch(n_mol=j + 1, xc="pbe")[j]
    assert g["seeds"] == p.meta["seeds"]
    print("case: batch member %d (%d atoms) PBE prec=%s" % (j, p.n_atoms, prec), flush=True)
    plan = Plan.from_problem(p, prec=prec, xc="pbe")
    check(plan, p, g, prec, "member %d" % j)
    plan.close()
