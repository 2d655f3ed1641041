"""GPU parity: libkldi (through its C ABI) against the FP64 CPU oracle on the same seeded inputs."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import reorder

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10363_amd.plan import Plan
    return Plan


def run(Plan, p, xc, prec="fp64", t_b=1e-10, t_d=1e-10, **kw):
    print("case: %s xc=%s prec=%s t_b=%g t_d=%g n_ao=%d n_points=%d" % (p.name, xc, prec, t_b, t_d, p.n_ao,
                                                                         p.n_points), flush=True)
    plan = Plan.from_problem(p, xc=xc, prec=prec, t_b=t_b, t_d=t_d, **kw)
    D = torch.from_numpy(p.D).cuda()
    rho, exc, vxc = plan.eval(D)
    st = plan.check()
    out = dict(rho=rho.cpu().numpy(), E=float(exc.item()), V=vxc.cpu().numpy(), stats=st, info=plan.info(),
               plan=plan)
    return out


def blocked_ref(p, xc, t_b=1e-10, t_d=1e-10):
    return oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc,
                               t_b=t_b, t_d=t_d, d_ao=32, G=128)


TINY = [
    # (n_atoms, n_rad, n_ang, n_occ, seed): ragged AO counts and grid lengths
    (2, 10, 26, 2, 41),
    (4, 16, 50, 4, 42),
    (5, 13, 38, 5, 43),
]


@pytest.mark.parametrize("xc", ["lda", "pbe", "pbe_x"])
@pytest.mark.parametrize("shape", TINY)
def test_tiny_fp64_matches_blocked_oracle(Plan, xc, shape):
    n_atoms, n_rad, n_ang, n_occ, seed = shape
    p = synth.tiny_problem(n_atoms=n_atoms, n_rad=n_rad, n_ang=n_ang, n_occ=n_occ, xc=xc, seed=seed, box_A=4.0)
    ref = blocked_ref(p, xc)
    g = run(Plan, p, xc)
    assert abs(g["E"] - ref["E"]) <= 1e-12 * max(1.0, abs(ref["E"]))
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * max(1.0, np.abs(ref["V"]).max())
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-12 * max(1.0, np.abs(ref["rho"]).max())
    assert np.array_equal(g["V"], g["V"].T)
    assert g["stats"]["n_pairs_x"] == ref["nP_X"]
    assert g["stats"]["n_pairs_v"] == ref["nP_M"]


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_tiny_unscreened_matches_dense_oracle(Plan, xc):
    p = synth.tiny_problem(n_atoms=4, n_rad=14, n_ang=26, n_occ=4, xc=xc, seed=44, box_A=5.0)
    ref = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    g = run(Plan, p, xc, t_b=0.0, t_d=0.0)
    assert g["info"]["retained_fraction"] == 1.0
    assert abs(g["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * np.abs(ref["V"]).max()
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-12 * np.abs(ref["rho"]).max()


def test_plan_structure_matches_oracle_orders_and_retention(Plan, cfg0):
    p = cfg0
    ref = blocked_ref(p, "lda")
    plan = Plan.from_problem(p, xc="lda")
    ao, pt, ret, bmax = plan.structure()
    assert np.array_equal(ao, ref["ao_perm"])
    assert np.array_equal(pt, ref["pt_perm"])
    s = ref["s"].T          # oracle [tile, block] -> [block, tile]
    sure = np.abs(s - 1e-10) > 1e-6 * 1e-10
    assert np.array_equal(ret.astype(bool)[sure], ref["S_phi"].T[sure])
    m = ret.astype(bool)
    assert np.allclose(bmax[m], ref["b"].T[m], rtol=1e-13, atol=0)
    plan.close()


def test_cfg0_fp64_and_fp32(Plan, cfg0):
    p = cfg0
    ref = blocked_ref(p, "lda")
    dense = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "lda")
    g = run(Plan, p, "lda", "fp64")
    assert abs(g["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * np.abs(ref["V"]).max()
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-12 * np.abs(ref["rho"]).max()
    assert (g["stats"]["n_pairs_x"], g["stats"]["n_pairs_v"]) == (ref["nP_X"], ref["nP_M"])
    assert g["stats"]["n_pairs_v_diag"] == 0
    # accuracy targets of the FP32 form (1e-6 Eh, 1e-7 in Vxc) against the unscreened FP64 oracle
    f = run(Plan, p, "lda", "fp32")
    # the FP32 plan runs the same triples, its diagonal ones (p, p, r) on the FP64 diagonal kernel
    assert (f["stats"]["n_pairs_x"], f["stats"]["n_pairs_v"]) == (ref["nP_X"], ref["nP_M"])
    assert f["stats"]["n_pairs_v_diag"] == ref["nP_M_diag"] > 0
    assert abs(f["E"] - dense["E"]) < 1e-6
    assert np.abs(f["V"] - dense["V"]).max() < 1e-7
    big = dense["rho"] > 1e-8
    assert np.max(np.abs(f["rho"][big] - dense["rho"][big]) / dense["rho"][big]) < 1e-5
    print("cfg0 fp32: dE %.3e dV %.3e" % (abs(f["E"] - dense["E"]), np.abs(f["V"] - dense["V"]).max()))


def test_cfg0_geometry_pbe_fp64(Plan, cfg0):
    p = cfg0
    ref = blocked_ref(p, "pbe")
    g = run(Plan, p, "pbe", "fp64")
    assert abs(g["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * np.abs(ref["V"]).max()
    assert (g["stats"]["n_pairs_x"], g["stats"]["n_pairs_v"]) == (ref["nP_X"], ref["nP_M"])


def test_bitwise_deterministic(Plan):
    p = synth.tiny_problem(n_atoms=5, n_rad=14, n_ang=38, n_occ=5, xc="pbe", seed=45, box_A=5.0)
    plan = Plan.from_problem(p, xc="pbe")
    D = torch.from_numpy(p.D).cuda()
    a = [t.cpu().numpy().copy() for t in plan.eval(D)]
    b = [t.cpu().numpy().copy() for t in plan.eval(D)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    plan.close()


def test_nonfinite_density_matrix_is_reported(Plan):
    p = synth.tiny_problem(n_atoms=2, n_rad=10, n_ang=26, n_occ=2, seed=46)
    plan = Plan.from_problem(p)
    D = torch.from_numpy(p.D).cuda()
    D[1, 2] = float("nan")
    plan.eval(D)
    from paper_2605_10363_amd._lib import KldiError
    with pytest.raises(KldiError) as e:
        plan.check()
    assert e.value.status == -6
    plan.close()


def test_rho_only_and_no_vxc(Plan):
    p = synth.tiny_problem(n_atoms=3, n_rad=12, n_ang=26, n_occ=3, xc="pbe", seed=47)
    ref = blocked_ref(p, "pbe")
    plan = Plan.from_problem(p, xc="pbe")
    rho, exc, vxc = plan.eval(torch.from_numpy(p.D).cuda(), vxc=False)
    assert vxc is None
    assert abs(float(exc.item()) - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(rho.cpu().numpy() - ref["rho"]).max() <= 1e-12 * np.abs(ref["rho"]).max()
    plan.close()


@pytest.mark.parametrize("xc,prec", [("lda", "fp64"), ("pbe", "fp64"), ("lda", "fp32"), ("pbe", "fp32"),
                                     ("pbe", "bf16x6")])
def test_grid_chunks_give_identical_results(Plan, cfg0, xc, prec):
    """Processing the grid in several chunks of whole Vxc segments (small Phi/Z workspaces) must give
    bit-identical results to one chunk: the same work items run, and every sum keeps its order.  With FP32
    operands the diagonal Vxc tiles of each chunk run on the side stream and must be joined before the
    next chunk overwrites the workspaces."""
    p = cfg0
    D = torch.from_numpy(p.D).cuda()
    outs = []
    for ct in (0, 40):
        plan = Plan.from_problem(p, xc=xc, prec=prec, v_segment=16, chunk_tiles=ct)
        info = plan.info()
        print("chunk_tiles=%d -> %d grid chunks" % (ct, info["n_grid_chunks"]), flush=True)
        outs.append(([t.cpu().numpy().copy() for t in plan.eval(D)], plan.check(), info["n_grid_chunks"]))
        plan.close()
    (a, sa, na), (b, sb, nb) = outs
    assert na == 1 and nb > 1
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert (sa["n_pairs_x"], sa["n_pairs_v"], sa["n_pairs_v_diag"]) == (sb["n_pairs_x"], sb["n_pairs_v"],
                                                                         sb["n_pairs_v_diag"])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_zero_density_matrix_gives_exact_zeros(Plan, prec):
    """D = 0: every a_pq is 0, so no (p, q) pair is executable (eq. block_pair_filter); rho = 0 gives
    f = v = 0 below the density floor, so Z, every Vxc pair and Vxc vanish.  The oracle gives the same
    exact zeros; the retained structure (which depends on the basis and grid only) is unchanged."""
    p = synth.tiny_problem(n_atoms=3, n_rad=12, n_ang=26, n_occ=3, xc="pbe", seed=47)
    Dz = np.zeros_like(p.D)
    ref = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, Dz, "pbe",
                              t_b=1e-10, t_d=1e-10, d_ao=32, G=128)
    assert ref["E"] == 0.0 and (ref["nP_X"], ref["nP_M"]) == (0, 0)
    print("case: zero D, pbe, prec=%s" % prec, flush=True)
    plan = Plan.from_problem(p, xc="pbe", prec=prec)
    assert plan.info()["n_retained_tiles"] > 0
    rho, exc, vxc = plan.eval(torch.zeros(p.n_ao, p.n_ao, dtype=torch.float64, device="cuda"))
    st = plan.check()
    assert float(exc.item()) == 0.0
    assert not torch.any(rho != 0).item() and not torch.any(vxc != 0).item()
    assert (st["n_pairs_x"], st["n_pairs_v"]) == (0, 0)
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_thresholds_that_retain_nothing(Plan, prec):
    """t_b = t_d = 1e300: no (tile, block) pair is retained (eq. retained_blocks_B), so the plan has no X or
    Vxc work items; every output is an exact zero, as in the oracle at the same thresholds."""
    p = synth.tiny_problem(n_atoms=3, n_rad=12, n_ang=26, n_occ=3, xc="pbe", seed=47)
    ref = blocked_ref(p, "pbe", t_b=1e300, t_d=1e300)
    assert ref["E"] == 0.0 and ref["S_phi"].sum() == 0
    g = run(Plan, p, "pbe", prec=prec, t_b=1e300, t_d=1e300)
    assert g["info"]["n_retained_tiles"] == 0 and g["info"]["n_v_items"] == 0
    assert g["E"] == 0.0 and not np.any(g["rho"]) and not np.any(g["V"])
    assert (g["stats"]["n_pairs_x"], g["stats"]["n_pairs_v"]) == (0, 0)
    g["plan"].close()


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_grid_smaller_than_one_block(Plan, xc):
    """One atom, 15 AOs (a tile with 17 padding rows) and 78 points (one block with 50 padding points of
    weight 0): FP64 to the blocked oracle at 1e-12, the mixed form within its targets."""
    p = synth.tiny_problem(n_atoms=1, n_rad=3, n_ang=26, n_occ=1, xc=xc, seed=48, box_A=3.0)
    assert p.n_ao < 32 and p.n_points < 128
    ref = blocked_ref(p, xc)
    g = run(Plan, p, xc, prec="fp64")
    assert abs(g["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * np.abs(ref["V"]).max()
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-12 * np.abs(ref["rho"]).max()
    assert (g["stats"]["n_pairs_x"], g["stats"]["n_pairs_v"]) == (ref["nP_X"], ref["nP_M"])
    g["plan"].close()
    for prec in ("fp32", "bf16x6"):
        f = run(Plan, p, xc, prec=prec)
        assert abs(f["E"] - ref["E"]) < 1e-6 and np.abs(f["V"] - ref["V"]).max() < 1e-7
        assert np.array_equal(f["V"], f["V"].T)
        f["plan"].close()


def _rho_abs(p):
    """sum_{mu nu} |Phi_mu,i| |D_mu nu| |Phi_nu,i| per point (dense oracle basis): the scale that bounds the
    rounding of rho = sum_{mu nu} Phi_mu,i D_mu nu Phi_nu,i whatever the signs of its terms."""
    from oracle import basis as obasis
    phi = obasis.eval_ao(p.atom_xyz, p.basis, p.grid.xyz, deriv=0)
    a = np.abs(phi[0] if isinstance(phi, tuple) else phi)
    return np.einsum("mi,mi->i", a, np.abs(p.D) @ a)


@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3"])
@pytest.mark.parametrize("xc", ["lda", "pbe"])
@pytest.mark.parametrize("shape", TINY + [None])
def test_split_bf16_forms_against_blocked_oracle(Plan, cfg0, prec, xc, shape):
    """The split-precision X product on BF16 MFMA against the blocked FP64 oracle.  With k pieces per
    operand each of D and Phi is represented to 2^(-8k) relative and the dropped products are of that
    order, so every term Phi_p D_pq Phi_q of rho carries a relative error below 3 * 2^(-8k); FP32
    accumulation of the 32-term products of a K tile and their FP64 flushes add at most 34 * 2^-24 of
    the terms' magnitudes.  Hence |rho - rho_ref| <= (3 * 2^(-8k) + 34 * 2^-24) sum |Phi||D||Phi| per
    point.  Six products (k = 3) also meet the precision targets of the mixed form (1e-6 Eh in E_xc,
    1e-7 in Vxc); three (k = 2) are reported."""
    if shape is None:
        p = cfg0
    else:
        n_atoms, n_rad, n_ang, n_occ, seed = shape
        p = synth.tiny_problem(n_atoms=n_atoms, n_rad=n_rad, n_ang=n_ang, n_occ=n_occ, xc=xc, seed=seed, box_A=4.0)
    ref = blocked_ref(p, xc)
    g = run(Plan, p, xc, prec=prec)
    k = 3 if prec == "bf16x6" else 2
    bound = (3 * 2.0 ** (-8 * k) + 34 * 2.0 ** -24) * _rho_abs(p)
    drho = np.abs(g["rho"] - ref["rho"])
    dE = abs(g["E"] - ref["E"])
    dV = np.abs(g["V"] - ref["V"]).max()
    print("%s %s %s: dE %.3e dV %.3e max drho/bound %.3f" % (p.name, xc, prec, dE, dV, (drho / bound).max()),
          flush=True)
    assert np.all(drho <= bound)
    assert np.array_equal(g["V"], g["V"].T)
    assert g["stats"]["n_pairs_x"] == ref["nP_X"]
    if prec == "bf16x6":
        assert dE < 1e-6 and dV < 1e-7
    g["plan"].close()


@pytest.mark.parametrize("xc", ["lda", "pbe"])
@pytest.mark.parametrize("which", ["tiny", "cfg0"])
def test_overlap_clustered_basis_order(Plan, cfg0, xc, which):
    """Plans whose basis functions follow the overlap-signature clustering (kldi_overlap_order, shell
    order in kldi_opts) against the blocked oracle run with the same shell order (oracle.cluster): FP64 to
    1e-12 with identical executed pair counts, and identical internal AO orders."""
    from paper_2605_10363_amd.plan import overlap_order
    from oracle import cluster
    p = cfg0 if which == "cfg0" else synth.tiny_problem(n_atoms=5, n_rad=14, n_ang=38, n_occ=5, xc=xc, seed=45,
                                                        box_A=5.0)
    S = synth.overlap_matrix(p.basis, p.atom_xyz)
    so_ref, _ = cluster.overlap_shell_order(S, p.basis)
    _, so = overlap_order(p.basis, S)
    assert np.array_equal(so, so_ref)
    ref = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc,
                              t_b=1e-10, t_d=1e-10, d_ao=32, G=128, shell_order=so_ref)
    g = run(Plan, p, xc, shell_order=so)
    ao, _, _, _ = g["plan"].structure()
    assert np.array_equal(ao, ref["ao_perm"])
    assert abs(g["E"] - ref["E"]) <= 1e-12 * max(1.0, abs(ref["E"]))
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * max(1.0, np.abs(ref["V"]).max())
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-12 * max(1.0, np.abs(ref["rho"]).max())
    assert (g["stats"]["n_pairs_x"], g["stats"]["n_pairs_v"]) == (ref["nP_X"], ref["nP_M"])
    print("%s %s: retained fraction %.4f (atom order %.4f)" % (which, xc, g["info"]["retained_fraction"],
                                                             Plan.from_problem(p, xc=xc).info()["retained_fraction"]),
          flush=True)
    g["plan"].close()


@pytest.mark.parametrize("xc", ["lda", "pbe"])
@pytest.mark.parametrize("which", ["tiny", "cfg0"])
def test_256_point_blocks_against_blocked_oracle(Plan, cfg0, xc, which):
    """Grid blocks of 256 points: the library screens and filters per 256-point block (the two 128-point
    blocks of its kernels share the retained tiles and the summaries b_pr, z_qr of the pair); results
    against the oracle run with G = 256 (FP64 to 1e-12, executed pairs counted per 128 points), FP32 within
    the mixed targets, and one grid chunk equal to several bit for bit."""
    p = cfg0 if which == "cfg0" else synth.tiny_problem(n_atoms=5, n_rad=14, n_ang=38, n_occ=5, xc=xc, seed=45,
                                                        box_A=5.0)
    ref = oracle.eval_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc,
                              t_b=1e-10, t_d=1e-10, d_ao=32, G=256, count_unit=128)
    g = run(Plan, p, xc, grid_block=256)
    assert abs(g["E"] - ref["E"]) <= 1e-12 * max(1.0, abs(ref["E"]))
    assert np.abs(g["V"] - ref["V"]).max() <= 1e-12 * max(1.0, np.abs(ref["V"]).max())
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-12 * max(1.0, np.abs(ref["rho"]).max())
    assert (g["stats"]["n_pairs_x"], g["stats"]["n_pairs_v"]) == (ref["nP_X"], ref["nP_M"])
    p128 = Plan.from_problem(p, xc=xc)
    g128 = p128.info()["retained_fraction"]
    p128.close()
    print("%s %s G=256: retained fraction %.4f (G=128 %.4f)" % (which, xc, g["info"]["retained_fraction"], g128),
          flush=True)
    g["plan"].close()
    f = run(Plan, p, xc, prec="fp32", grid_block=256)
    assert abs(f["E"] - ref["E"]) < 1e-6 and np.abs(f["V"] - ref["V"]).max() < 1e-7
    f["plan"].close()
    if which == "cfg0":
        D = torch.from_numpy(p.D).cuda()
        outs = []
        for ct in (0, 40):
            plan = Plan.from_problem(p, xc=xc, prec="fp32", grid_block=256, v_segment=16, chunk_tiles=ct)
            outs.append([t.cpu().numpy().copy() for t in plan.eval(D)] + [plan.info()["n_grid_chunks"]])
            plan.close()
        assert outs[0][3] == 1 and outs[1][3] > 1
        for x, y in zip(outs[0][:3], outs[1][:3]):
            assert np.array_equal(x, y)
