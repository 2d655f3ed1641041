"""GPU: the nuclear gradient of E_xc with the grid held fixed (kldi_eval_grad, FP64 and FP32 plans) against
the oracle (oracle.grad): the block-filtered gradient at the same thresholds element by element, the dense
gradient without screening, and at full size central differences of E_xc in atom positions.

FP32 plans round the products' operands to FP32 (relative 2^-24 each) and sum 32 points of a product in
FP32 (at most 32 roundings of 2^-24 of the sum of the terms' magnitudes) before the FP64 running sums, so
a gradient component moves by at most 34 * 2^-24 times the same sums over absolute values
(oracle.grad.exc_gradient_blocked(..., magnitude=True)); the FP32 X product moves rho, grad rho and with
them the products' coefficients by a bound of the same form.  The tests allow 64 * 2^-24 of it."""
import numpy as np
import pytest

import synth
from oracle import grad as og

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10363_amd.plan import Plan
    return Plan


U32 = 2.0 ** -24
FP32_BOUND = 64 * U32


def _grad(Plan, p, xc, with_count=False, prec="fp64", **kw):
    plan = Plan.from_problem(p, xc=xc, prec=prec, **kw)
    D = torch.from_numpy(p.D).cuda()
    exc = torch.empty(1, dtype=torch.float64, device="cuda")
    g = plan.grad(D, exc=exc).cpu().numpy()
    n_prod = plan.check()["n_pairs_v"]        # tile triples of the gradient products
    _, e, _ = plan.eval(D, vxc=False)
    torch.cuda.synchronize()
    assert float(exc.item()) == float(e.item())
    plan.close()
    return (g, n_prod) if with_count else g


@pytest.mark.parametrize("xc", ["lda", "pbe", "pbe_x"])
@pytest.mark.parametrize("shape", [(2, 10, 26, 2, 41), (4, 16, 50, 4, 42), (5, 13, 38, 5, 43)])
def test_tiny_gradient_matches_blocked_oracle(Plan, xc, shape):
    n_atoms, n_rad, n_ang, n_occ, seed = shape
    p = synth.tiny_problem(n_atoms=n_atoms, n_rad=n_rad, n_ang=n_ang, n_occ=n_occ, xc=xc, seed=seed, box_A=4.0)
    print("case: tiny gradient %s xc=%s" % (p.name, xc), flush=True)
    ref, n_ref = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D,
                                         xc, t_b=1e-10, return_count=True)
    g, n = _grad(Plan, p, xc, with_count=True)
    print("  max |dg| %.2e of max |g| %.2e, %d product triples" % (np.abs(g - ref).max(), np.abs(ref).max(), n),
          flush=True)
    assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert n == n_ref


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_gradient_pair_filter_against_blocked_oracle(Plan, xc):
    """A pair threshold large enough to drop product triples on a small molecule (t_d = 1e-6 with t_b =
    1e-10): the same executed triples as the oracle's filter a_pq max|A_pr| max|B_qr| >= t_d, and the same
    gradient to 1e-12."""
    p = synth.tiny_problem(n_atoms=5, n_rad=14, n_ang=38, n_occ=5, xc=xc, seed=47, box_A=5.0)
    print("case: gradient pair filter %s xc=%s" % (p.name, xc), flush=True)
    ref, n_ref = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D,
                                         xc, t_b=1e-10, t_d=1e-6, return_count=True)
    _, n_all = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D,
                                       xc, t_b=1e-10, t_d=1e-6, t_grad=0.0, return_count=True)
    g, n = _grad(Plan, p, xc, with_count=True, t_b=1e-10, t_d=1e-6)
    print("  %d of %d product triples, max |dg| %.2e" % (n, n_all, np.abs(g - ref).max()), flush=True)
    assert n_ref < n_all
    assert n == n_ref
    assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_unscreened_gradient_matches_dense_oracle(Plan, xc):
    p = synth.tiny_problem(n_atoms=4, n_rad=14, n_ang=26, n_occ=4, xc=xc, seed=44, box_A=5.0)
    print("case: unscreened gradient xc=%s" % xc, flush=True)
    ref = og.exc_gradient(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    g = _grad(Plan, p, xc, t_b=0.0, t_d=0.0)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_cfg0_gradient_matches_blocked_oracle(Plan, cfg0, xc):
    p = cfg0
    print("case: cfg0 gradient xc=%s" % xc, flush=True)
    ref = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc,
                                  t_b=1e-10)
    g = _grad(Plan, p, xc)
    print("  max |dg| %.2e of max |g| %.2e" % (np.abs(g - ref).max(), np.abs(ref).max()), flush=True)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("xc", ["lda", "pbe"])
@pytest.mark.parametrize("shape", [(2, 10, 26, 2, 41), (5, 13, 38, 5, 43)])
def test_fp32_gradient_within_rounding_bound_of_blocked_oracle(Plan, xc, shape):
    n_atoms, n_rad, n_ang, n_occ, seed = shape
    p = synth.tiny_problem(n_atoms=n_atoms, n_rad=n_rad, n_ang=n_ang, n_occ=n_occ, xc=xc, seed=seed, box_A=4.0)
    print("case: tiny FP32 gradient %s xc=%s" % (p.name, xc), flush=True)
    args = (p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc)
    ref, n_ref = og.exc_gradient_blocked(*args, t_b=1e-10, return_count=True)
    mag = og.exc_gradient_blocked(*args, t_b=1e-10, magnitude=True)
    g, n = _grad(Plan, p, xc, with_count=True, prec="fp32")
    err = np.abs(g - ref)
    print("  max |dg| %.2e, max |dg| / magnitude %.2e (bound %.2e), %d product triples"
          % (err.max(), (err / np.maximum(mag, 1e-300)).max(), FP32_BOUND, n), flush=True)
    assert np.all(err <= FP32_BOUND * mag + 1e-14)
    assert n == n_ref


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_fp32_gradient_pair_filter_and_unscreened(Plan, xc):
    """FP32 plans: with a pair threshold that drops product triples (t_d = 1e-6) the executed triples are the
    oracle's, and without screening the gradient meets the dense oracle; both within the rounding bound."""
    p = synth.tiny_problem(n_atoms=5, n_rad=14, n_ang=38, n_occ=5, xc=xc, seed=47, box_A=5.0)
    print("case: FP32 gradient pair filter / unscreened %s xc=%s" % (p.name, xc), flush=True)
    args = (p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc)
    for t_b, t_d in ((1e-10, 1e-6), (0.0, 0.0)):
        ref, n_ref = og.exc_gradient_blocked(*args, t_b=t_b, t_d=t_d, return_count=True)
        mag = og.exc_gradient_blocked(*args, t_b=t_b, t_d=t_d, magnitude=True)
        g, n = _grad(Plan, p, xc, with_count=True, prec="fp32", t_b=t_b, t_d=t_d)
        err = np.abs(g - ref)
        print("  t_b %.0e t_d %.0e: %d product triples, max |dg| / magnitude %.2e"
              % (t_b, t_d, n, (err / np.maximum(mag, 1e-300)).max()), flush=True)
        assert n == n_ref
        assert np.all(err <= FP32_BOUND * mag + 1e-14)
    dense = og.exc_gradient(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, xc)
    assert np.abs(ref - dense).max() <= 1e-12 * np.abs(dense).max()   # t = 0: the blocked form is the dense one


@pytest.mark.parametrize("xc", ["lda", "pbe"])
def test_cfg0_fp32_gradient_within_rounding_bound(Plan, cfg0, xc):
    p = cfg0
    print("case: cfg0 FP32 gradient xc=%s" % xc, flush=True)
    args = (p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, p.D, xc)
    ref, n_ref = og.exc_gradient_blocked(*args, t_b=1e-10, return_count=True)
    mag = og.exc_gradient_blocked(*args, t_b=1e-10, magnitude=True)
    g, n = _grad(Plan, p, xc, with_count=True, prec="fp32")
    err = np.abs(g - ref)
    print("  max |dg| %.2e of max |g| %.2e, max |dg| / magnitude %.2e" % (err.max(), np.abs(ref).max(),
          (err / np.maximum(mag, 1e-300)).max()), flush=True)
    assert np.all(err <= FP32_BOUND * mag + 1e-14)
    assert n == n_ref


@pytest.mark.parametrize("xc", ["lda", "pbe"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gradient_grid_chunks_give_identical_results(Plan, cfg0, xc, prec):
    """The gradient of a plan that processes the grid in several chunks (small Phi/Z workspaces) equals that
    of one chunk bit for bit: the same items run, each writes its own partial, and the reduction keeps
    its order."""
    p = cfg0
    outs = []
    for ct in (0, 40):
        print("case: cfg0 gradient xc=%s prec=%s chunk_tiles=%d" % (xc, prec, ct), flush=True)
        plan = Plan.from_problem(p, xc=xc, prec=prec, v_segment=16, chunk_tiles=ct)
        n_chunks = plan.info()["n_grid_chunks"]
        g = plan.grad(torch.from_numpy(p.D).cuda()).cpu().numpy()
        outs.append((g, plan.check()["n_pairs_v"], n_chunks))
        plan.close()
    (ga, na, ca), (gb, nb, cb) = outs
    assert ca == 1 and cb > 1
    assert na == nb
    assert np.array_equal(ga, gb)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gradient_degenerate_inputs_give_exact_zeros(Plan, prec):
    """D = 0 (no D block retained, rho = 0 below the density floor: every coefficient vanishes) and a
    threshold that retains no basis tile both give a gradient of exact zeros with no product executed, as
    the oracle's definition does."""
    p = synth.tiny_problem(n_atoms=3, n_rad=10, n_ang=26, n_occ=3, xc="pbe", seed=45, box_A=4.0)
    for D, t_b in ((np.zeros_like(p.D), 1e-10), (p.D, 1e30)):
        print("case: degenerate gradient prec=%s t_b=%.0e |D|=%.1f" % (prec, t_b, np.abs(D).max()), flush=True)
        plan = Plan.from_problem(p, xc="pbe", prec=prec, t_b=t_b, t_d=t_b)
        g = plan.grad(torch.from_numpy(np.ascontiguousarray(D)).cuda()).cpu().numpy()
        n = plan.check()["n_pairs_v"]
        plan.close()
        ref = og.exc_gradient_blocked(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, D, "pbe",
                                      t_b=t_b, t_d=t_b)
        assert np.all(ref == 0.0)
        assert np.all(g == 0.0)
        assert n == 0


def test_gradient_refuses_unsupported_plans(Plan):
    p = synth.tiny_problem(n_atoms=2, n_rad=10, n_ang=26, n_occ=2, seed=41)
    from paper_2605_10363_amd._lib import KldiError
    plan = Plan.from_problem(p, prec="bf16x6")
    with pytest.raises(KldiError) as e:
        plan.grad(torch.from_numpy(p.D).cuda())
    assert e.value.status == -4
    plan.close()


@pytest.mark.timeout(600)
def test_chain_gradient_matches_energy_differences(Plan):
    """200-atom chain (2000 AOs, 4.53M points, PBE): the FP64 and FP32 gradients of three atom coordinates
    against central differences of the FP64 E_xc (atoms moved with their basis functions, grid fixed) at
    thresholds 1e-14, where the screening sets hardly change with the displacement."""
    p = synth.make_problem(1)
    print("case: chain gradient vs energy differences", flush=True)
    plan = Plan.from_problem(p, prec="fp64", t_b=1e-14, t_d=1e-14)
    D = torch.from_numpy(p.D).cuda()
    g = plan.grad(D).cpu().numpy()
    plan.close()
    plan = Plan.from_problem(p, prec="fp32", t_b=1e-14, t_d=1e-14)
    g32 = plan.grad(D).cpu().numpy()
    plan.close()
    print("  FP32 against FP64 gradient: max |dg| %.2e of max |g| %.2e" % (np.abs(g32 - g).max(), np.abs(g).max()),
          flush=True)
    h = 1e-4
    for A, a in ((0, 0), (57, 1), (150, 2)):
        Es = []
        for sgn in (1, -1):
            xyz = p.atom_xyz.copy()
            xyz[A, a] += sgn * h
            pl = Plan(xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, xc="pbe", prec="fp64", t_b=1e-14,
                      t_d=1e-14)
            Es.append(float(pl.eval(D, vxc=False)[1].item()))
            pl.close()
        fd = (Es[0] - Es[1]) / (2 * h)
        print("  atom %d axis %d: gradient %.10f (FP32 plan %.10f), central difference %.10f"
              % (A, a, g[A, a], g32[A, a], fd), flush=True)
        assert abs(g[A, a] - fd) <= 1e-6 * max(1.0, abs(fd))
        assert abs(g32[A, a] - fd) <= 1e-6 * max(1.0, abs(fd))
