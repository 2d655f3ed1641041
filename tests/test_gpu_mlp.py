"""GPU: the learned functional surrogate and the auxiliary entry points, through the C ABI, against the
FP64 oracle (oracle.mlp, oracle.functionals, oracle.exc)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import functionals as fx
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10363_amd import plan as m
    return m


def test_xc_eval_arrays_match_oracle(mod):
    rng = np.random.default_rng(3)
    rho = 10 ** rng.uniform(-12, 2, 5000)
    sig = rho ** (8 / 3) * 10 ** rng.uniform(-4, 2, 5000)
    # PBE's mu = beta pi^2 / 3 makes the gradient terms of exchange and correlation cancel to leading
    # order in s, so v_sigma of "pbe" is a small difference of two larger parts: its rounding error is
    # bounded relative to |v_sigma,x| + |v_sigma,c|, not to |v_sigma|
    vs_scale = np.abs(fx.pbe_x(rho, sig)[2]) + np.abs(fx.pbe_c(rho, sig)[2])
    for xc in ("lda", "pbe", "pbe_x"):
        f, vr, vs = mod.xc_eval(xc, torch.from_numpy(rho).cuda(), torch.from_numpy(sig).cuda(), 1e-14)
        ef, evr, evs = fx.evaluate(xc, rho, sig, 1e-14)
        assert np.allclose(f.cpu().numpy(), ef, rtol=1e-12, atol=0)
        assert np.allclose(vr.cpu().numpy(), evr, rtol=1e-12, atol=0)
        if xc != "lda":
            dvs = np.abs(vs.cpu().numpy() - evs)
            print("%s: max |dv_sigma| / (|v_sigma,x| + |v_sigma,c|) = %.2e" % (xc, (dvs / vs_scale).max()))
            assert np.all(dvs <= 1e-12 * vs_scale)


def test_eval_grid_rho_and_sigma(mod):
    p = synth.tiny_problem(n_atoms=4, n_rad=14, n_ang=38, n_occ=4, xc="pbe", seed=61, box_A=4.0)
    ref = oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.D, "pbe", want_v=False)
    plan = mod.Plan.from_problem(p, xc="pbe", t_b=0.0, t_d=0.0)
    rho, sigma = plan.eval_grid(torch.from_numpy(p.D).cuda())
    assert np.allclose(rho.cpu().numpy(), ref["rho"], rtol=1e-12, atol=1e-300)
    assert np.allclose(sigma.cpu().numpy(), ref["sigma"], rtol=1e-11, atol=1e-300)
    plan.close()


def test_training_kernel_gradient_matches_fp64_oracle(mod):
    rng = np.random.default_rng(4)
    net = mod.Mlp(seed=11)
    theta = omlp.init_params(rng) + 0.05 * rng.normal(size=omlp.N_PARAMS)
    net.params(set_params=theta.astype(np.float32))
    th32 = theta.astype(np.float32).astype(np.float64)
    for n in (1, 63, 64, 1000, 4099):
        x = rng.uniform(-1, 1, size=(n, 2)).astype(np.float32)
        t = rng.normal(size=(n, 3)).astype(np.float32)
        L, g = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
        Lr, gr = omlp.loss_and_grad(th32, x.astype(np.float64), t.astype(np.float64))
        print("n=%d loss %.8f oracle %.8f  max|dg| %.2e  max|g| %.2e" % (n, L, Lr, np.abs(g - gr).max(),
                                                                       np.abs(gr).max()), flush=True)
        assert abs(L - Lr) <= 1e-5 * Lr
        assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()
    net.close()


@pytest.fixture(scope="module")
def trained(mod):
    """A surrogate trained on the (rho, sigma) points of the 12-atom workload's grid with PBE geometry."""
    p = synth.make_problem(0)
    plan = mod.Plan.from_problem(p, xc="pbe")
    rho, sigma = plan.eval_grid(torch.from_numpy(p.D).cuda())
    net = mod.Mlp(seed=5)
    losses = net.train(rho, sigma, epochs=40, batch=8192, lr=3e-3, seed=9, xc="pbe", rho_min=1e-8)
    print("training loss per epoch:", np.array2string(losses[[0, 9, 19, 39]], precision=5), flush=True)
    return p, plan, net, rho, sigma, losses


def test_training_reduces_loss(trained):
    p, plan, net, rho, sigma, losses = trained
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.05 * losses[0]


def test_adam_steps_match_oracle_update(mod):
    """Several kldi_mlp_step calls against oracle.mlp.adam_step, element by element.  Each step is fed
    the gradient the library computes for the batch (kldi_mlp_loss_grad returns exactly the reduced
    gradient the step uses), so the check isolates the update rule; the gradient itself is checked
    against the oracle above.  The oracle keeps its moments in FP64; the kernels keep FP32 moments
    and FP32 parameters, so each updated parameter may differ by the FP32 rounding of the update."""
    rng = np.random.default_rng(21)
    net = mod.Mlp(seed=3)
    theta = omlp.init_params(rng) + 0.05 * rng.normal(size=omlp.N_PARAMS)
    net.params(set_params=theta.astype(np.float32))
    m = np.zeros(omlp.N_PARAMS)
    v = np.zeros(omlp.N_PARAMS)
    lr = 1e-3
    for k in range(1, 7):
        n = int(rng.integers(50, 3000))
        x = torch.from_numpy(rng.uniform(-1, 1, size=(n, 2)).astype(np.float32)).cuda()
        t = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).cuda()
        th0 = net.params()[0].astype(np.float64)
        L0, g = net.loss_grad(x, t)
        L1 = net.step(x, t, lr)
        th1 = net.params()[0].astype(np.float64)
        ref, m, v = omlp.adam_step(th0, g.astype(np.float64), m, v, k, lr=lr)
        d = np.abs(th1 - ref)
        tol = 4 * 2.0 ** -24 * np.abs(ref) + 1e-5 * lr
        print("step %d (n=%d): loss %.6f, max|dtheta| %.2e (of tolerance %.2f), max|update| %.2e" % (
            k, n, L1, d.max(), (d / tol).max(), np.abs(ref - th0).max()), flush=True)
        assert L1 == L0
        assert np.all(d <= tol)
        assert np.abs(ref - th0).max() > 0.5 * lr           # the step moved the parameters
    net.close()


def test_inference_matches_oracle_forward_and_falls_back(mod, trained):
    """BF16 inference against the oracle network with the same weights rounded to BF16, within the
    oracle's running error bound for FP32 accumulation and BF16 activations (oracle.mlp.bf16_inference)."""
    p, plan, net, rho, sigma, losses = trained
    theta, box, tm, ts = net.params()
    r = rho.cpu().numpy()
    s = sigma.cpu().numpy()
    f, vr, vs, used = net.forward(rho, sigma)
    f, vr, vs, used = f.cpu().numpy(), vr.cpu().numpy(), vs.cpu().numpy(), used.cpu().numpy().astype(bool)
    assert np.array_equal(used, r >= 1e-8)             # the box is the training range
    x = omlp.features(r[used], s[used], box)
    y, ey = omlp.bf16_inference(theta.astype(np.float64), x)
    yg = (omlp.targets(r[used], f[used], vr[used], vs[used]) - tm) / ts
    dy = np.abs(yg - y)
    y64, _ = omlp.forward(theta.astype(np.float64), x)
    print("inference |dy| max %.3e mean %.3e, bound max %.3e, largest share of the bound %.3f; BF16 weights "
          "alone move the heads by up to %.3e" % (dy.max(), dy.mean(), ey.max(), (dy / ey).max(),
                                                np.abs(y - y64).max()), flush=True)
    assert np.all(dy <= ey * (1 + 1e-6) + 1e-12)
    # fallback points are the analytic functional
    af, avr, avs = fx.evaluate("pbe", r[~used], s[~used], 0.0)
    assert np.allclose(f[~used], af, rtol=1e-12, atol=1e-300)
    assert np.allclose(vr[~used], avr, rtol=1e-12, atol=1e-300)


def _network_energy(net, rho, sigma, w):
    """E_xc of the oracle network (BF16-rounded weights, FP64) on the library's rho, sigma: the network
    where the library used it, PBE elsewhere; and the bound on the library's E from the inference bound."""
    theta, box, tm, ts = net.params()
    r, s = rho.cpu().numpy(), sigma.cpu().numpy()
    used = net.forward(rho, sigma)[3].cpu().numpy().astype(bool)
    f = fx.evaluate("pbe", r, s, 1e-14)[0]
    y, ey = omlp.bf16_inference(theta.astype(np.float64), omlp.features(r[used], s[used], box))
    r43 = r[used] ** (4.0 / 3.0)
    f[used] = (y[:, 0] * ts[0] + tm[0]) * r43
    bound = float(np.sum(np.abs(w[used]) * ey[:, 0] * ts[0] * r43)) + 1e-12 * float(np.sum(np.abs(w * f)))
    return float(np.sum(w * f)), bound, used


def test_attached_surrogate_in_evaluation(mod, trained):
    """The trained network replaces the analytic PBE inside kldi_eval: E_xc equals the oracle network's
    energy within the inference bound; what the network gains over the analytic functional (time of
    the functional stage, error) is reported."""
    p, plan, net, rho, sigma, losses = trained
    D = torch.from_numpy(p.D).cuda()
    _, e_an, v_an = plan.eval(D)
    plan.timing(True)
    for _ in range(3):
        plan.eval(D)
    st_an, _ = plan.stage_ms()
    plan.attach_mlp(net)
    _, e_ml, v_ml = plan.eval(D)
    stats = plan.check()
    plan.timing(True)
    for _ in range(3):
        plan.eval(D)
    st_ml, _ = plan.stage_ms()
    E_an, E_ml = float(e_an.item()), float(e_ml.item())
    E_net, bound, used = _network_energy(net, rho, sigma, p.grid.weight)
    dV = float((v_ml - v_an).abs().max().item())
    frac = stats["n_points_mlp"] / p.n_points
    print("surrogate: E %.10f, oracle network %.10f (|d| %.2e, bound %.2e); analytic %.10f (rel %.2e), "
          "max|dV| vs analytic %.2e, network on %.1f%% of points, functional stage %.3f ms vs %.3f ms analytic" % (
              E_ml, E_net, abs(E_ml - E_net), bound, E_an, abs(E_ml - E_an) / abs(E_an), dV, 100 * frac,
              st_ml["xfunc"], st_an["xfunc"]), flush=True)
    assert stats["n_points_mlp"] == int(used.sum())
    assert abs(E_ml - E_net) <= bound
    plan.attach_mlp(None)
    _, e_back, _ = plan.eval(D)
    assert float(e_back.item()) == E_an


def test_retraining_after_attach_is_seen_by_the_plan(mod, trained):
    """A plan holds a view of the network's device memory: training again after attaching changes the
    weights, range box and target statistics, and the next evaluation (eager or a captured graph)
    uses the new ones.  The first training range (rho >= 1e-2) covers few grid points, the second
    (rho >= 1e-8) nearly all, so a plan that kept the first box would count the wrong number of
    network points."""
    p, plan, net0, rho, sigma, losses = trained
    D = torch.from_numpy(p.D).cuda()
    net = mod.Mlp(seed=8)
    with pytest.raises(mod.L.KldiError) as ei:
        plan.attach_mlp(net)                           # not trained yet
    assert ei.value.status == -5
    keep = rho >= 1e-2
    net.train(rho[keep].contiguous(), sigma[keep].contiguous(), epochs=5, batch=8192, lr=3e-3, seed=1, xc="pbe")
    plan.attach_mlp(net)
    counts = []
    for phase in (0, 1):
        if phase == 1:
            net.train(rho, sigma, epochs=5, batch=8192, lr=3e-3, seed=2, xc="pbe", rho_min=1e-8)
        E, b, used = _network_energy(net, rho, sigma, p.grid.weight)
        for use_graph in (False, True, True):
            plan.graph(use_graph)
            e = float(plan.eval(D)[1].item())
            n = plan.check()["n_points_mlp"]
            print("training %d, graph %d: E %.10f, oracle network %.10f (bound %.2e), network points %d of %d" % (
                phase, use_graph, e, E, b, n, p.n_points), flush=True)
            assert n == int(used.sum())
            assert abs(e - E) <= b
        counts.append(n)
    assert counts[1] > counts[0]
    plan.graph(False)
    plan.attach_mlp(None)
    pbex = mod.Mlp(seed=9)
    pbex.train(rho, sigma, epochs=1, batch=8192, lr=3e-3, seed=3, xc="pbe_x")
    with pytest.raises(mod.L.KldiError) as ei:
        plan.attach_mlp(pbex)                          # trained on another functional
    assert ei.value.status == -1
    net.close()
    pbex.close()
