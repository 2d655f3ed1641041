"""Benchmark: one block-filtered EXC evaluation (rho + E_xc + Vxc) per step on one MI355X.

Workload: the 200-atom chain (2000 cartesian AOs, 75 x 302 points per atom = 4.53M points,
128-point blocks, PBE, t_b = t_d = 1e-10), synthetic and seeded.  A step is one kldi_eval on a
ready plan with D already in HBM: D preparation, basis on retained tiles, X = D Phi block GEMMs
with the density epilogue, the functional, Z, the M = Phi Z^T block GEMMs, the FP64 reduction and
the symmetrised Vxc.  The mixed path (FP32 MFMA, FP64 accumulation) is the headline; the FP64
path is timed beside it on the same inputs.

Prints one JSON line.  --gpus N with N > 1 exits: libkldi runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DTYPE = {"fp32": "f32", "bf16x6": "bf16x6 (split)", "bf16x3": "bf16x3 (split)", "fp64": "f64"}
PATHS = {"fp32": "mixed: FP32 MFMA block GEMMs, FP64 functional and accumulation",
         "bf16x6": "mixed: X = D Phi as six BF16-MFMA products of three-piece splits, Vxc on FP32 MFMA, "
                   "FP64 functional and accumulation",
         "bf16x3": "mixed: X = D Phi as three BF16-MFMA products of two-piece splits, Vxc on FP32 MFMA, "
                   "FP64 functional and accumulation",
         "fp64": "FP64 MFMA block GEMMs"}
METRIC = "ms per EXC eval (rho+E_xc+Vxc) & TFLOP/s, mixed vs FP64, at 1e-6 Eh error"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}   # MI355X dense MFMA peaks
GOLDEN = os.path.join(ROOT, "tests", "golden", "cfg1_oracle.json")            # dense (unscreened)
GOLDEN_BLOCKED = os.path.join(ROOT, "tests", "golden", "cfg1_blocked.json")   # the method at t = 1e-10
GOLDEN_BLOCKED_OVERLAP = os.path.join(ROOT, "tests", "golden", "cfg1_overlap_blocked.json")  # same, clustered order
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


WORKLOADS = {
    0: "12-atom molecule, 100 cartesian AOs, 52,800 points (40x110 per atom), 128-point blocks, 32-AO tiles, "
       "LDA, t_b=t_d=1e-10",
    1: "200-atom chain, 2000 cartesian AOs (3s2p1d/2s1p), 4.53M points (75x302 per atom), 128-point blocks, "
       "32-AO tiles, PBE, t_b=t_d=1e-10",
    2: "1000-atom cluster, 10,000 cartesian AOs, 22.65M points (75x302 per atom), 128-point blocks, 32-AO tiles, "
       "PBE, t_b=t_d=1e-10",
}
# screening block (grid_block) of each workload's recipe: the 1000- and 500-atom clusters use 256 points
DEFAULT_G = {0: 128, 1: 128, 2: 256, 3: 128, 4: 256}


def workload_name(config, G):
    return WORKLOADS.get(config, "config %d" % config).replace("128-point blocks", "%d-point blocks" % G)


def kernels_sha1():
    """SHA-1 of the device sources (kernels, their device helpers and shared structs): the HBM counters
    in profiles/traffic.json describe the kernels built from exactly these files."""
    h = hashlib.sha1()
    for f in ("kernels.hip", "device.h", "kldi_impl.h"):
        h.update(open(os.path.join(ROOT, "paper_2605_10363_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_path(plan, D, steps, warmup, torch):
    for _ in range(warmup):
        plan.eval(D)
    torch.cuda.synchronize()
    plan.timing(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    outs = None
    for _ in range(steps):
        outs = plan.eval(D)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    stage, n = plan.stage_ms()
    st = plan.check()                      # counters of the last evaluation
    plan.timing(False)
    rho, exc, vxc = outs
    return ms, stage, st, float(exc.item()), vxc.cpu().numpy(), rho


UNIT_FLOP = 2.0 * 32 * 32 * 128   # one executed (p, q, r) tile triple
GEMM_KERNELS = {"fp32": ("k_xgemm_f32", "k_vgemm_f32"), "fp64": ("k_xgemm_f64", "k_vgemm_f64"),
                "bf16x6": ("k_xgemm_bf16", "k_vgemm_f32"), "bf16x3": ("k_xgemm_bf16", "k_vgemm_f32")}


def gemm_rooflines(prec, stats, stage):
    """Rates of the two block-GEMM kernels from the stage events of one plan (one grid chunk): X = D Phi is
    the whole xgemm stage; the Vxc stage also holds the pair-mask kernel and, for FP32 operands, the FP64
    diagonal kernel on a side stream, so its rate is a lower bound of the Vxc kernel's.  Work of FP32 plans'
    diagonal triples (FP64 MFMA) is counted apart."""
    kx, kv = GEMM_KERNELS[prec]
    peak = PEAK_TFLOPS["fp64" if prec == "fp64" else "fp32"]
    diag = stats.get("n_pairs_v_diag", 0)
    fx, fv, fd = UNIT_FLOP * stats["n_pairs_x"], UNIT_FLOP * (stats["n_pairs_v"] - diag), UNIT_FLOP * diag
    tx, tv = stage["xgemm"] * 1e-3, stage["vgemm"] * 1e-3
    out = {"x": {"kernel": kx, "tflop": round(fx / 1e12, 4), "ms": round(stage["xgemm"], 4),
                 "tflops": round(fx / tx / 1e12, 3), "frac": round(fx / tx / 1e12 / peak, 4)},
           "v": {"kernel": kv + (" (stage also holds k_vmask and the concurrent k_vdiag)" if diag else
                                 " (stage also holds k_vmask)"),
                 "tflop": round(fv / 1e12, 4), "ms": round(stage["vgemm"], 4),
                 "tflops": round(fv / tv / 1e12, 3), "frac": round(fv / tv / 1e12 / peak, 4)},
           "combined": {"tflops": round((fx + fv) / (tx + tv) / 1e12, 3),
                        "frac": round((fx + fv) / (tx + tv) / 1e12 / peak, 4)},
           "peak_tflops": peak}
    if diag:
        out["v_diag_fp64"] = {"kernel": "k_vdiag", "tflop": round(fd / 1e12, 4), "n_triples": diag,
                              "peak_tflops": PEAK_TFLOPS["fp64"]}
    return out


def cpu_baseline(p, n_sample=None, seed=0):
    """The FP64 oracle (dense, NumPy + host BLAS) on a random sample of grid points, scaled to one
    full evaluation (its cost is linear in the number of points).  The sample is sized for about 15 s of
    host work: 300,000 points at 2000 AOs, fewer for larger bases (the cost per point grows faster than
    the AO count)."""
    import oracle
    if n_sample is None:
        n_sample = int(300000 * min(1.0, (2000.0 / p.n_ao) ** 1.5))
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(p.n_points, size=min(n_sample, p.n_points), replace=False))
    t0 = time.perf_counter()
    oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz[idx], p.grid.weight[idx], p.D, p.xc)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return {"value": dt * 1e3 * p.n_points / len(idx), "unit": "ms/eval", "cores": cores, "kind": "oracle",
            "blas": blas_vendor(),
            "sample": "%d of %d grid points (seeded random subset), dense FP64 oracle, %.1f s measured, "
                      "scaled linearly to all points" % (len(idx), p.n_points, dt)}


def blas_vendor():
    """The BLAS library NumPy was built against (name and version), as NumPy reports it."""
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg["Build Dependencies"]["blas"]
        return "%s %s" % (b.get("name", "?"), b.get("version", ""))
    except Exception:   # older NumPy: no dict form
        return "unknown"


SWEEP_T = [(t, t) for t in (1e-8, 1e-9, 1e-10, 1e-11, 1e-12, 1e-14, 0.0)]
# the pair threshold alone (Sec. IV-A's t_d sensitivity) at the paper's block threshold t_b = 1e-12
SWEEP_TD = [(1e-12, t) for t in (1e-4, 1e-6, 1e-8, 1e-10, 1e-12, 0.0)]


def sweep(p, D, steps, warmup, torch, Plan, gd, so=None, pairs=SWEEP_T, precs=("fp32", "fp64")):
    """Thresholds (t_b, t_d) on the mixed path (and the FP64 path): retained fraction, executed pairs,
    ms/eval, and the errors of E_xc and of sampled Vxc entries against the unscreened FP64 oracle (gd) and
    against the FP64 GPU path at the same thresholds."""
    ij = np.array(gd["v_ij"])
    rows = []
    for t_b, t_d in pairs:
        t = t_d
        r = {"t": t_d, "t_b": t_b, "t_d": t_d}
        for prec in precs:
            plan = Plan.from_problem(p, prec=prec, t_b=t_b, t_d=t_d, shell_order=so)
            info = plan.info()
            ms, stage, st, E, V, rho = time_path(plan, D, steps, warmup, torch)
            dv = max(np.abs(V[ij[:, 0], ij[:, 1]] - np.array(gd["v"])).max(),
                     np.abs(np.diag(V) - np.array(gd["v_diag"])).max())
            r[prec] = {"ms": round(ms, 3), "E": E, "dE_vs_dense": abs(E - gd["E"]), "dV_vs_dense_sampled": dv,
                       "V": V}
            if prec == "fp32":
                r.update(retained_fraction=info["retained_fraction"], n_pairs_x=st["n_pairs_x"],
                         n_pairs_v=st["n_pairs_v"], chunks=info["n_grid_chunks"])
            plan.close()
            del rho
            torch.cuda.empty_cache()
            log("sweep t_b=%g t_d=%g %s: %.2f ms, retained %.4f, pairs x %d v %d, dE vs dense %.2e, dV %.2e" % (
                t_b, t, prec, ms, info["retained_fraction"], st["n_pairs_x"], st["n_pairs_v"], abs(E - gd["E"]), dv))
        if "fp64" in r and "fp32" in r:
            r["fp32"]["dE_vs_fp64"] = abs(r["fp32"]["E"] - r["fp64"]["E"])
            r["fp32"]["dV_vs_fp64"] = float(np.abs(r["fp32"]["V"] - r["fp64"]["V"]).max())
        for prec in precs:
            del r[prec]["V"]
        rows.append(r)
    return rows


def time_batch(B, D, steps, warmup, torch):
    for _ in range(warmup):
        B.eval(D)
    torch.cuda.synchronize()
    st = B.check()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    outs = None
    for _ in range(steps):
        outs = B.eval(D)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, st, outs


def cpu_baseline_batch(ps, n_mol_sample=8, pts_per_mol=20000, seed=0):
    """The FP64 oracle on a sample of the batch: n_mol_sample seeded molecules, pts_per_mol seeded points
    each; per molecule the time is scaled to all its points, and the batch total by the cost model
    n_points * n_ao^2 (the dense oracle's work) fitted on the sampled molecules."""
    import oracle
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(len(ps), size=min(n_mol_sample, len(ps)), replace=False))
    t_full, w_s = 0.0, 0.0
    t_meas = 0.0
    for m in pick:
        p = ps[m]
        idx = np.sort(rng.choice(p.n_points, size=min(pts_per_mol, p.n_points), replace=False))
        t0 = time.perf_counter()
        oracle.eval_exc(p.atom_xyz, p.basis, p.grid.xyz[idx], p.grid.weight[idx], p.D, p.xc)
        dt = time.perf_counter() - t0
        t_meas += dt
        t_full += dt * p.n_points / len(idx)
        w_s += float(p.n_points) * p.n_ao ** 2
    w_all = sum(float(p.n_points) * p.n_ao ** 2 for p in ps)
    return {"value": t_full * (w_all / w_s) * 1e3, "unit": "ms/eval", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": "%d of %d molecules, %d seeded points each (%.1f s measured), scaled to each molecule's "
                      "points and to the batch by n_points * n_ao^2" % (len(pick), len(ps), pts_per_mol, t_meas)}


def bench_batch(args, torch):
    """The batching form: 256 uneven molecules in one plan, replayed as a captured graph; the schedule and
    Vxc segment length are the autotuner's (--schedule auto) or given."""
    import synth
    from paper_2605_10363_amd.plan import Batch
    t0 = time.time()
    ps = synth.make_batch(xc=args.xc)
    log("inputs: %d molecules, %d atoms, %d AOs, %d points (%.1f s)" % (
        len(ps), sum(p.n_atoms for p in ps), sum(p.n_ao for p in ps), sum(p.n_points for p in ps), time.time() - t0))
    res = {}
    for prec in (["fp32"] if args.no_fp64 else ["fp32", "fp64"]):
        B = Batch(ps, xc=args.xc, prec=prec, v_segment=args.v_segment,
                  schedule="grid" if args.schedule == "auto" else args.schedule)
        info = B.info()
        D = B.pack([p.D for p in ps])
        if args.schedule == "auto":
            tune = B.autotune(D, reps=2)
        else:
            inf = B.info()
            tune = {"v_segment": inf["v_segment"], "schedule": inf["schedule"], "ms": None, "n_tried": 0}
        B.graph(True)
        log("%s batch plan: %.0f ms, retained fraction %.4f, %d X items, %d V items, %.1f GB; autotune %s" % (
            prec, info["plan_ms"], info["retained_fraction"], info["n_x_items"], info["n_v_items"],
            info["workspace_bytes"] / 1e9, tune))
        ms, st, (rho, exc, V) = time_batch(B, D, args.steps, args.warmup, torch)
        log("%s: %.3f ms/eval (all %d molecules), pairs x %d v %d" % (prec, ms, len(ps), st["n_pairs_x"],
                                                                      st["n_pairs_v"]))
        res[prec] = dict(ms=ms, stats=st, E=exc.cpu().numpy(), V=V, tune=tune, info=B.info())
        B.close()
        torch.cuda.empty_cache()
    mix = res["fp32"]
    flops = mix["stats"]["gemm_flops"]
    out = {
        "metric": METRIC, "value": round(mix["ms"], 4), "unit": "ms/eval", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mix["ms"], 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch of 256 molecules, 5-60 atoms each (%d atoms, %d cartesian AOs, %d points, 50x194 "
                               "per atom), 128-point blocks, 32-AO tiles, %s, t_b=t_d=1e-10, one plan, captured graph"
                               % (sum(p.n_atoms for p in ps), sum(p.n_ao for p in ps), sum(p.n_points for p in ps),
                                  args.xc.upper()),
                   "path": "mixed: FP32 MFMA block GEMMs, FP64 functional and accumulation",
                   "autotune": {k: mix["tune"][k] for k in ("v_segment", "schedule", "ms")}},
        "tflops": round(flops / (mix["ms"] * 1e-3) / 1e12, 3),
        "gemm_flops_per_eval": flops,
        "retained_fraction": mix["info"]["retained_fraction"],
    }
    if "fp64" in res:
        f64 = res["fp64"]
        out["fp64"] = {"ms": round(f64["ms"], 4),
                       "tflops": round(f64["stats"]["gemm_flops"] / (f64["ms"] * 1e-3) / 1e12, 3),
                       "autotune": {k: f64["tune"][k] for k in ("v_segment", "schedule", "ms")}}
        out["speedup_mixed_vs_fp64"] = round(f64["ms"] / mix["ms"], 3)
        out["err_mixed_vs_fp64"] = {"E_xc_max": float(np.abs(mix["E"] - f64["E"]).max()),
                                    "V_maxabs": float((mix["V"] - f64["V"]).abs().max().item())}
    # a replayed graph records no stage events: the GEMM work of the whole evaluation over its time (a lower
    # bound of the rate of the two block-GEMM kernels)
    achieved = flops / (mix["ms"] * 1e-3) / 1e12
    out["roofline"] = {"bound": "mfma", "kernel": "k_xgemm_f32 + k_vgemm_f32 (captured graph: whole evaluation)",
                       "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                       "frac": round(achieved / PEAK_TFLOPS["fp32"], 4), "traffic": None}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(ps)
    print(json.dumps(out), flush=True)


def bench_learned(args, torch):
    """The learned form: a 2-64-64-64-3 SiLU network trained on the GPU on (rho, sigma) points of the
    200-atom chain and the 1000-atom cluster stands in for PBE on the 500-atom cluster."""
    import synth
    from paper_2605_10363_amd.plan import Plan, Mlp
    from oracle import functionals as fx
    t0 = time.time()
    rs, ss = [], []
    for k, n_take in ((1, 4_530_000), (2, 5_470_000)):
        p = synth.make_problem(k)
        plan = Plan.from_problem(p, prec="fp32")
        r, s = plan.eval_grid(torch.from_numpy(p.D).cuda())
        g = torch.Generator(device="cpu").manual_seed(5000 + k)
        idx = torch.randperm(p.n_points, generator=g)[:n_take].cuda()
        rs.append(r[idx])
        ss.append(s[idx])
        plan.close()
        del r, s
        torch.cuda.empty_cache()
        log("training points from %s: %d of %d (%.1f s)" % (p.name, n_take, p.n_points, time.time() - t0))
    rho_t, sig_t = torch.cat(rs), torch.cat(ss)
    n_train = int(rho_t.numel())
    net = Mlp(seed=7)
    t1 = time.time()
    phases = [args.epochs // 3 + (1 if k < args.epochs % 3 else 0) for k in range(3)]
    losses = np.concatenate([net.train(rho_t, sig_t, epochs=ne, batch=16384, lr=lr, seed=11 + k, xc="pbe", rho_min=1e-8)
                             for k, (ne, lr) in enumerate(zip(phases, (2e-3, 5e-4, 1.25e-4))) if ne > 0])
    torch.cuda.synchronize()
    train_s = time.time() - t1
    log("trained %d epochs on %d points in %.1f s; loss %s" % (args.epochs, rho_t.numel(), train_s,
                                                               np.array2string(losses[::max(1, len(losses) // 5)], precision=4)))
    # inference against the analytic functional (and the oracle's functional) on training-range samples
    sel = torch.randperm(rho_t.numel(), generator=torch.Generator().manual_seed(3))[:200000].cuda()
    f, vr, vs, used = net.forward(rho_t[sel], sig_t[sel])
    r_np, s_np = rho_t[sel].cpu().numpy(), sig_t[sel].cpu().numpy()
    ef, evr, evs = fx.evaluate("pbe", r_np, s_np, 1e-14)
    u = used.cpu().numpy().astype(bool)
    rel_f = np.abs(f.cpu().numpy()[u] - ef[u]) / np.abs(ef[u])
    del rho_t, sig_t, rs, ss
    torch.cuda.empty_cache()

    p4 = synth.make_problem(4)
    D4 = torch.from_numpy(p4.D).cuda()
    log("inputs: %s n_atoms=%d n_ao=%d n_points=%d" % (p4.name, p4.n_atoms, p4.n_ao, p4.n_points))
    # the functional alone on this workload's (rho, sigma): analytic PBE (FP64) vs the network
    plan = Plan.from_problem(p4, prec="fp32", xc="pbe", grid_block=args.grid_block)
    r4, s4 = plan.eval_grid(D4)
    plan.close()
    torch.cuda.synchronize()
    from paper_2605_10363_amd.plan import xc_eval
    fn_ms = {}
    for tag, fn in (("analytic", lambda: xc_eval("pbe", r4, s4, 1e-14)), ("mlp", lambda: net.forward(r4, s4))):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        fn_ms[tag] = e0.elapsed_time(e1) / 5
    log("functional alone on %d points: analytic %.3f ms, network %.3f ms" % (r4.numel(), fn_ms["analytic"], fn_ms["mlp"]))
    del r4, s4
    torch.cuda.empty_cache()
    out_runs = {}
    for tag in ("analytic", "mlp"):
        plan = Plan.from_problem(p4, prec="fp32", xc="pbe", grid_block=args.grid_block)
        if tag == "mlp":
            plan.attach_mlp(net)
        ms, stage, st, E, V, rho = time_path(plan, D4, args.steps, args.warmup, torch)
        out_runs[tag] = dict(ms=ms, stage=stage, st=st, E=E, V=V, chunks=plan.info()["n_grid_chunks"])
        log("%s: %.3f ms/eval, functional stage %.3f ms, E %.10f, surrogate points %d" % (
            tag, ms, stage["xfunc"], E, st["n_points_mlp"]))
        plan.close()
        del rho
        torch.cuda.empty_cache()
    plan = Plan.from_problem(p4, prec="fp64", xc="pbe", grid_block=args.grid_block)
    ms64, stage64, st64, E64, V64, rho64 = time_path(plan, D4, 1, 1, torch)
    plan.close()
    a, m = out_runs["analytic"], out_runs["mlp"]
    out = {
        "metric": METRIC, "value": round(m["ms"], 4), "unit": "ms/eval", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(m["ms"], 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "500-atom cluster, 5000 cartesian AOs, %d points (75x302 per atom), %d-point blocks, "
                               "PBE replaced by the trained network where it covers a point" % (p4.n_points,
                                                                                                 args.grid_block),
                   "path": "mixed FP32 block GEMMs; BF16-weight MLP functional, analytic fallback"},
        "learned": {
            "train_points": n_train, "train_sources": "4.53M points of the 200-atom chain + 5.47M of the 1000-atom cluster",
            "epochs": args.epochs, "learning_rates": "2e-3, 5e-4, 1.25e-4 (one third of the epochs each)",
            "train_s": round(train_s, 2), "final_loss": float(losses[-1]),
            "points_on_network": int(m["st"]["n_points_mlp"]), "fraction_on_network": m["st"]["n_points_mlp"] / p4.n_points,
            "functional_kernel_ms": {"mlp": round(fn_ms["mlp"], 4), "analytic": round(fn_ms["analytic"], 4),
                                     "what": "f, v_rho, v_sigma at every grid point of this workload, alone"},
            "functional_and_z_stage_ms": {"mlp": round(m["stage"]["xfunc"], 4), "analytic": round(a["stage"]["xfunc"], 4)},
            "eval_ms": {"mlp": round(m["ms"], 4), "analytic": round(a["ms"], 4), "fp64_analytic": round(ms64, 4)},
            "E_xc": {"mlp": m["E"], "analytic": a["E"], "fp64_analytic": E64},
            "err_vs_analytic": {"E_xc": abs(m["E"] - a["E"]), "E_xc_rel": abs(m["E"] - a["E"]) / abs(a["E"]),
                                "V_maxabs": float(np.abs(m["V"] - a["V"]).max())},
            "err_vs_fp64": {"E_xc": abs(m["E"] - E64), "V_maxabs": float(np.abs(m["V"] - V64).max())},
            "f_rel_err_vs_oracle_functional": {"median": float(np.median(rel_f)), "p99": float(np.quantile(rel_f, 0.99)),
                                               "sample": "200000 training-range points"},
        },
    }
    # roofline of the dominant block-GEMM kernel of the run with the network (as for the single-molecule
    # line; with several grid chunks the combined stage and the GEMM work of the whole evaluation)
    if m["chunks"] > 1:
        kernel = "k_xgemm_f32 + k_vgemm_f32 (%d grid chunks: combined stage)" % m["chunks"]
        achieved = m["st"]["gemm_flops"] / (m["stage"]["vgemm"] * 1e-3) / 1e12
    else:
        dom = "xgemm" if m["stage"]["xgemm"] >= m["stage"]["vgemm"] else "vgemm"
        g = gemm_rooflines("fp32", m["st"], m["stage"])["x" if dom == "xgemm" else "v"]
        kernel, achieved = g["kernel"], g["tflops"]
    out["roofline"] = {"bound": "mfma", "kernel": kernel, "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["fp32"],
                       "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["fp32"], 4), "traffic": None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1,
                    help="1: 200-atom chain (default); 2: 1000-atom cluster; 3: batch of 256 molecules; "
                         "4: 500-atom cluster with the learned functional")
    ap.add_argument("--xc", default="lda", help="functional of the batch workload (lda or pbe)")
    ap.add_argument("--epochs", type=int, default=60,
                    help="training epochs of the learned form (--config 4), in three equal phases at learning rates "
                         "2e-3, 5e-4 and 1.25e-4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dense", action="store_true",
                    help="also time the unscreened comparator at workloads other than 0 and 1 (size sweep)")
    ap.add_argument("--no-learned", action="store_true",
                    help="workload 4: time the analytic functional on the main path instead of the learned form")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="threshold sweep t_b = t_d on workload 1 (retained fraction, time, errors) instead of the bench")
    ap.add_argument("--no-dense", action="store_true", help="skip the unscreened (t_b = t_d = 0) GPU comparator")
    ap.add_argument("--no-other-order", action="store_true",
                    help="workload 1: skip the timing of the other basis order (for profiler runs)")
    ap.add_argument("--ao-order", default="overlap", choices=["overlap", "atom"],
                    help="basis order of the timed plans on workloads 1 and 2: overlap-signature clustering (the "
                         "paper's reordering; default) or atom order; workload 1 also times the other order once")
    ap.add_argument("--precs", default="fp32,bf16x6,bf16x3",
                    help="precision forms timed beside FP64 (workloads 1 and 2); the first is the headline value")
    ap.add_argument("--v-segment", type=int, default=0, help="grid blocks per Vxc segment (0 = plan's choice)")
    ap.add_argument("--grid-block", type=int, default=0,
                    help="points per screening block, 128 or 256 (0 = the workload's recipe: 256 for workloads 2 "
                         "and 4, else 128)")
    ap.add_argument("--schedule", default="grid", choices=["grid", "queue", "auto"],
                    help="work-item schedule of the GEMM kernels (auto: the plan's autotuner picks it and the "
                         "Vxc segment length, outside the timed region)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (HBM-counter calibration for profiling)")
    args = ap.parse_args()
    if args.grid_block == 0:
        args.grid_block = DEFAULT_G.get(args.config, 128)
    if args.gpus != 1:
        print("bench.py runs on one GPU only (libkldi has no multi-GPU path); got --gpus %d" % args.gpus)
        sys.exit(2)

    import torch
    import synth
    from paper_2605_10363_amd.plan import Plan

    if args.config == 3:
        bench_batch(args, torch)
        return
    if args.config == 4 and not args.no_learned:
        bench_learned(args, torch)
        return

    t0 = time.time()
    p = synth.make_problem(args.config)
    log("inputs: %s n_atoms=%d n_ao=%d n_points=%d (%.1f s)" % (p.name, p.n_atoms, p.n_ao, p.n_points,
                                                                time.time() - t0))
    D = torch.from_numpy(p.D).cuda()
    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    so, order_ms = None, 0.0
    if args.ao_order == "overlap":
        from paper_2605_10363_amd.plan import overlap_order
        S = synth.overlap_matrix(p.basis, p.atom_xyz)   # an input (the SCF setup has it), not timed
        t0 = time.time()
        _, so = overlap_order(p.basis, S)
        order_ms = (time.time() - t0) * 1e3
        del S
        log("overlap-signature basis order: %.0f ms" % order_ms)
    if args.sweep:
        gd = json.load(open(GOLDEN))
        rows = sweep(p, D, args.steps, args.warmup, torch, Plan, gd, so)
        rows_td = sweep(p, D, args.steps, args.warmup, torch, Plan, gd, so, pairs=SWEEP_TD, precs=("fp32",))
        print(json.dumps({"workload": workload_name(args.config, args.grid_block), "sweep": rows,
                          "sweep_td_at_tb_1e-12": rows_td}), flush=True)
        return
    res = {}
    forms = [f for f in args.precs.split(",") if f]
    for prec in (forms if args.no_fp64 else forms + ["fp64"]):
        torch.cuda.synchronize()
        t0 = time.time()
        plan = Plan.from_problem(p, prec=prec, v_segment=args.v_segment, shell_order=so, grid_block=args.grid_block,
                                 schedule="grid" if args.schedule == "auto" else args.schedule)
        tune = plan.autotune(D, reps=2) if args.schedule == "auto" else None
        info = plan.info()
        if tune is not None:
            log("%s autotune: %s" % (prec, tune))
        log("%s plan: %.0f ms, retained fraction %.4f, n_ret %d, max tiles/block %d, %d V items, %.1f GB" % (
            prec, info["plan_ms"], info["retained_fraction"], info["n_retained_tiles"], info["max_tiles_per_block"],
            info["n_v_items"], info["workspace_bytes"] / 1e9))
        plan.eval(D)
        torch.cuda.synchronize()
        cold_ms = (time.time() - t0) * 1e3 + order_ms
        ms, stage, st, E, V, rho = time_path(plan, D, args.steps, args.warmup, torch)
        log("%s: %.3f ms/eval, stages %s, pairs x %d v %d, E %.12f" % (
            prec, ms, {k: round(v, 3) for k, v in stage.items()}, st["n_pairs_x"], st["n_pairs_v"], E))
        res[prec] = dict(ms=ms, stage=stage, stats=st, E=E, V=V, info=info, cold_ms=cold_ms,
                         elec=float(torch.dot(rho, torch.from_numpy(p.grid.weight).cuda()).item()))
        plan.close()
        del rho
        torch.cuda.empty_cache()

    mix = res[forms[0]]
    flops = mix["stats"]["gemm_flops"]
    out = {
        "metric": METRIC, "value": round(mix["ms"], 4), "unit": "ms/eval", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mix["ms"], 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[forms[0]], "data": "synthetic",
        "config": {"workload": workload_name(args.config, args.grid_block),
                   "path": PATHS[forms[0]],
                   "basis_order": "overlap-signature clustering" if so is not None else "atom order",
                   "seeds": p.meta.get("seeds")},
        "tflops": round(flops / (mix["ms"] * 1e-3) / 1e12, 3),
        "gemm_flops_per_eval": flops,
        "retained_fraction": mix["info"]["retained_fraction"],
        "stage_ms": {k: round(v, 4) for k, v in mix["stage"].items()},
        "plan_ms": round(mix["info"]["plan_ms"] + order_ms, 1),
        "basis_order_ms": round(order_ms, 1),
        "cold_ms": round(mix["cold_ms"], 1),
        "electrons": mix["elec"], "n_occ": p.n_occ,
    }
    if mix["info"]["n_grid_chunks"] == 1:
        out["gemms"] = gemm_rooflines(forms[0], mix["stats"], mix["stage"])
    if "fp64" in res:
        f64 = res["fp64"]
        out["fp64"] = {"ms": round(f64["ms"], 4), "tflops": round(f64["stats"]["gemm_flops"] / (f64["ms"] * 1e-3) / 1e12, 3),
                       "stage_ms": {k: round(v, 4) for k, v in f64["stage"].items()}}
        if f64["info"]["n_grid_chunks"] == 1:
            out["fp64"]["gemms"] = gemm_rooflines("fp64", f64["stats"], f64["stage"])
        out["speedup_mixed_vs_fp64"] = round(f64["ms"] / mix["ms"], 3)
        out["err_mixed_vs_fp64"] = {"E_xc": abs(mix["E"] - f64["E"]), "V_maxabs": float(np.abs(mix["V"] - f64["V"]).max())}
    out["precision_forms"] = {}
    for prec in forms:
        r = res[prec]
        d = {"ms": round(r["ms"], 4), "tflops": round(r["stats"]["gemm_flops"] / (r["ms"] * 1e-3) / 1e12, 3),
             "stage_ms": {k: round(v, 4) for k, v in r["stage"].items()}, "path": PATHS[prec]}
        if "fp64" in res:
            d["err_vs_fp64"] = {"E_xc": abs(r["E"] - res["fp64"]["E"]),
                                "V_maxabs": float(np.abs(r["V"] - res["fp64"]["V"]).max())}
        out["precision_forms"][prec] = d
    if args.config == 1:
        out["err_vs_oracle"] = {}
        for tag, path in (("blocked", GOLDEN_BLOCKED_OVERLAP if so is not None else GOLDEN_BLOCKED), ("dense", GOLDEN)):
            if not os.path.exists(path):
                continue
            g = json.load(open(path))
            ij = np.array(g["v_ij"])
            for prec, r in res.items():
                V = r["V"]
                dv = max(np.abs(V[ij[:, 0], ij[:, 1]] - np.array(g["v"])).max(),
                         np.abs(np.diag(V) - np.array(g["v_diag"])).max())
                out["err_vs_oracle"]["%s_%s" % (tag, prec)] = {"E_xc": abs(r["E"] - g["E"]), "V_maxabs_sampled": dv}

    if args.config == 1 and not args.no_fp64:
        # the nuclear gradient of E_xc with the grid held fixed, on an FP64 plan and on an FP32 plan, beside the
        # energy evaluation
        grads = {}
        for gprec in ("fp64", "fp32"):
            plan = Plan.from_problem(p, prec=gprec, shell_order=so)
            g = plan.grad(D)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = max(2, args.steps // 2)
            e0.record()
            for _ in range(reps):
                g = plan.grad(D)
            e1.record()
            torch.cuda.synchronize()
            gms = e0.elapsed_time(e1) / reps
            grads[gprec] = (gms, g.cpu().numpy())
            log("%s gradient: %.3f ms, max |dE/dR| %.3e" % (gprec, gms, np.abs(grads[gprec][1]).max()))
            plan.close()
            torch.cuda.empty_cache()
        gms, gn = grads["fp64"]
        out["gradient"] = {"what": "dE_xc/dR of all %d atoms (grid held fixed), FP64 plan, one kldi_eval_grad call "
                                   "(its own rho, functional and the gradient products)" % p.n_atoms,
                           "ms": round(gms, 3), "ratio_to_fp64_energy_eval": round(gms / res["fp64"]["ms"], 3)
                           if "fp64" in res else None, "max_abs": float(np.abs(gn).max()),
                           "fp32_plan": {"ms": round(grads["fp32"][0], 3),
                                         "max_abs_diff_vs_fp64": float(np.abs(grads["fp32"][1] - gn).max())}}
    if (args.config in (0, 1) or args.dense) and not args.no_dense:
        plan = Plan.from_problem(p, prec=forms[0], t_b=0.0, t_d=0.0, shell_order=so, grid_block=args.grid_block)
        info = plan.info()
        ms, stage, st, E, V, rho = time_path(plan, D, max(3, args.steps // 2), 1, torch)
        log("%s unscreened (t_b = t_d = 0): %.3f ms/eval, %d chunks, pairs x %d v %d" % (
            forms[0], ms, info["n_grid_chunks"], st["n_pairs_x"], st["n_pairs_v"]))
        out["dense"] = {"what": "the same kernels with every candidate tile retained and every pair executed "
                                "(t_b = t_d = 0): the dense-GPU comparator", "ms": round(ms, 3),
                        "speedup_block_filtered": round(ms / mix["ms"], 3), "n_pairs_x": st["n_pairs_x"],
                        "n_pairs_v": st["n_pairs_v"], "grid_chunks": info["n_grid_chunks"],
                        "tflops": round(st["gemm_flops"] / (ms * 1e-3) / 1e12, 3)}
        plan.close()
        del rho
        torch.cuda.empty_cache()
    if args.config == 1 and not args.no_other_order:
        other = "atom order" if so is not None else "overlap-signature clustering"
        so2 = None
        if so is None:
            from paper_2605_10363_amd.plan import overlap_order
            _, so2 = overlap_order(p.basis, synth.overlap_matrix(p.basis, p.atom_xyz))
        plan = Plan.from_problem(p, prec=forms[0], v_segment=args.v_segment, shell_order=so2, grid_block=args.grid_block)
        info = plan.info()
        ms, stage, st, E, V, rho = time_path(plan, D, args.steps, args.warmup, torch)
        log("%s, %s: %.3f ms/eval, retained fraction %.4f, pairs x %d v %d" % (
            forms[0], other, ms, info["retained_fraction"], st["n_pairs_x"], st["n_pairs_v"]))
        out["other_basis_order"] = {
            "order": other, "ms": round(ms, 4), "stage_ms": {k: round(v, 4) for k, v in stage.items()},
            "retained_fraction": info["retained_fraction"], "n_retained_tiles": info["n_retained_tiles"],
            "n_pairs_x": st["n_pairs_x"], "n_pairs_v": st["n_pairs_v"], "E_xc_diff": abs(E - mix["E"]),
            "headline": {"ms": round(mix["ms"], 4), "retained_fraction": mix["info"]["retained_fraction"],
                         "n_retained_tiles": mix["info"]["n_retained_tiles"], "n_pairs_x": mix["stats"]["n_pairs_x"],
                         "n_pairs_v": mix["stats"]["n_pairs_v"]}}
        plan.close()
        del rho
        torch.cuda.empty_cache()

    # roofline of the dominant kernel (the larger of the two block-GEMM stages), timed live above.  A plan
    # that processes the grid in several chunks interleaves the stages, so only the GEMM work of the whole
    # evaluation over that combined stage is known (a lower bound of the GEMM rate).
    traffic = None
    if mix["info"]["n_grid_chunks"] > 1:
        achieved = flops / (mix["stage"]["vgemm"] * 1e-3) / 1e12
        kernel = "%s + %s (%d grid chunks: combined stage, all kernels between D preparation and "\
                 "the final sums)" % (GEMM_KERNELS[forms[0]] + (mix["info"]["n_grid_chunks"],))
    else:
        dom = "xgemm" if mix["stage"]["xgemm"] >= mix["stage"]["vgemm"] else "vgemm"
        g = out["gemms"]["x" if dom == "xgemm" else "v"]
        achieved = g["tflops"]
        kernel = g["kernel"]
        # the counters in TRAFFIC were taken on the 200-atom chain (workload 1) from these exact sources
        if args.config == 1 and os.path.exists(TRAFFIC):
            t = json.load(open(TRAFFIC))
            if t.get("kernels_sha1") == kernels_sha1() and dom in t.get("bytes_per_launch", {}):
                traffic = t["bytes_per_launch"][dom]
    out["roofline"] = {"bound": "mfma", "kernel": kernel, "achieved": round(achieved, 3),
                       "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["fp32"], 4),
                       "traffic": traffic}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
