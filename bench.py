#!/usr/bin/env python3
"""Throughput of CLAMP's forward-model hot path on one MI355X.

A step is one CLAMP iteration (the loop body of Alg. 2) over every look of
the full-size synthetic workload: all forward agents (aperture operator,
exact mu-step, surrogate r-update), the Gaussian prior agent and the Mann
consensus step.  Inputs are generated on the host, uploaded, and the state is
initialised before the timed region.  `value` is voxel-looks per second of
whole iterations; per-stage HIP-event times give the roofline figure of the
dominant kernel, and the float64 oracle is timed on a sample of the same work.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash(group):
    """sha256 over the kernel sources of one group (forward path or CNN)."""
    from paper_2406_13651_amd.profsum import kernel_source_hash as h
    return h(group)


def counter_traffic(record, group):
    """The committed counter record (profiles/counter_traffic.json) for a
    workload, or None when it is missing or the kernel sources have changed
    since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "counter_traffic.json")) as f:
            rec = json.load(f)[record]
    except (OSError, KeyError, ValueError):
        return None
    return rec if rec.get("source_sha256") == kernel_source_hash(group) else None


def warmup_and_time(C, plan, iterate, warmup, steps, sb, after=None, breakdown=10):
    """Warm-up, then `breakdown` iterations with every stage timed (HIP events
    around each stage), which give the per-stage figures and pick the dominant
    stage: the one with the most time among those with algorithmic bytes in
    sb.  Then the timed region, with events around the dominant stage only (a
    pair of events around every stage costs about 4% of an iteration), then
    `after()` (results read from the state the timed region leaves).
    Returns (seconds of the timed region, {stage: (ms, launches)} with the
    dominant stage's entry from the timed region, dominant stage)."""
    import torch
    for _ in range(warmup):
        iterate()
    torch.cuda.synchronize()
    C.clamp_plan_set_timing(plan, True)
    for _ in range(max(breakdown, 1)):
        iterate()
    torch.cuda.synchronize()
    C.clamp_plan_set_timing(plan, False)
    stages = dict(C.clamp_plan_get_timing(plan))
    dom = max((k for k in stages if k in sb), key=lambda k: stages[k][0])
    C.clamp_plan_set_timing_stages(plan, [dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        iterate()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    C.clamp_plan_set_timing(plan, False)
    timed = C.clamp_plan_get_timing(plan)
    if after is not None:
        after()
    stages[dom] = timed[dom]
    return elapsed, stages, dom


def host_cpu():
    """Host CPU model, os.cpu_count() and the threads this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def oracle_state(g):
    """The GPU state as a float64 oracle state."""
    import numpy as np
    import oracle
    return oracle.ClampState(mu=g.mu.cpu().numpy().astype(np.complex128), r=g.r.cpu().numpy().astype(np.float64),
                             w=g.state_w().cpu().numpy().astype(np.float64), k=g.k,
                             ahy2=g.ahy2.cpu().numpy().astype(np.float64))


def oracle_check_and_cpu_baseline(spec, y, g, sigma2, threads):
    """One more CLAMP iteration on the GPU from the timed run's state (after a
    residual refresh, so both sides start from resid = D(a)(y - A mu)),
    against the float64 oracle's iteration from the same state (relative
    error per result), and the oracle's wall time for that iteration on
    `threads` host threads and on one."""
    import copy

    import numpy as np
    import oracle
    import torch

    g.refresh()
    torch.cuda.synchronize()
    st0 = oracle_state(g)
    g.iterate()
    torch.cuda.synchronize()
    got = {"mu": g.mu.cpu().numpy(), "r": g.r.cpu().numpy(), "w": g.state_w().cpu().numpy(),
           "wbar": g.wbar.cpu().numpy()}
    conv = g.conv_err()
    mres = g.mu_residual()
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    s2w = float(np.float32(g.sigma_w2))
    s2 = float(np.float32(sigma2))
    prior = lambda x: oracle.gaussian_smooth(x, g.prior_sigma)  # noqa: E731

    def rel(a, b):
        a = np.asarray(a)
        b = np.asarray(b, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    st = copy.deepcopy(st0)
    t0 = time.perf_counter()
    h = oracle.clamp_iteration(st, y, mask, s2w, s2, g.rho, prior, workers=threads)
    t_multi = time.perf_counter() - t0
    # the mu-residual is ||d|| / ||A^H y / sigma_w^2|| with d the difference of
    # two terms of the size of A^H y / sigma_w^2: float32 bounds its error in
    # absolute terms (a few units of 2^-24), not relative to a small residual
    check = {"mu": rel(got["mu"], st.mu), "r": rel(got["r"], st.r), "w": rel(got["w"], st.w),
             "wbar": rel(got["wbar"], h["wbar"]), "conv_err": abs(conv - h["conv_err"]) / h["conv_err"],
             "bound": 1e-5,
             "mu_residual": {"gpu": mres, "oracle": h["mu_residual"], "abs_diff": abs(mres - h["mu_residual"]),
                             "bound_abs": 1e-6},
             "what": "one CLAMP iteration from the timed run's state (iteration %d), GPU float32 against the "
                     "float64 oracle: relative L2 of mu, r, w, w_bar, relative error of the convergence error, "
                     "absolute error of the mu-residual" % (st0.k + 1)}
    del st
    st = copy.deepcopy(st0)
    t0 = time.perf_counter()
    oracle.clamp_iteration(st, y, mask, s2w, s2, g.rho, prior, workers=1)
    t_single = time.perf_counter() - t0
    del st, st0
    units = spec.looks * spec.n
    model, ncpu, avail = host_cpu()
    base = {
        "value": units / t_multi,
        "unit": "voxel-looks/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "float64 numpy oracle: one whole CLAMP iteration (%d forward agents, Gaussian prior, Mann "
                  "step, convergence measures) at %dx%dx%d, the looks' agents on %d threads (%.2f s)"
                  % (spec.looks, spec.nx, spec.ny, spec.nz, threads, t_multi),
        "single_thread": {"value": units / t_single, "seconds": round(t_single, 3), "cores": 1},
        "host": {"cpu_model": model, "os_cpu_count": ncpu, "usable_threads": avail},
    }
    return check, base


def run_batch(args):
    """Uneven batch: 32 scenes drawn from the batch recipe, one batched step
    per iteration replayed from a HIP graph, against scene-by-scene launches
    of the same iterations."""
    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import _clamp as C
    from paper_2406_13651_amd.perf import stage_bytes

    specs = synth.batch_specs(32, seed=0, cap_voxel_looks=args.batch_cap)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    scenes = []
    for i, sp in enumerate(specs):
        r = synth.facet_scene(sp, np.random.Generator(np.random.PCG64(synth.seed_sequence(sp.config_id, i).spawn(1)[0])))
        scenes.append(dict(nx=sp.nx, ny=sp.ny, nz=sp.nz, looks=sp.looks, radius=sp.radius,
                           sigma_w2=synth.noise_variance(r, sp.snr_db), sigma2=args.sigma2, with_prior=True))
    total = sum(sp.n * sp.looks for sp in specs)
    log("batch of %d scenes, %.3g voxel-looks per iteration" % (len(specs), total))
    b = G.ClampBatchGPU(scenes, device=dev)
    ys = []
    for i, sp in enumerate(specs):
        _, y, s2 = synth.make_problem(sp, i, workers=16)
        assert np.float32(s2) == np.float32(scenes[i]["sigma_w2"])
        ys.append(torch.from_numpy(y).to(dev))
        del y
        b.init_scene(i, ys[-1])
    b.restart()
    torch.cuda.synchronize()
    log("scenes initialised; autotuning grids")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tuned = b.autotune(stream)
        for _ in range(args.warmup):
            b.step(stream)
        stream.synchronize()
        # per-stage times of eager batched steps
        C.clamp_plan_set_timing(b.plan, True)
        for _ in range(3):
            b.step(stream)
        stream.synchronize()
        C.clamp_plan_set_timing(b.plan, False)
        stages = C.clamp_plan_get_timing(b.plan)
        b.capture(stream)
        stream.synchronize()
        log("timing %d graph replays" % args.steps)
        t0 = time.perf_counter()
        b.replay(args.steps, stream)
        stream.synchronize()
        t1 = time.perf_counter()
        log("timing 3 iterations launched scene by scene")
        t2 = time.perf_counter()
        for _ in range(3):
            b.step_per_scene()
        stream.synchronize()
        t3 = time.perf_counter()
    torch.cuda.synchronize()
    elapsed = t1 - t0
    per_scene_ms = (t3 - t2) / 3 * 1e3
    fault = int(b.fault.item())
    sb = {}
    for i, sp in enumerate(specs):
        info = b.plan.info[i]
        for k, v in stage_bytes(sp.nx, sp.ny, sp.nz, sp.looks, info["P"], info["B"], sp.looks + 1,
                                fused=b.fused).items():
            sb[k] = sb.get(k, 0) + v
    fused_form = b.fused
    del b
    torch.cuda.empty_cache()
    # the same scenes through the single-scene driver (the update pass with
    # the Mann step fused in), one scene after another
    log("timing 3 iterations of single-scene drivers (fused update and Mann step), scene by scene")
    gs = []
    for i, sc in enumerate(scenes):
        g1 = G.ClampGPU(sc["nx"], sc["ny"], sc["nz"], sc["looks"], sc["radius"], sc["sigma_w2"], sc["sigma2"],
                        with_prior=True, device=dev)
        g1.init(ys[i])
        gs.append(g1)
    for g1 in gs:
        g1.iterate()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(3):
        for g1 in gs:
            g1.iterate()
    torch.cuda.synchronize()
    fused_ms = (time.perf_counter() - t4) / 3 * 1e3
    del gs, ys
    torch.cuda.empty_cache()
    per_stage = {}
    for name, (ms, cnt) in stages.items():
        avg = ms / cnt
        e = {"avg_ms": round(avg, 4), "launches": cnt}
        if name in sb:
            e["alg_GBps"] = round(sb[name] / (avg * 1e-3) / 1e9, 1)
        per_stage[name] = e
    dom = max((k for k in per_stage if k in sb), key=lambda k: stages[k][0])
    dom_ms = stages[dom][0] / stages[dom][1]
    achieved = sb[dom] / (dom_ms * 1e-3) / 1e9
    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": total * args.steps / elapsed,
        "unit": "voxel-looks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch of %d uneven scenes (N in {128,192,256,384,512}, nz in {32,64,128}, "
                               "4-32 looks, R = N/4, SNR 10 dB), %.3g voxel-looks per iteration, one graph "
                               "replay per CLAMP iteration" % (len(specs), total),
                   "mann_step": "fused into the update pass" if fused_form else "a pass of its own",
                   "scenes": [[sp.nx, sp.nz, sp.looks] for sp in specs], "sigma2": args.sigma2},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "per_scene_launch": {"ms_per_step": round(per_scene_ms, 3),
                             "voxel_looks_per_s": total / (per_scene_ms * 1e-3),
                             "what": "the batch's iteration through the single-scene calls of the same form, "
                                     "scene after scene, on the batch's state"},
        "per_scene_fused": {"ms_per_step": round(fused_ms, 3), "voxel_looks_per_s": total / (fused_ms * 1e-3),
                            "what": "single-scene drivers with the Mann step fused into the update pass, "
                                    "scene after scene"},
        "batched_over_per_scene": round(per_scene_ms / (elapsed / args.steps * 1e3), 3),
        "batched_over_per_scene_fused": round(fused_ms / (elapsed / args.steps * 1e3), 3),
        "autotune": tuned,
        "stages": per_stage,
        "fault": fault,
    }
    print(json.dumps(result), flush=True)


CNN_FWD_FLOP = 335_232      # per voxel: 2 * 27 * (1*32 + 6*32*32 + 32*1)
CNN_TRAIN_FLOP = 1_003_968  # forward + input gradients of layers 2-8 + weight gradients of all 8
# U-Net forward, algorithmic flop per full-resolution voxel: 3x3x3
# convolutions (1 -> 32: 1,728; 32 -> 32: 55,296) at level k cost 1/8^k per
# voxel (level 0: 1 + 3 of 32 -> 32, levels 1 and 2: 4 each), transposed
# convolutions 2,048 per output voxel at levels 0, 1, 2, the output layer 1,728
UNET_FWD_FLOP = 1728 + 3 * 55296 + 4 * 55296 // 8 + 4 * 55296 // 64 + 2048 + 2048 // 8 + 2048 // 64 + 1728
# training: forward, input gradients (none for the first layer) and weight gradients
UNET_TRAIN_FLOP = 3 * UNET_FWD_FLOP - 1728
BF16_PEAK_TFLOPS = 2500.0


def copy_probe(args, dev):
    """A device copy of --copy-probe MiB, the known-size reference for the
    hardware byte counters (FETCH_SIZE, WRITE_SIZE)."""
    import torch
    if args.copy_probe <= 0:
        return
    nfl = args.copy_probe * (1 << 20) // 4
    src = torch.ones(nfl, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: %d bytes read, %d bytes written" % (nfl * 4, nfl * 4))
    del src, dst


def equal_nrmse_summary(out, iters):
    """Iterations and wall time of each form to bring the scale-fit NRMSE
    (Sec. V-A) 10% below that of the speckle average, the comparison
    reconstruction and every form's initial image (nrmse[0]); counted from
    iteration 1, within the evaluation window."""
    sa = out["plain"]["nrmse"][0]
    target = round(0.9 * sa, 5)
    equal = {"target_nrmse": target,
             "target": "10%% below the speckle average's NRMSE %.4f (every form's initial image): the first "
                       "iteration k >= 1 at or below it, within %d iterations" % (sa, iters)}
    for name, o_ in out.items():
        tr = o_["nrmse"]
        hit = next((k for k, v in enumerate(tr) if k >= 1 and v <= target), None)
        best = min(range(1, len(tr)), key=lambda k: tr[k])
        equal[name] = {"iterations": hit, "ms_to_target": None if hit is None else round(hit * o_["ms_per_iter"], 3),
                       "ms_per_iter": round(o_["ms_per_iter"], 4), "iters_per_s": round(1e3 / o_["ms_per_iter"], 2),
                       "nrmse_final": tr[-1], "nrmse_best": tr[best], "best_iteration": best}
    lh, ph = equal["learned"]["ms_to_target"], equal["plain"]["ms_to_target"]
    equal["learned_faster_than_plain"] = lh is not None and (ph is None or lh < ph)
    return equal


def learned_eval(args, dev):
    """Train the prior agent on seeded pairs, then reconstruct the evaluation
    scene with the learned prior, the Gaussian prior (the plain form) and the
    forward agents alone; NRMSE after every iteration and the wall time per
    iteration of each form."""
    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import learned as Lm

    unet = args.prior == "unet"
    # U-Net patches: nx a multiple of 128 (32-voxel tiles at the third level)
    pz, py, px = (32, 32, 128) if unet else (32, 64, 64)
    log("training pairs: %d volumes of %dx%dx%d (%s inputs%s)" % (
        args.train_pairs, px, py, pz, args.train_mode,
        ", noise %g" % args.train_noise if args.train_mode == "awgn" else ", looks simulated on the GPU"))
    t0 = time.perf_counter()
    X, T = Lm.make_pairs(args.train_pairs, seed=0, nz=pz, ny=py, nx=px, mode=args.train_mode, noise=args.train_noise)
    t_pairs = time.perf_counter() - t0
    prior = (Lm.UnetPrior(Lm.unet_init_params(0), device=dev) if unet else Lm.CnnPrior(Lm.init_params(0), device=dev))
    log("training %d epochs, lr %g" % (args.train_epochs, args.lr))
    hist = Lm.train(prior, X, T, epochs=args.train_epochs, lr=args.lr,
                    log=lambda m: log("  " + m))
    del X, T

    spec = synth.CONFIGS["learned"]
    log("evaluation scene %dx%dx%d, %d looks" % (spec.nx, spec.ny, spec.nz, spec.looks))
    r_true, y, s2w = synth.make_problem(spec, 0, workers=16)
    yt = torch.from_numpy(y).to(dev)
    rt = torch.from_numpy(r_true.astype(np.float32)).to(dev)
    del y
    geo = (spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, args.sigma2)
    forms = {
        "plain": lambda: G.ClampGPU(*geo, with_prior=True, device=dev),
        "learned": lambda: Lm.LearnedClamp(*geo, prior=prior, device=dev),
        "forward_only": lambda: G.ClampGPU(*geo, with_prior=False, device=dev),
    }
    iters = args.eval_iters
    out = {}
    for name, make in forms.items():
        g = make()
        g.init(yt)
        trace = [Lm.nrmse(torch.tensordot(torch.tensor(g.upsilon, device=dev, dtype=torch.float32), g.w, 1), rt)]
        for _ in range(iters):
            g.iterate()
            trace.append(Lm.nrmse(g.wbar, rt))
        conv = g.conv_err()
        fault = int(g.fault.item())
        # wall time per iteration, timed without the NRMSE checks
        g.init(yt)
        for _ in range(args.warmup):
            g.iterate()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.iterate()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        out[name] = {"nrmse": [round(v, 5) for v in trace], "ms_per_iter": ms, "conv_err": conv, "fault": fault}
        log("%-12s nrmse it0 %.4f it%d %.4f min %.4f, %.3f ms/iter, conv %.2e" %
            (name, trace[0], iters, trace[-1], min(trace), ms, conv))
        del g
        torch.cuda.empty_cache()
    training = {"mode": args.train_mode, "pairs": args.train_pairs, "patch": [pz, py, px],
                "pair_synthesis_s": round(t_pairs, 2), "epochs": args.train_epochs, "lr": args.lr,
                "steps": hist["steps"], "seconds": round(hist["seconds"], 2), "best_val": hist["best_val"]}
    return {"out": out, "equal": equal_nrmse_summary(out, iters), "hist": hist, "training": training,
            "prior": prior, "spec": spec, "unet": unet, "patch": (pz, py, px)}


def run_learned(args):
    """Learned form: train the CNN prior agent, reconstruct the evaluation
    scene with the three forms, time the prior agent alone, and report the
    equal-NRMSE comparison."""
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    copy_probe(args, dev)
    ev = learned_eval(args, dev)
    out, hist, prior, spec, unet = ev["out"], ev["hist"], ev["prior"], ev["spec"], ev["unet"]
    pz, py, px = ev["patch"]
    fwd_flop, train_flop = (UNET_FWD_FLOP, UNET_TRAIN_FLOP) if unet else (CNN_FWD_FLOP, CNN_TRAIN_FLOP)
    train_tflops = hist["voxels"] * train_flop / hist["seconds"] / 1e12
    t_pairs = ev["training"]["pair_synthesis_s"]

    # the learned prior alone, timed with events on the stream it runs on
    w = torch.rand(spec.nz, spec.ny, spec.nx, device=dev) + 0.05
    o = torch.empty_like(w)
    for _ in range(3):
        prior.apply(w, o)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    ev0.record()
    for _ in range(reps):
        prior.apply(w, o)
    ev1.record()
    torch.cuda.synchronize()
    cnn_ms = ev0.elapsed_time(ev1) / reps
    cnn_tflops = spec.n * fwd_flop / (cnn_ms * 1e-3) / 1e12

    rec = None if unet else counter_traffic("cnn_apply_64x256x256", "cnn")
    cnn_traffic = round(rec["read_bytes"] + rec["write_bytes"]) if rec is not None else None
    equal = ev["equal"]
    lt = out["learned"]
    units = spec.looks * spec.n
    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": units / (lt["ms_per_iter"] * 1e-3),
        "unit": "voxel-looks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lt["ms_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (forward agents), bf16 with f32 accumulation (%s)" % ("U-Net" if unet else "CNN"),
        "data": "synthetic",
        "config": {"workload": "learned form: CLAMP iteration with the %s prior agent, %dx%dx%d, %d looks, "
                               "pupil radius %g, SNR %g dB; trained on %d seeded %dx%dx%d denoising pairs"
                               % ("U-Net" if unet else "CNN", spec.nx, spec.ny, spec.nz, spec.looks, spec.radius,
                                  spec.snr_db, args.train_pairs, px, py, pz),
                   "prior": args.prior, "sigma2": args.sigma2, "train_epochs": args.train_epochs, "lr": args.lr,
                   "train_mode": args.train_mode, "train_noise": args.train_noise},
        "roofline": {"bound": "mfma",
                     "kernel": ("unet_apply (13 convolutions, 3 transposed)" if unet
                                else "cnn_apply (8 convolutions)"),
                     "achieved": round(cnn_tflops, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(cnn_tflops / BF16_PEAK_TFLOPS, 4), "traffic": cnn_traffic},
        "prior_apply_ms": round(cnn_ms, 3),
        "cnn_apply_ms": None if unet else round(cnn_ms, 3),
        "training": {"mode": args.train_mode, "pairs": args.train_pairs, "pair_synthesis_s": t_pairs,
                     "steps": hist["steps"],
                     "seconds": round(hist["seconds"], 2), "voxels_per_s": hist["voxels"] / hist["seconds"],
                     "tflops": round(train_tflops, 2), "frac_bf16_peak": round(train_tflops / BF16_PEAK_TFLOPS, 4),
                     "val_loss": [round(v, 6) for v in hist["val"]], "best_val": hist["best_val"]},
        "equal_nrmse": equal,
        "forms": out,
    }
    print(json.dumps(result), flush=True)


def large_eval(args, dev, prior=None):
    """Large reconstruction: 512x512x128, 32 looks, SNR 5 dB, four objects;
    CLAMP with the learned prior for `--eval-iters` iterations through the
    forward-only fallback driver, and the forward-only reconstruction beside
    it as the reference for its error.  prior: a trained CnnPrior, or None to
    train one as in the learned workload.  Returns the figures as a dict."""
    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import _clamp as C
    from paper_2406_13651_amd import learned as Lm
    from paper_2406_13651_amd.perf import stage_bytes

    train_s = None
    if prior is None:
        log("training pairs: %d volumes of 64x64x32" % args.train_pairs)
        X, T = Lm.make_pairs(args.train_pairs, seed=0, mode=args.train_mode, noise=args.train_noise)
        prior = Lm.CnnPrior(Lm.init_params(0), device=dev)
        train_s = Lm.train(prior, X, T, epochs=args.train_epochs, lr=args.lr)["seconds"]
        del X, T
    spec = synth.CONFIGS["large"]
    log("synthesising %dx%dx%d, %d looks" % (spec.nx, spec.ny, spec.nz, spec.looks))
    t0 = time.perf_counter()
    r_true, y, s2w = synth.make_problem(spec, 0, workers=16)
    t_syn = time.perf_counter() - t0
    yt = torch.from_numpy(y).to(dev)
    rt = torch.from_numpy(r_true.astype(np.float32)).to(dev)
    del y, r_true
    geo = (spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, args.sigma2)
    iters = args.eval_iters
    units = spec.looks * spec.n

    log("large: learned form, %d iterations" % iters)
    g = Lm.LearnedClamp(*geo, prior=prior, device=dev)
    sb = stage_bytes(spec.nx, spec.ny, spec.nz, spec.looks, g.info["P"], g.info["B"], spec.looks + 1, fused=g.fused)
    g.init(yt)
    # after the warm-up, 5 iterations with every stage timed give the
    # per-stage breakdown and pick the dominant stage; the timed run,
    # restarted from the initialisation, carries events around it only
    for _ in range(args.warmup):
        g.iterate()
    torch.cuda.synchronize()
    C.clamp_plan_set_timing(g.plan, True)
    for _ in range(5):
        g.iterate()
    torch.cuda.synchronize()
    C.clamp_plan_set_timing(g.plan, False)
    stages = dict(C.clamp_plan_get_timing(g.plan))
    dom = max((k for k in stages if k in sb), key=lambda k: stages[k][0])
    g.init(yt)
    C.clamp_plan_set_timing_stages(g.plan, [dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, info = Lm.run_with_fallback(lambda: g, lambda: G.ClampGPU(*geo, with_prior=False, device=dev), yt, iters)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    C.clamp_plan_set_timing(g.plan, False)
    timed = C.clamp_plan_get_timing(g.plan)
    learned_nrmse = Lm.nrmse(out, rt)
    learned_out = out.clone()
    fault = int(g.fault.item())
    conv = g.conv_err()
    if dom in timed:
        stages[dom] = timed[dom]
    del g, out
    torch.cuda.empty_cache()

    log("large: forward-only reference, %d iterations" % iters)
    f = G.ClampGPU(*geo, with_prior=False, device=dev)
    f.init(yt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.run(iters)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    fwd_nrmse = Lm.nrmse(f.wbar, rt)
    diff = Lm.nrmse(learned_out, f.wbar)
    del f, learned_out, yt, rt
    torch.cuda.empty_cache()
    per_stage = {}
    for name, (ms, cnt) in stages.items():
        e = {"avg_ms": round(ms / cnt, 4), "launches": cnt}
        if name in sb:
            e["alg_GBps"] = round(sb[name] / (ms / cnt * 1e-3) / 1e9, 1)
        per_stage[name] = e
    dom_ms = stages[dom][0] / stages[dom][1]
    achieved = sb[dom] / (dom_ms * 1e-3) / 1e9
    ms_iter = t_learned / iters * 1e3
    return {
        "workload": "CLAMP with the learned prior, %dx%dx%d, %d looks, pupil radius %g, SNR %g dB, %d objects; "
                    "%.2f GB of complex64 looks" % (spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, spec.snr_db,
                                                    spec.n_objects, spec.n * spec.looks * 8 / 1e9),
        "iterations": iters,
        "ms_per_iter": round(ms_iter, 3),
        "voxel_looks_per_s": units / (ms_iter * 1e-3),
        "forward_only_voxel_looks_per_s": units * iters / t_fwd,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)},
        "nrmse": {"learned": learned_nrmse, "forward_only": fwd_nrmse, "learned_vs_forward_only": diff},
        "conv_err": conv,
        "reductions": "float64 (step sizes, h, convergence error, mu-residual)",
        "fallback": info,
        "wall_s": {"learned": round(t_learned, 3), "forward_only": round(t_fwd, 3), "synthesis": round(t_syn, 1),
                   "training": None if train_s is None else round(train_s, 2)},
        "stages": per_stage,
        "fault": fault,
    }


def run_large(args):
    """The large reconstruction as its own bench line (large_eval)."""
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lg = large_eval(args, dev)
    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": lg["voxel_looks_per_s"],
        "unit": "voxel-looks/s",
        "n_gpus": 1,
        "steps": lg["iterations"],
        "warmup": args.warmup,
        "ms_per_step": lg["ms_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (forward agents), bf16 with f32 accumulation (CNN)",
        "data": "synthetic",
        "config": {"workload": "large: " + lg["workload"], "sigma2": args.sigma2, "iterations": lg["iterations"]},
        "roofline": dict(lg["roofline"], traffic=None),
        "large": lg,
    }
    print(json.dumps(result), flush=True)


def run_compare(args):
    """The comparison of Sec. V (the paper's Table 2 is on its own synthetic
    train scene) on the full-size synthetic scene: the speckle average, and
    CLAMP with the l2,1 agent, the TV agent, the Gaussian prior (the plain
    form), the forward agents alone and, with --compare-learned, the trained
    CNN prior; PSNR and volumetric NRMSE (eq. psnr, scale-fit) and the
    point-cloud metrics (eqs. pc-distance, nrmse) after --eval-iters
    iterations.  The l2,1 and TV weights are chosen from a grid on scene 1,
    never on the evaluation scene 0."""
    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import metrics as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = synth.CONFIGS["full"]
    iters = args.eval_iters
    geo = (spec.nx, spec.ny, spec.nz, spec.looks, spec.radius)

    def run(y, s2w, **kw):
        g = G.ClampGPU(*geo, s2w, args.sigma2, device=dev, **kw)
        g.init(y)
        sa = g.speckle_average()
        t0 = time.perf_counter()
        g.run(iters)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / iters * 1e3
        out = g.wbar.cpu().numpy().astype(np.float64)
        info = {"conv_err": g.conv_err(), "ms_per_iter": round(ms, 3), "fault": int(g.fault.item())}
        return out, sa.cpu().numpy().astype(np.float64), info

    def weights(sa):
        """Candidate weights scaled to the initial image: the l2,1 threshold
        against the median range-slice norm, the TV weight against the mean."""
        norms = np.sqrt(np.sum(sa ** 2, axis=(1, 2)))
        return ({"l21": [f * float(np.median(norms)) for f in (0.05, 0.2, 0.5)],
                 "tv": [f * float(sa.mean()) for f in (0.05, 0.2, 0.5)]})

    log("tuning the l2,1 and TV weights on scene 1")
    r1, y1, s21 = synth.make_problem(spec, 1, workers=16)
    y1t = torch.from_numpy(y1).to(dev)
    del y1
    _, sa1, _ = run(y1t, s21, with_prior=False)
    chosen = {}
    for kind, cands in weights(sa1).items():
        best = None
        for wgt in cands:
            out, _, _ = run(y1t, s21, prior=kind, prior_weight=wgt, tv_iters=args.tv_iters)
            e = M.nrmse(out, r1)
            log("  %s weight %.4g: NRMSE %.4f" % (kind, wgt, e))
            if best is None or e < best[1]:
                best = (wgt, e)
        chosen[kind] = best[0]
    del y1t
    torch.cuda.empty_cache()

    log("evaluation scene 0")
    r0, y0, s20 = synth.make_problem(spec, 0, workers=16)
    y0t = torch.from_numpy(y0).to(dev)
    del y0
    mask_alpha = G.clamp_plan_create([G.Scene(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius)]).info[0]["alpha"]
    floor = s20 / mask_alpha
    thr_true = spec.r_min
    cutoff = M.rayleigh_cutoff(spec.nx, spec.radius)

    def quality(img):
        b = M.scale_fit(img, r0)
        pc = M.point_cloud_metrics(b * img, r0, spec.r_min + floor, thr_true, cutoff)
        return {"psnr": M.psnr(img, r0), "nrmse": M.nrmse(img, r0),
                "point_cloud": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in pc.items()}}

    forms = {"l21": dict(prior="l21", prior_weight=chosen["l21"], tv_iters=args.tv_iters),
             "tv": dict(prior="tv", prior_weight=chosen["tv"], tv_iters=args.tv_iters),
             "gaussian": dict(prior="gauss"),
             "forward_only": dict(with_prior=False)}
    rows = {}
    sa = None
    for name, kw in forms.items():
        out, sa, info = run(y0t, s20, **kw)
        rows[name] = dict(quality(out), **info)
        log("  %-12s PSNR %.2f dB, NRMSE %.4f, pc distance %.3f, FPR %.3f" % (
            name, rows[name]["psnr"], rows[name]["nrmse"], rows[name]["point_cloud"]["distance"],
            rows[name]["point_cloud"]["false_positive_rate"]))
    rows["speckle_average"] = quality(sa)
    if args.compare_learned:
        from paper_2406_13651_amd import learned as Lm
        X, T = Lm.make_pairs(args.train_pairs, seed=0, mode=args.train_mode, noise=args.train_noise)
        prior = Lm.CnnPrior(Lm.init_params(0), device=dev)
        Lm.train(prior, X, T, epochs=args.train_epochs, lr=args.lr)
        del X, T
        g = Lm.LearnedClamp(*geo, s20, args.sigma2, prior=prior, device=dev)
        g.init(y0t)
        t0 = time.perf_counter()
        g.run(iters)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / iters * 1e3
        rows["learned"] = dict(quality(g.wbar.cpu().numpy().astype(np.float64)), conv_err=g.conv_err(),
                               ms_per_iter=round(ms, 3), fault=int(g.fault.item()))
    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": spec.looks * spec.n / (rows["gaussian"]["ms_per_iter"] * 1e-3),
        "unit": "voxel-looks/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": 0,
        "ms_per_step": rows["gaussian"]["ms_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "comparison of Sec. V on the full-size scene (256x256x64, 16 looks, SNR 10 dB): "
                               "speckle average and CLAMP with l2,1, TV, Gaussian and no prior agent, %d "
                               "iterations; value: the Gaussian form's rate" % iters,
                   "sigma2": args.sigma2, "weights": chosen, "tv_iters": args.tv_iters,
                   "point_cloud": {"truth": "voxels above the background %g" % thr_true,
                                   "reconstruction": "voxels of beta* r_hat above the background plus the "
                                                     "noise floor sigma_w^2/alpha = %.4g" % floor,
                                   "cutoff_voxels": round(cutoff, 3)}},
        "forms": rows,
    }
    print(json.dumps(result), flush=True)


# The paper's own configuration (Sec. III-D and Sec. V): a 128^3 image from
# 64 range samples zero-padded by q = 2, 9 looks, the U-Net prior; it states
# under 0.5 s per CLAMP iteration on one NVIDIA Quadro RTX 8000.
PAPER_CONFIG = dict(n=128, looks=9, radius=32.0, range_box=64)
PAPER_SECONDS_PER_ITERATION = 0.5


def run_paper(args):
    """CLAMP iterations at the paper's configuration with its U-Net prior, and
    with the Gaussian and CNN priors beside it (untrained weights: the time
    of an iteration does not depend on them).  The paper's figure is an upper
    bound on its time per iteration, so vs_baseline is a lower bound on the
    ratio of iteration rates."""
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import learned as Lm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c = PAPER_CONFIG
    n, L, R, K = c["n"], c["looks"], c["radius"], c["range_box"]
    spec = synth.SceneSpec("paper", n, n, n, L, R, 10.0, 24, 0.05, 1, 1)
    log("paper configuration: %dx%dx%d, %d looks, range box %d (q = %g)" % (n, n, n, L, K, n / K))
    r_true, y, s2w = synth.make_problem(spec, 0, workers=16, range_support=K)
    yt = torch.from_numpy(y).to(dev)
    del y
    geo = (n, n, n, L, R, s2w, args.sigma2)
    forms = {
        "unet": lambda: Lm.LearnedClamp(*geo, prior=Lm.UnetPrior(Lm.unet_init_params(0), device=dev),
                                        range_support=K, device=dev),
        "gaussian": lambda: G.ClampGPU(*geo, with_prior=True, range_support=K, device=dev),
        "cnn": lambda: Lm.LearnedClamp(*geo, prior=Lm.CnnPrior(Lm.init_params(0), device=dev), range_support=K,
                                       device=dev),
    }
    out = {}
    for name, make in forms.items():
        g = make()
        g.init(yt)
        for _ in range(args.warmup):
            g.iterate()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.iterate()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        out[name] = {"ms_per_iter": round(ms, 4), "fault": int(g.fault.item())}
        log("  %-8s %.3f ms per iteration" % (name, ms))
        del g
        torch.cuda.empty_cache()
    ms = out["unet"]["ms_per_iter"]
    units = n ** 3 * L
    print(json.dumps({
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": units / (ms * 1e-3), "unit": "voxel-looks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "iters_per_s": 1e3 / ms,
        "vs_baseline": (1e3 / ms) / (1.0 / PAPER_SECONDS_PER_ITERATION),
        "baseline": {"value": 1.0 / PAPER_SECONDS_PER_ITERATION, "unit": "iterations/s",
                     "source": "Sec. III-D: under 0.5 s per CLAMP iteration at 128^3 on one NVIDIA Quadro RTX 8000",
                     "note": "an upper bound on the paper's time, another machine; context, not a target"},
        "dtype": "f32 (forward agents), bf16 with f32 accumulation (U-Net)", "data": "synthetic",
        "config": {"workload": "the paper's configuration: CLAMP with the U-Net prior, %dx%dx%d from %d range "
                               "samples (q = %g, 3D operator), %d looks, pupil radius %g, SNR 10 dB" % (
                                   n, n, n, K, n / K, L, R)},
        "forms": out,
    }))


def run_tiny(args):
    """The tiny forward-only scene (32x32x16, 4 looks, pupil radius 8, SNR
    20 dB; the looks' forward agents and the Mann step, no prior): latency
    per CLAMP iteration, launched call by call through the single-scene
    driver, as eager one-scene batched steps, and replayed from the batch's
    captured HIP graph (one graph launch per iteration).  At this size an
    iteration moves about 3.5 MB and is bound by launch latency, so no
    roofline is reported.  The graph-replayed state is compared with the
    single-scene driver's after the same iterations; the CPU baseline is
    the float64 oracle's time per iteration of the same run."""
    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G

    spec = synth.CONFIGS["tiny"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    r_true, y, s2w = synth.make_problem(spec, 0)
    yt = torch.from_numpy(y).to(dev)
    log("tiny forward-only scene %dx%dx%d, %d looks: %d warmup and %d timed iterations per form"
        % (spec.nx, spec.ny, spec.nz, spec.looks, args.warmup, args.steps))
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, args.sigma2, with_prior=False,
                   device=dev)
    g.init(yt)
    g.run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(args.steps)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t0) / args.steps * 1e3

    b = G.ClampBatchGPU([dict(nx=spec.nx, ny=spec.ny, nz=spec.nz, looks=spec.looks, radius=spec.radius,
                              sigma_w2=s2w, sigma2=args.sigma2, with_prior=False)], device=dev)
    b.init([yt])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            b.step(stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.step(stream)
        stream.synchronize()
        batch_ms = (time.perf_counter() - t0) / args.steps * 1e3
        b.capture(stream)
        b.replay(1, stream)
        stream.synchronize()
        t0 = time.perf_counter()
        b.replay(args.steps, stream)
        stream.synchronize()
        graph_ms = (time.perf_counter() - t0) / args.steps * 1e3
    torch.cuda.synchronize()
    # the single-scene driver brought to the batch's iteration count
    g.run(b.k - g.k)
    torch.cuda.synchronize()
    w_b, w_g = b.states[0]["wbar"].cpu().numpy(), g.wbar.cpu().numpy()
    gap = float(np.linalg.norm(w_b - w_g) / np.linalg.norm(w_g))
    fault = int(b.fault.item()) | int(g.fault.item())
    log("  single-scene %.4f ms, batch eager %.4f ms, graph replay %.4f ms per iteration; "
        "graph vs single-scene rel. L2 %.2e after %d iterations" % (single_ms, batch_ms, graph_ms, gap, b.k))
    units = spec.looks * spec.n
    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": units / (graph_ms * 1e-3), "unit": "voxel-looks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": graph_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tiny forward-only CLAMP (looks' forward agents + Mann step, no prior), %dx%dx%d, "
                               "%d looks, pupil radius %g, SNR %g dB, one graph replay per iteration"
                               % (spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, spec.snr_db)},
        "latency_us": {"graph_replay": round(graph_ms * 1e3, 2), "batch_eager": round(batch_ms * 1e3, 2),
                       "single_scene_calls": round(single_ms * 1e3, 2)},
        "roofline": None,
        "graph_vs_single_scene_rel_l2": gap,
        "iterations_compared": b.k,
        "fault": fault,
    }
    if not args.no_cpu_baseline:
        import oracle
        f32 = lambda v: float(np.float32(v))  # noqa: E731
        iters = 20
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.clamp_run(y, spec.radius, f32(s2w), f32(args.sigma2), iters, with_prior=False, keep_hist=False)
            times.append(time.perf_counter() - t0)
        t = sorted(times)[1]
        result["cpu_baseline"] = {"value": units * iters / t, "unit": "voxel-looks/s", "cores": 1,
                                  "kind": "oracle", "ms_per_iter": round(t / iters * 1e3, 3),
                                  "sample": "%d forward-only iterations of the same scene in float64, median of 3"
                                            % iters}
    print(json.dumps(result), flush=True)


# The padded workload's cases: (name, zero-padding factor q, all-pass
# aperture); q = 1, 1.5, 2 are the factors of Sec. V.
PADDED_CASES = [("q=1", 1.0, False), ("q=1.5", 1.5, False), ("q=2", 2.0, False), ("ablation a=1, q=1", 1.0, True)]


def run_padded(args):
    """The 3D operator with zero-padding in range (Sec. II-A): the full-size
    scene with its 64 range samples padded by q in {1, 1.5, 2} (nz = 64 q, a
    range box of K = 64 frequencies), 16 looks, Gaussian prior; and the
    aperture ablation a = 1 (all-pass pupil and range box).  Reports time per
    iteration, the range passes' bandwidth and the NRMSE after the timed
    iterations for each."""
    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import _clamp as C
    from paper_2406_13651_amd.perf import stage_bytes
    from paper_2406_13651_amd.learned import nrmse

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = synth.CONFIGS["full"]
    K = base.nz
    rows = {}
    for name, q, allpass in PADDED_CASES:
        nz = int(round(base.nz * q))
        spec = synth.SceneSpec(base.name, base.nx, base.ny, nz, base.looks, base.radius, base.snr_db,
                               base.n_facets, base.r_min, base.n_objects, base.config_id)
        log("%s: %dx%dx%d, range box %d, %d looks" % (name, spec.nx, spec.ny, nz, K, spec.looks))
        mask = np.ones((spec.ny, spec.nx), np.uint8) if allpass else None
        if allpass:
            # a = 1: every sample of the 3D frequency grid holds data (a pupil radius
            # beyond the grid and a full range box)
            r_true, y, s2w = synth.make_problem(
                synth.SceneSpec(spec.name, spec.nx, spec.ny, spec.nz, spec.looks, 1e9, spec.snr_db, spec.n_facets,
                                spec.r_min, spec.n_objects, spec.config_id), 0, workers=16, range_support=nz)
        else:
            r_true, y, s2w = synth.make_problem(spec, 0, workers=16, range_support=K)
        yt = torch.from_numpy(y).to(dev)
        del y
        rt = torch.from_numpy(r_true.astype(np.float32)).to(dev)
        g = G.ClampGPU(spec.nx, spec.ny, nz, spec.looks, spec.radius, s2w, args.sigma2, with_prior=True,
                       device=dev, mask=mask, range_support=nz if allpass else K)
        g.init(yt)
        info = g.info
        sb = stage_bytes(spec.nx, spec.ny, nz, spec.looks, info["P"], info["B"], g.N, g.scene.range_support,
                         fused=g.fused)
        res = {}

        def after():
            res.update(nrmse=nrmse(g.wbar, rt), conv_err=g.conv_err(), fault=int(g.fault.item()))

        el, stages, _ = warmup_and_time(C, g.plan, g.iterate, args.warmup, args.steps, sb, after)
        per = {}
        for k, (ms, cnt) in stages.items():
            e = {"avg_ms": round(ms / cnt, 4)}
            if k in sb:
                e["alg_GBps"] = round(sb[k] / (ms / cnt * 1e-3) / 1e9, 1)
            per[k] = e
        rows[name] = {"nz": nz, "range_support": g.scene.range_support, "alpha": info["alpha"],
                      "ms_per_iter": el / args.steps * 1e3,
                      "voxel_looks_per_s": spec.n * spec.looks * args.steps / el,
                      "nrmse": res["nrmse"], "conv_err": res["conv_err"], "fault": res["fault"],
                      "stages": per}
        log("  %.3f ms/iter, NRMSE %.4f, conv %.2e" % (rows[name]["ms_per_iter"], rows[name]["nrmse"],
                                                       rows[name]["conv_err"]))
        del g, yt, rt
        torch.cuda.empty_cache()
    q1 = rows["q=1"]
    dom = max((k for k in q1["stages"] if "alg_GBps" in q1["stages"][k]), key=lambda k: q1["stages"][k]["avg_ms"])
    achieved = q1["stages"][dom]["alg_GBps"]
    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": q1["voxel_looks_per_s"],
        "unit": "voxel-looks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": q1["ms_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D operator with range zero-padding: 256x256x(64 q), range box of 64 frequencies, "
                               "16 looks, pupil radius 64, SNR 10 dB, Gaussian prior; value at q = 1",
                   "sigma2": args.sigma2},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "cases": rows,
    }
    print(json.dumps(result), flush=True)


def parser():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="full")
    ap.add_argument("--sigma2", type=float, default=1e-3)
    ap.add_argument("--r-update", default="quadratic", choices=("quadratic", "exact"),
                    help="forward-agent r-update: the quadratic surrogate (App. A) or the exact surrogate prox")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="full workload: skip the large configuration (512x512x128, 32 looks, learned prior)")
    ap.add_argument("--no-learned", action="store_true",
                    help="full workload: skip the equal-NRMSE comparison (CNN training and three 50-iteration runs)")
    ap.add_argument("--batch-cap", type=float, default=2.5e9,
                    help="largest total voxel-looks of the uneven batch draw (--workload batch)")
    ap.add_argument("--train-pairs", type=int, default=2000, help="training volumes (--workload learned)")
    ap.add_argument("--train-epochs", type=int, default=30)
    ap.add_argument("--prior", default="cnn", choices=("cnn", "unet"),
                    help="learned workload: the 8-layer CNN or the U-Net prior")
    ap.add_argument("--train-mode", default="speckle", choices=("speckle", "clamp", "awgn"),
                    help="training inputs: speckle averages of looks the forward model simulates (default), "
                         "consensus images of forward-only CLAMP runs on them, or the target plus white noise")
    ap.add_argument("--train-noise", type=float, default=0.3,
                    help="awgn pairs: noise standard deviation U[0, train_noise] max(target)")
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--eval-iters", type=int, default=50)
    ap.add_argument("--tv-iters", type=int, default=20, help="Chambolle steps per TV prior application")
    ap.add_argument("--compare-learned", action="store_true",
                    help="compare workload: also train the CNN prior and include the learned form")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy MIB mebibytes once with a plain device copy, as a "
                         "known-size reference for hardware byte counters")
    return ap


def main():
    args = parser().parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on one GPU and has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "learned":
        run_learned(args)
        return
    if args.workload == "large":
        run_large(args)
        return
    if args.workload == "padded":
        run_padded(args)
        return
    if args.workload == "compare":
        run_compare(args)
        return
    if args.workload == "paper":
        run_paper(args)
        return
    if args.workload == "tiny":
        run_tiny(args)
        return

    import numpy as np
    import torch

    import synth
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import _clamp as C
    from paper_2406_13651_amd.perf import agent_bytes_min, stage_bytes

    spec = synth.CONFIGS[args.workload]
    log("generating %s workload %dx%dx%d, %d looks" % (spec.name, spec.nx, spec.ny, spec.nz, spec.looks))
    r_true, y, s2w = synth.make_problem(spec, 0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, args.sigma2, with_prior=True,
                   device=dev, r_update=args.r_update)
    yt = torch.from_numpy(y).to(dev)
    g.init(yt)
    copy_probe(args, dev)
    info = g.info
    sb = stage_bytes(spec.nx, spec.ny, spec.nz, spec.looks, info["P"], info["B"], g.N, fused=g.fused)
    log("warmup %d iterations, a 10-iteration per-stage breakdown, then %d timed iterations"
        % (args.warmup, args.steps))
    res = {}

    def after():
        res["fault"] = int(g.fault.item())
        res["conv"] = g.conv_err()
        wbar = g.wbar.cpu().numpy().astype(np.float64)
        bs = float(wbar.ravel() @ r_true.ravel() / (wbar.ravel() @ wbar.ravel()))
        res["nrmse"] = float(np.linalg.norm(bs * wbar - r_true) / np.linalg.norm(r_true))

    elapsed, stages, dom = warmup_and_time(C, g.plan, g.iterate, args.warmup, args.steps, sb, after)
    fault, conv, nrmse = res["fault"], res["conv"], res["nrmse"]

    units = spec.looks * spec.n
    value = units * args.steps / elapsed
    per_stage = {}
    for name, (ms, cnt) in stages.items():
        avg = ms / cnt
        entry = {"avg_ms": round(avg, 5), "launches": cnt}
        if name in sb:
            entry["alg_bytes"] = sb[name]
            entry["alg_GBps"] = round(sb[name] / (avg * 1e-3) / 1e9, 1)
        per_stage[name] = entry
    dom_avg_ms = stages[dom][0] / stages[dom][1]
    achieved = sb[dom] / (dom_avg_ms * 1e-3) / 1e9
    traffic = None
    rec = (counter_traffic("clamp_iteration_256x256x64_L16", "fwd")
           if args.workload == "full" and args.r_update == "quadratic" else None)
    if rec is not None and dom in rec["stages"]:
        traffic = round(rec["stages"][dom]["read_bytes"] + rec["stages"][dom]["write_bytes"])
    agent_stage_names = ("col_inv", "row_grad", "col_fwd", "gamma", "row_update", "row_update_mann",
                         "resid_update", "diag_after")
    # the per-stage events of the breakdown add a few percent to each stage,
    # so the agents' time is the clean timed iteration less the stages that
    # are not the forward agents' (prior and the Mann step's own launch)
    other_ms = sum(stages[k][0] / stages[k][1] for k in stages if k not in agent_stage_names)
    mann_ms = stages["mace_step"][0] / stages["mace_step"][1] if "mace_step" in stages else 0.0
    agent_ms = elapsed / args.steps * 1e3 - other_ms
    agent_min = agent_bytes_min(spec.nx, spec.ny, spec.nz, spec.looks, info["P"])

    def agent_roof(ms, what):
        gbps = agent_min / (ms * 1e-3) / 1e9
        return {"what": what, "ms": round(ms, 4), "voxel_looks_per_s": units / (ms * 1e-3),
                "min_bytes": agent_min, "GBps_vs_min_bytes": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBS, 4)}

    result = {
        "metric": "fwd-agent voxel-looks/s + HBM GB/s vs peak; CLAMP iters/s at fixed NRMSE",
        "value": value,
        "unit": "voxel-looks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "CLAMP iteration (forward agents + Gaussian prior + Mann step), %dx%dx%d, "
                               "%d looks, pupil radius %g, SNR %g dB" % (spec.nx, spec.ny, spec.nz, spec.looks,
                                                                         spec.radius, spec.snr_db),
                   "nx": spec.nx, "ny": spec.ny, "nz": spec.nz, "looks": spec.looks, "pupil_radius": spec.radius,
                   "sigma2": args.sigma2, "r_update": args.r_update, "mann_step": "fused into the update pass",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "iters_per_s": args.steps / elapsed,
        # the lower bound (48 + 32 alpha bytes per voxel-look) counts the Mann
        # update's w traffic as fused into the agent's last pass, as the fused
        # update pass does (the Mann step's own launch is then only its final
        # reduction, counted in the second figure)
        "fwd_agent": agent_roof(agent_ms, "forward-agent stages (col_inv .. diag_after, the update pass with the "
                                          "Mann step fused in): the timed iteration less the other stages' "
                                          "breakdown means, against the lower bound of one application"),
        "fwd_agent_with_mann": agent_roof(agent_ms + mann_ms, "forward-agent stages plus the Mann step's launch"),
        "stages": per_stage,
        "conv_err": conv,
        "nrmse": nrmse,
        "fault": fault,
    }
    if not args.no_cpu_baseline:
        threads = max(1, min(16, host_cpu()[2]))
        log("one more iteration against the float64 oracle, timed on %d threads and on one" % threads)
        check, base = oracle_check_and_cpu_baseline(spec, y, g, args.sigma2, threads)
        result["oracle_check"] = check
        result["cpu_baseline"] = base
    if args.workload == "full" and not args.no_learned:
        # the second half of the metric: the learned form against the plain
        # form at a fixed NRMSE, on the learned workload's evaluation scene
        del g, yt
        torch.cuda.empty_cache()
        log("equal-NRMSE comparison: train the CNN prior, then 3 forms x %d iterations" % args.eval_iters)
        ev = learned_eval(args, dev)
        sp = ev["spec"]
        result["equal_nrmse"] = dict(ev["equal"], workload="CNN prior agent trained on the GPU; evaluation scene "
                                     "%dx%dx%d, %d looks, pupil radius %g, SNR %g dB" %
                                     (sp.nx, sp.ny, sp.nz, sp.looks, sp.radius, sp.snr_db),
                                     training=ev["training"])
        if not args.no_large:
            # the large configuration with the same trained prior
            lg = large_eval(args, dev, ev["prior"])
            lg.pop("stages")
            result["large"] = lg
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
