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


def cpu_baseline(spec, y, g, sigma2, budget_s=12.0):
    """Time the float64 oracle on a bounded sample of one iteration."""
    import numpy as np
    import oracle

    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    alpha = oracle.aperture_fraction(mask)
    mu = g.mu.cpu().numpy()
    r = g.r.cpu().numpy().astype(np.float64)
    w = g.w.cpu().numpy().astype(np.float64)
    s2w = float(np.float32(g.sigma_w2))
    t_agents, looks_done = 0.0, 0
    for l in range(spec.looks):
        t0 = time.perf_counter()
        oracle.forward_agent(mu[l].astype(np.complex128), y[l].astype(np.complex128), r[l], w[l], mask, s2w,
                             sigma2, alpha, 1.5)
        t_agents += time.perf_counter() - t0
        looks_done += 1
        if t_agents > budget_s:
            break
    t0 = time.perf_counter()
    rr = r.copy()
    rr[spec.looks] = oracle.gaussian_smooth(w[spec.looks], 1.0)
    ups = oracle.agent_weights(spec.looks, True)
    oracle.convergence_error(rr, w, ups)
    oracle.mann_step(w, rr, ups, 0.5)
    t_rest = time.perf_counter() - t0
    t_iter = t_agents / looks_done * spec.looks + t_rest
    return {
        "value": spec.looks * spec.n / t_iter,
        "unit": "voxel-looks/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "float64 numpy oracle: forward agents of %d of %d looks plus one Gaussian prior and Mann "
                  "step at %dx%dx%d, scaled to a whole iteration (%.1f s measured)"
                  % (looks_done, spec.looks, spec.nx, spec.ny, spec.nz, t_agents + t_rest),
    }


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
    for i, sp in enumerate(specs):
        _, y, s2 = synth.make_problem(sp, i, workers=16)
        assert np.float32(s2) == np.float32(scenes[i]["sigma_w2"])
        yt = torch.from_numpy(y).to(dev)
        del y
        b.init_scene(i, yt)
        del yt
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
    sb = {}
    for i, sp in enumerate(specs):
        info = b.plan.info[i]
        for k, v in stage_bytes(sp.nx, sp.ny, sp.nz, sp.looks, info["P"], info["B"], sp.looks + 1).items():
            sb[k] = sb.get(k, 0) + v
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
                   "scenes": [[sp.nx, sp.nz, sp.looks] for sp in specs], "sigma2": args.sigma2},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "per_scene_launch": {"ms_per_step": round(per_scene_ms, 3),
                             "voxel_looks_per_s": total / (per_scene_ms * 1e-3)},
        "batched_over_per_scene": round(per_scene_ms / (elapsed / args.steps * 1e3), 3),
        "autotune": tuned,
        "stages": per_stage,
        "fault": int(b.fault.item()),
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="full")
    ap.add_argument("--sigma2", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-cap", type=float, default=2.5e9,
                    help="largest total voxel-looks of the uneven batch draw (--workload batch)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy MIB mebibytes once with a plain device copy, as a "
                         "known-size reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        run_batch(args)
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
                   device=dev)
    yt = torch.from_numpy(y).to(dev)
    g.init(yt)
    if args.copy_probe > 0:
        nfl = args.copy_probe * (1 << 20) // 4
        src = torch.ones(nfl, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (nfl * 4, nfl * 4))
        del src, dst
    log("warmup %d iterations" % args.warmup)
    for _ in range(args.warmup):
        g.iterate()
    torch.cuda.synchronize()
    C.clamp_plan_set_timing(g.plan, True)
    log("timing %d iterations" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.iterate()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    C.clamp_plan_set_timing(g.plan, False)
    stages = C.clamp_plan_get_timing(g.plan)
    fault = int(g.fault.item())
    conv = g.conv_err()
    wbar = g.wbar.cpu().numpy().astype(np.float64)
    bs = float(wbar.ravel() @ r_true.ravel() / (wbar.ravel() @ wbar.ravel()))
    nrmse = float(np.linalg.norm(bs * wbar - r_true) / np.linalg.norm(r_true))

    elapsed = t1 - t0
    units = spec.looks * spec.n
    value = units * args.steps / elapsed
    info = g.info
    sb = stage_bytes(spec.nx, spec.ny, spec.nz, spec.looks, info["P"], info["B"], g.N)
    per_stage = {}
    for name, (ms, cnt) in stages.items():
        avg = ms / cnt
        entry = {"avg_ms": round(avg, 5), "launches": cnt}
        if name in sb:
            entry["alg_bytes"] = sb[name]
            entry["alg_GBps"] = round(sb[name] / (avg * 1e-3) / 1e9, 1)
        per_stage[name] = entry
    dom = max((k for k in per_stage if k in sb), key=lambda k: stages[k][0])
    dom_avg_ms = stages[dom][0] / stages[dom][1]
    achieved = sb[dom] / (dom_avg_ms * 1e-3) / 1e9
    agent_stage_names = ("col_inv", "row_grad", "col_fwd", "gamma", "row_update", "resid_update", "diag_after")
    agent_ms = sum(stages[k][0] for k in agent_stage_names if k in stages) / args.steps
    agent_min = agent_bytes_min(spec.nx, spec.ny, spec.nz, spec.looks, info["P"])

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
                   "sigma2": args.sigma2, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "iters_per_s": args.steps / elapsed,
        "fwd_agent": {"ms": round(agent_ms, 4), "voxel_looks_per_s": units / (agent_ms * 1e-3),
                      "GBps_vs_min_bytes": round(agent_min / (agent_ms * 1e-3) / 1e9, 1),
                      "min_bytes": agent_min},
        "stages": per_stage,
        "conv_err": conv,
        "nrmse": nrmse,
        "fault": fault,
    }
    if not args.no_cpu_baseline:
        log("timing the float64 oracle on a sample")
        result["cpu_baseline"] = cpu_baseline(spec, y, g, args.sigma2)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
