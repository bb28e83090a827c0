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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="full")
    ap.add_argument("--sigma2", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy MIB mebibytes once with a plain device copy, as a "
                         "known-size reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

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
