"""Throughput benchmark of the fused thread-safe LB + Allen-Cahn step.

One step = one pass of the whole fused update over every node of the
workload.  Prints ONE JSON line:
  value        MLUPS (million lattice updates per second) of the headline
               precision, wall clock over K steps with inputs resident in HBM
  roofline     achieved HBM GB/s of the fused kernel from its algorithmic bytes
               (11 state fields read + 11 written per node) over the kernel
               time measured with HIP events on the library's stream
  cpu_baseline the FP64 CPU oracle timed on this host on a bounded sample
  modes        the same figures for every storage precision that was run

Workloads (seeded, synthetic; lattice units):
  C1  static droplet 32^3, periodic
  C2  rising bubble 128 x 128 x 256, no-slip walls on all faces (default)
  C3  binary droplet collision 256^3, periodic
  C4  ensemble of 64 periodic boxes with edges in [24, 96]
  C5  drop falling into a pool 512^3, walls on +-z
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PAPER_CONTEXT = {"glups": 1.49, "hardware": "1x NVIDIA A100 64GB", "workload": "512^3 two-phase, water-air",
                 "precision": "not stated"}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16_os": "f32 (fp16 offset-scale storage)",
         "bf16_os": "f32 (bf16 offset-scale storage)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_cases(config):
    from paper_2501_00846_amd import workloads as WL

    if config == "C1":
        return [WL.static_droplet()], "static droplet 32^3 periodic, rho ratio 1000, mu ratio 100"
    if config == "C2":
        return [WL.rising_bubble()], ("rising bubble 128x128x256, no-slip walls all faces, rho ratio 1000, "
                                      "mu ratio 100, Eo 10, Mo 1e-3")
    if config == "C3":
        return [WL.droplet_collision()], "binary droplet collision 256^3 periodic, rho ratio 800, mu ratio 50"
    if config == "C4":
        return WL.ensemble(64), "ensemble of 64 periodic droplet boxes, edges in [24, 96]"
    if config == "C5":
        return [WL.drop_into_pool()], "drop into pool 512^3, walls on +-z, rho ratio 1000, mu ratio 100"
    raise SystemExit("unknown config " + config)


def kernel_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2501_00846_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config, precision, nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get("%s/%s" % (config, precision))
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent["bytes_per_launch"]


def run_mode(cases, precision, steps, warmup, tune, unbatched=False):
    import torch

    from paper_2501_00846_amd import lbm

    ctx = lbm.Context([c.problem for c in cases], precision)
    for i, c in enumerate(cases):
        ctx.init_case(i, c)
    if tune:
        ctx.autotune(steps=max(4, min(20, steps // 10)))
    step = ctx.step_unbatched if unbatched else ctx.step
    step(warmup)
    ctx.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(ctx.stream)
    step(steps)
    e1.record(ctx.stream)
    ctx.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = e0.elapsed_time(e1) / steps
    nodes = ctx.total_nodes
    bpl = ctx.bytes_per_update
    diag = ctx.diagnostics(0)
    tuning = ctx.tuning()
    ctx.close()
    mlups = nodes * steps / wall / 1e6
    achieved = nodes * bpl / (kern_ms * 1e-3) / 1e9
    return dict(mlups=mlups, ms_per_step=wall / steps * 1e3, kernel_ms=kern_ms, nodes=nodes,
                bytes_per_update=bpl, achieved_gbs=achieved, frac=achieved / PEAK_HBM_GBS,
                tuning=tuning, phase_mass=diag["phase_mass"], nonfinite=diag["nonfinite"])


def cpu_baseline(config):
    """FP64 oracle on a bounded sample of the workload, timed on this host."""
    from oracle import scheme as S
    from paper_2501_00846_amd import workloads as WL

    if config in ("C2",):
        case = WL.rising_bubble(nz=64, zc=48.0)
        sample = "rising-bubble configuration restricted to 128x128x64 (bottom quarter, bubble included), 2 steps"
        nsteps = 2
    elif config == "C1":
        case = WL.static_droplet()
        sample = "static droplet 32^3, 50 steps"
        nsteps = 50
    elif config == "C4":
        case = WL.ensemble_box(0)
        sample = "ensemble box 0 (%dx%dx%d), 10 steps" % (case.problem.nx, case.problem.ny, case.problem.nz)
        nsteps = 10
    else:
        n = 96
        if config == "C3":
            case = WL.droplet_collision(n=n, radius=24.0 * n / 256)
        else:
            case = WL.drop_into_pool(n=n)
        sample = "%s configuration scaled to %d^3, 2 steps" % (config, n)
        nsteps = 2
    st = S.initial_state(case.phi, case.u, case.pstar)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        st = S.step(st, case.problem)
    dt = time.perf_counter() - t0
    return {"value": case.problem.n_nodes * nsteps / dt / 1e6, "unit": "MLUPS", "cores": 1,
            "kind": "oracle", "sample": sample, "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--config", default="C2", choices=["C1", "C2", "C3", "C4", "C5"])
    ap.add_argument("--precision", default=None,
                    help="comma list of fp64,fp32,fp16_os,bf16_os (default depends on config)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--unbatched", action="store_true", help="C4: one launch per box per step")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only (the path is a single-GPU kernel; multi-GPU slab "
              "decomposition is not built): --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    defaults = {"C1": "fp64", "C2": "fp64,fp32", "C3": "fp32,fp16_os,bf16_os", "C4": "fp32",
                "C5": "fp32,fp16_os,fp64"}
    precisions = (args.precision or defaults[args.config]).split(",")
    log("bench: building cases for %s" % args.config)
    cases, desc = make_cases(args.config)
    modes = {}
    for prec in precisions:
        log("bench: %s %s: %d warmup + %d timed steps" % (args.config, prec, args.warmup, args.steps))
        modes[prec] = run_mode(cases, prec, args.steps, args.warmup, not args.no_tune, args.unbatched)
        log("bench: %s %s: %.0f MLUPS, kernel %.3f ms/step, %.0f GB/s (%.1f%% of HBM peak)" % (
            args.config, prec, modes[prec]["mlups"], modes[prec]["kernel_ms"], modes[prec]["achieved_gbs"],
            100 * modes[prec]["frac"]))
    head = precisions[0]
    m = modes[head]
    traffic = measured_traffic(args.config, head, m["nodes"])
    roof = {"bound": "hbm", "achieved": round(m["achieved_gbs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(m["frac"], 4), "traffic": traffic,
            "kernel": "fused_step (%s)" % head, "bytes_per_update": m["bytes_per_update"],
            "nodes_per_launch": m["nodes"]}
    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.config)
    out = {
        "metric": "MLUPS (million lattice updates per second) of the fused thread-safe LB + Allen-Cahn step",
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic (seeded initial droplet/bubble fields)",
        "config": {"workload": desc, "config": args.config, "nodes": m["nodes"], "precision": head,
                   "tuning": m["tuning"], "steps_per_launch": 1},
        "roofline": roof,
        "cpu_baseline": cpu,
        "modes": {p: {"mlups": round(v["mlups"], 1), "kernel_ms": round(v["kernel_ms"], 4),
                      "achieved_gbs": round(v["achieved_gbs"], 1), "frac": round(v["frac"], 4),
                      "bytes_per_update": v["bytes_per_update"], "tuning": v["tuning"],
                      "nonfinite": v["nonfinite"]} for p, v in modes.items()},
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
