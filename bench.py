"""Throughput benchmark of the fused thread-safe LB + Allen-Cahn step.

One step = one pass of the whole fused update over every node of the
workload.  Prints ONE JSON line:
  value        MLUPS (million lattice updates per second) of the headline
               precision (the first of --precision), wall clock over K steps
               with inputs resident in HBM
  roofline     achieved HBM GB/s of the fused kernel from its algorithmic bytes
               (11 state fields read + 11 written per node) over the kernel
               time measured with HIP events on the library's stream, and the
               vector-ALU ceiling beside it (committed SQ_INSTS_VALU count
               over the issue rate of the 256 CUs)
  cpu_baseline the FP64 CPU oracle timed on this host on a bounded sample
  modes        the same figures for every storage precision that was run,
               each with its per-field error against the FP64 run of the same
               step count (phi, rho, u, p; relative L2 and max norms)

Workloads (seeded, synthetic; lattice units):
  C1  static droplet 32^3, periodic
  C2  rising bubble 128 x 128 x 256, no-slip walls on all faces
  C3  binary droplet collision 256^3, periodic
  C4  ensemble of 64 periodic boxes with edges in [24, 96]
  C5  drop falling into a pool 512^3, walls on +-z (default: the largest
      single-domain workload, FP64 headline with FP32 and FP16-os storage)
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
# vector-ALU issue ceiling in wave64 instructions per second: 256 CUs x 4 SIMDs
# at 2.4 GHz, each SIMD (16 lanes) retiring one wave64 instruction per 4
# cycles (FP64 and unpacked FP32 alike; packed FP32 is not used)
CUS, SIMDS, CLOCK_HZ = 256, 4, 2.4e9
VALU_ISSUE_PER_S = CUS * SIMDS * CLOCK_HZ / 4.0
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
    if config == "raindrop":
        return [WL.raindrop_train(dtype=np.float32)], ("train of 5 drops onto a substrate, 500x500x3000, walls on "
                                                       "+-z, We 40, rho ratio 1000, mu ratio 100")
    if config == "eoga":
        return WL.eo_ga_sweep(), ("Eo-Ga rising-bubble sweep: 12 periodic 200x200x400 boxes in one launch, "
                                  "rho ratio 1000, mu ratio 100")
    raise SystemExit("unknown config " + config)


def kernel_hash():
    """Hash of the sources the fused step is compiled from (its kernel, the
    device helpers it shares, the state layout it reads), which keys the
    committed counter summaries."""
    h = hashlib.sha256()
    for f in ("fused_step.hip", "device_common.h", "state_layout.h"):
        with open(os.path.join(ROOT, "paper_2501_00846_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(config, precision, tuning, path=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source at the same tile shape and z-chunk;
    else None."""
    path = path or TRAFFIC_JSON
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    launch = [tuning[k] for k in ("block_x", "block_y", "z_chunk")]
    ent = data.get(traffic_key(config, precision, launch))
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent["bytes_per_launch"]


def traffic_key(config, precision, launch):
    """Entry name in profiles/traffic.json: workload, closure and precision
    (config is e.g. "C2" or "C5/gc"), then tile shape and z-chunk."""
    return "%s/%s@%s" % (config, precision, ",".join(str(v) for v in launch[:3]))


def copy_bandwidth(nbytes=1 << 31, reps=10):
    """Device-to-device copy rate (GB/s, bytes read + written) of torch's copy
    kernel on the current stream: the attainable-bandwidth reference beside the
    8 TB/s specification."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


VALU_JSON = os.path.join(ROOT, "profiles", "valu.json")


def wave_planes(problems, tuning):
    """Wave64-planes one launch of the fused step executes: every item (a tile
    of (block_x - 2) x (block_y - 2) output columns over z_chunk output planes)
    marches its output planes plus one staging plane on each side that is not
    a z wall, with ceil(block_x * block_y / 64) wavefronts.  Mirrors the tile
    list of the runtime and the plane loop of the kernel."""
    bx, by, zc0 = (int(tuning[k]) for k in ("block_x", "block_y", "z_chunk"))
    tx, ty = bx - 2, by - 2
    waves = -(-bx * by // 64)
    total = 0
    for p in problems:
        wz = p.bc[2] == 1
        zc = max(1, min(zc0, p.nz))
        cols = -(-p.nx // tx) * -(-p.ny // ty)
        planes = 0
        for z0 in range(0, p.nz, zc):
            z1 = min(z0 + zc, p.nz)
            first = 0 if (wz and z0 == 0) else z0 - 1
            last = p.nz - 1 if (wz and z1 == p.nz) else z1
            planes += last - first + 1
        total += cols * planes * waves
    return total


def valu_key(config, precision, tuning):
    """Entry name in profiles/valu.json: workload (with "/gc" for the gradient
    closure), precision and tile shape."""
    return "%s/%s@%d,%d" % (config, precision, int(tuning["block_x"]), int(tuning["block_y"]))


def valu_per_launch(config, precision, problems, tuning, path=None):
    """Vector-ALU wave instructions of one launch: the committed SQ_INSTS_VALU
    count per wave-plane (same kernel source and tile shape) times the
    wave-planes of this launch; None when no such count is committed."""
    path = path or VALU_JSON
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(valu_key(config, precision, tuning))
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent["valu_per_wave_plane"] * wave_planes(problems, tuning)


def alu_ceiling(valu, nodes, kernel_ms):
    """The vector-ALU floor of a launch of `valu` wave instructions at the
    issue rate VALU_ISSUE_PER_S, as time, MLUPS and the fraction of the
    measured kernel time it accounts for."""
    if valu is None:
        return None
    floor_ms = valu / VALU_ISSUE_PER_S * 1e3
    return {"valu_per_launch": int(round(valu)), "valu_per_update": round(valu * 64 / nodes, 1),
            "issue_peak_ginst_s": round(VALU_ISSUE_PER_S / 1e9, 1), "floor_ms": round(floor_ms, 4),
            "ceiling_mlups": round(nodes / (floor_ms * 1e-3) / 1e6, 1),
            "achieved_ginst_s": round(valu / (kernel_ms * 1e-3) / 1e9, 1),
            "frac": round(floor_ms / kernel_ms, 4)}


def run_mode(cases, precision, steps, warmup, tune, unbatched=False, tuning=None, fields=False):
    """Autotune (or take `tuning`), restart from the initial fields, run
    `warmup` steps, time `steps` steps.  The state after the timed region is
    therefore warmup + steps steps from the initial fields in every mode, and
    with fields=True the observables of box 0 are returned for the error
    against the FP64 run."""
    import torch

    from paper_2501_00846_amd import lbm

    ctx = lbm.Context([c.problem for c in cases], precision)
    for i, c in enumerate(cases):
        ctx.init_case(i, c)
    if tuning is not None:
        ctx.set_tuning(*tuning)
    elif tune:
        ctx.autotune(steps=max(4, min(20, steps // 10)))
        # the tuner advanced the state: restart from the initial fields
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
    step = ctx.step_unbatched if unbatched else ctx.step
    step(warmup)
    ctx.synchronize()
    # the timed steps run as five consecutive segments with HIP events on the
    # library's stream between them (no synchronisation inside the region):
    # the per-step kernel time is the whole region's, and the five segment
    # times give its median and spread
    nseg = 5 if steps >= 5 else 1
    bounds = [steps * i // nseg for i in range(nseg + 1)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nseg + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(ctx.stream)
    for i in range(nseg):
        step(bounds[i + 1] - bounds[i])
        ev[i + 1].record(ctx.stream)
    ctx.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = ev[0].elapsed_time(ev[nseg]) / steps
    seg_ms = [ev[i].elapsed_time(ev[i + 1]) / (bounds[i + 1] - bounds[i]) for i in range(nseg)]
    nodes = ctx.total_nodes
    bpl = ctx.bytes_per_update
    if getattr(cases[0].problem, "fine_phase", False):
        # the fine phase field is state too: 8 fine nodes read and written per update
        bpl += 16 * (8 if precision == "fp64" else 4)
    diag = ctx.diagnostics(0)
    # cost of the FP64 reductions of every box (one launch, synchronised):
    # best of three calls
    diag_ms = []
    for _ in range(3):
        t1 = time.perf_counter()
        ctx.diagnostics_all()
        diag_ms.append((time.perf_counter() - t1) * 1e3)
    tuning = ctx.tuning()
    obs = ctx.fields(0) if fields else None
    ctx.close()
    mlups = nodes * steps / wall / 1e6
    achieved = nodes * bpl / (kern_ms * 1e-3) / 1e9
    return dict(mlups=mlups, ms_per_step=wall / steps * 1e3, kernel_ms=kern_ms,
                kernel_ms_segments=[round(v, 5) for v in seg_ms],
                kernel_ms_median=float(np.median(seg_ms)), nodes=nodes,
                bytes_per_update=bpl, achieved_gbs=achieved, frac=achieved / PEAK_HBM_GBS,
                tuning=tuning, phase_mass=diag["phase_mass"], nonfinite=diag["nonfinite"],
                diagnostics_ms=min(diag_ms), fields=obs)


def field_errors(got, ref):
    """Per-field error of a run against the FP64 run of the same step count:
    relative L2 and max norms of phi, rho, u_x, u_y, u_z and p."""
    out = {}
    for name in ("phi", "rho", "p"):
        out[name] = _rel(got[name], ref[name])
    for c, cn in enumerate("xyz"):
        out["u" + cn] = _rel(got["u"][c], ref["u"][c])
    return {k: {kk: float("%.3g" % vv) for kk, vv in v.items()} for k, v in out.items()}


def cpu_baseline(config):
    """FP64 oracle on a bounded sample of the workload, timed on this host."""
    from oracle import scheme as S
    from paper_2501_00846_amd import workloads as WL

    if config in ("C2",):
        case = WL.rising_bubble(nz=64, zc=48.0)
        sample = "rising-bubble configuration restricted to 128x128x64 (bottom quarter, bubble included), 4 steps"
        nsteps = 4
    elif config == "C1":
        case = WL.static_droplet()
        sample = "static droplet 32^3, 50 steps"
        nsteps = 50
    elif config == "C4":
        case = WL.ensemble_box(0)
        sample = "ensemble box 0 (%dx%dx%d), 10 steps" % (case.problem.nx, case.problem.ny, case.problem.nz)
        nsteps = 10
    elif config == "raindrop":
        case = WL.raindrop_train(nx=64, ny=64, nz=240, radius=8.0)
        sample = "raindrop train scaled to 64x64x240 (R 8), 4 steps"
        nsteps = 4
    elif config == "eoga":
        case = WL.eo_ga_bubble(30.0, 100.0, nx=64, ny=64, nz=128, radius=16.0)
        sample = "one Eo-Ga bubble (Eo 30, Ga 100) scaled to 64x64x128 (R 16), 8 steps"
        nsteps = 8
    else:
        n = 96
        if config == "C3":
            case = WL.droplet_collision(n=n, radius=24.0 * n / 256)
        else:
            case = WL.drop_into_pool(n=n)
        nsteps = 4  # about 12 s of one core
        sample = "%s configuration scaled to %d^3, %d steps" % (config, n, nsteps)
    from threadpoolctl import threadpool_limits

    st = S.initial_state(case.phi, case.u, case.pstar)
    # the oracle is NumPy elementwise code; any native thread pool it could
    # reach (BLAS, OpenMP) is held to one thread, so the figure is one core's
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(nsteps):
            st = S.step(st, case.problem)
        dt = time.perf_counter() - t0
    return {"value": case.problem.n_nodes * nsteps / dt / 1e6, "unit": "MLUPS", "cores": 1,
            "kind": "oracle", "sample": sample, "seconds": round(dt, 2)}


def _fields_and_diag(case, precision, steps, every=None):
    """Run `steps` steps with diagnostics every `every` steps.  Returns
    (fields, trace, failed_at): fields None and failed_at the step count of
    the first non-finite diagnostics if the run lost stability."""
    from paper_2501_00846_amd import lbm

    ctx = lbm.Context(case.problem, precision)
    ctx.init_case(0, case)
    trace = []
    done = 0
    every = every or steps
    try:
        while done < steps:
            k = min(every, steps - done)
            ctx.step(k)
            done += k
            trace.append((done, ctx.diagnostics(0)))
        f = ctx.fields(0)
    except lbm.LbmError:
        ctx.close()
        return None, trace, done
    ctx.close()
    return f, trace, None


def _rel(a, b):
    return {"l2": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
            "max": float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))}


def precision_study(args):
    """Per-field error of each reduced-precision storage mode against the FP64
    run of the same GPU path (itself pinned to the oracle), at the lengths the
    workloads are defined with: relative L2 and max norms of phi, rho, u, p;
    the Laplace pressure jump of the static droplet (500 steps); the rising
    bubble's centre-of-mass velocity over 20,000 steps and its terminal value
    (mean over the last 2,000 steps); the 256^3 collision after 5,000 steps."""
    from paper_2501_00846_amd import workloads as WL

    modes = ["fp32", "fp16_os", "bf16_os"]
    studies = {
        "C1": (WL.static_droplet(), 500, 50, "laplace"),
        "C2": (WL.rising_bubble(), 20000, 500, "ucom"),
        "C3": (WL.droplet_collision(), 5000, 500, None),
    }
    if args.closure == "gradient":
        # every mode, FP64 included, runs the gradient closure
        for case, _, _, _ in studies.values():
            case.problem.gradient_closure = True
    out = {"closure": args.closure}
    for name, (case, steps, every, extra) in studies.items():
        log("precision study %s: %d steps" % (name, steps))
        ref, rtrace, rfail = _fields_and_diag(case, "fp64", steps, every)
        res = {"steps": steps, "workload": case.name}
        if rfail is not None:
            res["fp64"] = {"nonfinite_at_step": rfail}
            out[name] = res
            continue
        ur = np.array([t[1]["velocity_g"][2] for t in rtrace]) if extra == "ucom" else None
        for m in modes:
            got, gtrace, gfail = _fields_and_diag(case, m, steps, every)
            if gfail is not None:
                res[m] = {"nonfinite_at_step": gfail}
                log("  %s: non-finite by step %d" % (m, gfail))
                continue
            errs = {}
            for fld in ("phi", "rho", "p"):
                errs[fld] = _rel(got[fld], ref[fld])
            for c, cn in enumerate("xyz"):
                errs["u" + cn] = _rel(got["u"][c], ref["u"][c])
            if extra == "laplace":
                dr = rtrace[-1][1]["p_l"] - rtrace[-1][1]["p_g"]
                dg = gtrace[-1][1]["p_l"] - gtrace[-1][1]["p_g"]
                errs["laplace_dp"] = {"fp64": dr, "mode": dg, "rel": abs(dg - dr) / abs(dr),
                                      "vs_2sigma_over_R": dr / (2 * case.problem.sigma / 8.0)}
            if extra == "ucom":
                ug = np.array([t[1]["velocity_g"][2] for t in gtrace])
                tail = max(1, len(ur) // 10)
                term_r, term_g = float(ur[-tail:].mean()), float(ug[-tail:].mean())
                errs["u_com"] = {"fp64_terminal": term_r, "mode_terminal": term_g,
                                 "terminal_rel": abs(term_g - term_r) / abs(term_r),
                                 "rel_max_over_time": float(np.abs(ug - ur).max() / np.abs(ur).max()),
                                 "fp64_trace": [float(v) for v in ur]}
            errs["phase_mass_drift"] = float((gtrace[-1][1]["phase_mass"] - rtrace[-1][1]["phase_mass"])
                                             / rtrace[-1][1]["phase_mass"])
            res[m] = errs
            log("  %s: phi %.2e rho %.2e uz %.2e p %.2e (rel L2)" % (
                m, errs["phi"]["l2"], errs["rho"]["l2"], errs["uz"]["l2"], errs["p"]["l2"]))
        out[name] = res
    print(json.dumps({"precision_study": out}), flush=True)


COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written
# the calibration copy's kernel name; the run also launches torch's fill kernel
# (torch.ones: nothing read, 1 GiB written), which must not enter the average
COPY_KERNEL = "MulFunctor"


def copy_calibration(reps):
    """A plain device copy of known size (torch's copy kernel), for scaling the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch

    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)  # one elementwise kernel: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    log("bench: copy calibration: %d copies of %d bytes" % (reps, COPY_BYTES))


def _read_counter_csv(path, counter, name_part):
    """Mean per-dispatch value (KiB as reported) of `counter` over dispatches whose
    kernel name contains name_part, from a rocprofv3 counter_collection.csv."""
    import csv

    vals = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter or name_part not in row.get("Kernel_Name", ""):
                continue
            key = row.get("Dispatch_Id") or row.get("Correlation_Id")
            vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
    if not vals:
        raise SystemExit("no %s rows for %s in %s" % (counter, name_part, path))
    return sum(vals.values()) / len(vals)


def summarize_counters(args):
    """Turn four rocprofv3 --pmc runs (fused step FETCH_SIZE and WRITE_SIZE,
    copy kernel FETCH_SIZE and WRITE_SIZE) into profiles/traffic.json."""
    fetch = _read_counter_csv(args.fetch_csv, "FETCH_SIZE", "fused_step")
    write = _read_counter_csv(args.write_csv, "WRITE_SIZE", "fused_step")
    cf = _read_counter_csv(args.copy_fetch_csv, "FETCH_SIZE", args.copy_kernel)
    cw = _read_counter_csv(args.copy_write_csv, "WRITE_SIZE", args.copy_kernel)
    f_fetch = COPY_BYTES / (cf * 1024.0)
    f_write = COPY_BYTES / (cw * 1024.0)
    traffic = fetch * 1024.0 * f_fetch + write * 1024.0 * f_write
    path = getattr(args, "traffic_json", None) or TRAFFIC_JSON
    data = json.load(open(path)) if os.path.exists(path) else {}
    cases, _ = make_cases(args.config)
    nodes = sum(c.problem.n_nodes for c in cases)
    prec = args.precision.split(",")[0]
    gc = args.closure == "gradient"
    # algorithmic bytes per update: phi + moment fields, read and written
    bpl = 2 * ({"fp64": 8, "fp32": 4}.get(prec, 4) + (4 if gc else 10) * {"fp64": 8, "fp32": 4}.get(prec, 2))
    tuning = [int(v) for v in args.tuning.split(",")] if args.tuning else None
    if tuning is None:
        raise SystemExit("--summarize-counters needs the --tuning the counters were taken with")
    key = traffic_key(args.config + ("/gc" if gc else ""), prec, tuning)
    data[key] = {
        "kernel_hash": kernel_hash(), "tuning": tuning,
        "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
        "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": f_fetch, "write_scale": f_write,
        "bytes_per_launch": traffic, "nodes": nodes, "bytes_per_update_measured": traffic / nodes,
        "bytes_per_update_algorithmic": bpl}
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps(data[key]))


def summarize_valu(args):
    """SQ_INSTS_VALU of the fused step from a rocprofv3 --pmc run into
    profiles/valu.json, as wave instructions per wave-plane of the launch the
    counters were taken with (--tuning)."""
    valu = _read_counter_csv(args.valu_csv, "SQ_INSTS_VALU", "fused_step")
    if not args.tuning:
        raise SystemExit("--summarize-valu needs the --tuning the counters were taken with")
    t = [int(v) for v in args.tuning.split(",")]
    tuning = {"block_x": t[0], "block_y": t[1], "z_chunk": t[2]}
    cases, _ = make_cases(args.config)
    gc = args.closure == "gradient"
    planes = wave_planes([c.problem for c in cases], tuning)
    prec = args.precision.split(",")[0]
    key = valu_key(args.config + ("/gc" if gc else ""), prec, tuning)
    path = getattr(args, "valu_json", None) or VALU_JSON
    data = json.load(open(path)) if os.path.exists(path) else {}
    nodes = sum(c.problem.n_nodes for c in cases)
    data[key] = {"kernel_hash": kernel_hash(), "tuning": t[:3], "valu_per_dispatch": valu,
                 "wave_planes": planes, "valu_per_wave_plane": valu / planes,
                 "valu_per_update": valu * 64 / nodes}
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps(data[key]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own run length, 400 for the second workloads)")
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--config", default="C5", choices=["C1", "C2", "C3", "C4", "C5", "raindrop", "eoga"])
    ap.add_argument("--precision", default=None,
                    help="comma list of fp64,fp32,fp16_os,bf16_os (default depends on config; the first "
                         "is the headline)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true",
                    help="skip the per-field error against the FP64 run")
    ap.add_argument("--unbatched", action="store_true", help="C4: one launch per box per step")
    ap.add_argument("--precision-study", action="store_true",
                    help="per-field errors of the reduced-precision modes against FP64")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="REPS",
                    help="only run REPS plain 1 GiB device copies (counter calibration)")
    ap.add_argument("--summarize-counters", action="store_true",
                    help="write profiles/traffic.json from rocprofv3 counter CSVs")
    ap.add_argument("--summarize-valu", action="store_true",
                    help="write profiles/valu.json from a rocprofv3 SQ_INSTS_VALU counter CSV")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--copy-fetch-csv")
    ap.add_argument("--copy-write-csv")
    ap.add_argument("--valu-csv")
    ap.add_argument("--copy-kernel", default=COPY_KERNEL)
    ap.add_argument("--closure", default="moment", choices=["moment", "gradient"],
                    help="a2 from the stored second moment (the paper's algorithm) or from the "
                         "velocity gradient (5-field state)")
    ap.add_argument("--high-order", action="store_true",
                    help="fourth-order phase-field update (the flow solver keeps its stencils)")
    ap.add_argument("--fine-phase", action="store_true",
                    help="phase field on a grid refined by 2 per axis (the flow solver reads its restriction)")
    ap.add_argument("--tuning", default=None, metavar="BX,BY,ZCHUNK,PERSISTENT",
                    help="fixed launch configuration instead of autotuning")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.precision_study:
        precision_study(args)
        return
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.summarize_valu:
        summarize_valu(args)
        return

    if args.gpus != 1:
        print("bench.py runs on one GPU only (the path is a single-GPU kernel; multi-GPU slab "
              "decomposition is not built): --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    defaults = {"C1": "fp64", "C2": "fp64,fp32", "C3": "fp32,fp16_os,bf16_os", "C4": "fp32",
                "C5": "fp64,fp32,fp16_os", "raindrop": "fp32", "eoga": "fp32"}
    if args.steps is None:
        # each workload is timed over its own run length
        args.steps = {"C1": 500, "C2": 20000, "C3": 5000, "C4": 2000, "C5": 2000}.get(args.config, 400)
    precisions = (args.precision or defaults[args.config]).split(",")
    log("bench: building cases for %s" % args.config)
    cases, desc = make_cases(args.config)
    gc = args.closure == "gradient"
    if gc:
        for c in cases:
            c.problem.gradient_closure = True
        desc += ", gradient closure (state phi, P, J)"
    if args.high_order:
        for c in cases:
            c.problem.high_order_ac = True
        desc += ", fourth-order phase-field update"
    if args.fine_phase:
        if args.high_order:
            raise SystemExit("--fine-phase and --high-order are separate variants")
        for c in cases:
            c.problem.fine_phase = True
        desc += ", phase field on the grid refined by 2"
    cfg_key = args.config + ("/gc" if gc else "") + ("/ho" if args.high_order else "") + \
        ("/fine" if args.fine_phase else "")
    problems = [c.problem for c in cases]
    # per-field error against the FP64 run: only for single-box workloads
    # that run FP64 among their modes
    errors = (not args.no_error and not args.unbatched and "fp64" in precisions and len(cases) == 1
              and len(precisions) > 1)
    order = (["fp64"] + [p for p in precisions if p != "fp64"]) if errors else precisions
    modes = {}
    ref_fields = None
    tuning_arg = tuple(int(v) for v in args.tuning.split(",")) if args.tuning else None
    for prec in order:
        log("bench: %s %s: %d warmup + %d timed steps" % (args.config, prec, args.warmup, args.steps))
        m = run_mode(cases, prec, args.steps, args.warmup, not args.no_tune, args.unbatched, tuning_arg,
                     fields=errors)
        obs = m.pop("fields")
        if errors:
            if prec == "fp64":
                ref_fields = obs
            else:
                m["error_vs_fp64"] = field_errors(obs, ref_fields)
                log("bench: %s error vs fp64 after %d steps: phi %.2e rho %.2e uz %.2e p %.2e (rel L2)" % (
                    prec, args.warmup + args.steps, m["error_vs_fp64"]["phi"]["l2"],
                    m["error_vs_fp64"]["rho"]["l2"], m["error_vs_fp64"]["uz"]["l2"],
                    m["error_vs_fp64"]["p"]["l2"]))
            del obs
        m["alu"] = alu_ceiling(valu_per_launch(cfg_key, prec, problems, m["tuning"]), m["nodes"],
                               m["kernel_ms"])
        modes[prec] = m
        log("bench: %s %s: %.0f MLUPS, kernel %.3f ms/step, %.0f GB/s (%.1f%% of HBM peak)" % (
            args.config, prec, m["mlups"], m["kernel_ms"], m["achieved_gbs"], 100 * m["frac"]))
    ref_fields = None
    if args.config == "C4" and not args.unbatched:
        # the unbatched baseline: one launch per box per step (no graphs)
        prec = precisions[0]
        log("bench: C4 %s unbatched baseline" % prec)
        mu = run_mode(cases, prec, args.steps, args.warmup, False, True,
                      tuple(modes[prec]["tuning"].values()))
        mu.pop("fields")
        modes[prec + "_unbatched"] = mu
        log("bench: C4 unbatched: %.0f MLUPS" % mu["mlups"])
    head = precisions[0]
    m = modes[head]
    traffic = measured_traffic(cfg_key, head, m["tuning"])
    copy_gbs = copy_bandwidth()
    log("bench: device copy %.0f GB/s" % copy_gbs)
    hbm_floor_ms = m["nodes"] * m["bytes_per_update"] / (PEAK_HBM_GBS * 1e9) * 1e3
    alu = m["alu"]
    # the roofline that bounds the kernel: the larger of the HBM floor
    # (algorithmic bytes at 8 TB/s) and the vector-ALU floor
    bound = "alu" if (alu is not None and alu["floor_ms"] > hbm_floor_ms) else "hbm"
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": round(m["achieved_gbs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(m["frac"], 4)}
    else:
        roof = {"bound": "alu", "achieved": alu["achieved_ginst_s"], "peak": alu["issue_peak_ginst_s"],
                "unit": "G VALU wave-instructions/s", "frac": alu["frac"],
                "hbm_achieved_gbs": round(m["achieved_gbs"], 1), "hbm_frac": round(m["frac"], 4)}
    roof.update({"traffic": traffic, "copy_gbs": round(copy_gbs, 1),
                 "frac_of_copy": round(m["achieved_gbs"] / copy_gbs, 4),
                 "hbm_floor_ms": round(hbm_floor_ms, 4), "alu": alu,
                 "kernel": "fused_step (%s)" % head + (" + ho_flux + ho_phase" if args.high_order else "") +
                           (" + ho_flux (u) + fine_step + fine_restrict" if args.fine_phase else ""),
                 "kernel_ms": round(m["kernel_ms"], 4),
                 "bytes_per_update": m["bytes_per_update"], "nodes_per_launch": m["nodes"]})
    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.config)
    out = {
        "metric": "MLUPS (million lattice updates per second) of the fused thread-safe LB + Allen-Cahn step, "
                  "with % of HBM roofline; reduced-precision storage modes with their per-field error vs FP64",
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": None,
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic (seeded initial droplet/bubble fields)",
        "config": {"workload": desc, "config": args.config, "closure": args.closure,
                   "phase_update": ("fourth-order" if args.high_order else
                                    "second-order on the grid refined by 2" if args.fine_phase else "second-order"),
                   "nodes": m["nodes"],
                   "precision": head, "tuning": m["tuning"], "steps_per_launch": 1},
        "roofline": roof,
        "cpu_baseline": cpu,
        "modes": {p: {"mlups": round(v["mlups"], 1), "kernel_ms": round(v["kernel_ms"], 4),
                      "kernel_ms_median_of_5": round(v["kernel_ms_median"], 4),
                      "kernel_ms_segments": v["kernel_ms_segments"],
                      "achieved_gbs": round(v["achieved_gbs"], 1), "frac": round(v["frac"], 4),
                      "bytes_per_update": v["bytes_per_update"], "tuning": v["tuning"],
                      "alu": v.get("alu"), "error_vs_fp64": v.get("error_vs_fp64"),
                      "diagnostics_ms": round(v["diagnostics_ms"], 3),
                      "nonfinite": v["nonfinite"]} for p, v in modes.items()},
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
