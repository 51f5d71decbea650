"""Throughput of the coupled flow + thermal lattice Boltzmann step on one GPU.

One "step" is one whole coupled time step (pull-streaming, moments, EOS and
psi, force, velocity, thermal source, both MRT collisions, store) over every
node of the workload, i.e. one launch of the fused step kernel.  The headline
workload is the 4096 x 4096 periodic spinodal case in FP64 (seeded synthetic
input, the HBM-bound configuration); the reduced-precision storage forms of
the same workload are reported under "variants".

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS (coupled flow+thermal) and % HBM roofline, FP64 vs "
          "reduced-precision/batched")
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per lattice update: 9 f + 9 g read and written, plus the
# phi history read and written (storage bytes / phi bytes per precision)
BYTES_PER_LUP = {0: 36 * 8 + 2 * 8, 1: 36 * 4 + 2 * 4, 2: 36 * 4 + 2 * 4,
                 3: 36 * 2 + 2 * 4}
PREC_NAME = {0: "FP64", 1: "FP32", 2: "FP32_SHIFTED", 3: "FP16_SHIFTED"}
PREC_DTYPE = {0: "f64", 1: "f32", 2: "f32", 3: "f16-storage/f32"}


def gpu_run(n, prec, steps, warmup, per_launch=40, model=0):
    import torch
    from paper_1709_04400_amd import inputs, lbpc
    cfg, fl = inputs.spinodal(n, precision=prec)
    cfg["thermal_model"] = model
    sim = lbpc.Simulation(cfg)
    sim.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    del fl
    stream = sim.stream
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    # average duration of one step-kernel launch: an event pair around each
    # launch, on the stream the library launches on
    evs = [(torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(per_launch)]
    for a, b in evs:
        a.record(stream)
        sim.step(1)
        b.record(stream)
    torch.cuda.synchronize()
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / per_launch
    d = sim.diag()
    sim.close()
    if d["nonfinite"]:
        raise RuntimeError("non-finite state in the benchmark run")
    return ms_total / steps, kern_ms, cfg


def batch_run(count, steps, warmup, tiles=None):
    """The batched sweep: `count` heated-wall droplets of sizes drawn from
    {64, 96, ..., 512}, FP32 storage, one persistent launch per step,
    autotuned tiles.  With `tiles` (the autotuner's earlier pick) the steady
    steps are replayed from a captured hipGraph instead."""
    import torch
    from paper_1709_04400_amd import inputs, lbpc
    cases = inputs.batch_cases(count=count, seed=1709,
                               precision=inputs.FP32)
    # the graph switch is read when the batch is created
    old = os.environ.get("LBPC_BATCH_GRAPH")
    os.environ["LBPC_BATCH_GRAPH"] = "1" if tiles else "0"
    try:
        b = lbpc.Batch([c for c, _ in cases])
    finally:
        if old is None:
            os.environ.pop("LBPC_BATCH_GRAPH")
        else:
            os.environ["LBPC_BATCH_GRAPH"] = old
    for k, (_, f) in enumerate(cases):
        b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    del cases
    stream = b.stream
    b.step(warmup)
    if tiles:
        b.set_tiles(tiles["block_width"], tiles["rows"])
        tune = dict(tiles)
    else:
        tune = b.autotune(steps=3)   # steady-state timings, state unchanged
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nodes = b.nodes()
    bad = sum(b.diag(k)["nonfinite"] for k in range(0, count, 17))
    b.close()
    if bad:
        raise RuntimeError("non-finite state in the batched run")
    return ms, nodes, tune


def cpu_baseline(n_sample=512, steps=150):
    """The FP64 oracle, single thread, on a crop of the same recipe."""
    import oracle
    from paper_1709_04400_amd import inputs
    cfg, fl = inputs.spinodal(n_sample)
    o = oracle.Oracle(cfg)
    o.init_fields(**fl)
    o.step(2)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": n_sample * n_sample * steps / dt / 1e6, "unit": "MLUPS",
            "cores": 1, "kind": "oracle",
            "sample": f"spinodal recipe (seed 4400) on a {n_sample}x{n_sample} "
                      f"periodic lattice, {steps} steps, single thread, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--variants", type=int, default=1,
                    help="also time the reduced-precision storage forms")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256,
                    help="lattices in the batched sweep (0: skip it)")
    ap.add_argument("--per-launch", type=int, default=40)
    ap.add_argument("--traffic-file", default=os.path.join(
        ROOT, "profiles", "traffic_k_step_fp64_spinodal4096.md"))
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        copy_calibration(args.calibrate_copy_mib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no "
              "multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    ms, kern_ms, cfg = gpu_run(args.n, 0, args.steps, args.warmup,
                               args.per_launch)
    nodes = args.n * args.n
    mlups = nodes / ms / 1e3
    alg_bytes = BYTES_PER_LUP[0] * nodes
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = read_traffic(args.traffic_file, args.n)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded spinodal recipe; the paper uses no "
                "dataset)",
        "config": {"workload": f"spinodal {args.n}x{args.n} periodic D2Q9, "
                               "T = 0.86 Tc, rho and T with seeded uniform "
                               "noise, FP64 storage and arithmetic",
                   "nx": args.n, "ny": args.n, "precision": "FP64",
                   "kernel": "k_step<0,false> (fused, one launch per step)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel_avg_ms": round(kern_ms, 5),
                     "alg_bytes_per_launch": alg_bytes},
    }
    if args.variants:
        var = {}
        for prec in (1, 2, 3):
            vms, vk, _ = gpu_run(args.n, prec, max(args.steps // 4, 50),
                                 args.warmup)
            vb = BYTES_PER_LUP[prec] * nodes / (vk * 1e-3) / 1e9
            var[PREC_NAME[prec]] = {
                "MLUPS": round(nodes / vms / 1e3, 1),
                "ms_per_step": round(vms, 5), "dtype": PREC_DTYPE[prec],
                "alg_GBs": round(vb, 1),
                "frac": round(vb / HBM_PEAK_GBS, 4),
                "bytes_per_lup": BYTES_PER_LUP[prec]}
        # the other thermal models on the same workload (FP64): the
        # Gong-Cheng BGK collision, and the BGK form of the improved model,
        # which also reads and writes T v of the previous step
        for model, name, bpl in ((2, "GONG_CHENG_FP64", BYTES_PER_LUP[0]),
                                 (3, "IMPROVED_BGK_FP64",
                                  BYTES_PER_LUP[0] + 4 * 8)):
            try:
                vms, vk, _ = gpu_run(args.n, 0, max(args.steps // 8, 50),
                                     args.warmup, model=model)
            except RuntimeError as e:
                var[name] = {"error": str(e)}
                continue
            vb = bpl * nodes / (vk * 1e-3) / 1e9
            var[name] = {
                "MLUPS": round(nodes / vms / 1e3, 1),
                "ms_per_step": round(vms, 5), "dtype": "f64",
                "alg_GBs": round(vb, 1), "frac": round(vb / HBM_PEAK_GBS, 4),
                "bytes_per_lup": bpl}
        out["variants"] = var
    if args.batch:
        bsteps = max(args.steps // 10, 50)
        bms, bnodes, tune = batch_run(args.batch, bsteps, args.warmup)
        bb = BYTES_PER_LUP[1] * bnodes / (bms * 1e-3) / 1e9
        out.setdefault("variants", {})["BATCHED_FP32"] = {
            "MLUPS": round(bnodes / bms / 1e3, 1), "ms_per_step": round(bms, 5),
            "dtype": "f32", "lattices": args.batch, "nodes": bnodes,
            "steps": bsteps, "alg_GBs": round(bb, 1),
            "frac": round(bb / HBM_PEAK_GBS, 4), "tiles": tune,
            "workload": "heated-wall droplets, sizes U{64..512 step 32}, "
                        "R = 0.2 N, T_w ~ U[1.02, 1.2] T_sat, seed 1709"}
        gms, gnodes, _ = batch_run(args.batch, bsteps, args.warmup, tune)
        gb = BYTES_PER_LUP[1] * gnodes / (gms * 1e-3) / 1e9
        out["variants"]["BATCHED_FP32_GRAPH"] = {
            "MLUPS": round(gnodes / gms / 1e3, 1),
            "ms_per_step": round(gms, 5), "dtype": "f32",
            "lattices": args.batch, "steps": bsteps,
            "alg_GBs": round(gb, 1), "frac": round(gb / HBM_PEAK_GBS, 4),
            "replay": "hipGraph of one ping-pong period, same tiles"}
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """A plain device-to-device copy of `mib` MiB (read mib, write mib)."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "copies": 3}), flush=True)


def read_traffic(path, n):
    """HBM bytes per step launch from the committed counter summary, used
    only while the kernel source and the host code that picks its tile
    shape are the ones the counters were taken on."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    try:
        if int(vals.get("n", -1)) != n or \
                vals.get("kernel_source_hash") != _kernel_hash():
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("lbpc_step.hip", "lbpc_device.h", "lbpc_host.h"):
        with open(os.path.join(ROOT, "paper_1709_04400_amd", "csrc",
                               name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
