#!/usr/bin/env python3
"""Benchmark of the coupled three-lattice lattice Boltzmann step on one MI355X.

Metric: MLUPS (million lattice-node updates per second; one update advances
all three lattices f, g, h), with the achieved fraction of the HBM roofline,
on the sessile-droplet-on-an-adsorbing-solid workload (256 x 128 D2Q9,
half-way bounce-back wetting/adsorbing bottom wall, free-slip top, semicircle
R0 = 40, psi_b = 0.02, theta0 = 60 deg, adsorption strength drawn from seed 2),
FP32 storage with FP64 reductions.  A second, cache-exceeding grid (4096^2
periodic drop, same physics family) is timed to show the HBM-bound regime.

Prints one JSON line.  `value` is the sessile workload's MLUPS.  `roofline`
is taken on the 4096^2 grid, whose 5 GB of state streams from HBM every step
(the sessile grid's 10 MB stay in the on-die caches, so HBM does not bound
it; its kernel figures are under `headline_kernel`).  Beside the published
HBM peak the roofline carries two ceilings measured in the same run: a plain
device copy and the library's bandwidth probe (the step's bytes and access
pattern without its arithmetic).  The batched sweep's step (512 cases of the
sweep distribution) and the surrogate ensemble's inference rate follow.  The
FP64 CPU oracle is timed beside it on the host (bounded sample) as
cpu_baseline.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def gpu_run(cfg, precision, steps, warmup, kernel_steps):
    """Wall-clock run of `steps` steps (graph-replayed, as a user calls
    lbm_step), then `kernel_steps` more with per-kernel HIP-event timing (those
    launch one by one) for the roofline."""
    import torch
    from paper_2609_26332_amd import lbm

    sim = lbm.Sim(cfg, precision)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.timing_begin(kernel_steps)
    sim.step(kernel_steps)
    kt = sim.timing_end()
    inv = sim.invariants(check=False)
    N = cfg["nx"] * cfg["ny"]
    return dict(sim=sim, wall=wall, kernels=kt, N=N, inv=inv, bytes_node=sim.bytes_per_node_step())


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2609_26332_amd", "csrc", "lbm_kernels.hip")


def measured_traffic(key):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's
    readings), or None when that summary was taken on other kernel source."""
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    if not m or m.group(1) != src:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*(.*)", text)
    if not m:
        return None
    vals = dict(kv.split("=") for kv in m.group(1).replace(",", " ").split())
    return float(vals[key]) if key in vals else None


def roofline(res, key, cfg, precision):
    """Achieved HBM bandwidth of the dominant kernel (the fused step kernel,
    which moves all of a step's algorithmic bytes) on those bytes, from its
    HIP-event durations on the stream it runs on.  Beside the published peak,
    `pattern_ceiling` is what the library's bandwidth probe (the same bytes per
    node in the step's access pattern, without the arithmetic) reaches on the
    same grid in the same run."""
    from paper_2609_26332_amd import lbm
    kt = res["kernels"]
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms = kt[dom][0] / max(kt[dom][1], 1)
    bytes_launch = res["bytes_node"] * res["N"]
    achieved = bytes_launch / (dom_ms * 1e-3) / 1e9
    pr = lbm.probe_stream(cfg["nx"], cfg["ny"], precision, reps=20)
    cp = copy_rate()
    return {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(key),
        "kernel": dom, "bytes_per_node_step": res["bytes_node"], "nodes_per_launch": res["N"],
        "kernel_ms_per_launch": {k: round(v[0] / max(v[1], 1), 5) for k, v in kt.items()},
        "copy_ceiling": {"achieved": round(cp, 2), "unit": "GB/s", "frac_of_peak": round(cp / HBM_PEAK_GBS, 4),
                         "what": "plain 1 GiB device copy (torch copy_), read + write bytes"},
        "pattern_ceiling": {"achieved": round(pr["gbs"], 2), "unit": "GB/s", "frac_of_peak": round(pr["gbs"] / HBM_PEAK_GBS, 4),
                            "frac": round(achieved / pr["gbs"], 4), "ms_per_launch": round(pr["ms"], 5),
                            "what": "lbm_probe_stream: the step's bytes per node and access pattern, no arithmetic"},
    }


def storage_line(cfg, precision, steps):
    """The same grid in another storage: MLUPS and the step kernel's achieved
    bandwidth on that storage's algorithmic bytes (HIP events), against the
    peak."""
    import torch

    r = gpu_run(cfg, precision, steps, 10, steps)
    kt = r["kernels"]
    dom = max(kt, key=lambda k: kt[k][0])
    ms = kt[dom][0] / max(kt[dom][1], 1)
    gbs = r["bytes_node"] * r["N"] / (ms * 1e-3) / 1e9
    out = {"mlups": round(r["N"] * steps / r["wall"] / 1e6, 1), "kernel": dom, "kernel_ms_per_launch": round(ms, 5),
           "bytes_per_node_step": r["bytes_node"], "achieved": round(gbs, 2), "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del r
    torch.cuda.empty_cache()
    return out


def batch_run(seed: int = 2000, count: int = 512, steps: int = 1024):
    """The batched sweep's step: `count` cases of the sweep distribution (uneven
    grids, angles, adsorption, surfactant load, shear) advanced together, one
    launch of the batched step kernel per step (graph-replayed), segment height
    from the batch's own autotuner.  Timed over `steps` steps."""
    import torch
    from paper_2609_26332_amd import lbm, sweep

    cases = sweep.batch_cases(seed, count)
    b = lbm.Batch(cases, "fp32")
    seg = b.autotune(trial_steps=10)
    b.step(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    inv = b.invariants(check=False)
    b.close()
    return {"workload": "%d cases of the sweep distribution (seed %d), grids %dx%d .. %dx%d, FP32 storage"
                        % (count, seed, min(c["nx"] for c in cases), min(c["ny"] for c in cases),
                           max(c["nx"] for c in cases), max(c["ny"] for c in cases)),
            "nodes": nodes, "seg_rows": seg, "steps": steps, "ms_per_step": round(wall * 1e3 / steps, 4),
            "mlups": round(nodes * steps / wall / 1e6, 1), "case_steps_per_s": round(count * steps / wall, 1),
            "nonfinite_cases": int(sum(1 for v in inv if v["nonfinite"]))}


def copy_rate(gib: float = 1.0, reps: int = 10) -> float:
    """GB/s of a plain device-to-device copy of `gib` GiB (read + write bytes),
    timed with HIP events on the current stream."""
    import torch

    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * n * 4 / ms / 1e6


def surrogate_rate(n: int = 4096, reps: int = 20) -> dict:
    """Inference rate of the 5-member surrogate ensemble (mean and spread of
    both outputs per case) on n cases, and one training step's time at the
    training batch size, with initial (untrained) parameters."""
    import numpy as np
    import torch
    from paper_2609_26332_amd import surrogate

    net = surrogate.Mlp(members=5, max_batch=n)
    for k in range(5):
        net.set_params(k, surrogate.glorot_params(k + 1, net.n_params))
    x = torch.as_tensor(np.random.default_rng(0).uniform(-1, 1, size=(n, 5)).astype(np.float32)).cuda()
    net.predict(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.predict(x)
    torch.cuda.synchronize()
    t_pred = (time.perf_counter() - t0) / reps
    b = 256
    t, m = torch.zeros(b, 2, device="cuda"), torch.ones(b, 2, device="cuda")
    xb = x[:b].contiguous()
    net.train_step(0, xb, t, m, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(0, xb, t, m, 1e-3)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / reps
    net.close()
    return {"members": 5, "cases": n, "predict_ms": round(t_pred * 1e3, 4), "predict_cases_per_s": round(n / t_pred, 1),
            "train_step_ms_batch256": round(t_train * 1e3, 4)}


def copy_calibration():
    import torch

    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "copies": 5}))


def cpu_baseline(cfg, budget_s=15.0):
    import oracle

    oracle.build(force=False)
    s = oracle.OracleSim(cfg)
    t0 = time.perf_counter()
    s.step(10)
    t1 = time.perf_counter()
    per = max((t1 - t0) / 10, 1e-6)
    n = max(10, int(budget_s / per))
    t0 = time.perf_counter()
    s.step(n)
    dt = time.perf_counter() - t0
    N = cfg["nx"] * cfg["ny"]
    return {"value": round(N * n / dt / 1e6, 4), "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d steps of the same %dx%d workload after 10 warm-up steps, FP64 oracle, %.1f s"
                      % (n, cfg["nx"], cfg["ny"], dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--large-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=1024)
    ap.add_argument("--workload", default="both", choices=["both", "sessile", "large"],
                    help="profiling aid: run one of the two workloads only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling aid: five device copies of 1 GiB (the reference for the HBM byte counters), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_2609_26332_amd import inputs

    if args.workload == "large":
        big = inputs.roofline_grid()
        rb = gpu_run(big, args.precision, args.large_steps, 10, args.large_steps)
        print(json.dumps({"workload": "periodic drop 4096x4096", "roofline": roofline(rb, "large_" + args.precision, big, args.precision)}))
        return
    cfg = inputs.sessile_drop()
    res = gpu_run(cfg, args.precision, args.steps, args.warmup, min(args.steps, 2000))
    mlups = res["N"] * args.steps / res["wall"] / 1e6
    head = roofline(res, "sessile_" + args.precision, cfg, args.precision)
    out = {
        "metric": "MLUPS (3 coupled lattices) + HBM roofline %",
        "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["wall"] * 1e3 / args.steps, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "sessile drop on adsorbing solid, 256x128 D2Q9, %s storage, FP64 reductions"
                               % args.precision.upper(),
                   "nx": cfg["nx"], "ny": cfg["ny"], "theta0_deg": cfg["theta0_deg"], "psi_b": cfg["psi_b"],
                   "beta_sg": round(cfg["beta_sg"], 6), "precision": args.precision},
        "lattice_mlups": round(3 * mlups, 2),
    }
    if res["inv"]["nonfinite"]:
        out["warning"] = "non-finite fields after the timed run"
    del res
    if not args.no_large and args.workload == "both":
        big = inputs.roofline_grid()
        rb = gpu_run(big, args.precision, args.large_steps, 10, args.large_steps)
        rl = roofline(rb, "large_" + args.precision, big, args.precision)
        rl = dict(workload="periodic drop 4096x4096, %s storage (5 GB of state, beyond the on-die caches)"
                  % args.precision.upper(), mlups=round(rb["N"] * args.large_steps / rb["wall"] / 1e6, 1), **rl)
        out["roofline"] = rl
        del rb
        if args.precision == "fp32":
            out["roofline_other_storages"] = {prec: storage_line(big, prec, 40) for prec in ("fp64", "fp16")}
    if "roofline" not in out:   # the large grid was not run: the headline workload's kernel stands in
        out["roofline"] = head
    out["headline_kernel"] = dict(workload="the sessile workload above (state resident in the on-die caches)", **head)
    if not args.no_batch and args.workload == "both" and args.precision == "fp32":
        out["batched_sweep"] = batch_run(steps=args.batch_steps)
        out["surrogate"] = surrogate_rate()
    if not args.no_cpu_baseline and args.workload == "both":
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
