#!/usr/bin/env python3
"""Benchmark of the coupled three-lattice lattice Boltzmann step on one MI355X.

Headline workload: the batched sweep, 512 independent sessile / sheared
droplets of the sweep distribution (grids 64x32 .. 384x192, theta0 U[30,150]
deg, adsorption strength U[0,0.5], psi_b U[0.005,0.05], Ca U[0,0.2], radius
U[12,60]; SplitMix64 seed 2000), advanced together by one batched step launch
per step (graph-replayed), FP32 storage with FP64 multiplier reductions.  One
step advances every case by one time step of all three lattices; `value` is
the batch's MLUPS (fluid nodes x steps / wall seconds / 1e6), with the state
already resident in HBM.

`roofline` is the batched step kernel's achieved HBM bandwidth on the
algorithmic bytes of a node-step (27 populations and 4 history planes, read
and written: 248 B in FP32 storage, 496 B in FP64, 140 B with FP16
populations), timed with HIP events on the batch's stream.  The bytes the
kernel actually moves by design (FP64 phi/psi planes, advecting-velocity and
source history) are reported beside it with their ratio.

Further lines: the same batch in FP64 and FP16 storage; a 4096^2 periodic grid
(state far beyond the on-die caches) in all three storages with a plain-copy
and an access-pattern ceiling; the single 256x128 sessile drop and the 64^2
stationary drop; the surrogate ensemble's rates.  The FP64 CPU oracle is timed
beside them on the host cores (bounded samples, stated) as cpu_baseline.
"""
import argparse
import concurrent.futures
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per node-step: 27 populations and 4 history planes
# (phi, psi, u_x, u_y of the previous step), each read and written once.
ALGO_BYTES = {"fp32": 2 * (27 * 4 + 4 * 4), "fp64": 2 * (27 * 8 + 4 * 8), "fp16": 2 * (27 * 2 + 4 * 4)}
SEED = 2000
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2609_26332_amd", "csrc", "lbm_kernels.hip")


def sync():
    import torch

    torch.cuda.synchronize()


def measured_traffic(key):
    """HBM bytes per launch of a step kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's
    readings), when that summary was taken on the current kernel source;
    None otherwise."""
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


def kernel_line(kt, nodes, prec, design_bytes):
    """Roofline figures of the dominant (step) kernel from HIP-event times."""
    ms = kt["k_step"][0] / max(kt["k_step"][1], 1)
    algo = ALGO_BYTES[prec]
    gbs = algo * nodes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_node_step": algo,
            "kernel_ms_per_launch": round(ms, 5),
            "finish_ms_per_launch": round(kt["k_step_finish"][0] / max(kt["k_step_finish"][1], 1), 5),
            "design_bytes_per_node_step": design_bytes,
            "design_over_algorithmic": round(design_bytes / algo, 4),
            "design_bytes_achieved_gbs": round(design_bytes * nodes / (ms * 1e-3) / 1e9, 2)}


def batch_run(prec, steps, warmup, kernel_steps, count=512):
    """The batched sweep: `count` cases, one batched step launch per step,
    segment height from the batch's autotuner; wall-clock steps (graph
    replays) and then event-timed eager steps for the kernel figures."""
    from paper_2609_26332_amd import lbm, sweep

    cases = sweep.batch_cases(SEED, count)
    b = lbm.Batch(cases, prec)
    seg = b.autotune(trial_steps=10)
    tune = b.autotune_report()
    info = b.info()
    b.step(warmup)
    sync()
    t0 = time.perf_counter()
    b.step(steps)
    sync()
    wall = time.perf_counter() - t0
    b.timing_begin(kernel_steps)
    b.step(kernel_steps)
    kt = b.timing_end()
    inv = b.invariants(check=False)
    nodes = info["nodes"]
    out = {"workload": "%d cases of the sweep distribution (seed %d), grids %dx%d .. %dx%d, %s storage, FP64 reductions"
                       % (count, SEED, min(c["nx"] for c in cases), min(c["ny"] for c in cases),
                          max(c["nx"] for c in cases), max(c["ny"] for c in cases), prec.upper()),
           "nodes": nodes, "cases": count, "seg_rows": seg, "workgroups": info["workgroups"],
           "wall_s": wall, "mlups": nodes * steps / wall / 1e6, "ms_per_step": wall * 1e3 / steps,
           "case_steps_per_s": count * steps / wall, "nonfinite_cases": int(sum(1 for v in inv if v["nonfinite"])),
           "kernels": kt,
           "autotune": [dict(seg_rows=r["seg_rows"], trial_ms=round(r["ms"], 3), max_rel_dev=float("%.3g" % r["max_rel_dev"]),
                             passed=r["passed"]) for r in tune]}
    b.close()
    return out


def design_bytes(prec):
    """Bytes per node-step the step kernels move by design in this storage
    (with surfactant): the populations, the FP64 phi/psi planes and six
    history planes, read and written (lbm_bytes_per_node_step)."""
    return {"fp32": 296.0, "fp64": 560.0, "fp16": 196.0}[prec]


def grid_run(cfg, prec, steps, warmup, kernel_steps):
    from paper_2609_26332_amd import lbm

    sim = lbm.Sim(cfg, prec)
    sim.step(warmup)
    sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sync()
    wall = time.perf_counter() - t0
    sim.timing_begin(kernel_steps)
    sim.step(kernel_steps)
    kt = sim.timing_end()
    N = cfg["nx"] * cfg["ny"]
    out = {"mlups": round(N * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 5),
           "step_kernel": sim.step_kernel(), "nonfinite": sim.invariants(check=False)["nonfinite"],
           **kernel_line(kt, N, prec, sim.bytes_per_node_step())}
    sim.close()
    return out


# Algorithmic bytes of a D3Q19 node-step: 57 populations and 5 history planes
# (phi, psi, u_x, u_y, u_z of the previous step), read and written.
ALGO_BYTES_3D = {"fp32": 2 * (57 * 4 + 5 * 4), "fp64": 2 * (57 * 8 + 5 * 8)}


def grid3d_run(n, prec, steps, warmup):
    """The 3-D (D3Q19) step on an n^3 periodic drop: whole-step rate (its five
    kernels) on the algorithmic bytes of a D3Q19 node-step."""
    from paper_2609_26332_amd import inputs, lbm3d

    sim = lbm3d.Sim3(inputs.drop3d(n, n / 4.0, psi_b=0.01), prec)
    sim.step(warmup)
    sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sync()
    wall = time.perf_counter() - t0
    N = n ** 3
    ms = wall * 1e3 / steps
    gbs = ALGO_BYTES_3D[prec] * N / (ms * 1e-3) / 1e9
    out = {"workload": "periodic drop %d^3, D3Q19, %s storage" % (n, prec.upper()), "mlups": round(N * steps / wall / 1e6, 1),
           "ms_per_step": round(ms, 5), "bytes_per_node_step": ALGO_BYTES_3D[prec], "achieved": round(gbs, 2),
           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "design_bytes_per_node_step": sim.bytes_per_node_step(),
           "what": "whole step (five kernels), wall clock over %d steps" % steps,
           "nonfinite": sim.invariants(check=False)["nonfinite"]}
    sim.close()
    return out


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
    """Inference rate of the 5-member surrogate ensemble on n cases and one
    training step's time at the training batch size (initial parameters)."""
    import numpy as np
    import torch
    from paper_2609_26332_amd import surrogate

    net = surrogate.Mlp(members=5, max_batch=n)
    for k in range(5):
        net.set_params(k, surrogate.glorot_params(k + 1, net.n_params))
    x = torch.as_tensor(np.random.default_rng(0).uniform(-1, 1, size=(n, 5)).astype(np.float32)).cuda()
    net.predict(x)
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.predict(x)
    sync()
    t_pred = (time.perf_counter() - t0) / reps
    b = 256
    t, m = torch.zeros(5, b, 2, device="cuda"), torch.ones(5, b, 2, device="cuda")
    xb = x[:b].unsqueeze(0).repeat(5, 1, 1).contiguous()
    net.train_step_ensemble(xb, t, m, 1e-3)
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step_ensemble(xb, t, m, 1e-3)
    sync()
    t_train = (time.perf_counter() - t0) / reps
    net.close()
    return {"members": 5, "cases": n, "predict_ms": round(t_pred * 1e3, 4), "predict_cases_per_s": round(n / t_pred, 1),
            "train_step_ms_batch256_all_members": round(t_train * 1e3, 4)}


DATA_DIR = os.path.join(ROOT, "paper_2609_26332_amd", "data")
TRAIN_SEEDS = list(range(1000, 1015))
CALIB_SEEDS = [1015, 1016]


def sweep_file(seed):
    return os.path.join(DATA_DIR, "sweep_seed%d.npz" % seed)


def stream_sweep(n_cases: int, slots: int, cap: int, seed: int = 3000) -> dict:
    """A stream of sweep cases longer than the batch: n_cases cases of the
    sweep distribution through `slots` batch slots, each finished slot
    refilled with the next waiting case, against the same cases run as
    consecutive batches of `slots` cases each; 16-row segments in both, so
    every case's results must agree exactly."""
    from paper_2609_26332_amd import inputs, sweep

    cases = inputs.sweep_batch(seed, n_cases)
    kw = dict(precision="fp32", seg_rows=16, autotune=False, cap=cap)
    print("stream: %d cases through %d slots, cap %d" % (n_cases, slots, cap), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    refill = sweep.run_sweep(cases, slots=slots, **kw)
    t_refill = time.perf_counter() - t0
    print("stream: refilled run %.1f s" % t_refill, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    seq = []
    for i in range(0, n_cases, slots):
        seq += sweep.run_sweep(cases[i:i + slots], **kw)["results"]
        print("stream: consecutive batch %d done" % (i // slots), file=sys.stderr, flush=True)
    t_seq = time.perf_counter() - t0
    same = all(a["status"] == b["status"] and a["step"] == b["step"] and a["mass_psi"] == b["mass_psi"]
               for a, b in zip(refill["results"], seq))
    status = {}
    for r in refill["results"]:
        status[r["status"]] = status.get(r["status"], 0) + 1
    return {"workload": "stream of %d sweep cases (seed %d) through %d slots, stop rule capped at %d steps"
                        % (n_cases, seed, slots, cap),
            "refill_seconds": round(t_refill, 2), "refill_cases_per_s": round(n_cases / t_refill, 3),
            "refills": refill["refills"], "consecutive_batches_seconds": round(t_seq, 2),
            "consecutive_cases_per_s": round(n_cases / t_seq, 3), "speedup": round(t_seq / t_refill, 3),
            "identical_results": bool(same), "status": status}


def surrogate_sweep(cap: int = 50000) -> dict:
    """The second half of the metric: the 512 held-out cases of the sweep
    distribution (seed 2000) delivered by the batched solver alone and by the
    surrogate with its calibrated fallback to the solver, both timed here.
    The ensemble trains on the committed solver runs of seeds 1000-1014
    (7680 cases) and calibrates its fallback threshold on seeds 1015-1016;
    the accuracy of the delivered angles is judged against this run's own
    plain sweep."""
    import numpy as np
    from paper_2609_26332_amd import sweep, train_surrogate as ts

    cases = sweep.batch_cases(SEED, 512)
    t0 = time.perf_counter()
    r = sweep.run_sweep(cases, cap=cap)
    plain_s = time.perf_counter() - t0
    truth = ts.labels(cases, r, cap)
    sur, train_s, _, n_train = ts.train([sweep_file(k) for k in TRAIN_SEEDS], log=None)
    cal = ts.calibrate(sur, [sweep_file(k) for k in CALIB_SEEDS], log=None)
    delivered, pred, fb, pred_s, fb_s = ts.deliver(sur, cases, cal["threshold_deg"], cap)
    acc = ts.accuracy(delivered, pred, fb, truth)
    stored = np.load(sweep_file(SEED))["angle"]
    both = np.isfinite(stored) & np.isfinite(truth["angle"])
    n = len(cases)
    return {"what": "512 held-out sweep cases (seed 2000) to their stop rule: plain batched solver vs surrogate with "
                    "calibrated fallback to the solver; training and calibration on committed solver runs",
            "plain_cases_per_s": round(n / plain_s, 3), "plain_seconds": round(plain_s, 2),
            "cases_per_s": round(n / (pred_s + fb_s), 3), "gain": round(plain_s / (pred_s + fb_s), 2),
            "predict_seconds": round(pred_s, 4), "fallback_seconds": round(fb_s, 2),
            "threshold_deg": round(cal["threshold_deg"], 4), "calibration": cal,
            "train_cases": n_train, "train_seconds": round(train_s, 2), **acc,
            "plain_angles_vs_committed_max_abs_deg": float(np.abs(stored[both] - truth["angle"][both]).max())
            if both.any() else None}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s=8.0):
    """The FP64 oracle on the host cores, on bounded samples:
    * the headline workload: cases of the same sweep batch, one case per
      thread on every host core, each run for a bounded number of steps;
    * one thread on the 64^2 stationary drop (1000 steps) and on a 512^2
      periodic drop (a bounded number of steps)."""
    import oracle
    from paper_2609_26332_amd import inputs, sweep

    oracle.build(force=False)
    ncores = len(os.sched_getaffinity(0))
    oracle.set_parallel(False)   # one case per thread; no nested threads
    try:
        cases = sweep.batch_cases(SEED, 512)[:ncores]
        sims = [oracle.OracleSim(c) for c in cases]
        sims[0].step(2)
        t0 = time.perf_counter()
        sims[0].step(5)
        per_node_step = (time.perf_counter() - t0) / (5 * cases[0]["nx"] * cases[0]["ny"])
        mean_nodes = sum(c["nx"] * c["ny"] for c in cases) / len(cases)
        steps = max(10, int(budget_s / (per_node_step * mean_nodes)))

        def run(s):
            s.step(steps)

        with concurrent.futures.ThreadPoolExecutor(max_workers=ncores) as ex:
            t0 = time.perf_counter()
            list(ex.map(run, sims))
            wall = time.perf_counter() - t0
        node_steps = steps * sum(c["nx"] * c["ny"] for c in cases)
        sweep_mlups = node_steps / wall / 1e6
        del sims
        c1 = inputs.stationary_drop()
        s = oracle.OracleSim(c1)
        t0 = time.perf_counter()
        s.step(1000)
        t_c1 = time.perf_counter() - t0
        big = inputs.stationary_drop(nx=512, ny=512, R=128.0)
        s = oracle.OracleSim(big)
        s.step(1)
        t0 = time.perf_counter()
        s.step(1)
        per = time.perf_counter() - t0
        n512 = max(2, min(200, int(budget_s / per)))
        t0 = time.perf_counter()
        s.step(n512)
        t_512 = time.perf_counter() - t0
    finally:
        oracle.set_parallel(True)
    return {"value": round(sweep_mlups, 4), "unit": "MLUPS", "cores": ncores, "kind": "oracle",
            "sample": "%d cases of the same sweep batch (seed %d), one per host thread, %d steps each, FP64 oracle, "
                      "%.1f s (the full batch is 512 cases; MLUPS is per node-step, so it extrapolates directly)"
                      % (len(cases), SEED, steps, wall),
            "case_steps_per_s": round(len(cases) * steps / wall, 2),
            "single_thread": {"stationary_drop_64x64_1000_steps_mlups": round(4096 * 1000 / t_c1 / 1e6, 4),
                              "periodic_drop_512x512_mlups": round(512 * 512 * n512 / t_512 / 1e6, 4),
                              "periodic_drop_512x512_steps": n512},
            "nproc": ncores, "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--kernel-steps", type=int, default=20, help="event-timed steps for the kernel figures")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline batch (profiling aid)")
    ap.add_argument("--workload", default="all",
                    choices=["all", "batch", "grid4096", "grid3d", "surrogate", "mlp", "stream"],
                    help="profiling aid: one workload only (stream: a case stream longer than the batch, with refill)")
    ap.add_argument("--stream-cases", type=int, default=1024)
    ap.add_argument("--stream-slots", type=int, default=512)
    ap.add_argument("--stream-cap", type=int, default=10000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp16"],
                    help="profiling aid: storage of the single workload run with --workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling aid: five device copies of 1 GiB (the reference for the HBM byte counters), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (the batch would shard by cases, "
              "see the design notes); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        sync()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "copies": 5}))
        return
    from paper_2609_26332_amd import inputs

    if args.workload == "surrogate":
        print(json.dumps(surrogate_sweep()), flush=True)
        return
    if args.workload == "mlp":
        print(json.dumps(surrogate_rate()), flush=True)
        return
    if args.workload == "stream":
        print(json.dumps(stream_sweep(args.stream_cases, args.stream_slots, args.stream_cap)), flush=True)
        return
    if args.workload == "grid3d":
        p3 = args.precision if args.precision in ("fp32", "fp64") else "fp32"
        print(json.dumps(grid3d_run(128, p3, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "grid4096":
        r = grid_run(inputs.roofline_grid(), args.precision, args.steps, args.warmup, args.kernel_steps)
        print(json.dumps({"workload": "periodic drop 4096x4096 %s" % args.precision, **r}), flush=True)
        return
    prec = args.precision if args.workload == "batch" else "fp32"
    hb = batch_run(prec, args.steps, args.warmup, args.kernel_steps)
    rl = kernel_line(hb["kernels"], hb["nodes"], prec, design_bytes(prec))
    rl.update(kernel="k_step_batch", nodes_per_launch=hb["nodes"],
              traffic=measured_traffic("batch_" + prec))
    if rl["traffic"] is not None:
        rl["traffic_source"] = ("rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel source, scaled by a 1 GiB copy's "
                                "readings (profiles/k_step_traffic.md); not counted in this run")
    from paper_2609_26332_amd import lbm as _lbm
    hc = _lbm.probe_copy(1.0, 10)
    rl.update(copy_ceiling_gbs=round(hc["gbs"], 2), frac_of_copy_ceiling=round(rl["achieved"] / hc["gbs"], 4))
    torch.cuda.empty_cache()
    out = {
        "metric": "MLUPS (3 coupled lattices) + HBM roofline %; batched sweep cases/s at ±0.5°",
        "value": round(hb["mlups"], 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(hb["ms_per_step"], 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == "fp32" else prec.replace("fp", "f"),
        "data": "synthetic",
        "config": {"workload": "batched sweep: " + hb["workload"], "cases": hb["cases"], "nodes": hb["nodes"],
                   "seed": SEED, "seg_rows": hb["seg_rows"], "workgroups": hb["workgroups"], "precision": prec},
        "lattice_mlups": round(3 * hb["mlups"], 2),
        "case_steps_per_s": round(hb["case_steps_per_s"], 1),
        "roofline": rl,
        "autotune": {"what": "segment heights tried on the batch, 10 timed steps each from the initial state; a "
                             "candidate counts only if its sums agree with the first's (relative 1e-6 in FP32)",
                     "candidates": hb["autotune"]},
    }
    if hb["nonfinite_cases"]:
        out["warning"] = "%d cases with non-finite fields after the timed run" % hb["nonfinite_cases"]
    if args.workload == "all" and not args.no_extras:
        out["batch_other_storages"] = {}
        for p in ("fp64", "fp16"):
            r = batch_run(p, max(50, args.steps // 4), 10, args.kernel_steps)
            out["batch_other_storages"][p] = dict(mlups=round(r["mlups"], 1), ms_per_step=round(r["ms_per_step"], 5),
                                                  seg_rows=r["seg_rows"], nonfinite_cases=r["nonfinite_cases"],
                                                  **kernel_line(r["kernels"], r["nodes"], p, design_bytes(p)))
            torch.cuda.empty_cache()
        big = inputs.roofline_grid()
        g = {}
        for p in ("fp32", "fp64", "fp16"):
            g[p] = grid_run(big, p, 100, 10, args.kernel_steps)
            g[p]["traffic"] = measured_traffic("grid_" + p)
            torch.cuda.empty_cache()
        from paper_2609_26332_amd import lbm
        pr = lbm.probe_stream(big["nx"], big["ny"], "fp32", reps=20)
        cp = copy_rate()
        g["copy_ceiling"] = {"achieved": round(cp, 2), "unit": "GB/s", "frac_of_peak": round(cp / HBM_PEAK_GBS, 4),
                             "what": "plain 1 GiB device copy (torch copy_), read + write bytes"}
        hc = lbm.probe_copy(1.0, 10)
        g["copy_ceiling_hip"] = {"achieved": round(hc["gbs"], 2), "unit": "GB/s", "frac_of_peak": round(hc["gbs"] / HBM_PEAK_GBS, 4),
                                 "ms_per_copy": round(hc["ms"], 5), "copied": hc["copied"],
                                 "what": "lbm_probe_copy: 1 GiB streaming copy, 16-byte non-temporal loads and stores, "
                                         "read + write bytes"}
        g["pattern_ceiling_fp32"] = {"achieved": round(pr["gbs"], 2), "unit": "GB/s",
                                     "frac_of_peak": round(pr["gbs"] / HBM_PEAK_GBS, 4), "ms_per_launch": round(pr["ms"], 5),
                                     "what": "lbm_probe_stream: the FP32 step's design bytes (296 B/node) in its access "
                                             "pattern, without arithmetic"}
        out["grid_4096x4096"] = dict(workload="periodic drop 4096x4096 (state far beyond the on-die caches)", **g)
        torch.cuda.empty_cache()
        out["sessile_256x128_fp32"] = grid_run(inputs.sessile_drop(), "fp32", 2000, 100, args.kernel_steps)
        out["stationary_64x64_fp64"] = grid_run(inputs.stationary_drop(), "fp64", 2000, 100, args.kernel_steps)
        out["grid3d_128"] = {p: grid3d_run(128, p, 40, 5) for p in ("fp32", "fp64")}
        torch.cuda.empty_cache()
        out["surrogate"] = surrogate_rate()
        torch.cuda.empty_cache()
        out["sweep_with_surrogate"] = surrogate_sweep()
    if not args.no_cpu_baseline and args.workload == "all":
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
