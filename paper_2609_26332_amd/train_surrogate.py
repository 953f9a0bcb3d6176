"""Training data, training and evaluation of the sweep surrogate.

  python -m paper_2609_26332_amd.train_surrogate generate --seed 1000 --count 512 --out d1000.npz
  python -m paper_2609_26332_amd.train_surrogate evaluate --train d1000.npz d1001.npz ... --val d2000.npz

`generate` runs a batch of the sweep distribution (inputs.sweep_batch(seed))
to its stop rule with the lattice Boltzmann batch and stores, per case, the
five inputs, the delivered apparent angle, the detachment time scaled by the
cap (tau) with its censoring mask, and the run's wall time.  `evaluate` trains
the ensemble on the training files, predicts the held-out file, sends the
cases whose ensemble spread exceeds the threshold back to the solver (run
and timed), and reports the accuracy of the delivered angles against the
solver's and the throughput against the plain solver sweep of the same cases.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import sweep

STATUS = {"steady": 0, "capped": 1, "detached": 2, "fault": 3}


def generate(seed: int, count: int, cap: int, out: str, log=print):
    cases = sweep.batch_cases(seed, count)
    r = sweep.run_sweep(cases, cap=cap, log=None)
    X = np.array([sweep.sweep_inputs(c) for c in cases])
    res = r["results"]
    st = np.array([STATUS[x["status"]] for x in res])
    angle = np.array([x.get("theta_app_deg", np.nan) for x in res], dtype=np.float64)
    t_cap = np.array([sweep.detach_time_star(c, cap) for c in cases])
    t_det = np.array([x.get("detach_t_star", 0.0) for x in res], dtype=np.float64)
    tau = np.where(t_cap > 0, np.minimum(t_det, t_cap) / np.where(t_cap > 0, t_cap, 1.0), 0.0)
    tau_mask = (st == STATUS["detached"]).astype(np.float64)
    np.savez(out, X=X, angle=angle, tau=tau, tau_mask=tau_mask, status=st, seed=seed, cap=cap,
             seconds=r["total_seconds"], run_seconds=r["run_seconds"], node_steps=r["node_steps"])
    log(json.dumps(dict(seed=seed, count=count, cap=cap, seconds=round(r["total_seconds"], 2),
                        status={k: int((st == v).sum()) for k, v in STATUS.items()})))
    return out


def load(files):
    parts = [np.load(f) for f in files]
    keys = ["X", "angle", "tau", "tau_mask", "status"]
    return {k: np.concatenate([p[k] for p in parts]) for k in keys}, parts


def evaluate(train_files, val_file, threshold: float = 0.5, epochs: int = 300, members: int = 5, log=print) -> dict:
    from .surrogate import Surrogate
    import torch

    tr, _ = load(train_files)
    ok = tr["status"] != STATUS["fault"]
    t0 = time.perf_counter()
    sur = Surrogate(members=members, threshold_deg=threshold)
    losses = sur.fit(tr["X"][ok], tr["angle"][ok], tr["tau"][ok], tr["tau_mask"][ok], epochs=epochs, log=log)
    torch.cuda.synchronize()
    train_seconds = time.perf_counter() - t0
    va, vparts = load([val_file])
    cap = int(vparts[0]["cap"])
    seed = int(vparts[0]["seed"])
    cases = sweep.batch_cases(seed, len(va["angle"]))
    truth = va["angle"]
    plain_seconds = float(vparts[0]["seconds"])           # the plain solver sweep of these cases
    # surrogate pass (timed), then the solver on the cases it declines (timed)
    t0 = time.perf_counter()
    angle, spread, tau, tau_sd = sur.predict(va["X"])
    torch.cuda.synchronize()
    predict_seconds = time.perf_counter() - t0
    fb = spread > threshold
    fb_seconds = 0.0
    delivered = angle.copy()
    if fb.any():
        sub = [c for c, f in zip(cases, fb) if f]
        t0 = time.perf_counter()
        r = sweep.run_sweep(sub, cap=cap)
        fb_seconds = time.perf_counter() - t0
        delivered[fb] = np.array([x.get("theta_app_deg", np.nan) for x in r["results"]])
    valid = np.isfinite(truth)
    err = np.abs(delivered - truth)[valid]
    err_sur = np.abs(angle - truth)[valid & ~fb]
    n = len(truth)
    out = dict(train_cases=int(ok.sum()), val_cases=n, members=members, epochs=epochs, threshold_deg=threshold,
               train_seconds=round(train_seconds, 2), final_losses=[round(float(x), 5) for x in losses],
               fallback_fraction=round(float(fb.mean()), 4),
               within_0p5_deg=round(float((err <= 0.5).mean()), 4), max_err_deg=round(float(err.max()), 4),
               mean_err_deg=round(float(err.mean()), 4),
               surrogate_only_mean_err_deg=round(float(err_sur.mean()), 4) if err_sur.size else None,
               surrogate_only_within_0p5=round(float((err_sur <= 0.5).mean()), 4) if err_sur.size else None,
               plain_seconds=round(plain_seconds, 3), predict_seconds=round(predict_seconds, 4),
               fallback_seconds=round(fb_seconds, 3),
               plain_cases_per_s=round(n / plain_seconds, 3),
               surrogate_cases_per_s=round(n / (predict_seconds + fb_seconds), 3),
               gain=round(plain_seconds / (predict_seconds + fb_seconds), 2))
    log(json.dumps(out))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--seed", type=int, required=True)
    g.add_argument("--count", type=int, default=512)
    g.add_argument("--cap", type=int, default=50000)
    g.add_argument("--out", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--train", nargs="+", required=True)
    e.add_argument("--val", required=True)
    e.add_argument("--epochs", type=int, default=300)
    e.add_argument("--threshold", type=float, default=0.5)
    e.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        generate(a.seed, a.count, a.cap, a.out)
    else:
        r = evaluate(a.train, a.val, a.threshold, a.epochs)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(r, f, indent=1)


if __name__ == "__main__":
    main()
