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
    lb = labels(cases, r, cap)
    st = lb["status"]
    np.savez(out, **lb, seed=seed, cap=cap, seconds=r["total_seconds"], run_seconds=r["run_seconds"],
             node_steps=r["node_steps"])
    log(json.dumps(dict(seed=seed, count=count, cap=cap, seconds=round(r["total_seconds"], 2),
                        status={k: int((st == v).sum()) for k, v in STATUS.items()})))
    return out


def load(files):
    parts = [np.load(f) for f in files]
    keys = ["X", "angle", "tau", "tau_mask", "status"]
    return {k: np.concatenate([p[k] for p in parts]) for k in keys}, parts


def calibrate(sur, calib_files, tol_deg: float = 0.5, target: float = 0.99, confidence: float = 0.95,
              max_spread_deg: float = 0.5, log=print) -> dict:
    """Fallback threshold from calibration cases the ensemble did not train on.

    The ensemble's spread is not an error bound: members trained on the same
    data share a bias the spread cannot show.  On the calibration cases (the
    solver's results known) the cases are ordered by spread; accepting those
    with spread <= t, a case is a miss when it is accepted and its predicted
    angle is off by more than tol_deg (or the solver's drop detached, so there
    is no angle to predict).  t is the largest spread, at most max_spread_deg,
    for which the one-sided Clopper-Pearson upper bound (at `confidence`) on
    the fraction of misses among all cases stays within 1 - target; cases
    above t go to the solver, whose angles are exact by definition.  So at
    least `target` of delivered angles lie within tol_deg, with that
    confidence, for cases drawn from the calibration cases' distribution."""
    from scipy.stats import beta

    ca, _ = load(calib_files)
    use = ca["status"] != STATUS["fault"]
    angle, spread, tau, _ = sur.predict(ca["X"][use])
    det = ca["tau_mask"][use] > 0
    err = np.abs(angle - ca["angle"][use])
    miss = ~(err <= tol_deg)                       # NaN truth (detached) counts as a miss
    N = int(use.sum())
    order = np.argsort(spread, kind="stable")
    k = np.cumsum(miss[order])
    upper = beta.ppf(confidence, k + 1, N - k)     # Clopper-Pearson bound for k misses in N cases
    ok = (upper <= 1.0 - target) & (spread[order] <= max_spread_deg)
    # the accepted set must be a prefix: stop at the first spread where the bound fails
    stop = int(np.argmin(ok)) if not ok.all() else N
    t = float(spread[order][stop - 1]) if stop > 0 else 0.0
    acc = spread <= t
    out = dict(threshold_deg=t, calib_cases=N, target_within=target, confidence=confidence,
               calib_accepted=round(float(acc.mean()), 4), calib_misses=int((miss & acc).sum()),
               calib_miss_bound=round(float(upper[stop - 1]), 5) if stop > 0 else None,
               calib_detached=int(det.sum()),
               calib_detach_tau_mean_abs_err=round(float(np.abs(tau - ca["tau"][use])[det].mean()), 4)
               if det.any() else None)
    if log:
        log(json.dumps(dict(calibration=out)))
    return out


def labels(cases, r, cap: int) -> dict:
    """Per-case labels of a finished sweep (sweep.run_sweep's result)."""
    res = r["results"]
    st = np.array([STATUS[x["status"]] for x in res])
    angle = np.array([x.get("theta_app_deg", np.nan) for x in res], dtype=np.float64)
    t_cap = np.array([sweep.detach_time_star(c, cap) for c in cases])
    t_det = np.array([x.get("detach_t_star", 0.0) for x in res], dtype=np.float64)
    tau = np.where(t_cap > 0, np.minimum(t_det, t_cap) / np.where(t_cap > 0, t_cap, 1.0), 0.0)
    return dict(X=np.array([sweep.sweep_inputs(c) for c in cases]), angle=angle, tau=tau,
                tau_mask=(st == STATUS["detached"]).astype(np.float64), status=st)


def train(train_files, epochs: int = 1000, members: int = 5, log=print):
    """The ensemble trained on the committed sweep files; returns (surrogate, seconds, final losses)."""
    from .surrogate import Surrogate
    import torch

    tr, _ = load(train_files)
    ok = tr["status"] != STATUS["fault"]
    t0 = time.perf_counter()
    sur = Surrogate(members=members)
    losses = sur.fit(tr["X"][ok], tr["angle"][ok], tr["tau"][ok], tr["tau_mask"][ok], epochs=epochs, log=log)
    torch.cuda.synchronize()
    return sur, time.perf_counter() - t0, losses, int(ok.sum())


def deliver(sur, cases, threshold: float, cap: int):
    """Angles of `cases`: the ensemble's where its spread is within the
    threshold, else the batched solver's (run on the declined cases only).
    Returns the delivered angles, the ensemble's predictions (angle, spread,
    tau), the fallback mask and the two timed phases in seconds."""
    import torch

    X = np.array([sweep.sweep_inputs(c) for c in cases])
    t0 = time.perf_counter()
    angle, spread, tau, _ = sur.predict(X)
    torch.cuda.synchronize()
    predict_seconds = time.perf_counter() - t0
    fb = spread > threshold
    delivered = angle.copy()
    fb_seconds = 0.0
    if fb.any():
        sub = [c for c, f in zip(cases, fb) if f]
        t0 = time.perf_counter()
        r = sweep.run_sweep(sub, cap=cap)
        fb_seconds = time.perf_counter() - t0
        delivered[fb] = np.array([x.get("theta_app_deg", np.nan) for x in r["results"]])
    return delivered, (angle, spread, tau), fb, predict_seconds, fb_seconds


def accuracy(delivered, pred, fb, truth: dict) -> dict:
    """Delivered angles against the solver's: within 0.5 degree over the cases
    with an angle (and by stop status), the detachment-time error of the
    cases that detached, and the ensemble's own accuracy where it was used."""
    angle, spread, tau = pred
    t = truth["angle"]
    valid = np.isfinite(t)
    err = np.abs(delivered - t)
    steady = valid & (truth["status"] == STATUS["steady"])
    capped = valid & (truth["status"] == STATUS["capped"])
    det = truth["tau_mask"] > 0
    used = valid & ~fb
    e_used = np.abs(angle - t)[used]
    return dict(
        cases=len(t), fallback_fraction=round(float(fb.mean()), 4),
        within_0p5_deg=round(float((err[valid] <= 0.5).mean()), 4),
        max_err_deg=round(float(err[valid].max()), 4), mean_err_deg=round(float(err[valid].mean()), 4),
        steady_cases=int(steady.sum()),
        steady_within_0p5_deg=round(float((err[steady] <= 0.5).mean()), 4) if steady.any() else None,
        capped_cases=int(capped.sum()),
        capped_within_0p5_deg=round(float((err[capped] <= 0.5).mean()), 4) if capped.any() else None,
        detached_cases=int(det.sum()),
        detached_taken_from_surrogate=int((det & ~fb).sum()),
        detach_tau_mean_abs_err=round(float(np.abs(tau - truth["tau"])[det].mean()), 4) if det.any() else None,
        surrogate_used_cases=int(used.sum()),
        surrogate_used_within_0p5_deg=round(float((e_used <= 0.5).mean()), 4) if used.any() else None)


def evaluate(train_files, val_file, threshold: float = 0.5, epochs: int = 1000, members: int = 5, log=print,
             calib_files=None) -> dict:
    """Train, calibrate the fallback (when calibration files are given) and
    deliver the held-out file's cases; the plain sweep time is the one stored
    with the held-out file."""
    sur, train_seconds, losses, n_train = train(train_files, epochs, members, log)
    calib = None
    if calib_files:
        calib = calibrate(sur, calib_files, tol_deg=0.5, max_spread_deg=threshold, log=log)
        threshold = calib["threshold_deg"]
    va, vparts = load([val_file])
    cap, seed = int(vparts[0]["cap"]), int(vparts[0]["seed"])
    cases = sweep.batch_cases(seed, len(va["angle"]))
    plain_seconds = float(vparts[0]["seconds"])
    delivered, pred, fb, predict_seconds, fb_seconds = deliver(sur, cases, threshold, cap)
    n = len(cases)
    out = dict(train_cases=n_train, members=members, epochs=epochs, threshold_deg=threshold,
               train_seconds=round(train_seconds, 2), final_losses=[round(float(x), 5) for x in losses],
               plain_seconds=round(plain_seconds, 3), predict_seconds=round(predict_seconds, 4),
               fallback_seconds=round(fb_seconds, 3), plain_cases_per_s=round(n / plain_seconds, 3),
               surrogate_cases_per_s=round(n / (predict_seconds + fb_seconds), 3),
               gain=round(plain_seconds / (predict_seconds + fb_seconds), 2),
               **accuracy(delivered, pred, fb, va), calibration=calib)
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
    e.add_argument("--epochs", type=int, default=1000)
    e.add_argument("--threshold", type=float, default=0.5)
    e.add_argument("--calib", nargs="+", help="calibration files: the fallback threshold is fitted on them")
    e.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        generate(a.seed, a.count, a.cap, a.out)
    else:
        r = evaluate(a.train, a.val, a.threshold, a.epochs, calib_files=a.calib)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(r, f, indent=1)


if __name__ == "__main__":
    main()
