"""Batched parameter sweep of sessile / sheared droplets on the GPU.

Runs cases of the sweep distribution (inputs.sweep_case: contact angle,
adsorption strength, surfactant load, capillary number, drop radius) to their
stop rule in lbm_batch launches and returns, per case, the steady apparent
contact angle and the detachment time:

* steady: the apparent angle (circular-cap estimate from contact width and
  height) moves less than `steady_tol` degrees over `steady_window` steps,
  checked every `check_every` steps;
* detached: the contact width on the wall row falls to zero (the detachment
  time t* = u_w t / (2 R0) is recorded);
* otherwise the case stops at `cap` steps (detachment censored at the cap).

Finished cases retire (their workgroups return at once) while the rest of the
batch continues.  Everything that computes runs in the HIP kernels; this
module only schedules.
"""
from __future__ import annotations

import math
import time

from . import inputs


def detach_time_star(cfg: dict, steps: int) -> float:
    """t* = u_w t / (2 R0); the cap is used for cases without wall motion."""
    uw = abs(cfg.get("u_wall_top", 0.0))
    return uw * steps / (2.0 * cfg["R0"]) if uw > 0 else 0.0


def run_sweep(cases: list, precision: str = "fp32", seg_rows: int = 0, autotune: bool = True,
              check_every: int = 500, steady_window: int = 2000, steady_tol: float = 0.05, cap: int = 50000,
              log=None) -> dict:
    """Run `cases` (configuration dicts) in one batch; returns a dict with the
    per-case results and the timing of the run."""
    from . import lbm

    t_start = time.perf_counter()
    b = lbm.Batch(cases, precision, seg_rows=seg_rows)
    seg = b.autotune(trial_steps=10) if autotune else b.info()["seg_rows"]
    info = b.info()
    n = len(cases)
    active = [True] * n
    history = [[] for _ in range(n)]   # (step, theta_app)
    result = [None] * n
    step = 0
    t_run = time.perf_counter()
    node_steps = 0
    while any(active):
        b.step(check_every)
        node_steps += check_every * sum(c["nx"] * c["ny"] for c, a in zip(cases, active) if a)
        step += check_every
        inv = b.invariants(check=False)
        changed = False
        for k in range(n):
            if not active[k]:
                continue
            iv = inv[k]
            done = None
            if iv["nonfinite"] or iv["psi_out_of_range"]:
                done = dict(status="fault", step=step)
            elif iv["contact_width"] <= 0.0:
                done = dict(status="detached", step=step, theta_app_deg=float("nan"),
                            detach_t_star=detach_time_star(cases[k], step))
            else:
                history[k].append((step, iv["theta_app_deg"]))
                lag = steady_window // check_every
                if len(history[k]) > lag and abs(history[k][-1][1] - history[k][-1 - lag][1]) < steady_tol:
                    done = dict(status="steady", step=step, theta_app_deg=iv["theta_app_deg"],
                                detach_t_star=detach_time_star(cases[k], cap))
                elif step >= cap:
                    done = dict(status="capped", step=step, theta_app_deg=iv["theta_app_deg"],
                                detach_t_star=detach_time_star(cases[k], cap))
            if done is not None:
                done.update(contact_width=iv["contact_width"], cap_height=iv["cap_height"],
                            mass_psi=iv["mass_psi"])
                result[k] = done
                active[k] = False
                changed = True
        if changed and any(active):
            b.set_active(active)
        if log is not None:
            log(f"step {step}: {sum(active)} of {n} cases running")
    t_end = time.perf_counter()
    b.close()
    return dict(results=result, seg_rows=seg, workgroups=info["workgroups"], nodes=info["nodes"],
                node_steps=node_steps, run_seconds=t_end - t_run, total_seconds=t_end - t_start,
                cases_per_second=n / (t_end - t_start))


def sweep_inputs(cfg: dict) -> list:
    """The five surrogate inputs of a case: theta0, adsorption strength, psi_b, Ca, R."""
    si = cfg["sweep_inputs"]
    return [si["theta0_deg"], si["adsorption"], si["psi_b"], si["Ca"], si["R"]]


def batch_cases(seed: int, count: int) -> list:
    return inputs.sweep_batch(seed, count)
