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
batch continues; with fewer batch slots than cases, a finished case's slot is
refilled with the next waiting case.  Everything that computes runs in the HIP
kernels; this module only schedules.
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
              slots: "int | None" = None, log=None) -> dict:
    """Run `cases` (configuration dicts) to their stop rule; returns a dict with
    the per-case results and the timing of the run.

    slots: batch slots (default: one per case).  With fewer slots than cases the
    largest cases open the slots and every slot whose case finishes takes the
    next waiting case (lbm_batch_replace_case: any grid that fits the slot), so
    the batch stays full while cases remain.  A case's steps, checks and stop
    rule count from its own start, and its results do not depend on the slot it
    ran in or on the cases beside it."""
    from . import lbm

    t_start = time.perf_counter()
    n = len(cases)
    nslot = n if slots is None else max(1, min(int(slots), n))
    if nslot < n:   # largest first: every later case then fits any slot
        need = [lbm.required_bytes(c, precision) for c in cases]
        order = sorted(range(n), key=lambda k: (-need[k], k))
    else:
        need, order = None, list(range(n))
    b = lbm.Batch([cases[k] for k in order[:nslot]], precision, seg_rows=seg_rows)
    seg = b.autotune(trial_steps=10) if autotune else b.info()["seg_rows"]
    info = b.info()
    waiting = order[nslot:]
    slot_case = list(order[:nslot])   # case index each slot runs
    start = [0] * nslot               # batch step at which the slot's case started
    active = [True] * nslot
    history = [[] for _ in range(n)]  # (case step, theta_app)
    result = [None] * n
    step = 0
    refills = 0
    t_run = time.perf_counter()
    node_steps = 0
    while any(active):
        b.step(check_every)
        node_steps += check_every * sum(cases[slot_case[s]]["nx"] * cases[slot_case[s]]["ny"]
                                        for s in range(nslot) if active[s])
        step += check_every
        inv = b.invariants(check=False)
        changed = False
        for s in range(nslot):
            if not active[s]:
                continue
            k, iv, own = slot_case[s], inv[s], step - start[s]
            done = None
            if iv["nonfinite"] or iv["psi_out_of_range"]:
                done = dict(status="fault", step=own)
            elif iv["contact_width"] <= 0.0:
                done = dict(status="detached", step=own, theta_app_deg=float("nan"),
                            detach_t_star=detach_time_star(cases[k], own))
            else:
                history[k].append((own, iv["theta_app_deg"]))
                lag = steady_window // check_every
                if len(history[k]) > lag and abs(history[k][-1][1] - history[k][-1 - lag][1]) < steady_tol:
                    done = dict(status="steady", step=own, theta_app_deg=iv["theta_app_deg"],
                                detach_t_star=detach_time_star(cases[k], cap))
                elif own >= cap:
                    done = dict(status="capped", step=own, theta_app_deg=iv["theta_app_deg"],
                                detach_t_star=detach_time_star(cases[k], cap))
            if done is not None:
                done.update(contact_width=iv["contact_width"], cap_height=iv["cap_height"],
                            mass_psi=iv["mass_psi"])
                result[k] = done
                active[s] = False
                changed = True
                fit = next((j for j, q in enumerate(waiting) if need[q] <= b.slot_bytes(s)), None) if waiting else None
                if fit is not None:
                    q = waiting.pop(fit)
                    b.replace_case(s, cases[q])
                    slot_case[s], start[s], active[s] = q, step, True
                    refills += 1
        if changed and any(active):
            b.set_active(active)
        if log is not None:
            log(f"step {step}: {sum(active)} of {nslot} slots running, {len(waiting)} cases waiting")
    t_end = time.perf_counter()
    b.close()
    return dict(results=result, seg_rows=seg, workgroups=info["workgroups"], nodes=info["nodes"],
                node_steps=node_steps, run_seconds=t_end - t_run, total_seconds=t_end - t_start,
                cases_per_second=n / (t_end - t_start), slots=nslot, refills=refills)


def sweep_inputs(cfg: dict) -> list:
    """The five surrogate inputs of a case: theta0, adsorption strength, psi_b, Ca, R."""
    si = cfg["sweep_inputs"]
    return [si["theta0_deg"], si["adsorption"], si["psi_b"], si["Ca"], si["R"]]


def batch_cases(seed: int, count: int) -> list:
    return inputs.sweep_batch(seed, count)
