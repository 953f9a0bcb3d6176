"""Comparison helpers for the GPU-vs-oracle parity tests (test code only)."""
import numpy as np

FIELDS = ["phi", "psi", "ux", "uy", "p", "mu_phi", "mu_psi"]


def field_errors(gpu: dict, orc: dict, u_floor: float, p_floor: float = 0.0) -> dict:
    """Per field: max |gpu - oracle| / max(max |oracle|, floor).  Near-zero
    fields are normalised by a physical scale: velocities by u_floor (a
    fraction of the velocity scale of the case), pressure by p_floor."""
    out = {}
    for k in FIELDS:
        if k not in gpu or k not in orc:
            continue
        ref = np.abs(orc[k]).max()
        floor = u_floor if k in ("ux", "uy") else (p_floor if k == "p" else 0.0)
        scale = max(ref, floor)
        diff = np.abs(gpu[k] - orc[k]).max()
        out[k] = diff / scale if scale > 0 else diff
    return out


def assert_fields_close(gpu: dict, orc: dict, tol: float, u_floor: float, p_floor: float = 0.0, label: str = ""):
    errs = field_errors(gpu, orc, u_floor, p_floor)
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, f"{label}: fields beyond {tol:g}: {bad} (all: {errs})"
    return errs
