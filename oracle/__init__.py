"""FP64 CPU oracle of the coupled three-population lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  The oracle is the yardstick the HIP path is
checked against: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP library (``paper_2609_26332_amd``); the two only share the seeded input
generators in ``paper_2609_26332_amd/inputs.py``, which hold none of the
method's arithmetic.

The C source (``lbm_oracle.c``) follows the model of Section 2 and the MRT
scheme of Section 3 of the paper step by step; this module only marshals
arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC3 = os.path.join(_HERE, "lbm3d_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

PERIODIC, WALL_WET, NOSLIP, FREESLIP = 0, 1, 2, 3
NONLINEAR, LINEAR = 0, 1
INIT_DROP, INIT_SLAB, INIT_BUBBLE = 0, 1, 2
F_PHI, F_PSI, F_UX, F_UY, F_P, F_RHO, F_MU_PHI, F_MU_PSI = 1, 2, 4, 8, 16, 32, 64, 128
FIELD_NAMES = ["phi", "psi", "ux", "uy", "p", "rho", "mu_phi", "mu_psi"]
DERIVED_NAMES = ["kappa", "beta", "W", "kBT", "phi_b", "sigma_sg0", "sigma_sl0",
                 "lambda_s", "M0", "eta_phi", "eta_psi", "psi_c"]


def build(force: bool = True) -> str:
    """Compile the oracle with plain -O2, no FMA contraction (gcc, OpenMP loops)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in (_SRC, _SRC3))
    if force or stale:
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB, _SRC, _SRC3, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_bottom", ctypes.c_int32), ("bc_top", ctypes.c_int32),
        ("constraint_phi", ctypes.c_int32), ("init_kind", ctypes.c_int32),
        ("mms", ctypes.c_int32), ("adv_raw", ctypes.c_int32),
        ("phi_hold", ctypes.c_int32), ("sat_cap", ctypes.c_int32),
        ("sigma_gl0", ctypes.c_double), ("eps", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("M_psi", ctypes.c_double),
        ("lambda_s", ctypes.c_double), ("kBT", ctypes.c_double), ("W", ctypes.c_double),
        ("Ex", ctypes.c_double), ("Pi", ctypes.c_double),
        ("psi_b", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("theta0_deg", ctypes.c_double), ("sigma_sg0", ctypes.c_double), ("sigma_sl0", ctypes.c_double),
        ("beta_sg", ctypes.c_double), ("beta_sl", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
        ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double), ("u_wall_top", ctypes.c_double),
        ("eta_phi", ctypes.c_double), ("eta_psi", ctypes.c_double), ("M0", ctypes.c_double),
        ("s_f", ctypes.c_double * 5), ("s_g", ctypes.c_double * 5), ("s_h", ctypes.c_double * 5),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("R0", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("mms_dx", ctypes.c_double),
    ]


class Invariants(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
        ("psi_out_of_range", ctypes.c_int64), ("cap_violations", ctypes.c_int64),
        ("mass_psi", ctypes.c_double), ("m_phi_h", ctypes.c_double), ("sum_phi", ctypes.c_double),
        ("area_phi_pos", ctypes.c_double), ("kinetic", ctypes.c_double),
        ("free_energy", ctypes.c_double), ("umax", ctypes.c_double),
        ("lambda_phi", ctypes.c_double), ("mubar_psi", ctypes.c_double),
        ("contact_width", ctypes.c_double), ("cap_height", ctypes.c_double),
        ("theta_app_deg", ctypes.c_double),
        ("sum_R_psi", ctypes.c_double), ("orthogonality", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(Params), ctypes.c_char_p, ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_derived.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        L.orc_fields.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double)]
        L.orc_invariants.argtypes = [ctypes.c_void_p, ctypes.POINTER(Invariants)]
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_load_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.orc_get_populations.argtypes = [ctypes.c_void_p, dp]
        L.orc_mms_errors.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_area_positive.restype = ctypes.c_double
        L.orc_area_positive.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_contact.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_parallel.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(cfg: dict) -> Params:
    """Map a configuration dictionary (see paper_2609_26332_amd.inputs) to the
    oracle's own parameter struct.  Unset entries take the 'derive' defaults."""
    p = Params()
    defaults = dict(lambda_s=-1.0, kBT=0.0, W=0.0, Ex=0.5, Pi=1.35, phi_b=0.0,
                    sigma_sg0=-1.0, sigma_sl0=-1.0, eta_phi=0.0, eta_psi=0.0, M0=-1.0,
                    theta0_deg=90.0, rho_l=1.0, rho_g=1.0, mu_l=0.1, mu_g=0.1)
    merged = dict(defaults)
    merged.update(cfg)
    names = {f for f, _ in Params._fields_}
    for k, v in merged.items():
        if k not in names:
            continue
        if k in ("s_f", "s_g", "s_h"):
            arr = (ctypes.c_double * 5)(*v)
            setattr(p, k, arr)
        else:
            setattr(p, k, v)
    return p


class OracleSim:
    """One oracle simulation.  Fields are FP64 arrays of shape (ny, nx)."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.params = make_params(cfg)
        self.nx, self.ny = self.params.nx, self.params.ny
        err = ctypes.create_string_buffer(256)
        h = lib().orc_create(ctypes.byref(self.params), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def derived(self) -> dict:
        out = np.zeros(len(DERIVED_NAMES))
        lib().orc_derived(self._h, _dptr(out))
        return dict(zip(DERIVED_NAMES, out.tolist()))

    def fields(self, names=None) -> dict:
        names = names or FIELD_NAMES
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES.index(nm)
        sel = [nm for nm in FIELD_NAMES if mask & (1 << FIELD_NAMES.index(nm))]
        out = np.zeros((len(sel), self.ny, self.nx))
        lib().orc_fields(self._h, mask, _dptr(out))
        return {nm: out[k] for k, nm in enumerate(sel)}

    def invariants(self) -> dict:
        inv = Invariants()
        lib().orc_invariants(self._h, ctypes.byref(inv))
        return inv.as_dict()

    def load_fields(self, phi, psi, ux=None, uy=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        uxp = _dptr(np.ascontiguousarray(ux, dtype=np.float64)) if ux is not None else None
        uyp = _dptr(np.ascontiguousarray(uy, dtype=np.float64)) if uy is not None else None
        lib().orc_load_fields(self._h, _dptr(phi), _dptr(psi), uxp, uyp)

    def populations(self) -> np.ndarray:
        out = np.zeros((27, self.ny, self.nx))
        lib().orc_get_populations(self._h, _dptr(out))
        return out

    def mms_errors(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        lib().orc_mms_errors(self._h, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value


def area_positive(phi: np.ndarray, wall_bottom=False, wall_top=False, periodic_y=True) -> float:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    return lib().orc_area_positive(_dptr(phi), nx, ny, int(wall_bottom), int(wall_top), int(periodic_y))


def contact(phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    w, h, t = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_contact(_dptr(phi), nx, ny, ctypes.byref(w), ctypes.byref(h), ctypes.byref(t))
    return w.value, h.value, t.value


def threads() -> int:
    return lib().orc_threads()


def set_parallel(on: bool) -> None:
    """Switch the oracle's OpenMP node loops on (default) or off process-wide."""
    lib().orc_set_parallel(1 if on else 0)


# ------------------------------------------------------------------ 3-D
FIELD_NAMES_3D = ["phi", "psi", "ux", "uy", "uz", "p", "rho", "mu_phi", "mu_psi"]


class Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc_bottom", ctypes.c_int32), ("bc_top", ctypes.c_int32),
        ("constraint_phi", ctypes.c_int32), ("init_kind", ctypes.c_int32),
        ("adv_raw", ctypes.c_int32), ("phi_hold", ctypes.c_int32), ("solid_wet", ctypes.c_int32),
        ("sigma_gl0", ctypes.c_double), ("eps", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("M_psi", ctypes.c_double), ("lambda_s", ctypes.c_double),
        ("kBT", ctypes.c_double), ("W", ctypes.c_double), ("Ex", ctypes.c_double), ("Pi", ctypes.c_double),
        ("psi_b", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("theta0_deg", ctypes.c_double), ("sigma_sg0", ctypes.c_double), ("sigma_sl0", ctypes.c_double),
        ("beta_sg", ctypes.c_double), ("beta_sl", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double), ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double), ("u_wall_top", ctypes.c_double),
        ("eta_phi", ctypes.c_double), ("eta_psi", ctypes.c_double), ("M0", ctypes.c_double),
        ("s_f", ctypes.c_double * 5), ("s_g", ctypes.c_double * 5), ("s_h", ctypes.c_double * 5),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
        ("R0", ctypes.c_double), ("a", ctypes.c_double),
    ]


class Invariants3(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64), ("psi_out_of_range", ctypes.c_int64),
        ("mass_psi", ctypes.c_double), ("m_phi_h", ctypes.c_double), ("sum_phi", ctypes.c_double),
        ("kinetic", ctypes.c_double), ("umax", ctypes.c_double), ("lambda_phi", ctypes.c_double),
        ("mubar_psi", ctypes.c_double), ("sum_R_psi", ctypes.c_double), ("orthogonality", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib3_ready = False


def lib3():
    global _lib3_ready
    L = lib()
    if not _lib3_ready:
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc3_create.restype = ctypes.c_void_p
        L.orc3_create.argtypes = [ctypes.POINTER(Params3), ctypes.c_char_p, ctypes.c_int]
        L.orc3_destroy.argtypes = [ctypes.c_void_p]
        L.orc3_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc3_derived.argtypes = [ctypes.c_void_p, dp]
        L.orc3_fields.argtypes = [ctypes.c_void_p, ctypes.c_uint32, dp]
        L.orc3_invariants.argtypes = [ctypes.c_void_p, ctypes.POINTER(Invariants3)]
        L.orc3_load_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc3_get_populations.argtypes = [ctypes.c_void_p, dp]
        L.orc3_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), dp]
        L.orc3_set_solid.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
        _lib3_ready = True
    return L


def make_params3(cfg: dict) -> Params3:
    p = Params3()
    defaults = dict(lambda_s=-1.0, kBT=0.0, W=0.0, Ex=0.5, Pi=1.35, phi_b=0.0, sigma_sg0=-1.0, sigma_sl0=-1.0,
                    eta_phi=0.0, eta_psi=0.0, M0=-1.0, theta0_deg=90.0, rho_l=1.0, rho_g=1.0, mu_l=0.1, mu_g=0.1)
    merged = dict(defaults)
    merged.update(cfg)
    names = {f for f, _ in Params3._fields_}
    for k, v in merged.items():
        if k not in names:
            continue
        if k in ("s_f", "s_g", "s_h"):
            setattr(p, k, (ctypes.c_double * 5)(*v))
        else:
            setattr(p, k, v)
    return p


class Oracle3Sim:
    """One 3-D oracle simulation.  Fields are FP64 arrays of shape (nz, ny, nx)."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.params = make_params3(cfg)
        self.nx, self.ny, self.nz = self.params.nx, self.params.ny, self.params.nz
        err = ctypes.create_string_buffer(256)
        h = lib3().orc3_create(ctypes.byref(self.params), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib3().orc3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        lib3().orc3_step(self._h, int(n))

    def derived(self) -> dict:
        out = np.zeros(len(DERIVED_NAMES))
        lib3().orc3_derived(self._h, _dptr(out))
        return dict(zip(DERIVED_NAMES, out.tolist()))

    def fields(self, names=None) -> dict:
        names = names or FIELD_NAMES_3D
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES_3D.index(nm)
        sel = [nm for nm in FIELD_NAMES_3D if mask & (1 << FIELD_NAMES_3D.index(nm))]
        out = np.zeros((len(sel), self.nz, self.ny, self.nx))
        lib3().orc3_fields(self._h, mask, _dptr(out))
        return {nm: out[k] for k, nm in enumerate(sel)}

    def invariants(self) -> dict:
        inv = Invariants3()
        lib3().orc3_invariants(self._h, ctypes.byref(inv))
        return inv.as_dict()

    def load_fields(self, phi, psi, u=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        up = _dptr(np.ascontiguousarray(u, dtype=np.float64)) if u is not None else None
        lib3().orc3_load_fields(self._h, _dptr(phi), _dptr(psi), up)

    def set_solid(self, mask):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        assert m.shape == (self.nz, self.ny, self.nx)
        if lib3().orc3_set_solid(self._h, m.tobytes()) != 0:
            raise ValueError("no fluid node left")

    def populations(self) -> np.ndarray:
        out = np.zeros((57, self.nz, self.ny, self.nx))
        lib3().orc3_get_populations(self._h, _dptr(out))
        return out


def lattice3():
    """The oracle's D3Q19 velocities (19 x 3) and weights."""
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    lib3().orc3_lattice(c, _dptr(w))
    return np.array(list(c)).reshape(19, 3), w
