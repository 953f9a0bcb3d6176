"""Python binding of the 3-D (D3Q19) library entry points (include/lbm3d.h).

Argument marshalling only: every step runs in the HIP kernels of
``liblbm_hip.so``.  PyTorch supplies the device memory (one uint8 tensor per
simulation) and the stream; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lbm as _lbm

ABI_VERSION = 2
FIELD_NAMES = ["phi", "psi", "ux", "uy", "uz", "p", "rho", "mu_phi", "mu_psi"]
EXPORTS = ["lbm3d_required_bytes", "lbm3d_init", "lbm3d_step", "lbm3d_reduce_invariants", "lbm3d_fetch_fields",
           "lbm3d_load_fields", "lbm3d_set_solid", "lbm3d_bytes_per_node_step", "lbm3d_destroy",
           "lbm3d_last_error"]


class Params3(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc_bottom", ctypes.c_int32), ("bc_top", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("constraint_phi", ctypes.c_int32), ("init_kind", ctypes.c_int32), ("adv_raw", ctypes.c_int32),
        ("phi_hold", ctypes.c_int32), ("solid_wet", ctypes.c_int32),
        ("sigma_gl0", ctypes.c_double), ("eps", ctypes.c_double), ("M_phi", ctypes.c_double),
        ("M_psi", ctypes.c_double), ("lambda_s", ctypes.c_double), ("kBT", ctypes.c_double), ("W", ctypes.c_double),
        ("Ex", ctypes.c_double), ("Pi", ctypes.c_double), ("psi_b", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("theta0_deg", ctypes.c_double), ("sigma_sg0", ctypes.c_double), ("sigma_sl0", ctypes.c_double),
        ("beta_sg", ctypes.c_double), ("beta_sl", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double), ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double), ("u_wall_top", ctypes.c_double),
        ("eta_phi", ctypes.c_double), ("eta_psi", ctypes.c_double), ("M0", ctypes.c_double),
        ("s_f", ctypes.c_double * 5), ("s_g", ctypes.c_double * 5), ("s_h", ctypes.c_double * 5),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double), ("R0", ctypes.c_double),
        ("a", ctypes.c_double),
    ]


class Invariants3(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64), ("psi_out_of_range", ctypes.c_int64),
        ("mass_psi", ctypes.c_double), ("m_phi_h", ctypes.c_double), ("sum_phi", ctypes.c_double),
        ("kinetic", ctypes.c_double), ("umax", ctypes.c_double), ("lambda_phi", ctypes.c_double),
        ("mubar_psi", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_ready = False


def lib():
    global _ready
    L = _lbm.lib()
    if not _ready:
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        L.lbm3d_required_bytes.argtypes = [ctypes.POINTER(Params3), ctypes.POINTER(sz)]
        L.lbm3d_init.argtypes = [ctypes.POINTER(Params3), vp, sz, vp, ctypes.POINTER(vp)]
        L.lbm3d_step.argtypes = [vp, ctypes.c_int64]
        L.lbm3d_reduce_invariants.argtypes = [vp, ctypes.POINTER(Invariants3)]
        L.lbm3d_fetch_fields.argtypes = [vp, ctypes.c_uint32, dp, sz]
        L.lbm3d_load_fields.argtypes = [vp, ctypes.c_int32, dp, sz]
        L.lbm3d_bytes_per_node_step.argtypes = [vp, dp]
        L.lbm3d_set_solid.argtypes = [vp, ctypes.c_char_p, sz]
        L.lbm3d_destroy.argtypes = [vp]
        L.lbm3d_last_error.argtypes = [vp]
        L.lbm3d_last_error.restype = ctypes.c_char_p
        for nm in EXPORTS[:-1]:
            getattr(L, nm).restype = ctypes.c_int
        _ready = True
    return L


def make_params(cfg: dict, precision: int) -> Params3:
    p = Params3()
    defaults = dict(lambda_s=-1.0, kBT=0.0, W=0.0, Ex=0.5, Pi=1.35, phi_b=0.0, sigma_sg0=-1.0, sigma_sl0=-1.0,
                    eta_phi=0.0, eta_psi=0.0, M0=-1.0, theta0_deg=90.0, rho_l=1.0, rho_g=1.0, mu_l=0.1, mu_g=0.1)
    merged = dict(defaults)
    merged.update(cfg)
    names = {f for f, _ in Params3._fields_}
    for k, v in merged.items():
        if k in names:
            setattr(p, k, (ctypes.c_double * 5)(*v) if k in ("s_f", "s_g", "s_h") else v)
    p.abi_version = ABI_VERSION
    p.precision = precision
    return p


def _check(rc, h=None):
    if rc != 0:
        raise _lbm.LbmError(rc, lib().lbm3d_last_error(h).decode())


class Sim3:
    """One 3-D simulation on the current HIP device; fields (nz, ny, nx)."""

    def __init__(self, cfg: dict, precision: str = "fp64", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch; the lattice Boltzmann path has no CPU fallback")
        self.cfg = dict(cfg)
        self.params = make_params(cfg, _lbm.PRECISIONS[precision])
        self.nx, self.ny, self.nz = self.params.nx, self.params.ny, self.params.nz
        nb = ctypes.c_size_t()
        _check(lib().lbm3d_required_bytes(ctypes.byref(self.params), ctypes.byref(nb)))
        self.buffer = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().lbm3d_init(ctypes.byref(self.params), ctypes.c_void_p(self.buffer.data_ptr()), nb.value,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(lib().lbm3d_step(self._h, int(n)), self._h)

    def invariants(self, check: bool = True) -> dict:
        inv = Invariants3()
        rc = lib().lbm3d_reduce_invariants(self._h, ctypes.byref(inv))
        if check:
            _check(rc, self._h)
        d = inv.as_dict()
        d["status"] = rc
        return d

    def fields(self, names=None) -> dict:
        names = names or FIELD_NAMES
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES.index(nm)
        sel = [nm for nm in FIELD_NAMES if mask & (1 << FIELD_NAMES.index(nm))]
        out = np.zeros((len(sel), self.nz, self.ny, self.nx))
        _check(lib().lbm3d_fetch_fields(self._h, mask, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
               self._h)
        return {nm: out[k] for k, nm in enumerate(sel)}

    def load_fields(self, phi, psi, u=None):
        planes = [phi, psi] + (list(u) if u is not None else [])
        arr = np.ascontiguousarray(np.stack([np.asarray(a, dtype=np.float64) for a in planes]))
        _check(lib().lbm3d_load_fields(self._h, 1 if u is not None else 0,
                                       arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), arr.size), self._h)

    def set_solid(self, mask):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        assert m.shape == (self.nz, self.ny, self.nx)
        _check(lib().lbm3d_set_solid(self._h, m.tobytes(), m.size), self._h)

    def bytes_per_node_step(self) -> float:
        b = ctypes.c_double()
        _check(lib().lbm3d_bytes_per_node_step(self._h, ctypes.byref(b)), self._h)
        return b.value
