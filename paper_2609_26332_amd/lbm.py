"""Python binding of the gfx950 lattice Boltzmann library (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbm_hip.so``.  PyTorch supplies the device memory (one uint8 tensor
per simulation, handed to ``lbm_init`` as ``dev_buf``) and the HIP stream.
There is no CPU fallback: without the built library or a gfx950 device every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  -- loads torch's HIP runtime first so one runtime serves both

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_hip.so")

ABI_VERSION = 4
PERIODIC, WALL_WET, NOSLIP, FREESLIP = 0, 1, 2, 3
FP64, FP32, FP16_SHIFTED = 0, 1, 2
NONLINEAR, LINEAR = 0, 1
INIT_DROP, INIT_SLAB, INIT_BUBBLE = 0, 1, 2
FIELD_NAMES = ["phi", "psi", "ux", "uy", "p", "rho", "mu_phi", "mu_psi"]
DERIVED_NAMES = ["kappa", "beta", "W", "kBT", "phi_b", "sigma_sg0", "sigma_sl0",
                 "lambda_s", "M0", "eta_phi", "eta_psi", "psi_c"]
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16_SHIFTED}
STATUS = {0: "LBM_OK", -1: "LBM_E_ARG", -2: "LBM_E_UNSUPPORTED", -3: "LBM_E_OOM", -4: "LBM_E_DEVICE",
          -5: "LBM_E_NONFINITE", -6: "LBM_E_RANGE", -7: "LBM_E_STATE"}

# Every symbol the header declares; the test suite checks the library exports them.
EXPORTS = ["lbm_required_bytes", "lbm_init", "lbm_step", "lbm_reduce_invariants", "lbm_fetch_fields",
           "lbm_load_fields", "lbm_state_bytes", "lbm_save_state", "lbm_load_state", "lbm_derived",
           "lbm_fetch_populations", "lbm_destroy", "lbm_last_error", "lbm_timing_begin", "lbm_timing_end",
           "lbm_bytes_per_node_step", "lbm_probe_bytes", "lbm_probe_stream", "lbm_probe_copy", "lbm_step_kernel",
           "lbm_batch_required_bytes", "lbm_batch_init", "lbm_batch_step", "lbm_batch_set_active",
           "lbm_batch_reduce_invariants", "lbm_batch_fetch_fields", "lbm_batch_replace_case", "lbm_batch_slot_bytes", "lbm_batch_autotune",
           "lbm_batch_autotune_report",
           "lbm_batch_info", "lbm_batch_timing_begin", "lbm_batch_timing_end", "lbm_batch_destroy",
           "lbm_batch_last_error"]
KERNEL_NAMES = ["k_step", "k_step_finish"]
STEP_KERNELS = ["k_step_small", "k_step_mid", "k_step", "k_step (three workgroups per CU)"]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_bottom", ctypes.c_int32), ("bc_top", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("constraint_phi", ctypes.c_int32), ("init_kind", ctypes.c_int32),
        ("adv_raw", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("phi_hold", ctypes.c_int32), ("sat_cap", ctypes.c_int32),
        ("sigma_gl0", ctypes.c_double), ("eps", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("M_psi", ctypes.c_double), ("lambda_s", ctypes.c_double),
        ("kBT", ctypes.c_double), ("W", ctypes.c_double), ("Ex", ctypes.c_double), ("Pi", ctypes.c_double),
        ("psi_b", ctypes.c_double), ("phi_b", ctypes.c_double), ("theta0_deg", ctypes.c_double),
        ("sigma_sg0", ctypes.c_double), ("sigma_sl0", ctypes.c_double),
        ("beta_sg", ctypes.c_double), ("beta_sl", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double), ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double), ("u_wall_top", ctypes.c_double),
        ("eta_phi", ctypes.c_double), ("eta_psi", ctypes.c_double), ("M0", ctypes.c_double),
        ("s_f", ctypes.c_double * 5), ("s_g", ctypes.c_double * 5), ("s_h", ctypes.c_double * 5),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("R0", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("mms_dx", ctypes.c_double),
    ]


class Invariants(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64), ("psi_out_of_range", ctypes.c_int64),
        ("cap_violations", ctypes.c_int64),
        ("mass_psi", ctypes.c_double), ("m_phi_h", ctypes.c_double), ("sum_phi", ctypes.c_double),
        ("area_phi_pos", ctypes.c_double), ("kinetic", ctypes.c_double), ("free_energy", ctypes.c_double),
        ("umax", ctypes.c_double), ("lambda_phi", ctypes.c_double), ("mubar_psi", ctypes.c_double),
        ("contact_width", ctypes.c_double), ("cap_height", ctypes.c_double), ("theta_app_deg", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        L.lbm_required_bytes.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(sz)]
        L.lbm_init.argtypes = [ctypes.POINTER(Params), vp, sz, vp, ctypes.POINTER(vp)]
        L.lbm_step.argtypes = [vp, ctypes.c_int64]
        L.lbm_reduce_invariants.argtypes = [vp, ctypes.POINTER(Invariants)]
        L.lbm_fetch_fields.argtypes = [vp, ctypes.c_uint32, dp, sz]
        L.lbm_load_fields.argtypes = [vp, ctypes.c_uint32, dp, sz]
        L.lbm_state_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.lbm_save_state.argtypes = [vp, vp, sz]
        L.lbm_load_state.argtypes = [vp, vp, sz]
        L.lbm_derived.argtypes = [vp, dp]
        L.lbm_fetch_populations.argtypes = [vp, dp, sz]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_timing_begin.argtypes = [vp, ctypes.c_int64]
        L.lbm_timing_end.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.lbm_bytes_per_node_step.argtypes = [vp, dp]
        L.lbm_probe_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(sz)]
        L.lbm_probe_stream.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, sz, vp,
                                       ctypes.POINTER(ctypes.c_float)]
        L.lbm_probe_copy.argtypes = [vp, vp, sz, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_float)]
        L.lbm_step_kernel.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        L.lbm_batch_required_bytes.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(sz)]
        L.lbm_batch_init.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32, vp, sz, vp, ctypes.POINTER(vp)]
        L.lbm_batch_step.argtypes = [vp, ctypes.c_int64]
        L.lbm_batch_set_active.argtypes = [vp, i32p]
        L.lbm_batch_reduce_invariants.argtypes = [vp, ctypes.POINTER(Invariants)]
        L.lbm_batch_fetch_fields.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32, dp, sz]
        L.lbm_batch_replace_case.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Params)]
        L.lbm_batch_slot_bytes.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(sz)]
        L.lbm_batch_autotune.argtypes = [vp, ctypes.c_int32, i32p]
        L.lbm_batch_autotune_report.argtypes = [vp, ctypes.c_int32, i32p, dp, dp, i32p, i32p]
        L.lbm_batch_info.argtypes = [vp, i32p, i32p, i32p, i64p]
        L.lbm_batch_timing_begin.argtypes = [vp, ctypes.c_int64]
        L.lbm_batch_timing_end.argtypes = [vp, dp, i64p]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_last_error.argtypes = [vp]
        L.lbm_batch_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("lbm_last_error", "lbm_batch_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def make_params(cfg: dict, precision: int) -> Params:
    """Map a configuration dictionary (paper_2609_26332_amd.inputs) onto lbm_params."""
    p = Params()
    defaults = dict(lambda_s=-1.0, kBT=0.0, W=0.0, Ex=0.5, Pi=1.35, phi_b=0.0, sigma_sg0=-1.0, sigma_sl0=-1.0,
                    eta_phi=0.0, eta_psi=0.0, M0=-1.0, theta0_deg=90.0, rho_l=1.0, rho_g=1.0, mu_l=0.1, mu_g=0.1)
    merged = dict(defaults)
    merged.update(cfg)
    names = {f for f, _ in Params._fields_}
    for k, v in merged.items():
        if k not in names:
            continue
        if k in ("s_f", "s_g", "s_h"):
            setattr(p, k, (ctypes.c_double * 5)(*v))
        else:
            setattr(p, k, v)
    p.abi_version = ABI_VERSION
    p.precision = precision
    return p


def _check(rc: int, handle=None):
    if rc != 0:
        msg = lib().lbm_last_error(handle).decode()
        raise LbmError(rc, msg)


def required_bytes(cfg: dict, precision: str = "fp64") -> int:
    p = make_params(cfg, PRECISIONS[precision])
    n = ctypes.c_size_t()
    _check(lib().lbm_required_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


class Sim:
    """One simulation on the current HIP device.

    Device memory comes from a torch uint8 tensor owned by this object and
    work is ordered on torch's current stream (or the stream given).  `fill`,
    if given, is a byte value written over that memory before lbm_init (the
    tests fill it with 0xFF, a NaN in every floating-point format, to show that
    nothing reads state the library has not written)."""

    def __init__(self, cfg: dict, precision: str = "fp64", stream: "torch.cuda.Stream | None" = None,
                 fill: "int | None" = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch; the lattice Boltzmann path has no CPU fallback")
        self.cfg = dict(cfg)
        self.precision = precision
        self.params = make_params(cfg, PRECISIONS[precision])
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = required_bytes(cfg, precision)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if fill is not None:
            with torch.cuda.stream(self.stream):
                self.buffer.fill_(int(fill))
        h = ctypes.c_void_p()
        rc = lib().lbm_init(ctypes.byref(self.params), ctypes.c_void_p(self.buffer.data_ptr()), nbytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc, None)
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(lib().lbm_step(self._h, int(n)), self._h)

    def invariants(self, check: bool = True) -> dict:
        inv = Invariants()
        rc = lib().lbm_reduce_invariants(self._h, ctypes.byref(inv))
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
        out = np.zeros((len(sel), self.ny, self.nx))
        _check(lib().lbm_fetch_fields(self._h, mask, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size), self._h)
        return {nm: out[k] for k, nm in enumerate(sel)}

    def load_fields(self, phi, psi, ux=None, uy=None):
        planes = [phi, psi] + ([ux, uy] if ux is not None else [])
        arr = np.ascontiguousarray(np.stack([np.asarray(a, dtype=np.float64) for a in planes]))
        mask = 1 | 2 | ((4 | 8) if ux is not None else 0)
        _check(lib().lbm_load_fields(self._h, mask, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), arr.size), self._h)

    def populations(self) -> np.ndarray:
        out = np.zeros((27, self.ny, self.nx))
        _check(lib().lbm_fetch_populations(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size), self._h)
        return out

    def derived(self) -> dict:
        out = np.zeros(len(DERIVED_NAMES))
        _check(lib().lbm_derived(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)
        return dict(zip(DERIVED_NAMES, out.tolist()))

    def save_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(lib().lbm_state_bytes(self._h, ctypes.byref(n)), self._h)
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().lbm_save_state(self._h, buf, n.value), self._h)
        return buf.raw

    def timing_begin(self, max_steps: int):
        _check(lib().lbm_timing_begin(self._h, int(max_steps)), self._h)

    def timing_end(self) -> dict:
        k = len(KERNEL_NAMES)
        ms = (ctypes.c_double * k)()
        n = (ctypes.c_int64 * k)()
        _check(lib().lbm_timing_end(self._h, ms, n), self._h)
        return {KERNEL_NAMES[j]: (ms[j], n[j]) for j in range(k)}

    def bytes_per_node_step(self) -> float:
        b = ctypes.c_double()
        _check(lib().lbm_bytes_per_node_step(self._h, ctypes.byref(b)), self._h)
        return b.value

    def step_kernel(self) -> dict:
        """The step kernel this handle launches (lbm_step_kernel)."""
        v, w, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_step_kernel(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(c)), self._h)
        return dict(variant=v.value, kernel=STEP_KERNELS[v.value], workgroups=w.value, cus=c.value)

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().lbm_load_state(self._h, buf, len(blob)), self._h)


def probe_stream(nx: int, ny: int, precision: str = "fp32", reps: int = 20) -> dict:
    """Mean time of the bandwidth probe (lbm_probe_stream: the step's memory
    traffic without its arithmetic) on an nx x ny grid, with the bytes it moves
    per node and the resulting rate."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to torch; the probe has no CPU fallback")
    prec = PRECISIONS[precision]
    L = lib()
    nb = ctypes.c_size_t()
    _check(L.lbm_probe_bytes(nx, ny, prec, ctypes.byref(nb)))
    buf = torch.zeros(nb.value, dtype=torch.uint8, device="cuda")
    ms = ctypes.c_float()
    st = torch.cuda.current_stream()
    _check(L.lbm_probe_stream(nx, ny, prec, reps, ctypes.c_void_p(buf.data_ptr()), nb.value,
                              ctypes.c_void_p(st.cuda_stream), ctypes.byref(ms)))
    per_node = {"fp64": 560.0, "fp32": 296.0, "fp16": 196.0}[precision]
    return dict(ms=ms.value, bytes_per_node=per_node, gbs=per_node * nx * ny / ms.value / 1e6)


def probe_copy(gib: float = 1.0, reps: int = 10) -> dict:
    """The device's streaming-copy ceiling (lbm_probe_copy: 16-byte
    non-temporal loads and stores) for gib GiB; rate over bytes read plus
    written."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to torch; the probe has no CPU fallback")
    n = int(gib * (1 << 30)) // 16 * 16
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    ms = ctypes.c_float()
    st = torch.cuda.current_stream()
    _check(lib().lbm_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, reps,
                                ctypes.c_void_p(st.cuda_stream), ctypes.byref(ms)))
    ok = bool(torch.equal(src[:: 1 << 20], dst[:: 1 << 20]))
    return dict(ms=ms.value, bytes=2 * n, gbs=2 * n / ms.value / 1e6, copied=ok)


def _bcheck(rc: int, b=None):
    if rc != 0:
        raise LbmError(rc, lib().lbm_batch_last_error(b).decode())


class Batch:
    """Independent cases advanced together (the batched sweep of the C ABI).

    cfgs: configuration dictionaries (inputs.py); all share the storage
    precision and the kind of y boundary.  seg_rows as lbm_batch_init (0: auto).
    Device memory is one torch uint8 tensor; work runs on torch's current
    stream (or the stream given)."""

    def __init__(self, cfgs: list, precision: str = "fp32", seg_rows: int = 0, stream=None, fill: "int | None" = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch; the lattice Boltzmann path has no CPU fallback")
        self.cfgs = [dict(c) for c in cfgs]
        self.precision = precision
        n = len(cfgs)
        self.params = (Params * n)(*[make_params(c, PRECISIONS[precision]) for c in cfgs])
        nbytes = ctypes.c_size_t()
        _bcheck(lib().lbm_batch_required_bytes(self.params, n, ctypes.byref(nbytes)))
        self.buffer = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if fill is not None:   # as Sim's fill
            with torch.cuda.stream(self.stream):
                self.buffer.fill_(int(fill))
        b = ctypes.c_void_p()
        _bcheck(lib().lbm_batch_init(self.params, n, int(seg_rows), ctypes.c_void_p(self.buffer.data_ptr()), nbytes.value,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b)))
        self._b = b
        self.count = n

    def close(self):
        if getattr(self, "_b", None):
            lib().lbm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _bcheck(lib().lbm_batch_step(self._b, int(n)), self._b)

    def set_active(self, active):
        arr = (ctypes.c_int32 * self.count)(*[1 if a else 0 for a in active])
        _bcheck(lib().lbm_batch_set_active(self._b, arr), self._b)

    def invariants(self, check: bool = True) -> list:
        inv = (Invariants * self.count)()
        rc = lib().lbm_batch_reduce_invariants(self._b, inv)
        if check:
            _bcheck(rc, self._b)
        return [x.as_dict() for x in inv]

    def fields(self, index: int, names=("phi", "psi")) -> dict:
        cfg = self.cfgs[index]
        nx, ny = cfg["nx"], cfg["ny"]
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES.index(nm)
        order = [nm for nm in FIELD_NAMES if mask & (1 << FIELD_NAMES.index(nm))]
        out = np.empty(len(order) * nx * ny, dtype=np.float64)
        _bcheck(lib().lbm_batch_fetch_fields(self._b, int(index), mask,
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size), self._b)
        return {nm: out[k * nx * ny:(k + 1) * nx * ny].reshape(ny, nx) for k, nm in enumerate(order)}

    def replace_case(self, index: int, cfg: dict):
        """Refill slot index with a new case of any grid that fits the slot
        (lbm_batch_replace_case)."""
        p = make_params(cfg, PRECISIONS[self.precision])
        _bcheck(lib().lbm_batch_replace_case(self._b, int(index), ctypes.byref(p)), self._b)
        self.cfgs[index] = dict(cfg)

    def slot_bytes(self, index: int) -> int:
        """Device bytes slot index holds (lbm_batch_slot_bytes)."""
        n = ctypes.c_size_t()
        _bcheck(lib().lbm_batch_slot_bytes(self._b, int(index), ctypes.byref(n)), self._b)
        return n.value

    def autotune(self, trial_steps: int = 20) -> int:
        seg = ctypes.c_int32()
        _bcheck(lib().lbm_batch_autotune(self._b, int(trial_steps), ctypes.byref(seg)), self._b)
        return seg.value

    def autotune_report(self) -> list:
        """The last autotune's candidates (lbm_batch_autotune_report): dicts of
        seg_rows, ms, max_rel_dev and passed, in the order tried."""
        m = 8
        seg, ok, rows = (ctypes.c_int32 * m)(), (ctypes.c_int32 * m)(), ctypes.c_int32()
        ms, dev = (ctypes.c_double * m)(), (ctypes.c_double * m)()
        _bcheck(lib().lbm_batch_autotune_report(self._b, m, seg, ms, dev, ok, ctypes.byref(rows)), self._b)
        return [dict(seg_rows=seg[k], ms=ms[k], max_rel_dev=dev[k], passed=bool(ok[k])) for k in range(rows.value)]

    def info(self) -> dict:
        c, s, w, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _bcheck(lib().lbm_batch_info(self._b, ctypes.byref(c), ctypes.byref(s), ctypes.byref(w), ctypes.byref(n)), self._b)
        return dict(count=c.value, seg_rows=s.value, workgroups=w.value, nodes=n.value)

    def timing_begin(self, max_steps: int):
        _bcheck(lib().lbm_batch_timing_begin(self._b, int(max_steps)), self._b)

    def timing_end(self) -> dict:
        k = len(KERNEL_NAMES)
        ms = (ctypes.c_double * k)()
        n = (ctypes.c_int64 * k)()
        _bcheck(lib().lbm_batch_timing_end(self._b, ms, n), self._b)
        return {KERNEL_NAMES[j]: (ms[j], n[j]) for j in range(k)}

