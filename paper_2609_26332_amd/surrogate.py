"""Learned surrogate of the batched sweep (ctypes binding of include/mlp.h).

An ensemble of MLPs (5 -> 256 -> 256 -> 256 -> 2, GELU, bfloat16 matrix-core
products with FP32 accumulation, FP32 master weights and Adam; all in the HIP
kernels of liblbm_hip.so) maps a case's five sweep inputs (clean contact angle,
adsorption strength, bulk surfactant, capillary number, radius) to its steady
apparent contact angle and detachment time.  The lattice Boltzmann batch stays
the fallback: a case whose ensemble spread of the predicted angle exceeds the
threshold (0.5 degree) is run by the solver instead, so every delivered angle
is either the solver's or agreed on by the ensemble.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lbm as _lbm

# Ranges of the sweep inputs (inputs.sweep_case), mapped to [-1, 1].
INPUT_RANGES = np.array([[30.0, 150.0], [0.0, 0.5], [0.005, 0.05], [0.0, 0.2], [12.0, 60.0]])

_mlp_ready = False


def lib():
    L = _lbm.lib()
    global _mlp_ready
    if not _mlp_ready:
        vp, fp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t
        i32 = ctypes.c_int32
        L.mlp_param_count.restype = i32
        L.mlp_required_bytes.argtypes = [i32, i32, ctypes.POINTER(sz)]
        L.mlp_init.argtypes = [i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
        L.mlp_set_params.argtypes = [vp, i32, fp]
        L.mlp_get_params.argtypes = [vp, i32, fp]
        L.mlp_forward.argtypes = [vp, i32, vp, i32, vp]
        L.mlp_loss_grad.argtypes = [vp, i32, vp, vp, vp, i32, fp, fp]
        L.mlp_train_step.argtypes = [vp, i32, vp, vp, vp, i32, ctypes.c_float, fp]
        L.mlp_train_step_ensemble.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, fp]
        L.mlp_predict_ensemble.argtypes = [vp, vp, i32, vp, vp]
        L.mlp_predict_ensemble_noalloc.argtypes = [vp, i32, vp, i32, vp, vp, vp]
        L.mlp_destroy.argtypes = [vp]
        L.mlp_last_error.argtypes = [vp]
        L.mlp_last_error.restype = ctypes.c_char_p
        for nm in ("mlp_required_bytes", "mlp_init", "mlp_set_params", "mlp_get_params", "mlp_forward",
                   "mlp_loss_grad", "mlp_train_step", "mlp_train_step_ensemble", "mlp_predict_ensemble",
                   "mlp_predict_ensemble_noalloc", "mlp_destroy"):
            getattr(L, nm).restype = ctypes.c_int
        _mlp_ready = True
    return L


EXPORTS = ["mlp_param_count", "mlp_required_bytes", "mlp_init", "mlp_set_params", "mlp_get_params", "mlp_forward",
           "mlp_loss_grad", "mlp_train_step", "mlp_train_step_ensemble", "mlp_predict_ensemble",
           "mlp_predict_ensemble_noalloc", "mlp_destroy", "mlp_last_error"]


def _check(rc, h=None):
    if rc != 0:
        raise _lbm.LbmError(rc, lib().mlp_last_error(h).decode())


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Mlp:
    """An ensemble of `members` networks on the current HIP device."""

    def __init__(self, members: int = 5, max_batch: int = 4096, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch; the surrogate has no CPU fallback")
        L = lib()
        self.members, self.max_batch = members, max_batch
        self.n_params = L.mlp_param_count()
        nb = ctypes.c_size_t()
        _check(L.mlp_required_bytes(members, max_batch, ctypes.byref(nb)))
        self.buffer = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.mlp_init(members, max_batch, _ptr(self.buffer), nb.value, ctypes.c_void_p(self.stream.cuda_stream),
                          ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, member: int, theta: np.ndarray):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.n_params
        _check(lib().mlp_set_params(self._h, member, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self._h)

    def get_params(self, member: int) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().mlp_get_params(self._h, member, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self._h)
        return a

    @staticmethod
    def _dev(a) -> torch.Tensor:
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32) if not isinstance(a, torch.Tensor) else a)
        return t.to(device="cuda", dtype=torch.float32).contiguous()

    def forward(self, member: int, x) -> torch.Tensor:
        x = self._dev(x)
        y = torch.empty((x.shape[0], 2), dtype=torch.float32, device="cuda")
        _check(lib().mlp_forward(self._h, member, _ptr(x), x.shape[0], _ptr(y)), self._h)
        return y

    def loss_grad(self, member: int, x, t, m):
        x, t, m = self._dev(x), self._dev(t), self._dev(m)
        loss = ctypes.c_float()
        g = np.empty(self.n_params, dtype=np.float32)
        _check(lib().mlp_loss_grad(self._h, member, _ptr(x), _ptr(t), _ptr(m), x.shape[0], ctypes.byref(loss),
                                   g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self._h)
        return loss.value, g

    def train_step(self, member: int, x, t, m, lr: float, want_loss: bool = False):
        loss = ctypes.c_float()
        _check(lib().mlp_train_step(self._h, member, _ptr(x), _ptr(t), _ptr(m), x.shape[0], float(lr),
                                    ctypes.byref(loss) if want_loss else None), self._h)
        return loss.value if want_loss else None

    def train_step_ensemble(self, x, t, m, lr: float, want_loss: bool = False):
        """One step of every member, each on its own batch: x [members][n][5],
        t and m [members][n][2], contiguous FP32 device tensors."""
        assert x.shape[0] == self.members and x.is_contiguous() and t.is_contiguous() and m.is_contiguous()
        loss = (ctypes.c_float * self.members)()
        _check(lib().mlp_train_step_ensemble(self._h, _ptr(x), _ptr(t), _ptr(m), x.shape[1], float(lr),
                                             loss if want_loss else None), self._h)
        return list(loss) if want_loss else None

    def predict(self, x):
        x = self._dev(x)
        mean = torch.empty((x.shape[0], 2), dtype=torch.float32, device="cuda")
        sd = torch.empty_like(mean)
        _check(lib().mlp_predict_ensemble(self._h, _ptr(x), x.shape[0], _ptr(mean), _ptr(sd)), self._h)
        return mean, sd


def predict_noalloc(params: torch.Tensor, x: torch.Tensor, mean: torch.Tensor, sd: torch.Tensor, stream=None):
    """mlp_predict_ensemble_noalloc: every argument is a caller-owned device
    tensor (params [members][n_params] FP32, x [n][5], mean and sd [n][2]);
    the call allocates nothing and does not synchronise."""
    st = stream if stream is not None else torch.cuda.current_stream()
    members, n = params.shape[0], x.shape[0]
    for t in (params, x, mean, sd):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    assert mean.shape == (n, 2) and sd.shape == (n, 2) and x.shape == (n, 5)
    _check(lib().mlp_predict_ensemble_noalloc(_ptr(params), members, _ptr(x), n, _ptr(mean), _ptr(sd),
                                              ctypes.c_void_p(st.cuda_stream)))


def glorot_params(seed: int, n_params: int) -> np.ndarray:
    """Initial parameters: W ~ U(-l, l), l = sqrt(6 / (in + out)), b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip([5, 256, 256, 256], [256, 256, 256, 2]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == n_params
    return theta


class Surrogate:
    """Ensemble surrogate with LBM fallback for the sweep.

    fit(): X [n][5] raw inputs, angle [n] (degrees), tau [n] (detachment time
    divided by the cap, in [0, 1]) and tau_mask [n] (0 where the detachment is
    censored by the cap or the case has no wall motion)."""

    def __init__(self, members: int = 5, threshold_deg: float = 0.5, max_batch: int = 4096):
        self.members, self.threshold = members, threshold_deg
        self.net = Mlp(members, max_batch)
        self.angle_mu = 0.0
        self.angle_sd = 1.0

    @staticmethod
    def scale_inputs(X) -> np.ndarray:
        X = np.asarray(X, dtype=np.float64)
        lo, hi = INPUT_RANGES[:, 0], INPUT_RANGES[:, 1]
        return (2.0 * (X - lo) / (hi - lo) - 1.0).astype(np.float32)

    def fit(self, X, angle, tau, tau_mask, epochs: int = 1000, batch: int = 256, lr: float = 2e-3, seed: int = 0,
            schedule: str = "cosine", log=None):
        """The angle output learns the standardised shift from the clean angle,
        theta_app - theta0 (a few degrees), rather than theta_app itself.  A case
        without an angle (NaN: the drop detached) is masked out of that output.

        Each member trains on its own bootstrap resample in its own order; the
        members step together (one mlp_train_step_ensemble per batch).  The
        rate follows a cosine decay from lr to zero over the run
        (schedule="cosine") or stays at lr ("constant")."""
        Xs = self.scale_inputs(X)
        shift = np.asarray(angle, dtype=np.float64) - np.asarray(X, dtype=np.float64)[:, 0]
        has = np.isfinite(shift)
        self.angle_mu, self.angle_sd = float(shift[has].mean()), float(shift[has].std() + 1e-12)
        T = np.stack([np.where(has, (shift - self.angle_mu) / self.angle_sd, 0.0), np.asarray(tau, dtype=np.float64)],
                     1).astype(np.float32)
        Mk = np.stack([has.astype(np.float64), np.asarray(tau_mask, dtype=np.float64)], 1).astype(np.float32)
        n, M = len(angle), self.members
        rngs = [np.random.default_rng(seed * 1000 + k) for k in range(M)]
        boots = [r.integers(0, n, size=n) for r in rngs]   # bootstrap resample per member
        for k in range(M):
            self.net.set_params(k, glorot_params(seed * 1000 + k + 1, self.net.n_params))
        xd, td, md = (torch.as_tensor(np.stack([a[bt] for bt in boots])).cuda() for a in (Xs, T, Mk))
        rows = torch.arange(M, device="cuda")[:, None]
        nb = max(1, n // batch)
        total, it = epochs * nb, 0
        losses = None
        for ep in range(epochs):
            perm = torch.as_tensor(np.stack([r.permutation(n) for r in rngs])).cuda()
            for b in range(nb):
                idx = perm[:, b * batch:(b + 1) * batch]
                last = ep == epochs - 1 and b == nb - 1
                rate = lr * 0.5 * (1.0 + np.cos(np.pi * it / total)) if schedule == "cosine" else lr
                out = self.net.train_step_ensemble(xd[rows, idx].contiguous(), td[rows, idx].contiguous(),
                                                   md[rows, idx].contiguous(), max(rate, 1e-12), want_loss=last)
                if last:
                    losses = out
                it += 1
        if log:
            for k, lo in enumerate(losses):
                log(f"member {k}: final batch loss {lo:.4g}")
        return losses

    def predict(self, X):
        """Ensemble mean and spread of (angle in degrees, tau) per case."""
        mean, sd = self.net.predict(self.scale_inputs(X))
        mean, sd = mean.cpu().numpy().astype(np.float64), sd.cpu().numpy().astype(np.float64)
        angle = np.asarray(X, dtype=np.float64)[:, 0] + mean[:, 0] * self.angle_sd + self.angle_mu
        angle_sd = sd[:, 0] * self.angle_sd
        return angle, angle_sd, mean[:, 1], sd[:, 1]

    def deliver(self, cases, run_lbm):
        """Angles for `cases`: the ensemble mean where its spread is within the
        threshold, else the solver's (run_lbm(list of cases) -> list of angles).
        Returns (angles, used_fallback mask)."""
        from .sweep import sweep_inputs
        X = np.array([sweep_inputs(c) for c in cases])
        angle, spread, _, _ = self.predict(X)
        fb = spread > self.threshold
        out = angle.copy()
        if fb.any():
            sub = [c for c, f in zip(cases, fb) if f]
            out[fb] = np.asarray(run_lbm(sub), dtype=np.float64)
        return out, fb
