"""The accuracy test of Sec. 4.1 (Table 1) on the GPU: the manufactured mode
of the C ABI (lbm_params.mms_dx) prescribes the velocity (0.05, -0.03) and
adds the test's sources.  First the mode against the FP64 oracle's own
manufactured mode on a 32^2 grid, then the relative L2 errors at t = 5 from
dx = 1/32 to 1/512 under diffusive scaling (dt = dx^2 / 0.15) against the
exact solution: second order, and the phi and psi sums conserved to round-off.
Table 1's magnitudes depend on eta and the non-hydrodynamic rates, which the
paper does not give; its orders (1.994 to 1.99999) are what is compared."""
import math

import numpy as np
import pytest

import oracle
from paper_2609_26332_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2609_26332_amd import lbm as binding

    return binding


def exact(n, t):
    """phi^e, psi^e of Sec. 4.1 at the nodes x = i/n, y = j/n ([ny][nx])."""
    y, x = np.mgrid[0:n, 0:n] / n
    X, Y = 2 * np.pi * (x - 0.05 * t), 2 * np.pi * (y + 0.03 * t)
    return 0.5 * np.exp(-t) * np.sin(X) * np.cos(Y), 0.5 + 0.05 * np.exp(-2 * t) * np.cos(X) * np.sin(Y)


def start(lbm, n):
    cfg = inputs.manufactured(n)
    g = lbm.Sim(cfg, "fp64")
    dx = 1.0 / n
    dt = dx * dx / 0.15
    ph, ps = exact(n, 0.0)
    g.load_fields(ph, ps, np.full_like(ph, 0.05 * dt / dx), np.full_like(ph, -0.03 * dt / dx))
    return cfg, g, dt


def test_manufactured_mode_matches_the_oracle(lbm):
    """The GPU's manufactured mode (the row sweep with the prescribed velocity
    and the sources) against the oracle's, 32^2, FP64, after 1, 20 and 300
    steps: every field within 1e-10 of the oracle's (relative to its largest
    value)."""
    cfg, g, _ = start(lbm, 32)
    assert g.step_kernel()["kernel"] == "k_step"
    o = oracle.OracleSim(cfg)
    done = 0
    for k in (1, 20, 300):
        g.step(k - done)
        o.step(k - done)
        done = k
        gf, of = g.fields(["phi", "psi", "mu_phi", "mu_psi"]), o.fields(["phi", "psi", "mu_phi", "mu_psi"])
        for nm in gf:
            err = np.abs(gf[nm] - of[nm]).max() / np.abs(of[nm]).max()
            assert err < 1e-10, (k, nm, err)


def test_manufactured_second_order_to_dx_1_512(lbm):
    """Sec. 4.1, Table 1: relative L2 errors of phi and psi at t = 5 for dx =
    1/32 .. 1/512 fall with order 2 (each successive order within [1.95,
    2.05]); sum psi is conserved to 1e-13 of itself and sum phi (zero) to
    1e-12 of sum |phi| at the start (round-off accumulating over up to 2e5 steps)."""
    errs = []
    for n in (32, 64, 128, 256, 512):
        cfg, g, dt = start(lbm, n)
        steps = int(round(5.0 / dt))
        i0 = g.invariants()
        ph0 = np.abs(g.fields(["phi"])["phi"]).sum()
        g.step(steps)
        i1 = g.invariants()
        assert i1["nonfinite"] == 0
        f = g.fields(["phi", "psi"])
        pe, se = exact(n, steps * dt)
        e = (math.sqrt(((f["phi"] - pe) ** 2).sum() / (pe ** 2).sum()),
             math.sqrt(((f["psi"] - se) ** 2).sum() / (se ** 2).sum()))
        errs.append(e)
        print(f"dx = 1/{n}: {steps} steps, E2 phi {e[0]:.5e}, E2 psi {e[1]:.5e}, "
              f"sum psi drift {(i1['mass_psi'] - i0['mass_psi']) / i0['mass_psi']:.2e}, "
              f"sum phi drift {i1['sum_phi'] - i0['sum_phi']:.2e}", flush=True)
        assert abs(i1["mass_psi"] - i0["mass_psi"]) / i0["mass_psi"] < 1e-13
        assert abs(i1["sum_phi"] - i0["sum_phi"]) < 1e-12 * ph0
    for k in range(len(errs) - 1):
        for c in range(2):
            order = math.log(errs[k][c] / errs[k + 1][c]) / math.log(2.0)
            print(f"order {k} field {c}: {order:.5f}", flush=True)
            assert 1.95 < order < 2.05, (k, c, order, errs)
