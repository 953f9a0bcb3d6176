"""Seeded synthetic workloads shared by the HIP path's callers and the oracle.

This module holds configuration dictionaries and seeded random draws only; it
contains none of the method's arithmetic (no derived constants, profiles or
populations).  Both the HIP binding and the oracle map these dictionaries onto
their own parameter structs and derive every lattice constant themselves.

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written out here so that every
draw is reproducible from the seed alone.
"""
from __future__ import annotations

import math

PERIODIC, WALL_WET, NOSLIP, FREESLIP = 0, 1, 2, 3
NONLINEAR, LINEAR = 0, 1
INIT_DROP, INIT_SLAB, INIT_BUBBLE = 0, 1, 2

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator: 64-bit state advanced by the golden-ratio
    increment, output mixed by two xor-shift-multiply rounds."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        """Uniform double in [lo, hi) from the top 53 bits."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / 9007199254740992.0))


def _base(**kw) -> dict:
    cfg = dict(
        sigma_gl0=0.01, eps=4.0, M_phi=0.05, M_psi=0.05,
        Ex=0.5, Pi=1.35, rho_l=1.0, rho_g=1.0, mu_l=0.1, mu_g=0.1,
        gx=0.0, gy=0.0, u_wall_bottom=0.0, u_wall_top=0.0,
        constraint_phi=NONLINEAR, init_kind=INIT_DROP,
        s_f=[1.0, 1.0, 0.0, 1.0, 1.0], s_g=[1.0, 1.0, 1.0, 1.0, 1.0], s_h=[1.0, 1.0, 1.0, 1.0, 1.0],
        beta_sg=0.0, beta_sl=0.0, theta0_deg=90.0,
    )
    cfg.update(kw)
    return cfg


def stationary_drop(nx: int = 64, ny: int = 64, R: float = 16.0, psi_b: float = 0.01, **kw) -> dict:
    """Plain method, 2-D periodic D2Q9 stationary droplet (interface width 4,
    density and viscosity ratio 1, tau_f = 0.8, mobilities 0.05, sigma0 = 0.01)."""
    return _base(nx=nx, ny=ny, bc_bottom=PERIODIC, bc_top=PERIODIC, psi_b=psi_b,
                 x0=nx / 2.0, y0=ny / 2.0, R0=R, **kw)


def static_drop_ratio1000(nx: int = 128, ny: int = 128, R: float = 32.0, psi_b: float = 0.01, **kw) -> dict:
    """Periodic surfactant-laden drop at the density and viscosity ratios of
    the paper's static-drop test (Sec. 4.2: rho_l/rho_g = 1000, mu_l/mu_g =
    100, light phase at unit density with mu_g = 0.1, sigma0 = 0.001; its
    W = 8 beta and k_B T = 5.4 beta are the defaults here), in lattice units:
    interface width 4, mobilities 0.05, nu_g = 0.1 and nu_l = 0.01."""
    cfg = _base(nx=nx, ny=ny, bc_bottom=PERIODIC, bc_top=PERIODIC, psi_b=psi_b,
                sigma_gl0=1e-3, rho_l=1000.0, rho_g=1.0, mu_l=10.0, mu_g=0.1,
                x0=nx / 2.0, y0=ny / 2.0, R0=R)
    cfg.update(kw)
    return cfg


def adsorption_strength(seed: int) -> float:
    """Adsorption strength drawn U[0, 0.5) from the seed (first SplitMix64 draw)."""
    return SplitMix64(seed).uniform(0.0, 0.5)


def sessile_drop(nx: int = 256, ny: int = 128, R: float = 40.0, theta0_deg: float = 60.0,
                 psi_b: float = 0.02, seed: int = 2, **kw) -> dict:
    """Sessile droplet on an adsorbing solid: half-way bounce-back bottom wall
    with wetting and adsorption, free-slip top, initial semicircle centred on
    the wall; the adsorption strength s is drawn from the seed and acts on the
    solid-gas interface (beta_sg = s, beta_sl = 0.01)."""
    s = adsorption_strength(seed)
    cfg = _base(nx=nx, ny=ny, bc_bottom=WALL_WET, bc_top=FREESLIP, psi_b=psi_b,
                theta0_deg=theta0_deg, beta_sg=s, beta_sl=0.01,
                x0=nx / 2.0, y0=-0.5, R0=R)
    cfg.update(kw)
    return cfg


def shear_drop(nx: int = 512, ny: int = 256, R: float = 64.0, Ca: float = 0.1,
               betas=(0.9, 0.01), psi_b: float = 0.01, **kw) -> dict:
    """Droplet under shear: top wall moving at u_w = Ca sigma0 / mu_l, density
    and viscosity ratio 10, theta0 = 90 deg, adsorption on the bottom wall.

    Units of the gas, as in the paper's high-density-ratio tests (Sec. 4):
    rho_g = 1, mu_g = 0.1, rho_l = 10, mu_l = 1, so nu = 0.1 in both phases.
    The same ratios with rho_g = 0.1 are unstable at sigma0 = 0.01 and W = 4:
    the capillary stiffness of phi makes a grid-scale compression mode
    oscillate at about one radian per step in the light phase."""
    mu_l = 1.0
    cfg = _base(nx=nx, ny=ny, bc_bottom=WALL_WET, bc_top=NOSLIP, psi_b=psi_b,
                theta0_deg=90.0, beta_sg=betas[0], beta_sl=betas[1],
                rho_l=10.0, rho_g=1.0, mu_l=mu_l, mu_g=0.1,
                u_wall_top=Ca * 0.01 / mu_l, x0=nx / 4.0, y0=-0.5, R0=R)
    cfg.update(kw)
    return cfg


def spreading_drop(theta0_deg: float = 90.0, nx: int = 200, ny: int = 100, R: float = 35.0,
                   psi_b: float = 0.0, **kw) -> dict:
    """Drop spreading on a wetting wall at the density and viscosity ratios of
    Sec. 4.3 (rho 1000:1, mu 100:1) in lattice units: a semicircle of radius R
    centred on the wall, interface width 6, sigma0 = 0.01, light phase at unit
    density with nu_g = 1, liquid nu_l = 0.1, no-slip top wall."""
    cfg = sessile_drop(nx=nx, ny=ny, R=R, theta0_deg=theta0_deg, psi_b=psi_b)
    cfg.update(eps=6.0, sigma_gl0=0.01, rho_l=1000.0, rho_g=1.0, mu_l=100.0, mu_g=1.0, bc_top=NOSLIP,
               beta_sg=0.0, beta_sl=0.0)
    cfg.update(kw)
    return cfg


def flat_slab(nx: int = 256, ny: int = 4, width: float = 128.0, psi_b: float = 0.0, **kw) -> dict:
    """Flat liquid slab across a periodic box (two planar interfaces)."""
    return _base(nx=nx, ny=ny, bc_bottom=PERIODIC, bc_top=PERIODIC, psi_b=psi_b,
                 init_kind=INIT_SLAB, x0=nx / 2.0, y0=0.0, a=width, R0=0.0, **kw)


def drop3d(n: int = 24, R: float = 7.0, psi_b: float = 0.01, ny: int = 0, nz: int = 0, **kw) -> dict:
    """Three-dimensional periodic stationary drop (stationary-drop physics of
    the 2-D case: interface width 4, sigma0 = 0.01, mobilities 0.05)."""
    ny, nz = ny or n, nz or n
    cfg = _base(nx=n, ny=ny, nz=nz, bc_bottom=PERIODIC, bc_top=PERIODIC, psi_b=psi_b,
                x0=n / 2.0, y0=ny / 2.0, z0=nz / 2.0, R0=R)
    cfg.update(kw)
    return cfg


def sessile3d(nx: int = 32, ny: int = 24, nz: int = 16, R: float = 8.0, theta0_deg: float = 60.0,
              psi_b: float = 0.02, beta_sg: float = 0.3, beta_sl: float = 0.01, **kw) -> dict:
    """Three-dimensional sessile drop on an adsorbing wetting wall at z = -1/2
    (hemisphere of radius R centred on the wall), free-slip top."""
    cfg = _base(nx=nx, ny=ny, nz=nz, bc_bottom=WALL_WET, bc_top=FREESLIP, psi_b=psi_b, theta0_deg=theta0_deg,
                beta_sg=beta_sg, beta_sl=beta_sl, x0=nx / 2.0, y0=ny / 2.0, z0=-0.5, R0=R)
    cfg.update(kw)
    return cfg


def roofline_grid(nx: int = 4096, ny: int = 4096, **kw) -> dict:
    """Large periodic grid (state far beyond the on-die caches) with one big
    drop, stationary-drop physics; used to measure the HBM-bound regime."""
    return stationary_drop(nx=nx, ny=ny, R=ny / 4.0, **kw)


def manufactured(n: int) -> dict:
    """Accuracy test of Sec. 4.1 on [0,1]^2 with n^2 nodes, in lattice units:
    eps = 0.025/dx and sigma0 = 0.001/dx reproduce beta = 0.03 and
    kappa = 9.375e-6/dx^2; the mobility 0.01 becomes 0.01*dt with
    dt = dx^2/0.15; k_BT = 0.162, W = 0.24, lambda_s = 0, linear constraints."""
    dx = 1.0 / n
    dt = dx * dx / 0.15
    return _base(nx=n, ny=n, bc_bottom=PERIODIC, bc_top=PERIODIC, psi_b=0.5, phi_b=1.0,
                 sigma_gl0=0.001 / dx, eps=0.025 / dx, M_phi=0.01 * dt, M_psi=0.01 * dt,
                 kBT=0.162, W=0.24, lambda_s=0.0, constraint_phi=LINEAR, mms=1, mms_dx=dx,
                 x0=0.0, y0=0.0, R0=0.0)


def sweep_case(rng: SplitMix64) -> dict:
    """One case of the batched sweep distribution: theta0 U[30,150] deg,
    adsorption strength U[0,0.5], psi_b U[0.005,0.05], Ca U[0,0.2],
    radius U[12,60]; grid nx = 16*floor(6.4 R/16), ny = nx/2."""
    theta = rng.uniform(30.0, 150.0)
    s = rng.uniform(0.0, 0.5)
    psi_b = rng.uniform(0.005, 0.05)
    Ca = rng.uniform(0.0, 0.2)
    R = rng.uniform(12.0, 60.0)
    nx = max(64, 16 * int(math.floor(6.4 * R / 16.0)))
    ny = nx // 2
    cfg = sessile_drop(nx=nx, ny=ny, R=R, theta0_deg=theta, psi_b=psi_b, seed=0)
    cfg.update(beta_sg=s, beta_sl=0.01, bc_top=NOSLIP, u_wall_top=Ca * 0.01 / 0.1)
    cfg["sweep_inputs"] = dict(theta0_deg=theta, adsorption=s, psi_b=psi_b, Ca=Ca, R=R)
    return cfg


def sweep_batch(seed: int, count: int = 512) -> list:
    rng = SplitMix64(seed)
    return [sweep_case(rng) for _ in range(count)]
