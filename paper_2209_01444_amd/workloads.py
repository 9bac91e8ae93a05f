"""Seeded synthetic workloads: parameter sets and random inputs.

This module holds numbers and random draws only, none of the method's
arithmetic, so both the GPU library and the CPU oracle can be fed from it.
All parameters are in lattice units (dx = 1, main step dt = 1).

Lattice mapping of the paper's runs: W0 = 1 lu and tau0 = 20 steps, so that
W0^2/tau0 = 0.05 lu^2/step, the lattice diffusivity of the paper's thermal
case (dx = 0.4 W0, dt = 0.008 tau0).  Diffusivities follow the paper's
dimensionless sets: thermal alpha = 4 W0^2/tau0 (Sec. 4.2), thermosolutal
alpha = D = 2 W0^2/tau0 (Sec. 4.4); viscosity from Pr = nu/alpha = 23.1
(Sec. 4.2); two-time-scaling N = 15 (Sec. 4 preamble).
"""
from __future__ import annotations

import math

import numpy as np

# Sec. 4.2: lambda = a1 W0 / d0 with a1 = 0.8839, d0 = 0.1385 W0
LAMBDA_THERMAL = 0.8839 / 0.1385


def pure_diffusion_128(precision: str = "f64") -> dict:
    """Plain method without flow: 128x128 periodic, one seed of radius 8 lu
    at node (64, 64), undercooling 0.55, eps4 = 0.05 at 0 degrees, uniform
    c (C = 1) and uniform theta; thermal coupling (Mc_inf = 0)."""
    return dict(
        name="pure_diffusion_128", nx=128, ny=128, use_c=1, use_t=1, use_ns=0, walls=0, n_sub=1,
        W0=1.0, tau0=20.0, eps4=0.05, orient=0.0, lambda_=LAMBDA_THERMAL, Mcinf=0.0, k=0.15,
        D=0.1, alpha=0.2, nu=0.0, rho0=1.0, u_in=(0.0, 0.0), theta0=-0.55, U0=0.0, C0=1.0,
        c_init_U=0, seed_R=8.0, seed_x=64.0, seed_y=64.0, noise_amp=0.0, precision=precision,
        steps=2000,
    )


def thermosolutal_flow(nx: int = 1024, ny: int = 1024, seed: int = 2, precision: str = "f32",
                       orient: float | None = None, u0: float = 0.01, delta: float = 0.55,
                       eps4: float = 0.05) -> tuple[dict, np.ndarray]:
    """Full thermosolutal coupling with melt flow (the paper's Sec. 4.4 set
    in lattice units): central seed of radius 10 lu with an orientation drawn
    from U[0, pi/4), undercooling 0.55, eps4 = 0.05, uniform inflow u0 from
    the west, unit Gaussian noise (scaled by noise_amp = 1e-3 where |phi| < 0.9).
    Returns (parameters, noise field of shape (ny, nx))."""
    rng = np.random.default_rng(seed)
    drawn = float(rng.uniform(0.0, math.pi / 4))
    noise = rng.standard_normal((ny, nx))
    cfg = dict(
        name=f"thermosolutal_flow_{nx}x{ny}", nx=nx, ny=ny, use_c=1, use_t=1, use_ns=1, walls=1,
        n_sub=15, W0=1.0, tau0=20.0, eps4=eps4, orient=drawn if orient is None else orient,
        lambda_=3.1913, Mcinf=0.5325, k=0.15, D=0.1, alpha=0.1, nu=23.1 * 0.1, rho0=1.0,
        u_in=(u0, 0.0), theta0=-delta, U0=0.0, C0=1.0, c_init_U=1, seed_R=10.0,
        seed_x=float(nx // 2), seed_y=float(ny // 2), noise_amp=1e-3, precision=precision,
        steps=20000,
    )
    return cfg, noise


def batched_sweep(count: int = 256, seed: int = 4,
                  sizes: tuple[int, ...] = (128, 256, 512, 1024)) -> list[tuple[dict, np.ndarray]]:
    """Independent seeds for a batched sweep: size drawn from `sizes` (square
    grids, {128..1024}^2 by default), undercooling ~ U[0.3, 0.65], eps4 ~
    U[0.02, 0.05], orientation ~ U[0, pi/4), u0 ~ U[0, 0.02]; otherwise the
    thermosolutal set."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(list(sizes)))
        delta = float(rng.uniform(0.3, 0.65))
        eps4 = float(rng.uniform(0.02, 0.05))
        orient = float(rng.uniform(0.0, math.pi / 4))
        u0 = float(rng.uniform(0.0, 0.02))
        nseed = int(rng.integers(0, 2**31 - 1))
        cfg, noise = thermosolutal_flow(n, n, seed=nseed, orient=orient, u0=u0, delta=delta,
                                        eps4=eps4)
        cfg["name"] = f"sweep_{i}_{n}"
        cfg["steps"] = 10000
        out.append((cfg, noise))
    return out


def thermal_dendrite(precision: str = "f32", L: int = 512, W0: float = 2.5, flow: bool = False) -> dict:
    """Thermal dendrite into an undercooled melt at the paper's resolution
    (Sec. 4.2): L x L nodes with dx = 0.4 W0 and dt = 0.008 tau0, i.e.
    W0 = 2.5 lu and tau0 = 125 steps (W0^2/tau0 = 0.05 lu^2/step as in the
    coarser mapping); Delta = 0.55, eps4 = 0.05, Mc_inf = 0, uniform c,
    alpha = 4 W0^2/tau0, lambda = 0.8839/0.1385, seed R = 10 dx at the centre,
    zero-gradient (symmetry) walls, no flow.

    flow=True: the melt-flow case of the same section, inflow u_in = W0/tau0
    along +x at the west wall, free outflow east, Pr = nu/alpha = 23.1, 15
    flow sub-steps per main step; the seed sits on the channel's centre
    line ((L - 1)/2) so that the two vertical arms mirror each other."""
    tau0 = W0 * W0 / 0.05
    alpha = 4.0 * W0 * W0 / tau0
    if not flow:
        return dict(
            name=f"thermal_dendrite_{L}", nx=L, ny=L, use_c=1, use_t=1, use_ns=0, walls=1, n_sub=1,
            W0=W0, tau0=tau0, eps4=0.05, orient=0.0, lambda_=LAMBDA_THERMAL, Mcinf=0.0, k=0.15,
            D=0.1, alpha=alpha, nu=0.1, rho0=1.0, u_in=(0.0, 0.0), theta0=-0.55, U0=0.0,
            C0=1.0, seed_R=10.0, seed_x=L / 2.0, seed_y=L / 2.0, noise_amp=0.0, precision=precision)
    c = (L - 1) / 2.0
    return dict(
        name=f"thermal_dendrite_flow_{L}", nx=L, ny=L, use_c=1, use_t=1, use_ns=1, walls=1, n_sub=15,
        W0=W0, tau0=tau0, eps4=0.05, orient=0.0, lambda_=LAMBDA_THERMAL, Mcinf=0.0, k=0.15,
        D=0.1, alpha=alpha, nu=23.1 * alpha, rho0=1.0, u_in=(W0 / tau0, 0.0), theta0=-0.55, U0=0.0,
        C0=1.0, seed_R=10.0, seed_x=c, seed_y=c, noise_amp=0.0, precision=precision)


def solutal_dendrite(precision: str = "f32", L: int = 1000, W0: float = 2.5, flow: bool = False) -> dict:
    """Isothermal alloy dendrite at the paper's resolution (Sec. 4.3):
    L x L nodes, dx = 0.4 W0, dt = 0.02 tau0 (W0 = 2.5 lu, tau0 = 50 steps),
    eps4 = 0.02, theta = 0 (no heat lattice), U0 = -0.55 (uniform initial
    supersaturation), D = 2 W0^2/tau0, Mc_inf = 1, k = 0.15, lambda = 3.191,
    seed R = 10 dx at the centre, zero-gradient walls, no flow.

    flow=True: the melt-flow case of the same section, which states neither
    inflow nor viscosity: the thermal case's inflow W0/tau0 and melt
    (nu = 23.1 x 4 W0^2/tau0, i.e. the same fluid), 15 flow sub-steps, the
    seed on the channel's centre line."""
    tau0 = W0 * W0 / 0.125
    base = dict(
        nx=L, ny=L, use_c=1, use_t=0, walls=1, c_init_U=1, W0=W0, tau0=tau0, eps4=0.02, orient=0.0,
        lambda_=3.191, Mcinf=1.0, k=0.15, D=2.0 * W0 * W0 / tau0, alpha=0.1, rho0=1.0, theta0=0.0, U0=-0.55,
        C0=1.0, seed_R=10.0, noise_amp=0.0, precision=precision)
    if not flow:
        return dict(base, name=f"solutal_dendrite_{L}", use_ns=0, n_sub=1, nu=0.1, u_in=(0.0, 0.0),
                    seed_x=L / 2.0, seed_y=L / 2.0)
    c = (L - 1) / 2.0
    return dict(base, name=f"solutal_dendrite_flow_{L}", use_ns=1, n_sub=15,
                nu=23.1 * 4.0 * W0 * W0 / tau0, u_in=(W0 / tau0, 0.0), seed_x=c, seed_y=c)


def thermosolutal_dendrite(precision: str = "f32", L: int = 2400, W0: float = 2.5, flow: bool = False) -> dict:
    """Thermosolutal dendrite with pure diffusion at the paper's resolution
    (Sec. 4.4): L x L nodes, dx = 0.4 W0 (the section gives no dx; Secs. 4.2
    and 4.3 use 0.4 W0), dt = tau0/55 (W0 = 2.5 lu, tau0 = 55 steps),
    eps4 = 0.02, theta0 = -0.55, U0 = 0, alpha = D = 2 W0^2/tau0 (Le = 1),
    Mc_inf = 0.5325, k = 0.15, lambda = 3.1913 (d0 = 0.2770 W0), seed
    R = 45 dx on the domain's centre, far-field walls (phi = -1, U = 0,
    theta = -0.55), no flow.

    flow=True: the section's melt-flow run, whose flow boundaries are those
    of the earlier sections: inflow W0/tau0 along +x at the west wall, free
    outflow east, free slip north and south, Pr = nu/alpha = 23.1, 15 flow
    sub-steps; phi, C and H take the channel's zero-gradient walls (the
    far-field walls are for the flow lattice off; the inflow carries the
    far-field melt in)."""
    tau0 = 55.0
    c = (L - 1) / 2.0
    alpha = 2.0 * W0 * W0 / tau0
    base = dict(
        nx=L, ny=L, use_c=1, use_t=1, n_sub=1, c_init_U=1, W0=W0, tau0=tau0, eps4=0.02, orient=0.0,
        lambda_=3.1913, Mcinf=0.5325, k=0.15, D=alpha, alpha=alpha, nu=0.1, rho0=1.0, u_in=(0.0, 0.0),
        theta0=-0.55, U0=0.0, C0=1.0, seed_R=45.0, seed_x=c, seed_y=c, noise_amp=0.0, precision=precision)
    if not flow:
        return dict(base, name=f"thermosolutal_dendrite_{L}", use_ns=0, walls=2)
    return dict(base, name=f"thermosolutal_dendrite_flow_{L}", use_ns=1, walls=1, n_sub=15,
                nu=23.1 * alpha, u_in=(W0 / tau0, 0.0))


def cylinder_flow(Re: float, R: int = 20, precision: str = "f32", n_sub: int = 15, length: int = 70,
                  height: int = 40) -> dict:
    """Flow past a stationary diffuse cylinder (Sec. 4.1): domain 70R x 40R
    nodes, cylinder of radius R lu centred at (20R, 20R), interface width
    W0 = 0.5 lu, s2 = 1.25 per flow sub-step (nu = 0.1 lu^2 per sub-step),
    inflow u0 = Re nu / (2R) per sub-step at the west wall, free outflow
    east, free slip north and south.  The paper's mesh is R = 20 (1400 x 800),
    u0 = 0.1 at Re = 40.  Main steps group n_sub flow sub-steps (phi, C and
    theta are frozen), so main-step velocity and viscosity are n_sub times
    the sub-step ones.  length, height: the domain in units of R (the
    cylinder stays 20R from the inlet, on the centre line)."""
    nu_sub = 0.1
    u0 = Re * nu_sub / (2.0 * R)
    return dict(
        name=f"cylinder_Re{Re:g}_R{R}", nx=length * R, ny=height * R, use_c=1, use_t=1, use_ns=1, walls=1,
        n_sub=n_sub, phi_static=1, W0=0.5, tau0=20.0, eps4=0.0, orient=0.0, lambda_=0.0, Mcinf=0.0,
        k=0.15, D=0.1, alpha=0.1, nu=nu_sub * n_sub, rho0=1.0, u_in=(u0 * n_sub, 0.0), theta0=0.0,
        U0=0.0, C0=1.0, seed_R=float(R), seed_x=20.0 * R, seed_y=height * R / 2.0, noise_amp=0.0,
        precision=precision)


def random_macro_tuples(count: int, seed: int = 11) -> np.ndarray:
    """Random macroscopic tuples (phi, C, U, theta, ux, uy, p) for equilibrium
    checks, in physically plausible ranges."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, 7))
    out[:, 0] = rng.uniform(-1.0, 1.0, count)
    out[:, 1] = rng.uniform(0.1, 1.5, count)
    out[:, 2] = rng.uniform(-1.0, 0.5, count)
    out[:, 3] = rng.uniform(-1.0, 0.2, count)
    out[:, 4] = rng.uniform(-0.05, 0.05, count)
    out[:, 5] = rng.uniform(-0.05, 0.05, count)
    out[:, 6] = rng.uniform(-1e-3, 1e-3, count)
    return out
