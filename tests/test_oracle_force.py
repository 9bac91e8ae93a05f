"""Pins of the oracle's external force (Sec. 3.4): a body force F enters the
velocity u* = sum c h + F/2, the first-order forcing as F + [1 - q] f, and,
through the adjustable parameter varphi, the second-order forcing
(uF + Fu) and the pressure term varphi K u.F with
K = 2 (s2 - 3 s4 + s2 s4) / (9 s2 s4).

What fixes them other than the oracle itself: the population form of the
forcing against the moment vector that Appendix B prints; a liquid under a
uniform force accelerates by exactly F per main step; in a uniform, partly
solid medium the force balances the diffuse drag at u = F (1/(1 - q) - 1/2)
per sub-step, and the pressure the scheme reports is stationary there for
any varphi (the K term makes the forced equilibrium a fixed point; without
it the pressure drifts linearly); a force-driven channel between diffuse
solid bands has the Stokes curvature u'' = -F/nu in its liquid core."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.golden_tables import read_blocks, evaluate

TABLES = read_blocks("appendix_b_tables.txt")


def test_forcing_populations_match_the_printed_moments():
    M = O.m_d2q9()
    rng = np.random.default_rng(5)
    for _ in range(20):
        Fx, Fy, fx, fy, u, v = rng.uniform(-1e-2, 1e-2, 6)
        vp = rng.uniform(-2.0, 2.0)
        m = M @ O.force_flow_full(Fx + fx, Fy + fy, Fx, Fy, u, v, vp)
        ref = evaluate(TABLES["d2q9_mF_full"], Fx=Fx, Fy=Fy, fx=fx, fy=fy, u=u, v=v, vp=vp)[0]
        np.testing.assert_allclose(m, ref, atol=1e-17, rtol=1e-12)


@pytest.mark.parametrize("varphi", [0.0, 1.0])
def test_liquid_accelerates_by_the_force(varphi):
    """phi = -1 everywhere (no diffuse drag), periodic, three flow sub-steps
    per main step: u grows by F per main step exactly."""
    F = (2e-4, -1e-4)
    cfg = dict(nx=6, ny=5, use_ns=1, n_sub=3, nu=0.3, force_x=F[0], force_y=F[1], varphi=varphi,
               lambda_=0.0)
    o = O.Oracle(cfg).set_fields(-np.ones((5, 6)), None, None, np.full((5, 6), 0.01), np.zeros((5, 6)))
    f0 = o.fields()
    o.step(10)
    f = o.fields()
    np.testing.assert_allclose(f["ux"] - f0["ux"], 10 * F[0], rtol=1e-11)
    np.testing.assert_allclose(f["uy"] - f0["uy"], 10 * F[1], rtol=1e-11)


@pytest.mark.parametrize("phi", [0.0, 0.6])
@pytest.mark.parametrize("varphi", [0.0, 1.0, 2.0])
def test_forced_porous_medium_is_steady(phi, varphi):
    """Uniform phi (a partly solid medium), uniform F, n_sub = 2: the force
    balances the diffuse drag, F + [1 - q] f = 0 with f = -u*, so
    u = N (F/N^2) (1/(1 - q) - 1/2) in main-step units, and the reported
    pressure does not move."""
    n, F = 2, (1e-4, 5e-5)
    cfg = dict(nx=5, ny=4, use_ns=1, n_sub=n, nu=0.5, force_x=F[0], force_y=F[1], varphi=varphi,
               lambda_=0.0, phi_static=1)
    o = O.Oracle(cfg).set_fields(np.full((4, 5), phi))
    o.step(200)
    f1 = o.fields()
    o.step(200)
    f2 = o.fields()
    solid = 0.5 * (1.0 + phi)
    for k, Fk in (("ux", F[0]), ("uy", F[1])):
        np.testing.assert_allclose(f2[k], n * (Fk / n**2) * (1.0 / solid - 0.5), rtol=1e-10)
    scale = (n * F[0]) ** 2
    assert np.abs(f2["p"] - f1["p"]).max() < 1e-12 * scale + 1e-20


def test_force_driven_channel_has_the_stokes_curvature():
    """Periodic channel between diffuse solid bands (phi = +1 outside
    |y - yc| < H/2, interface width W0 = 1), driven along x: in the liquid
    core the steady profile satisfies nu u'' + F = 0, and the peak velocity
    approaches the sharp-wall value F H^2 / (8 nu) as H grows (the diffuse
    drag shifts the effective wall into the liquid by a fixed distance)."""
    def run(H, nu=0.1, F=1e-6):
        ny, nx = H + 24, 4
        y = np.arange(ny)
        yc = (ny - 1) / 2
        phi = np.tanh((np.abs(y - yc) - H / 2) / math.sqrt(2.0))
        cfg = dict(nx=nx, ny=ny, use_ns=1, n_sub=1, nu=nu, phi_static=1, W0=1.0, force_x=F,
                   force_y=0.0, varphi=1.0, lambda_=0.0)
        o = O.Oracle(cfg).set_fields(np.repeat(phi[:, None], nx, 1))
        o.step(int(8 * H * H / nu))
        u = o.fields()["ux"][:, 0]
        c = int(yc)
        curv = -nu * (u[c + 1] - 2 * u[c] + u[c - 1]) / F
        return curv, u.max() / (F * H * H / (8 * nu)) - 1
    c20, e20 = run(20)
    c40, e40 = run(40)
    assert abs(c40 - 1) < 1e-3 and abs(c20 - 1) < 1e-2
    assert e20 < 0 and e40 < 0 and abs(e40) < 0.6 * abs(e20)
