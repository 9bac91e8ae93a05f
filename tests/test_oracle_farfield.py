"""Pins of the oracle's far-field walls (walls = 2): the outer ring of nodes
holds the far-field liquid of Sec. 4.4 (phi = -1, U = U0, theta = theta0)
by non-equilibrium extrapolation from the inward neighbour.

What fixes them other than the oracle itself: in a uniform liquid a product
of sines that vanishes on the wall ring is an eigenmode of diffusion with
Dirichlet walls, decaying at D (kx^2 + ky^2) with k = pi / (n - 1), at second
order in k; every disturbance relaxes to the far field exactly (zero-gradient
walls keep the mean instead); and the wall ring reports the far-field values
while a dendrite grows inside."""
import math

import numpy as np
import pytest

from oracle import oracle as O

TH0, U0, K = -0.3, -0.2, 0.15


def _liquid_cfg(n, **kw):
    cfg = dict(nx=n, ny=n, use_c=1, use_t=1, use_ns=0, walls=2, c_init_U=1, U0=U0, theta0=TH0,
               lambda_=0.0, k=K, D=0.1, alpha=0.2)
    cfg.update(kw)
    return cfg


def _mode(n):
    k = math.pi / (n - 1)
    x = np.arange(n)
    return np.sin(k * x)[None, :] * np.sin(k * x)[:, None], k


def _start(n, amp=0.05, **kw):
    m, k = _mode(n)
    theta = TH0 + amp * m
    U = U0 + amp * m
    C = 1.0 + (1.0 - K) * U  # C of U at phi = -1
    o = O.Oracle(_liquid_cfg(n, **kw)).set_fields(-np.ones((n, n)), C, theta)
    return o, m, k


def _amp(field, base, m):
    return float(np.sum((field - base) * m) / np.sum(m * m))


def _rate_errors(n, steps):
    o, m, k = _start(n)
    o.step(5)
    f1 = o.fields()
    o.step(steps)
    f2 = o.fields()
    out = {}
    for name, base, diff in (("theta", TH0, 0.2), ("U", U0, 0.1)):
        r = -math.log(_amp(f2[name], base, m) / _amp(f1[name], base, m)) / steps
        out[name] = abs(r / (diff * 2 * k * k) - 1)
    return out


def test_dirichlet_mode_decays_at_the_diffusion_rate():
    """theta (alpha = 0.2) and U (D = 0.1) modes vanishing on the wall ring
    decay at their diffusivities times 2 k^2, within 1% at n = 33 and at
    second order in k."""
    e33 = _rate_errors(33, 200)
    e65 = _rate_errors(65, 800)
    for name in ("theta", "U"):
        assert e33[name] < 1e-2, (name, e33)
        assert e33[name] / e65[name] > 3.0, (name, e33, e65)


def test_relaxes_to_the_far_field_zero_gradient_walls_do_not():
    n = 17
    o, m, _ = _start(n, amp=0.1)
    o.step(3000)
    f = o.fields()
    assert np.max(np.abs(f["theta"] - TH0)) < 1e-9
    assert np.max(np.abs(f["U"] - U0)) < 1e-9
    assert np.max(np.abs(f["phi"] + 1.0)) < 1e-12
    z, _, _ = _start(n, amp=0.1, walls=1)
    z.step(3000)
    fz = z.fields()
    # zero-gradient walls conserve heat: theta tends to the mean, off theta0
    assert np.max(np.abs(fz["theta"] - TH0)) > 1e-2


def test_wall_ring_holds_the_far_field_while_a_seed_grows():
    n = 40
    cfg = _liquid_cfg(n, lambda_=3.0, Mcinf=0.5, theta0=-0.55, U0=0.0, D=0.2, alpha=0.2,
                      seed_R=6.0, seed_x=14.0, seed_y=20.0, eps4=0.02)
    o = O.Oracle(cfg).init_seed()
    o.step(300)
    f = o.fields()
    ring = np.ones((n, n), bool)
    ring[1:-1, 1:-1] = False
    assert np.max(np.abs(f["phi"][ring] + 1.0)) < 1e-12
    assert np.max(np.abs(f["U"][ring])) < 1e-12
    assert np.max(np.abs(f["theta"][ring] + 0.55)) < 1e-12
    # the fields inside did change next to the wall (the seed's heat and
    # solute reach the ring within 300 steps)
    assert np.max(np.abs(f["theta"][1:-1, 1] + 0.55)) > 1e-4
    assert f["phi"][20, 14] > 0.9


@pytest.mark.parametrize("extra", [dict(use_ns=1, n_sub=2), dict(grad_stencil=1), dict(n_sub_t=2),
                                   dict(phi_static=1), dict(walls=3)])
def test_far_field_refusals(extra):
    with pytest.raises(ValueError):
        O.Oracle(dict(_liquid_cfg(20), **extra))
