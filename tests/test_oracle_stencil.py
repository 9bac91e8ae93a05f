"""Pins of the stencil-gradient ablation in the oracle (grad_stencil = 1):
grad phi from the isotropic nine-point difference of the node values of phi
instead of the local scheme of Sec. 3.1.  The stencil is exact on
quadratic fields and reduces to the central difference along an axis; the
phase-field equation with it keeps a planar front stationary at its
anisotropic width to second order, like the local scheme."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_dynamics import _planar


def test_stencil_is_exact_on_quadratics():
    rng = np.random.default_rng(5)
    a, b, c, d, e, f = rng.normal(size=6)
    ny, nx = 9, 11
    Y, X = np.mgrid[0:ny, 0:nx].astype(float)
    phi = a + b * X + c * Y + d * X * X + e * X * Y + f * Y * Y
    for (x, y) in [(1, 1), (5, 4), (9, 7), (3, 6)]:
        g = O.stencil_gradient({"walls": 1}, phi, x, y)
        np.testing.assert_allclose(g, [b + 2 * d * x + e * y, c + e * x + 2 * f * y], rtol=0, atol=1e-12)


def test_stencil_along_an_axis_is_the_central_difference_and_wraps():
    nx, ny = 12, 5
    k = 2 * math.pi / nx
    x = np.arange(nx)
    phi = np.repeat(np.sin(k * x)[None, :], ny, 0)
    for xx in (0, 5, nx - 1):  # wraps at both ends
        g = O.stencil_gradient({"walls": 0}, phi, xx, 2)
        exact = (math.sin(k * (xx + 1)) - math.sin(k * (xx - 1))) / 2
        assert g[0] == pytest.approx(exact, abs=1e-14)
        assert g[1] == pytest.approx(0.0, abs=1e-14)
    # the same field along y: the stencil is symmetric in its two axes
    g = O.stencil_gradient({"walls": 0}, phi.T.copy(), 2, 5)
    assert g[1] == pytest.approx((math.sin(k * 6) - math.sin(k * 4)) / 2, abs=1e-14)


@pytest.mark.parametrize("angle", [0, 45])
def test_planar_front_is_stationary_with_the_stencil_gradient(angle):
    """lambda = 0: -tanh(s/(sqrt(2) W0 a_s)) stays the stationary profile
    with the stencil gradient too, at second order in dx/W0."""
    errs = [_planar(angle, W0, grad_stencil=1) for W0 in (1.0, 2.0, 4.0)]
    assert errs[0] / errs[1] > 3.0
    assert errs[1] / errs[2] > 2.0
    assert errs[2] < 5e-3


def test_stencil_run_keeps_fourfold_symmetry_and_differs_from_local():
    cfg = dict(nx=48, ny=48, use_c=1, use_t=1, use_ns=0, W0=1.0, tau0=20.0, eps4=0.05,
               lambda_=0.8839 / 0.1385, alpha=0.2, theta0=-0.55, seed_R=6.0, seed_x=24.0, seed_y=24.0)
    st = O.Oracle(dict(cfg, grad_stencil=1)).init_seed().step(150)
    lo = O.Oracle(cfg).init_seed().step(150)
    a = st.fields()["phi"]
    np.testing.assert_allclose(a, a.T, atol=1e-12, rtol=0)
    mirror = np.roll(a[:, ::-1], 1, axis=1)  # x -> 48 - x about the seed column
    np.testing.assert_allclose(a, mirror, atol=1e-12, rtol=0)
    # both schemes grow the same seed; they differ at the discretisation level
    d = np.abs(a - lo.fields()["phi"]).max()
    assert 1e-6 < d < 0.2
