"""CPU pins of the anti-trapping current and of the hydrodynamic torque.

Anti-trapping current (Sec. 2, J_at): it is there so that the thin-interface
limit of the one-sided alloy model has no spurious solute trapping: the
solid freezes in at k times the liquid concentration at the interface (the
equilibrium partition that Sec. 4.3 checks on the dendrite axis through the
Gibbs-Thomson relation).  For a planar front (no curvature) the remaining
excess partition then falls like the square of the interface Peclet number
Pe = V W0 / D; without the current, or with a wrong sign or scale, it is of
first order (solute is trapped or over-rejected).

The factor 1 + (1 - k) U of the current is c / c_l^0 at the interface
(U's definition, Sec. 2): written for the concentration c, the solute
equation with the current is linear and homogeneous in c for a given phase
field history, so a melt without solute keeps none however the front
moves.  A current whose size does not vanish with c (the factor dropped, or
1 + U in its place) drives solute out of nothing, to negative
concentrations.

Torque and force (Sec. 3.4, Eq. HDforce): the force and torque on the solid
are minus the momentum and the angular momentum (about the centroid of the
solid) that the diffuse fluid-solid force gives the fluid in one collision
(Newton's third law), computed here from the collision itself, population
by population."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import oracle3 as O3

C9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)


def _front_run(dim=2, W0=2.0, U0=-0.8, steps=8000, every=25):
    """Isothermal alloy, planar front across x moving into a supersaturated
    melt (uniform U0) on a strip of the 2-D (D2Q5) or 3-D (D3Q7) oracle;
    returns the front history (t, position, U of the liquid extrapolated to
    the front) and the final U profile along x."""
    nx, ny = 320, (16 if dim == 2 else 4)
    tau0 = W0 * W0 / 0.05
    lam = 3.191
    # D = a2 lambda W0^2 / tau0 with a2 = 0.6267: zero interface kinetics
    D = 0.6267 * lam * W0 * W0 / tau0
    cfg = dict(nx=nx, ny=ny, use_c=1, use_t=0, use_ns=0, walls=1, c_init_U=1, W0=W0, tau0=tau0,
               eps4=0.0, lambda_=lam, Mcinf=1.0, k=0.15, D=D, theta0=0.0, U0=U0)
    x = np.arange(nx)
    x0 = 10 * W0
    prof = np.tanh((x0 - x) / (np.sqrt(2.0) * W0))
    if dim == 2:
        o = O.Oracle(cfg).set_fields(np.repeat(prof[None, :], ny, 0))
        line = lambda a: a[ny // 2]  # noqa: E731
    else:
        cfg3 = {k: v for k, v in cfg.items() if k not in ("use_c", "use_ns")}
        o = O3.Oracle3(dict(cfg3, nz=ny)).set_fields(np.broadcast_to(prof, (ny, ny, nx)))
        line = lambda a: a[ny // 2, ny // 2]  # noqa: E731
    hist = []
    for t in range(0, steps + 1, every):
        if t:
            o.step(every)
        f = o.fields()
        p, U = line(f["phi"]), line(f["U"])
        j = np.where((p[:-1] > 0) & (p[1:] <= 0))[0][-1]
        s = j + p[j] / (p[j] - p[j + 1])
        assert s + 9 * W0 < nx - 1, "front ran to the end of the strip"
        # the liquid's U, fitted 4..9 W0 ahead of the front, extrapolated back to it
        xs = np.arange(int(s + 4 * W0), int(s + 9 * W0))
        c = np.polyfit(xs - s, U[xs], 2)
        hist.append((t, s, np.polyval(c, 0.0)))
    return np.array(hist), line(o.fields()["U"]), cfg, x0


@pytest.mark.parametrize("dim", [2, 3])
def test_planar_alloy_front_does_not_trap_solute(dim):
    hist, U_end, cfg, x0 = _front_run(dim)
    W0, D, k, every = cfg["W0"], cfg["D"], cfg["k"], 25.0
    pe, excess = [], []
    for xs in np.arange(x0 + 6 * W0, hist[-1, 1] - 6 * W0, 2 * W0):
        j = np.searchsorted(hist[:, 1], xs)
        a = (xs - hist[j - 1, 1]) / (hist[j, 1] - hist[j - 1, 1])
        U_i = hist[j - 1, 2] + a * (hist[j, 2] - hist[j - 1, 2])  # liquid side when the front passed xs
        V = (hist[j, 1] - hist[j - 1, 1]) / every
        U_s = U_end[int(round(xs))]  # frozen into the solid (no diffusion there)
        pe.append(V * W0 / D)
        # c_s / (k c_l) - 1 with c_s = k (1 + (1-k) U_s) and c_l = 1 + (1-k) U_i
        excess.append((1 + (1 - k) * U_s) / (1 + (1 - k) * U_i) - 1)
    pe, excess = np.array(pe), np.array(excess)
    print("Pe", np.round(pe, 3), "\nexcess", np.round(excess, 4))
    assert len(pe) >= 8 and pe.min() < 0.12 and pe.max() > 0.3, "front too slow or too fast to test"
    low = pe <= 0.2
    assert low.sum() >= 3
    # second order in Pe where the thin-interface limit applies ...
    assert np.all(np.abs(excess[low]) <= 5.0 * pe[low] ** 2), (pe[low], excess[low])
    # ... and no first-order part: the fitted exponent over the samples is about 2
    slope = np.polyfit(np.log(pe), np.log(np.abs(excess)), 1)[0]
    print("exponent", slope)
    assert 1.7 <= slope <= 2.5


def _solute_free_front(dim, W0, theta0=-0.1, travel_W0=15.0):
    """Largest |C| left in a melt that holds no solute (C = 0) after a planar
    front, driven by a uniform undercooling theta0 alone (Mc_inf = 0, so the
    phase field does not see C), has swept travel_W0 interface widths of it;
    lattice units scale with W0 (tau0 = W0^2 / 0.05, D = 0.05 W0)."""
    tau0 = W0 * W0 / 0.05
    nx, ny = int(64 * W0), 4
    x0 = 8 * W0
    prof = np.tanh((x0 - np.arange(nx)) / (np.sqrt(2.0) * W0))
    cfg = dict(nx=nx, ny=ny, use_t=0, walls=1, W0=W0, tau0=tau0, eps4=0.0, lambda_=3.191,
               Mcinf=0.0, k=0.15, D=0.05 * W0, theta0=theta0)
    if dim == 2:
        o = O.Oracle(dict(cfg, use_c=1, use_ns=0)).set_fields(np.repeat(prof[None, :], ny, 0),
                                                             np.zeros((ny, nx)))
        line = lambda a: a[ny // 2]  # noqa: E731
    else:
        o = O3.Oracle3(dict(cfg, nz=ny)).set_fields(
            np.ascontiguousarray(np.broadcast_to(prof, (ny, ny, nx))), np.zeros((ny, ny, nx)))
        line = lambda a: a[ny // 2, ny // 2]  # noqa: E731
    s = x0
    while s < x0 + travel_W0 * W0:
        o.step(int(tau0))
        p = line(o.fields()["phi"])
        j = np.where((p[:-1] > 0) & (p[1:] <= 0))[0][-1]
        s = j + p[j] / (p[j] - p[j + 1])
        assert s + 8 * W0 < nx, "front ran to the end of the strip"
    return np.abs(o.fields()["C"]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_solute_free_melt_stays_free_under_a_moving_front(dim):
    """C = 0 is a solution of the solute equation with the anti-trapping
    current for any front motion; the lattice keeps it up to a
    discretisation error that falls faster than dx/W0 (C in units of c_l^0,
    the equilibrium liquid concentration)."""
    coarse, fine = (_solute_free_front(dim, W0) for W0 in (2.0, 4.0))
    print(f"max |C|: {coarse:.3e} at W0 = 2 lu, {fine:.3e} at W0 = 4 lu")
    assert coarse < 1e-2 and fine < 2.5e-3
    assert coarse / fine > 3.0


def _body_and_flow(nx=44, ny=38):
    """An off-centre, tilted elliptical solid body with a diffuse rim, in a
    stream that also rotates about a point away from the body."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    cx, cy, a, b, ang = 17.3, 21.6, 8.0, 4.5, 0.5
    xr = (x - cx) * np.cos(ang) + (y - cy) * np.sin(ang)
    yr = -(x - cx) * np.sin(ang) + (y - cy) * np.cos(ang)
    d = (np.sqrt((xr / a) ** 2 + (yr / b) ** 2) - 1.0) * min(a, b)
    phi = -np.tanh(d / np.sqrt(2.0))
    om, px, py = 2e-4, 25.0, 12.0
    ux = 0.01 - om * (y - py)
    uy = 0.003 + om * (x - px)
    return phi, ux, uy


@pytest.mark.parametrize("n_sub", [1, 15])
def test_force_and_torque_balance_the_fluid_momentum(n_sub):
    phi, ux, uy = _body_and_flow()
    ny, nx = phi.shape
    cfg = dict(nx=nx, ny=ny, use_ns=1, n_sub=n_sub, nu=0.3 * n_sub, walls=0, lambda_=0.0, phi_static=1)
    o = O.Oracle(cfg).set_fields(phi, None, None, ux * n_sub, uy * n_sub)
    h = o.pops(3)  # pre-collision flow populations
    dm = np.zeros((ny, nx, 2))
    for j in range(ny):
        for i in range(nx):
            post, _ = O.collide_flow(cfg, h[:, j, i].copy(), phi[j, i])
            dm[j, i] = C9.T @ (post - h[:, j, i])
    w = 0.5 * (1.0 + phi)  # solid fraction of a node
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    xs, ys = (w * x).sum() / w.sum(), (w * y).sum() / w.sum()
    dP = dm.sum(axis=(0, 1))
    dL = ((x - xs) * dm[..., 1] - (y - ys) * dm[..., 0]).sum()
    r = o.reduce()
    print(f"F = ({r['Fx']:.6e}, {r['Fy']:.6e}), T = {r['torque']:.6e}; dP = {dP}, dL = {dL:.6e}")
    assert abs(dL) > 1e-3 * np.abs(dP).max() * nx, "torque too small to test"
    np.testing.assert_allclose([r["Fx"], r["Fy"]], -dP, rtol=1e-11)
    assert r["torque"] == pytest.approx(-dL, rel=1e-11)
    np.testing.assert_allclose(r["centroid"], [xs, ys], rtol=1e-13)
