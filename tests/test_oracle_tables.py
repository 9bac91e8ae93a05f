"""Pins of the oracle's single-node pieces against closed forms the paper
prints or that follow from it (Appendix A moment conditions, Appendix B
tables, the 2-D anisotropy identity, the fully-solid node of Sec. 3.4)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.golden_tables import evaluate, read_blocks

TABLES = read_blocks("appendix_b_tables.txt")
C5 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1]], dtype=float)
C9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
              dtype=float)


def test_transform_matrices_as_printed():
    """Appendix B: M for D2Q5 and D2Q9, and the velocity order they imply."""
    np.testing.assert_array_equal(O.m_d2q5(), evaluate(TABLES["d2q5_M"]))
    np.testing.assert_array_equal(O.m_d2q9(), evaluate(TABLES["d2q9_M"]))


@pytest.mark.parametrize("s", [(1.0, 1.3, 1.0), (0.7, 1.538, 1.9), (1.2, 0.4, 0.3)])
def test_d2q5_lambda_equals_printed_matrix(s):
    """Appendix B prints Lambda = M^-1 S M for D2Q5 entry by entry."""
    s0, s1, s2 = s
    L = O.lambda_d2q5(s0, s1, s2)
    np.testing.assert_allclose(L, evaluate(TABLES["d2q5_lambda"], s0=s0, s1=s1, s2=s2),
                               atol=1e-15, rtol=0)


def test_lambda_eigen_conditions():
    """Appendix A: sum_i Lambda_ij = s0 and sum_i c_i Lambda_ij = s1 c_j."""
    L5 = O.lambda_d2q5(0.9, 1.4, 1.1)
    np.testing.assert_allclose(L5.sum(axis=0), 0.9, atol=1e-15)
    np.testing.assert_allclose(C5.T @ L5, 1.4 * C5.T, atol=1e-15)
    s9 = np.array([0.8, 1.2, 1.2, 1.04, 1.04, 1.04, 1.0, 1.0, 1.0])
    L9 = O.lambda_d2q9(s9)
    np.testing.assert_allclose(L9.sum(axis=0), 0.8, atol=1e-14)
    np.testing.assert_allclose(C9.T @ L9, 1.2 * C9.T, atol=1e-14)


def _rng():
    return np.random.default_rng(7)


def test_flow_equilibrium_moments_as_printed():
    """Appendix B: M h^eq = m_h^eq for random (rho0, p, u, v)."""
    M = O.m_d2q9()
    rng = _rng()
    for _ in range(50):
        rho0, p, u, v = rng.uniform(0.5, 1.5), rng.uniform(-1e-2, 1e-2), *rng.uniform(-0.1, 0.1, 2)
        m = M @ O.eq_flow(rho0, p, u, v)
        ref = evaluate(TABLES["d2q9_meq"], rho0=rho0, p=p, u=u, v=v)[0]
        np.testing.assert_allclose(m, ref, atol=1e-15, rtol=1e-14)


def test_flow_force_moments_as_printed():
    M = O.m_d2q9()
    rng = _rng()
    for _ in range(20):
        Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
        m = M @ O.force_flow(Fx, Fy)
        ref = evaluate(TABLES["d2q9_mF"], Fx=Fx, Fy=Fy)[0]
        np.testing.assert_allclose(m, ref, atol=1e-18, rtol=1e-13)


def test_cde_equilibrium_moment_conditions():
    """Appendix A: sum f^eq = A, sum c f^eq = B, sum c c f^eq = C cs^2 I with
    (A, B, C) = (phi, 0, phi) for the phase field, (C, C u, q U) for the
    solute, (H, H u, theta) for the heat lattice (Sec. 3.1-3.3)."""
    rng = _rng()
    cs2 = 1.0 / 3.0
    for _ in range(50):
        phi, C, U, th = rng.uniform(-1, 1), rng.uniform(0.2, 1.5), rng.uniform(-1, 0.5), rng.uniform(-1, 0)
        ux, uy = rng.uniform(-0.05, 0.05, 2)
        for quintic in (0, 1):
            e = O.eq_heat(th, phi, ux, uy, quintic)
            hphi = phi if not quintic else 15 * (phi - 2 * phi**3 / 3 + phi**5 / 5) / 8
            H = th - hphi / 2
            np.testing.assert_allclose(e.sum(), H, atol=1e-15)
            np.testing.assert_allclose(C5.T @ e, [H * ux, H * uy], atol=1e-16)
            np.testing.assert_allclose(np.einsum("i,ia,ib->ab", e, C5, C5), th * cs2 * np.eye(2),
                                       atol=1e-15)
        e = O.eq_phi(phi)
        np.testing.assert_allclose([e.sum(), *(C5.T @ e)], [phi, 0, 0], atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", e, C5, C5), phi * cs2 * np.eye(2),
                                   atol=1e-15)
        e = O.eq_solute(C, phi, U, ux, uy)
        q = (1 - phi) / 2
        np.testing.assert_allclose(e.sum(), C, atol=1e-15)
        np.testing.assert_allclose(C5.T @ e, [C * ux, C * uy], atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", e, C5, C5), q * U * cs2 * np.eye(2),
                                   atol=1e-15)


def test_weights_reproduce_lattice_isotropy():
    """cs^2 = 1/3 (Appendix B): sum w c c = cs^2 I for both lattices."""
    e5 = O.eq_phi(1.0)
    e9 = O.eq_flow(1.0, 0.0, 0.0, 0.0)  # p = 0, u = 0: h^eq = (rho0, 0...) ... only sigma
    assert e5.sum() == pytest.approx(1.0, abs=4e-16)
    np.testing.assert_allclose(e9, [1.0] + [0.0] * 8, atol=1e-16)
    w9 = O.eq_flow(0.0, 1.0 / 3.0, 0.0, 0.0)  # sigma_i = w_i p / cs^2 = w_i, sigma_0 = w0 - 1
    w9[0] += 1.0
    np.testing.assert_allclose(w9.sum(), 1.0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w9, C9, C9), np.eye(2) / 3, atol=1e-15)


@pytest.mark.parametrize("orient", [0.0, 0.3, math.pi / 5])
def test_anisotropy_matches_angle_form(orient):
    """Sec. 2: a_s = 1 - 3e + 4e sum n^4 equals the 2-D textbook form
    1 + e cos 4(psi - orient), and N = |g|^2 a_s grad_g a_s equals
    a_s a_s'(psi) (-g_y, g_x)."""
    rng = _rng()
    eps = 0.05
    for _ in range(100):
        g = rng.normal(size=2) * rng.uniform(1e-3, 1.0)
        a, Nx, Ny = O.anisotropy(eps, orient, *g)
        psi = math.atan2(g[1], g[0])
        a_ref = 1 + eps * math.cos(4 * (psi - orient))
        da = -4 * eps * math.sin(4 * (psi - orient))
        assert a == pytest.approx(a_ref, abs=1e-14)
        np.testing.assert_allclose([Nx, Ny], a_ref * da * np.array([-g[1], g[0]]),
                                   atol=1e-14 * (1 + np.abs(g).max()))


def test_anisotropy_extremes():
    """a_s = 1 + e along the axes and 1 - e along the diagonals (0 deg), and
    N vanishes in both directions."""
    eps = 0.05
    a, Nx, Ny = O.anisotropy(eps, 0.0, -0.3, 0.0)
    assert a == pytest.approx(1 + eps, abs=1e-15) and abs(Nx) < 1e-15 and abs(Ny) < 1e-15
    a, Nx, Ny = O.anisotropy(eps, 0.0, 0.2, 0.2)
    assert a == pytest.approx(1 - eps, abs=1e-15) and abs(Nx) < 1e-15 and abs(Ny) < 1e-15


def test_local_gradient_inverts_its_defining_relation():
    """Sec. 3.1 local scheme: for a gradient g the first moment
    m1 = -g/(3 s1(a_s(g))) - (W0^2/tau0) N(g) must map back to g."""
    cfg = dict(W0=1.0, tau0=20.0, eps4=0.05, orient=0.4, grad_tol=1e-15, grad_max_iter=200)
    rng = _rng()
    for _ in range(50):
        g = rng.normal(size=2) * rng.uniform(1e-3, 0.7)
        a, Nx, Ny = O.anisotropy(0.05, 0.4, *g)
        s1 = 1.0 / (3 * a * a * 0.05 + 0.5)
        m1 = -g / (3 * s1) - 0.05 * np.array([Nx, Ny])
        out = O.local_gradient(cfg, *m1)
        np.testing.assert_allclose(out[:2], g, rtol=1e-12, atol=1e-15)
        assert out[5] < 40


def test_local_gradient_bulk_guard():
    out = O.local_gradient(dict(W0=1.0, tau0=20.0, eps4=0.05), 1e-9, -2e-9)
    np.testing.assert_array_equal(out[:5], [0.0, 0.0, 1.0, 0.0, 0.0])


def test_fully_solid_node_stops_the_flow():
    """Sec. 3.4 with u_s = 0: at phi = 1 the diffuse force [1 - q] f cancels
    the momentum, so the post-collision momentum is exactly zero, and the
    post-collision mass is rho0 (s0 = 1)."""
    rng = _rng()
    cfg = dict(nu=2.31, n_sub=15, rho0=1.0)
    for _ in range(20):
        h = O.eq_flow(1.0, rng.uniform(-1e-4, 1e-4), *rng.uniform(-0.01, 0.01, 2))
        h += rng.normal(size=9) * 1e-4
        post, aux = O.collide_flow(cfg, h, 1.0)
        np.testing.assert_allclose(C9.T @ post, [0.0, 0.0], atol=1e-16)
        assert post.sum() == pytest.approx(1.0, abs=1e-15)
        # the reported velocity is u* + F/2 = u*/2 at phi = 1
        np.testing.assert_allclose(aux[2:], 0.5 * aux[:2], rtol=1e-14)


def test_liquid_node_momentum_is_conserved():
    """At phi = -1 the interface force vanishes: momentum is collision
    invariant (s1 = 1 relaxes towards u = u*)."""
    rng = _rng()
    cfg = dict(nu=0.3, n_sub=1, rho0=1.0)
    h = O.eq_flow(1.0, 1e-4, 0.01, -0.02) + rng.normal(size=9) * 1e-4
    post, aux = O.collide_flow(cfg, h, -1.0)
    np.testing.assert_allclose(C9.T @ post, C9.T @ h, atol=1e-16)
