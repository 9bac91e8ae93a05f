"""Host-side measurement helpers (no GPU): the cylinder's drag coefficient
and recirculation length, and the workloads' derived parameters."""
import math

import numpy as np
import pytest

from paper_2209_01444_amd import cylinder, workloads


def test_cylinder_workload_matches_the_paper_setup():
    cfg = workloads.cylinder_flow(40, R=20)
    assert (cfg["nx"], cfg["ny"]) == (1400, 800)          # 70 R x 40 R on the paper's mesh
    assert (cfg["seed_x"], cfg["seed_y"]) == (400.0, 400.0)
    u0 = cfg["u_in"][0] / cfg["n_sub"]
    nu = cfg["nu"] / cfg["n_sub"]
    assert u0 == pytest.approx(0.1) and 1.0 / (3.0 * nu + 0.5) == pytest.approx(1.25)
    assert 2 * u0 * cfg["seed_R"] / nu == pytest.approx(40.0)   # Re = 2 u0 R / nu


def test_drag_coefficient_uses_the_sub_step_inflow():
    cfg = workloads.cylinder_flow(20, R=20)
    u0 = 0.05
    red = {"Fx": 2.153 * 1.0 * 20 * u0 * u0, "Fx_solid": 0.0}
    assert cylinder.drag_coefficient(red, cfg) == pytest.approx(2.153)


def test_recirculation_length_from_a_synthetic_wake():
    cfg = workloads.cylinder_flow(20, R=20)
    ny, nx = cfg["ny"], cfg["nx"]
    x = np.arange(nx, dtype=float)
    rear = cfg["seed_x"] + cfg["seed_R"]
    L = 37.3
    row = np.where(x < rear, 0.0, np.tanh((x - rear - L) / 5.0))  # backward flow until rear + L
    ux = np.zeros((ny, nx))
    ux[int(cfg["seed_y"])] = row
    assert cylinder.recirculation_length(ux, cfg) == pytest.approx(L / cfg["seed_R"], abs=1e-3)
    ux[int(cfg["seed_y"])] = 1.0
    assert cylinder.recirculation_length(ux, cfg) == 0.0


def test_dendrite_workloads_use_the_paper_scales():
    th = workloads.thermal_dendrite()
    assert 1.0 / th["W0"] == pytest.approx(0.4) and th["tau0"] * 0.008 == pytest.approx(1.0)  # dx = 0.4 W0, dt = 0.008 tau0
    assert th["alpha"] == pytest.approx(4 * th["W0"] ** 2 / th["tau0"])
    so = workloads.solutal_dendrite()
    assert 1.0 / so["W0"] == pytest.approx(0.4) and so["tau0"] * 0.02 == pytest.approx(1.0) and so["use_t"] == 0
    assert so["D"] == pytest.approx(2 * so["W0"] ** 2 / so["tau0"])


def test_thermal_dendrite_flow_workload():
    # Sec. 4.2 with melt flow: inflow W0/tau0, Pr = nu/alpha = 23.1, seed on
    # the channel's centre line, 15 flow sub-steps with a stable rate
    fl = workloads.thermal_dendrite(flow=True)
    th = workloads.thermal_dendrite()
    assert fl["u_in"] == (pytest.approx(fl["W0"] / fl["tau0"]), 0.0) and fl["use_ns"] == 1
    assert fl["nu"] / fl["alpha"] == pytest.approx(23.1)
    assert fl["seed_x"] == fl["seed_y"] == (fl["nx"] - 1) / 2
    assert all(fl[k] == th[k] for k in ("W0", "tau0", "alpha", "lambda_", "eps4", "theta0", "seed_R"))
    s2 = 1.0 / (3.0 * fl["nu"] / fl["n_sub"] + 0.5)
    assert 0.0 < s2 < 2.0
    assert fl["u_in"][0] / fl["n_sub"] * 3 ** 0.5 < 0.1  # Mach number per sub-step


def test_solutal_dendrite_flow_workload():
    # Sec. 4.3 with melt flow: the section gives no inflow or viscosity; the
    # thermal case's inflow W0/tau0 and melt (nu = 23.1 x 4 W0^2/tau0)
    fl = workloads.solutal_dendrite(flow=True)
    so = workloads.solutal_dendrite()
    assert fl["u_in"] == (pytest.approx(fl["W0"] / fl["tau0"]), 0.0) and fl["use_ns"] == 1
    assert fl["nu"] == pytest.approx(23.1 * 4 * fl["W0"] ** 2 / fl["tau0"])
    assert fl["seed_x"] == fl["seed_y"] == (fl["nx"] - 1) / 2
    assert all(fl[k] == so[k] for k in ("W0", "tau0", "D", "lambda_", "eps4", "U0", "k", "Mcinf", "use_t"))
    assert 0.0 < 1.0 / (3.0 * fl["nu"] / fl["n_sub"] + 0.5) < 2.0
