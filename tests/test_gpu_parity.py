"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: FP64 GPU vs oracle <= 1e-10 relative L-inf per field; FP32 GPU vs
oracle <= 1e-4 relative L-inf per field and tip velocity within 0.5% after
2000 steps; equilibria bit-exact.  Relative L-inf error of a field is
max|a - b| / max|b| (absolute when the reference field is zero)."""
import ctypes
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2209_01444_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "C", "U", "theta", "ux", "uy", "p")


def _say(msg):
    print(msg, flush=True)


def rel_linf(a, b):
    s = np.abs(b).max()
    d = np.abs(a - b).max()
    return d / s if s > 0 else d


@pytest.fixture(scope="module")
def dlb():
    from paper_2209_01444_amd import dlb as mod
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mod.load_library()
    return mod


def compare(gf, of, tol, fields=FIELDS, label=""):
    errs = {f: rel_linf(gf[f], of[f]) for f in fields}
    _say(f"  {label} errors: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{label}: fields above {tol}: {bad}"
    return errs


# ---------------------------------------------------------------------------
# Equilibria: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("quintic", [0, 1])
def test_equilibria_bit_exact(dlb, quintic):
    _say(f"case: equilibria bit-exact, quintic={quintic}")
    m = W.random_macro_tuples(10000, seed=11 + quintic)
    rho0 = np.random.default_rng(3).uniform(0.5, 1.5, len(m))
    macros = np.column_stack([m, rho0])
    gpu = dlb.equilibria(macros, quintic)
    ref = np.empty_like(gpu)
    for i, (phi, C, U, th, ux, uy, p) in enumerate(m):
        ref[i, 0:5] = O.eq_phi(phi)
        ref[i, 5:10] = O.eq_solute(C, phi, U, ux, uy)
        ref[i, 10:15] = O.eq_heat(th, phi, ux, uy, quintic)
        ref[i, 15:24] = O.eq_flow(rho0[i], p, ux, uy)
    mism = np.argwhere(gpu != ref)
    assert mism.size == 0, f"{len(mism)} slots differ, first {mism[:5]}"


# ---------------------------------------------------------------------------
# Pure diffusion, 128^2 periodic (no flow), 2000 steps
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def pure_oracle():
    cfg = W.pure_diffusion_128()
    o = O.Oracle(cfg).init_seed()
    snaps, tips = {}, {}
    for t in (500, 1900, 2000):
        o.step(t - o.step_count)
        snaps[t] = o.fields()
        tips[t] = o.reduce()["tip_s"]
    return snaps, tips


def _run_gpu_pure(dlb, precision):
    cfg = W.pure_diffusion_128(precision)
    s = dlb.Solver(cfg).init_seed()
    r0 = s.reduce()
    snaps, tips, sums = {}, {}, [(r0["sum_C"], r0["sum_H"])]
    for t in (500, 1900, 2000):
        s.step(t - s.step_count)
        snaps[t] = s.fields()
        r = s.reduce()
        tips[t] = r["tip_s"]
        sums.append((r["sum_C"], r["sum_H"]))
    return snaps, tips, np.array(sums)


def test_pure_diffusion_f64_parity(dlb, pure_oracle):
    _say("case: pure diffusion 128x128 periodic FP64, 2000 steps")
    osn, otips = pure_oracle
    gsn, gtips, sums = _run_gpu_pure(dlb, "f64")
    for t in (500, 2000):
        compare(gsn[t], osn[t], 1e-10, fields=("phi", "C", "U", "theta"), label=f"f64 t={t}")
    np.testing.assert_allclose(gtips[2000], otips[2000], rtol=0, atol=1e-9)
    rel = np.abs(sums - sums[0]) / np.abs(sums[0])
    assert rel.max() < 1e-12  # solute and heat conservation on the GPU


@pytest.mark.parametrize("precision,tol", [("f32m", 1e-4), ("f32", 1e-4)])
def test_pure_diffusion_f32_parity(dlb, pure_oracle, precision, tol):
    """FP32 storage at the FP32 bar of 1e-4.  Both modes compute the
    phi/C/theta step in FP64 (f32m also the flow, which is off here): with
    FP32 arithmetic there the supersaturation U, whose 1/(1+k-(1-k)phi)
    factor magnifies phi errors sevenfold in the solid, missed it (1.4e-4)."""
    _say(f"case: pure diffusion 128x128 periodic {precision}, 2000 steps")
    osn, otips = pure_oracle
    gsn, gtips, sums = _run_gpu_pure(dlb, precision)
    for t in (500, 2000):
        compare(gsn[t], osn[t], tol, fields=("phi", "C", "U", "theta"), label=f"{precision} t={t}")
    v_gpu = (gtips[2000] - gtips[1900]) / 100
    v_orc = (otips[2000] - otips[1900]) / 100
    _say(f"  v_tip gpu {v_gpu} oracle {v_orc}")
    np.testing.assert_allclose(v_gpu, v_orc, rtol=5e-3)
    rel = np.abs(sums - sums[0]) / np.abs(sums[0])
    _say(f"  FP32 conservation drift {rel.max():.2e}")
    assert rel.max() < 1e-5


def test_pure_diffusion_fourfold_symmetry_on_gpu(dlb):
    _say("case: fourfold symmetry FP64 on the GPU")
    s = dlb.Solver(W.pure_diffusion_128("f64")).init_seed().step(300)
    f = s.fields()
    for name in ("phi", "C", "theta"):
        a = f[name]
        np.testing.assert_allclose(np.roll(a[:, ::-1], 1, axis=1), a, atol=1e-12, rtol=0)
        np.testing.assert_allclose(a.T, a, atol=1e-12, rtol=0)


# ---------------------------------------------------------------------------
# Thermosolutal coupling with flow, channel walls, ragged grid
# ---------------------------------------------------------------------------

def _flow_case(nx, ny, precision, seed=2):
    cfg, noise = W.thermosolutal_flow(nx, ny, seed=seed, precision=precision)
    return cfg, noise


@pytest.mark.parametrize("precision,tol,steps", [("f64", 1e-10, 300), ("f32", 1e-4, 300),
                                                  ("f32m", 1e-4, 300)])
def test_thermosolutal_flow_parity_ragged(dlb, precision, tol, steps):
    nx, ny = 96, 78  # two and a half tiles in x, ragged in y
    _say(f"case: thermosolutal flow {nx}x{ny} channel {precision}, {steps} steps")
    cfg, noise = _flow_case(nx, ny, precision)
    o = O.Oracle(cfg).init_seed(noise)
    s = dlb.Solver(cfg).init_seed(noise)
    for t in (1, 50, steps):
        o.step(t - o.step_count)
        s.step(t - s.step_count)
        compare(s.fields(), o.fields(), tol, label=f"{precision} t={t}")
    ro, rg = o.reduce(), s.reduce()
    for key in ("sum_C", "sum_H", "solid_fraction", "Fx", "Fy"):
        assert rg[key] == pytest.approx(ro[key], rel=max(tol, 1e-12) * 10, abs=1e-12), key


@pytest.mark.parametrize("case,precision,tol", [("channel", "f64", 1e-10), ("channel", "f32", 1e-4),
                                                ("periodic", "f64", 1e-10), ("periodic", "f32m", 1e-4)])
def test_external_force_parity(dlb, case, precision, tol):
    """External body force with varphi (Sec. 3.4): the coupled flow case with
    F = (2e-5, -1e-5) lu per main step^2 and varphi = 1 against the oracle,
    every field including the pressure; each flow sub-step is one launch."""
    nx, ny = 70, 54
    _say(f"case: external force {case} {nx}x{ny} {precision}")
    cfg, noise = _flow_case(nx, ny, precision)
    cfg = dict(cfg, force_x=2e-5, force_y=-1e-5, varphi=1.0, walls=1 if case == "channel" else 0)
    o = O.Oracle(cfg).init_seed(noise)
    s = dlb.Solver(cfg).init_seed(noise)
    for t in (1, 40, 200):
        o.step(t - o.step_count)
        s.step(t - s.step_count)
        compare(s.fields(), o.fields(), tol, label=f"force {case} {precision} t={t}")
    ro, rg = o.reduce(), s.reduce()
    for key in ("Fx", "Fy"):
        assert rg[key] == pytest.approx(ro[key], rel=max(tol, 1e-12) * 10, abs=1e-12), key


def test_force_driven_channel_on_gpu(dlb):
    """A channel between diffuse solid bands (H = 100, W0 = 1) driven by a
    body force, FP32, 15 flow sub-steps per main step: in the liquid core
    the steady profile has the Stokes curvature nu u'' = -F."""
    _say("case: force-driven channel 16x124, FP32, N_sub = 15")
    H, nx, n = 100, 16, 15
    ny = H + 24
    nu_sub, F_sub = 0.1, 1e-7
    y = np.arange(ny)
    yc = (ny - 1) / 2
    phi = np.repeat(np.tanh((np.abs(y - yc) - H / 2) / np.sqrt(2.0))[:, None], nx, 1)
    cfg = dict(nx=nx, ny=ny, use_ns=1, n_sub=n, nu=nu_sub * n, phi_static=1, W0=1.0, walls=0,
               force_x=F_sub * n * n, force_y=0.0, varphi=1.0, lambda_=0.0, precision="f32")
    s = dlb.Solver(cfg).set_fields(phi)
    s.step(8000)
    u = s.fields()["ux"][:, 3] / n  # per sub-step
    c = int(yc)
    curv = -nu_sub * (u[c + 1] - 2 * u[c] + u[c - 1]) / F_sub
    _say(f"  -nu u''/F = {curv:.5f}, u_max = {u.max():.4e} (sharp walls {F_sub * H * H / (8 * nu_sub):.4e})")
    assert abs(curv - 1) < 2e-3


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_quintic_interpolation_parity(dlb, precision, tol):
    """The quintic h(phi) = 15(phi - 2 phi^3/3 + phi^5/5)/8 that Sec. 2
    offers beside h = phi, in the heat equilibrium and in theta = H +
    h(phi)/2, on the coupled channel case: GPU against the oracle."""
    nx, ny = 64, 48
    _say(f"case: quintic h(phi), thermosolutal flow {nx}x{ny} channel {precision}, 200 steps")
    cfg, noise = _flow_case(nx, ny, precision)
    cfg = dict(cfg, h_quintic=1)
    o = O.Oracle(cfg).init_seed(noise).step(200)
    s = dlb.Solver(cfg).init_seed(noise).step(200)
    compare(s.fields(), o.fields(), tol, label=f"quintic {precision}")
    # the interpolation matters: h = phi gives a different temperature field
    lin = O.Oracle(dict(cfg, h_quintic=0)).init_seed(noise).step(200)
    assert np.abs(lin.fields()["theta"] - o.fields()["theta"]).max() > 1e-3


@pytest.mark.parametrize("case,precision,tol", [("periodic", "f64", 1e-10), ("channel", "f64", 1e-10),
                                               ("channel", "f32", 1e-4)])
def test_stencil_gradient_ablation_parity(dlb, case, precision, tol):
    """grad_stencil = 1 (grad phi from the nine-point stencil of the node
    values of phi instead of the local scheme of Sec. 3.1): GPU against the
    oracle on a periodic seed and on the coupled channel case."""
    _say(f"case: stencil gradient, {case} {precision}")
    if case == "periodic":
        cfg = dict(W.pure_diffusion_128(precision), nx=64, ny=64, seed_x=32.0, seed_y=32.0, grad_stencil=1)
        noise = None
    else:
        cfg, noise = _flow_case(64, 48, precision)
        cfg = dict(cfg, grad_stencil=1)
    o = O.Oracle(cfg).init_seed(noise).step(200)
    s = dlb.Solver(cfg).init_seed(noise).step(200)
    compare(s.fields(), o.fields(), tol, label=f"stencil {case} {precision}")
    # the ablation changes the result at the discretisation level
    local = O.Oracle(dict(cfg, grad_stencil=0)).init_seed(noise).step(200)
    assert np.abs(local.fields()["phi"] - o.fields()["phi"]).max() > 1e-6


@pytest.mark.parametrize("case,precision,tol,nt", [("channel", "f64", 1e-10, 4), ("channel", "f32", 1e-4, 3),
                                                   ("periodic", "f64", 1e-10, 8)])
def test_heat_sub_steps_parity(dlb, case, precision, tol, nt):
    """n_sub_t heat sub-steps per main step (multi-time-scaling for Le !=
    1), GPU against the oracle: the coupled channel case with alpha raised
    tenfold (Le = 10), and a periodic seed at alpha = 2."""
    _say(f"case: heat sub-steps n_sub_t={nt}, {case} {precision}")
    if case == "periodic":
        cfg = dict(W.pure_diffusion_128(precision), nx=64, ny=64, seed_x=32.0, seed_y=32.0, alpha=2.0,
                   n_sub_t=nt)
        noise = None
    else:
        cfg, noise = _flow_case(64, 48, precision)
        cfg = dict(cfg, alpha=10 * cfg["alpha"], n_sub_t=nt)
    o = O.Oracle(cfg).init_seed(noise).step(150)
    s = dlb.Solver(cfg).init_seed(noise).step(150)
    compare(s.fields(), o.fields(), tol, label=f"heat sub-steps {case} {precision}")


def test_heat_sub_steps_with_16bit_storage(dlb):
    """The heat sub-steps store their intermediate planes with the heat
    lattice's rest-state shifts: FP16-shifted storage follows the FP32 run
    to the storage tolerance of the fused-flow test."""
    _say("case: heat sub-steps n_sub_t=3 with FP16-shifted storage")
    runs = {}
    for precision in ("f32", "f16s"):
        cfg, noise = _flow_case(96, 78, precision)
        cfg = dict(cfg, alpha=10 * cfg["alpha"], n_sub_t=3)
        runs[precision] = dlb.Solver(cfg).init_seed(noise).step(30).fields()
    compare(runs["f16s"], runs["f32"], 6e-2, label="f16s vs f32, heat sub-steps")


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("walls", [1, 0])
def test_fused_flow_substeps_match_single_substeps(dlb, precision, walls):
    """Fusing 3 or 5 flow sub-steps per launch (registers + LDS tile) does
    the same arithmetic per node as one launch per sub-step: FP64 and FP32
    results agree to rounding; 16-bit storage is re-rounded only once per
    launch when fused, so there the check is the storage tolerance."""
    _say(f"case: fused flow sub-steps {precision} walls={walls}")
    cfg, noise = _flow_case(96, 78, precision)
    cfg["walls"] = walls
    runs = {}
    for fuse in (1, 3, 5):
        s = dlb.Solver(dict(cfg, flow_fuse=fuse)).init_seed(noise).step(30)
        runs[fuse] = s.fields()
    tol = {"f64": 1e-12, "f32": 2e-5, "f16s": 6e-2}[precision]
    for fuse in (3, 5):
        compare(runs[fuse], runs[1], tol, label=f"fuse {fuse} vs 1")


def test_thermosolutal_full_size_first_steps(dlb):
    """At the benchmark's size and launch shape (1024^2, FP32) the first
    main steps agree with the oracle field by field."""
    _say("case: thermosolutal flow 1024x1024 FP32, 3 steps vs oracle")
    cfg, noise = _flow_case(1024, 1024, "f32")
    o = O.Oracle(cfg).init_seed(noise).step(3)
    s = dlb.Solver(cfg).init_seed(noise).step(3)
    compare(s.fields(), o.fields(), 1e-4, label="1024^2 t=3")


def test_channel_mirror_symmetry_full_size(dlb):
    """Property at full size: with orientation 0, no noise and the seed on
    the mid-line y = (ny-1)/2, the channel problem is symmetric under
    y -> ny-1-y, so the GPU fields must be too after many steps."""
    _say("case: channel mirror symmetry 1024x1024 FP64, 200 steps")
    cfg, _ = _flow_case(1024, 1024, "f64")
    cfg.update(orient=0.0, seed_y=511.5, noise_amp=0.0)
    s = dlb.Solver(cfg).init_seed().step(200)
    f = s.fields()
    for name in ("phi", "C", "theta", "ux", "p"):
        np.testing.assert_allclose(f[name][::-1, :], f[name], atol=1e-11 * max(1, np.abs(f[name]).max()))
    np.testing.assert_allclose(-f["uy"][::-1, :], f["uy"], atol=1e-13)


def test_channel_mirror_symmetry_full_size_fp32_fused(dlb):
    """The same property in the benchmark's launch configuration (FP32,
    five fused flow sub-steps per launch, wave-row tiles with the row shift
    of the channel walls and the wall-free interior variant): the mirrored
    rows of the tiling are computed by different tiles and wall code, so a
    mistake in either breaks the symmetry."""
    _say("case: channel mirror symmetry 1024x1024 FP32 fused, 300 steps")
    cfg, _ = _flow_case(1024, 1024, "f32")
    cfg.update(orient=0.0, seed_y=511.5, noise_amp=0.0)
    s = dlb.Solver(cfg).init_seed().step(300)
    f = s.fields()
    for name in ("phi", "C", "theta", "ux", "p"):
        np.testing.assert_allclose(f[name][::-1, :], f[name], atol=1e-5 * max(1, np.abs(f[name]).max()))
    np.testing.assert_allclose(-f["uy"][::-1, :], f["uy"], atol=1e-5 * np.abs(f["ux"]).max())


# ---------------------------------------------------------------------------
# Edge cases and runtime behaviour
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,walls,fuse", [(16, 16, 0, 1), (17, 19, 0, 3), (16, 16, 1, 1),
                                              (16, 16, 1, 3), (65, 21, 1, 3), (40, 37, 0, 3)])
def test_small_and_ragged_grids(dlb, nx, ny, walls, fuse):
    _say(f"case: small grid {nx}x{ny} walls={walls} flow_fuse={fuse} FP64")
    cfg = dict(W.pure_diffusion_128("f64"), nx=nx, ny=ny, seed_x=nx / 2 - 0.3, seed_y=ny / 2 + 0.2,
               seed_R=3.0, walls=walls, use_ns=1, n_sub=3, nu=0.3, u_in=(0.01 * walls, 0.0),
               flow_fuse=fuse)
    o = O.Oracle(cfg).init_seed().step(40)
    s = dlb.Solver(cfg).init_seed().step(40)
    compare(s.fields(), o.fields(), 1e-10, label=f"{nx}x{ny}")


@pytest.mark.parametrize("nx,ny,walls,fuse", [(16, 16, 1, 5), (17, 19, 0, 5), (50, 23, 1, 5), (40, 37, 1, 3),
                                              (65, 21, 1, 5), (64, 64, 0, 5), (119, 61, 1, 5), (33, 25, 1, 3),
                                              (70, 24, 1, 5)])
def test_small_grids_fp32_fused_kernel(dlb, nx, ny, walls, fuse):
    """The FP32 wave-row fused kernel on grids where one tile holds both
    x walls (nx <= 54 at K = 5), both y walls (ny <= 22), or ragged edges,
    and with the tiling shifted by 0, 1 or 2 rows so that the wall row sits
    with its inward row (ny 23 and 24 at K = 5, 25 at K = 3 also put the
    bottom wall into the halo of the tile above the last): against the
    unfused path (same arithmetic) and against the oracle."""
    _say(f"case: FP32 fused kernel, small grid {nx}x{ny} walls={walls} fuse={fuse}")
    cfg = dict(W.pure_diffusion_128("f32"), nx=nx, ny=ny, seed_x=nx / 2 - 0.3, seed_y=ny / 2 + 0.2,
               seed_R=3.0, walls=walls, use_ns=1, n_sub=15, nu=0.3, u_in=(0.01, 0.004),
               flow_fuse=fuse)
    fused = dlb.Solver(cfg).init_seed().step(40)
    unfused = dlb.Solver(dict(cfg, flow_fuse=1)).init_seed().step(40)
    compare(fused.fields(), unfused.fields(), 2e-5, label=f"fused vs unfused {nx}x{ny}")
    o = O.Oracle(cfg).init_seed().step(40)
    compare(fused.fields(), o.fields(), 1e-4, fields=("phi", "C", "U", "theta", "ux", "uy"),
            label=f"fused vs oracle {nx}x{ny}")


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_static_cylinder_matches_oracle(dlb, precision, tol):
    """Frozen diffuse solid (the stationary-cylinder problem): only the flow
    lattice steps, with fused sub-steps on the GPU; fields and the
    hydrodynamic force agree with the oracle."""
    _say(f"case: static cylinder R=3, Re=5, 210x120, {precision}")
    cfg = W.cylinder_flow(5, R=3, precision=precision, n_sub=3)
    o = O.Oracle(cfg).init_seed()
    s = dlb.Solver(cfg).init_seed()
    phi0 = s.fields()["phi"]
    o.step(60)
    s.step(60)
    gf, of = s.fields(), o.fields()
    compare(gf, of, tol, fields=("phi", "ux", "uy", "p"), label=f"cylinder {precision}")
    assert np.array_equal(gf["phi"], phi0)
    rg, ro = s.reduce(), o.reduce()
    assert rg["Fx"] == pytest.approx(ro["Fx"], rel=10 * tol)
    assert ro["Fx"] > 0


@pytest.mark.parametrize("Re", [20, 40])
def test_cylinder_drag_and_wake_converge_to_the_paper(dlb, Re):
    """Pin of the flow lattice and the diffuse fluid-solid force against the
    paper's table of Sec. 4.1 (stationary cylinder; C_d = 2.153 / 1.598 and
    L_W = 1.853 / 4.491 at Re = 20 / 40), on the paper's mesh (R = 20 lu,
    1400 x 800) and at twice its resolution (R = 40 lu, the interface width
    W0 = 0.5 lu kept).  C_d: within 5% at both (measured +1.8% / -1.6% at
    Re 20, +2.7% / -0.2% at Re 40).  L_W is 9.9% / 8.6% long at R = 20 and
    5.4% / 4.3% at R = 40: the excess halves with the grid spacing, and the
    first-order extrapolation 2 L_W(40) - L_W(20) lands within 1% of the
    paper's value (bar 2%); the wake's length does not change with a twice
    longer domain and grows by 1-2% with twice the height (see the design
    notes), so neither explains it."""
    from paper_2209_01444_amd import cylinder
    _say(f"case: cylinder Re={Re}, R = 20 and 40 lu, FP32, to steady drag")
    cd_ref, lw_ref = cylinder.PAPER[Re]
    r20 = cylinder.run(Re, 20, "f32")
    r40 = cylinder.run(Re, 40, "f32", max_substeps=400000)
    lw_inf = 2.0 * r40["L_W"] - r20["L_W"]
    _say(f"  C_d {r20['Cd']:.4f} / {r40['Cd']:.4f} (paper {cd_ref}); L_W {r20['L_W']:.4f} / {r40['L_W']:.4f}, "
         f"extrapolated {lw_inf:.4f} (paper {lw_ref}); sub-steps {r20['substeps']} / {r40['substeps']}")
    assert abs(r20["Cd"] / cd_ref - 1) < 0.05 and abs(r40["Cd"] / cd_ref - 1) < 0.05
    assert abs(r40["L_W"] - lw_ref) < 0.7 * abs(r20["L_W"] - lw_ref)
    assert abs(lw_inf / lw_ref - 1) < 0.02


def test_thermal_dendrite_tip_velocity_matches_the_paper(dlb):
    """End-to-end pin of the phase-field and heat lattices against the value
    printed in Sec. 4.2: the thermal dendrite at the paper's resolution
    (512 x 512, dx = 0.4 W0, dt = 0.008 tau0, Delta = 0.55, eps4 = 0.05)
    reaches a steady tip velocity V d0/alpha = 0.0166 (0.017 from the
    Green's-function solution).  The solver gives 0.0167 over t = 100..148
    tau0; the bar is 3% on the window 112..128 tau0."""
    from paper_2209_01444_amd import dendrite
    _say("case: thermal dendrite 512x512 FP32, 16000 steps")
    r = dendrite.run(16000, 2000, "f32")
    v = np.mean(r["series"][-1]["V"])
    _say(f"  V d0/alpha over t = 112..128 tau0: {v:.5f} (paper {dendrite.PAPER_V})")
    assert abs(v / dendrite.PAPER_V - 1) < 0.03
    # fourfold symmetry at orientation 0: the four arms agree
    assert np.ptp(r["series"][-1]["V"]) < 1e-3 * v


def test_thermal_dendrite_with_melt_flow_follows_the_paper(dlb):
    """The melt-flow case of Sec. 4.2 (inflow W0/tau0 from the west, Pr =
    23.1, 15 flow sub-steps per main step) at 512 x 512 to t = 128 tau0,
    against what the section describes: the upstream arm (-x) grows fastest
    and speeds up, the arms across the flow settle at the pure-diffusion tip
    velocity (0.0166), and the downstream arm (+x) slows below them.  The
    solver gives 0.0255 upstream, 0.0168 across and 0.0114 downstream at
    t = 128 tau0."""
    from paper_2209_01444_amd import dendrite
    _say("case: thermal dendrite with melt flow 512x512 FP32, 16000 steps")
    r = dendrite.run(16000, 2000, "f32", flow=True)
    up, across, down = r["V_upstream"], r["V_vertical"], r["V_downstream"]
    _say(f"  V d0/alpha at 128 tau0: upstream {up:.5f}, across {across:.5f}, downstream {down:.5f}")
    assert up > 1.3 * across and down < 0.8 * across
    assert abs(across / dendrite.PAPER_V - 1) < 0.05
    mid, last = r["series"][3]["V"], r["series"][-1]["V"]  # t = 64 and 128 tau0
    assert last[2] > mid[2] and last[0] < mid[0]
    # the seed sits on the channel's centre line: the arms across the flow mirror each other
    assert abs(last[1] - last[3]) <= 1e-3 * across


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_isothermal_alloy_matches_oracle(dlb, precision, tol):
    """Isothermal runs (theta = theta0, no heat lattice) on both sides."""
    _say(f"case: isothermal alloy 96x80 channel walls, {precision}")
    cfg = dict(W.pure_diffusion_128(precision), nx=96, ny=80, use_t=0, walls=1, c_init_U=1, U0=-0.55,
               theta0=0.0, Mcinf=1.0, lambda_=3.191, eps4=0.02, seed_x=47.3, seed_y=40.2, seed_R=6.0)
    o = O.Oracle(cfg).init_seed().step(150)
    s = dlb.Solver(cfg).init_seed().step(150)
    compare(s.fields(), o.fields(), tol, fields=("phi", "C", "U", "theta"), label=f"isothermal {precision}")
    assert np.all(s.fields()["theta"] == 0.0)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_farfield_walls_match_oracle(dlb, precision, tol):
    """Far-field walls (Sec. 4.4): a thermosolutal seed next to the west wall
    of a ragged 70 x 54 grid, whose heat and solute reach the wall ring,
    against the oracle; the ring holds phi = -1, U0 and theta0."""
    _say(f"case: far-field walls 70x54 thermosolutal, {precision}")
    cfg = dict(W.pure_diffusion_128(precision), nx=70, ny=54, walls=2, c_init_U=1, U0=-0.1, theta0=-0.55,
               Mcinf=0.5325, lambda_=3.19, k=0.15, D=0.2, alpha=0.25, eps4=0.02, seed_R=6.0, seed_x=13.3,
               seed_y=26.6)
    o = O.Oracle(cfg).init_seed().step(200)
    s = dlb.Solver(cfg).init_seed().step(200)
    gf, of = s.fields(), o.fields()
    compare(gf, of, tol, fields=("phi", "C", "U", "theta"), label=f"far field {precision}")
    ring = np.ones((54, 70), bool)
    ring[1:-1, 1:-1] = False
    lim = 1e-12 if precision == "f64" else 1e-6
    assert np.abs(gf["phi"][ring] + 1.0).max() < lim
    assert np.abs(gf["U"][ring] + 0.1).max() < lim
    assert np.abs(gf["theta"][ring] + 0.55).max() < lim
    assert np.abs(gf["theta"][1:-1, 1] + 0.55).max() > 1e-4  # the seed's heat reached the wall
    r = s.reduce()
    assert r["nonfinite"] == 0


def test_thermosolutal_dendrite_with_far_field_walls(dlb):
    """Sec. 4.4's pure-diffusion run at its resolution (2400^2, far-field
    walls, Le = 1) to t D/d0^2 = 100000: the four arms grow alike (the seed
    sits on the domain's centre, 0 degrees), the tip velocity settles, the
    ring holds the far field, and ahead of the tip the rejected solute and
    the latent heat decay toward U0 and theta0."""
    from paper_2209_01444_amd import dendrite
    _say("case: thermosolutal dendrite 2400x2400 FP32, far-field walls, to tD/d0^2 = 100000")
    r = dendrite.run_thermosolutal(100000.0, 5, "f32", verbose=False)
    last, prev = r["series"][-1], r["series"][-2]
    _say(f"  V d0/D {last['V']}, rho/d0 {last['rho_d0']}, sigma {last['sigma']}, {r['MLUPS']:.0f} MLUPS")
    assert all(x["nonfinite"] == 0 for x in r["series"])
    v = np.array(last["V"])
    assert v.min() > 0 and (v.max() - v.min()) <= 1e-3 * v.mean()
    assert abs(np.mean(last["V"]) / np.mean(prev["V"]) - 1) < 0.1
    assert max(r["wall_max_dev"].values()) < 1e-6
    prof = np.array(r["axis_profile_x_d0_phi_U_theta"])
    ahead = prof[prof[:, 0] > 5.0]  # liquid ahead of the tip
    assert ahead[0, 2] > 0.0 and ahead[0, 3] > -0.55
    assert np.all(np.diff(ahead[:, 2]) <= 1e-6) and np.all(np.diff(ahead[:, 3]) <= 1e-6)


def test_thermosolutal_dendrite_with_melt_flow_follows_the_paper(dlb):
    """Sec. 4.4's melt-flow run at its resolution (2400^2, inflow W0/tau0,
    Pr = 23.1) to t D/d0^2 = 50000, against its description: the upstream
    arm grows fast, the arms across the flow grow clearly, and the
    downstream arm is suppressed (slow, with a blunt tip)."""
    from paper_2209_01444_amd import dendrite
    _say("case: thermosolutal dendrite with melt flow 2400x2400 FP32, to tD/d0^2 = 50000")
    r = dendrite.run_thermosolutal(50000.0, 4, "f32", verbose=False, flow=True)
    up, across, down = r["V_upstream"], r["V_vertical"], r["V_downstream"]
    last = r["series"][-1]
    _say(f"  V d0/D upstream {up:.5f}, across {across:.5f}, downstream {down:.5f}; rho/d0 {last['rho_d0']}")
    assert all(x["nonfinite"] == 0 for x in r["series"])
    assert up > 2.0 * across and down < 0.5 * across
    rho = last["rho_d0"]
    assert rho[0] > 2.0 * rho[1] and rho[2] < rho[1]  # blunt downstream tip, sharp upstream tip
    assert abs(last["V"][1] - last["V"][3]) <= 1e-3 * across  # arms across the flow mirror each other


def test_solutal_dendrite_with_melt_flow_follows_the_paper(dlb):
    """The melt-flow case of Sec. 4.3 at the paper's resolution (1000^2, to
    t = 600 tau0, the last time the section shows; inflow and viscosity are
    not given there: the thermal case's W0/tau0 and melt), against its
    description: the upstream arm outgrows the others, and while the
    upstream tip radius falls to a low value the radii of the tips across
    and down the flow grow again after a small decrease."""
    from paper_2209_01444_amd import dendrite
    _say("case: solutal dendrite with melt flow 1000x1000 FP32, 30000 steps")
    r = dendrite.run_solutal_flow(30000, 3000, "f32")
    up, across, down = r["V_upstream"], r["V_vertical"], r["V_downstream"]
    _say(f"  V d0/D at 600 tau0: upstream {up:.5f}, across {across:.5f}, downstream {down:.5f}")
    assert up > 1.5 * across and down < 0.6 * across
    first, mid, last = r["series"][0], r["series"][2], r["series"][-1]  # t = 60, 180 and 600 tau0
    rho_f, rho_m, rho_l = first["rho_d0"], mid["rho_d0"], last["rho_d0"]
    assert rho_l[2] < rho_f[2] and rho_l[2] < rho_l[1] and rho_l[2] < rho_l[0]  # upstream radius falls, stays low
    assert rho_l[0] > rho_m[0] and rho_l[1] > rho_m[1]  # downstream and across radii grow again
    assert abs(last["V"][1] - last["V"][3]) <= 1e-3 * across  # arms across the flow mirror each other


def test_solutal_dendrite_follows_gibbs_thomson(dlb):
    """Pin of the solute lattice and the anti-trapping current (Sec. 4.3):
    the isothermal alloy dendrite at the paper's resolution (1000 x 1000,
    dx = 0.4 W0, dt = 0.02 tau0) freezes into the solid on its central axis
    the concentration c_s/c_l^0 = k [1 - (1 - k) d0/r_tip] that the paper
    checks.  The solver: mean deviation 0.3%, at most 0.9% (without the
    anti-trapping current the solid traps solute: 18% mean deviation)."""
    from paper_2209_01444_amd import dendrite
    _say("case: solutal dendrite 1000x1000 FP32, 40000 steps, Gibbs-Thomson on the axis")
    r = dendrite.run_solutal(40000, 200, "f32")
    _say(f"  C_s mean {r['Cs_measured_mean']:.5f} vs Gibbs-Thomson {r['Cs_gibbs_thomson_mean']:.5f}, "
         f"mean err {r['mean_rel_err']:.4f}, max {r['max_rel_err']:.4f}")
    assert abs(r["mean_rel_err"]) < 0.01 and r["max_rel_err"] < 0.02
    assert r["Cs_measured_mean"] < 0.99 * r["trapping_free_value_k"]


def test_zero_steps_and_uniform_liquid(dlb):
    _say("case: step(0) and uniform liquid")
    cfg = dict(W.pure_diffusion_128("f64"), nx=32, ny=32)
    s = dlb.Solver(cfg).set_fields(-np.ones((32, 32)))
    f0 = s.fields()
    s.step(0)
    f1 = s.fields()
    for k in FIELDS:
        np.testing.assert_array_equal(f0[k], f1[k])
    s.step(50)
    f2 = s.fields()
    np.testing.assert_allclose(f2["phi"], -1.0, atol=1e-15)
    np.testing.assert_allclose(f2["theta"], cfg["theta0"], atol=1e-14)


def test_graph_replay_matches_single_steps(dlb):
    _say("case: graph replay vs single launches (bitwise)")
    cfg, noise = _flow_case(96, 64, "f32")
    a = dlb.Solver(cfg).init_seed(noise).step(11)
    b = dlb.Solver(cfg).init_seed(noise)
    for _ in range(11):
        b.step(1)
    fa, fb = a.fields(), b.fields()
    for k in FIELDS:
        np.testing.assert_array_equal(fa[k], fb[k])


def test_checkpoint_resume_is_bitwise(dlb):
    _say("case: checkpoint save/load resume")
    cfg, noise = _flow_case(96, 64, "f32")
    a = dlb.Solver(cfg).init_seed(noise).step(40)
    blob = a.save()
    a.step(40)
    b = dlb.Solver(cfg).load(blob)
    assert b.step_count == 40
    b.step(40)
    fa, fb = a.fields(), b.fields()
    for k in FIELDS:
        np.testing.assert_array_equal(fa[k], fb[k])


FIELDS5 = ("phi", "C", "theta", "ux", "uy")


def _smooth_noise(shape, seed, amp):
    """A smooth seeded perturbation (a few low Fourier modes)."""
    rng = np.random.default_rng(seed)
    ny, nx = shape
    Y, X = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for _ in range(4):
        kx, ky = rng.integers(1, 4, 2)
        ph = rng.uniform(0, 2 * np.pi)
        out += np.sin(2 * np.pi * (kx * X / nx + ky * Y / ny) + ph)
    return amp * out / 4


@pytest.mark.parametrize("flags", [{}, {"keep_flow": True}, {"keep_noneq": True},
                                   {"keep_flow": True, "keep_noneq": True}],
                         ids=["equilibrium", "keep_flow", "keep_noneq", "keep_both"])
def test_restart_at_new_fields_matches_oracle(dlb, flags):
    """Restart at perturbed fields with each continuation flag (FP64): the
    GPU and the oracle agree right after and 30 steps later."""
    _say(f"case: restart at perturbed fields, flags {flags}, 96x78 f64")
    cfg, noise = _flow_case(96, 78, "f64")
    o = O.Oracle(cfg).init_seed(noise).step(60)
    s = dlb.Solver(cfg).init_seed(noise).step(60)
    f = o.fields()
    new = {k: f[k] + _smooth_noise(f[k].shape, 5 + i, 1e-3 * (np.abs(f[k]).max() + 1e-3))
           for i, k in enumerate(FIELDS5)}
    o.set_fields(*[new[k] for k in FIELDS5], **flags)
    s.set_fields(*[new[k] for k in FIELDS5], **flags)
    gf, of = s.fields(), o.fields()
    if flags.get("keep_flow"):
        compare(gf, of, 1e-10, label="after restart")
    else:
        # the flow restarts at p = 0: p is then a small O(u^2) remainder whose
        # differences are rounding of O(1) populations; compare it absolutely
        compare(gf, of, 1e-10, fields=FIELDS[:-1], label="after restart")
        assert np.abs(gf["p"] - of["p"]).max() < 1e-13
    o.step(30)
    s.step(30)
    compare(s.fields(), o.fields(), 1e-10, label="30 steps later")


@pytest.mark.parametrize("precision,tol", [("f64", 1e-13), ("f32", 2e-5)])
def test_restart_at_own_fields_continues_the_run(dlb, precision, tol):
    """With both continuation flags, restarting at the solver's own fields
    (device FP64 fields) leaves the run unchanged up to rounding; a restart at
    equilibrium does not."""
    _say(f"case: restart at own fields, {precision}")
    cfg, noise = _flow_case(96, 78, precision)
    a = dlb.Solver(cfg).init_seed(noise).step(60)
    b = dlb.Solver(cfg).init_seed(noise).step(60)
    c = dlb.Solver(cfg).init_seed(noise).step(60)
    x = b.fields_device(FIELDS5, f32=False)
    b.set_fields(*[x[i] for i in range(5)], keep_flow=True, keep_noneq=True)
    c.set_fields(*[x[i] for i in range(5)])
    for sv in (a, b, c):
        sv.step(40)
    fa, fb, fc = a.fields(), b.fields(), c.fields()
    compare(fb, fa, tol, fields=("phi", "C", "theta", "ux", "uy"), label="continued")
    assert rel_linf(fc["phi"], fa["phi"]) > 1e-5


def test_nonfinite_is_reported(dlb):
    _say("case: NaN injection -> DLB_ENAN")
    cfg = dict(W.pure_diffusion_128("f32"), nx=32, ny=32)
    phi = -np.ones((32, 32))
    phi[5, 7] = np.nan
    s = dlb.Solver(cfg).set_fields(phi)
    with pytest.raises(dlb.DlbError) as e:
        s.reduce()
    assert e.value.code == dlb.DLB_ENAN
    assert s.reduce(allow_nonfinite=True)["nonfinite"] >= 1


def test_create_rejects_small_buffer(dlb):
    _say("case: dlb_create with a short buffer")
    import torch
    lib = dlb.load_library()
    p = dlb.make_params(W.pure_diffusion_128("f32"))
    need = lib.dlb_state_bytes(ctypes.byref(p))
    buf = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    rc = lib.dlb_create(ctypes.byref(p), ctypes.c_void_p(buf.data_ptr()), need // 2, None, ctypes.byref(h))
    assert rc == dlb.DLB_ENOMEM


# ---------------------------------------------------------------------------
# Batched launches
# ---------------------------------------------------------------------------

def _sweep_cfgs(precision="f32", fuse=5):
    import math as _m
    sizes = [(64, 64), (96, 80), (128, 128), (40, 48), (70, 33), (128, 96)]
    rng = np.random.default_rng(9)
    out = []
    for i, (nx, ny) in enumerate(sizes):
        cfg, noise = W.thermosolutal_flow(nx, ny, seed=100 + i, precision=precision,
                                          orient=float(rng.uniform(0, _m.pi / 4)),
                                          u0=float(rng.uniform(0, 0.02)),
                                          delta=float(rng.uniform(0.3, 0.65)),
                                          eps4=float(rng.uniform(0.02, 0.05)))
        cfg.update(seed_R=6.0, flow_fuse=fuse)
        out.append((cfg, noise))
    return out


@pytest.mark.parametrize("precision,fuse", [("f32", 5), ("f64", 3), ("f32", 1)])
def test_batch_members_match_single_runs(dlb, precision, fuse):
    """A batch of seeds of different sizes and parameters, stepped by one
    launch per kernel class, evolves every member bit for bit like a single
    solver with the same settings."""
    _say(f"case: batch of 6 seeds {precision} fuse={fuse} vs single runs")
    cases = _sweep_cfgs(precision, fuse)
    b = dlb.Batch([c for c, _ in cases])
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    b.set_config(fuse, 8, 2)
    b.step(23)
    assert b.step_count == 23
    for i, (m, (cfg, noise)) in enumerate(zip(b.members, cases)):
        s = dlb.Solver(cfg).init_seed(noise).step(23)
        fb, fs = m.fields(), s.fields()
        for k in FIELDS:
            assert np.array_equal(fb[k], fs[k]), f"member {i} field {k} differs"
        assert m.step_count == 23


@pytest.mark.parametrize("fuse", [5, 1])
def test_batch_workgroups_looping_over_tiles_give_the_same_members(dlb, fuse):
    """The smallest grids (one workgroup per compute unit) on a batch with
    more tiles than workgroups: each workgroup takes several tiles of its
    XCD's band in turn, and every member still evolves bit for bit like a
    single solver."""
    _say(f"case: batch of 3 seeds, 1 workgroup per CU, f32 fuse={fuse} vs single runs")
    cases = []
    for i, (nx, ny) in enumerate([(1024, 512), (200, 200), (64, 64)]):
        cfg, noise = W.thermosolutal_flow(nx, ny, seed=300 + i, precision="f32")
        cfg.update(seed_R=8.0, flow_fuse=fuse)
        cases.append((cfg, noise))
    b = dlb.Batch([c for c, _ in cases])
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    b.set_config(fuse, 1, 1)
    b.step(12)
    for i, (m, (cfg, noise)) in enumerate(zip(b.members, cases)):
        s = dlb.Solver(cfg).init_seed(noise).step(12)
        fb, fs = m.fields(), s.fields()
        for k in FIELDS:
            assert np.array_equal(fb[k], fs[k]), f"member {i} field {k} differs"


@pytest.mark.parametrize("walls,precision,fuse,shape", [(1, "f32", 5, (333, 271)), (0, "f32", 5, (200, 150)),
                                                      (1, "f16sm", 5, (150, 203)), (1, "f32", 3, (97, 300))])
def test_tall_fused_tiles_store_the_same_values(dlb, walls, precision, fuse, shape):
    """The fused flow launch with 48-row tiles (12 waves) against 32-row
    tiles (8 waves) on ragged channel and periodic grids: the stored fields
    are bit for bit the same (each stored node's arithmetic does not depend
    on the tiling).  A 48-row request with FP64 flow arithmetic is refused."""
    nx, ny = shape
    _say(f"case: tall fused tiles {nx}x{ny} walls={walls} {precision} fuse={fuse}")
    cfg, noise = W.thermosolutal_flow(nx, ny, seed=2, precision=precision)
    cfg.update(walls=walls, flow_fuse=fuse)
    a = dlb.Solver(dict(cfg, tile_rows=32)).init_seed(noise).step(30).fields()
    b = dlb.Solver(dict(cfg, tile_rows=48)).init_seed(noise).step(30).fields()
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
    with pytest.raises(dlb.DlbError):
        dlb.Solver(dict(cfg, precision="f64", tile_rows=48))


@pytest.mark.parametrize("width", [32, 128, 256])
def test_batch_node_tile_shapes_give_the_same_members(dlb, width):
    """The node tile of the batched node kernels (width x 256/width nodes)
    changes only which threads handle which nodes: with fuse 1 every flow
    sub-step also runs on node tiles, and each member is bit for bit the
    single solver's at every width.  Widths other than 32/64/128/256 are
    refused."""
    _say(f"case: batch node tile {width} x {256 // width}, f32 fuse=1 vs single runs")
    cases = _sweep_cfgs("f32", 1)
    b = dlb.Batch([c for c, _ in cases])
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    b.set_config(1, 8, 2)
    b.set_node_tile(width)
    assert b.node_tile == width
    b.step(11)
    for i, (m, (cfg, noise)) in enumerate(zip(b.members, cases)):
        s = dlb.Solver(cfg).init_seed(noise).step(11)
        fb, fs = m.fields(), s.fields()
        for k in FIELDS:
            assert np.array_equal(fb[k], fs[k]), f"member {i} field {k} differs at node tile {width}"
    for bad in (0, 16, 48, 512):
        with pytest.raises(dlb.DlbError):
            b.set_node_tile(bad)
    assert b.node_tile == width


@pytest.mark.parametrize("precision,fuse,tol", [("f64", 3, 1e-10), ("f32", 5, 1e-4)])
def test_batch_members_match_the_oracle(dlb, precision, fuse, tol):
    """Batch members against the CPU oracle directly: three members of
    different sizes, orientations, inflows, undercoolings and anisotropies
    (64x64, 40x48 and 70x33, the last ragged in both directions) after 120
    main steps of the persistent launches, every field at the parity bar."""
    _say(f"case: batch of 6 seeds {precision} fuse={fuse} vs the oracle")
    cases = _sweep_cfgs(precision, fuse)
    b = dlb.Batch([c for c, _ in cases])
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    b.set_config(fuse, 8, 2)
    b.step(120)
    for i in (0, 3, 4):
        cfg, noise = cases[i]
        o = O.Oracle(cfg).init_seed(noise).step(120)
        compare(b.members[i].fields(), o.fields(), tol, label=f"member {i} {cfg['nx']}x{cfg['ny']}")
        rg, ro = b.members[i].reduce(), o.reduce()
        for key in ("sum_C", "sum_H", "solid_fraction"):
            assert rg[key] == pytest.approx(ro[key], rel=max(tol, 1e-12)), key


def test_batch_autotune_and_member_rules(dlb):
    _say("case: batch autotune, member stepping refused")
    cases = _sweep_cfgs("f32", 5)
    b = dlb.Batch([c for c, _ in cases])
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    ms = b.autotune(3)
    fuse, bn, bt = b.config()
    _say(f"  tuned: fuse={fuse} node blocks/CU={bn} fused blocks/CU={bt} node tile {b.node_tile}, "
         f"{ms:.4f} ms/step")
    assert ms > 0 and fuse in (1, 3, 5) and b.node_tile in (32, 64, 128, 256)
    assert bn in (4, 16, 64, 256, 1024, 4096) and bt in (1, 2, 3, 4, 32, 4096)
    for bad in ((5, 4097, 2), (5, 0, 2), (4, 64, 2), (5, 64, 4097), (5, 64, 0)):
        with pytest.raises(dlb.DlbError):
            b.set_config(*bad)
    # tuning again from another node tile searches the same candidates
    b.set_node_tile(256)
    assert b.autotune(3) > 0 and b.node_tile in (32, 64, 128, 256)
    with pytest.raises(dlb.DlbError):
        b.members[0].step(1)
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    b.step(5)
    r = b.members[2].reduce()
    assert r["nonfinite"] == 0
    # solver options that batches do not carry are refused
    for opt in ({"phi_static": 1}, {"grad_stencil": 1}, {"n_sub_t": 2}, {"walls": 2, "use_ns": 0},
                {"force_x": 1e-5, "flow_fuse": 1}):
        with pytest.raises(dlb.DlbError):
            dlb.Batch([dict(cases[0][0], **opt)])
