"""Restart from given fields (orc_set_fields_ex): the continuation flags.

Pins: restarting at the state's own fields with both flags must leave the
evolution unchanged (nothing is lost that the method carries: non-equilibrium
parts, the flow lattice, time derivatives), while a restart at equilibrium
visibly perturbs it; the new state's macroscopic fields are the ones given."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2209_01444_amd import workloads as W

FIELDS5 = ("phi", "C", "theta", "ux", "uy")


def _case(kind):
    if kind == "channel":
        cfg, noise = W.thermosolutal_flow(48, 40, seed=3, precision="f64")
        return cfg, noise
    cfg = dict(W.pure_diffusion_128("f64"))
    cfg.update(nx=48, ny=48, seed_x=24.0, seed_y=24.0, seed_R=6.0)
    return cfg, None


def _run(cfg, noise, t0, t1, restart=None):
    o = O.Oracle(cfg).init_seed(noise)
    o.step(t0)
    if restart is not None:
        f = o.fields()
        o.set_fields(*[f[k] for k in FIELDS5], **restart)
    o.step(t1 - t0)
    return o.fields()


@pytest.mark.parametrize("kind", ["channel", "periodic"])
def test_restart_at_own_fields_with_both_flags_changes_nothing(kind):
    cfg, noise = _case(kind)
    ref = _run(cfg, noise, 60, 90)
    got = _run(cfg, noise, 60, 90, dict(keep_flow=True, keep_noneq=True))
    plain = _run(cfg, noise, 60, 90, {})
    for k in ("phi", "C", "theta", "ux", "uy"):
        scale = max(np.abs(ref[k]).max(), 1e-300)
        assert np.abs(got[k] - ref[k]).max() <= 1e-13 * scale, k
    # the equilibrium restart is a visible perturbation (the pin has power)
    assert np.abs(plain["phi"] - ref["phi"]).max() > 1e-4


def test_keep_noneq_sets_the_given_fields():
    cfg, noise = _case("channel")
    o = O.Oracle(cfg).init_seed(noise)
    o.step(40)
    f = o.fields()
    rng = np.random.default_rng(0)
    new = {k: f[k] + 1e-3 * rng.standard_normal(f[k].shape) for k in ("phi", "C", "theta")}
    o.set_fields(new["phi"], new["C"], new["theta"], None, None, keep_flow=True, keep_noneq=True)
    g = o.fields()
    inner = (slice(1, -1), slice(1, -1))  # wall nodes are rebuilt from the inward node
    for k in ("phi", "C", "theta"):
        np.testing.assert_allclose(g[k][inner], new[k][inner], rtol=0, atol=1e-14)
    # the flow lattice was kept
    np.testing.assert_array_equal(o.pops(3)[:, 1:-1, 1:-1], O.Oracle(cfg).init_seed(noise).step(40).pops(3)[:, 1:-1, 1:-1])


def test_unknown_flag_is_rejected():
    cfg, noise = _case("periodic")
    o = O.Oracle(cfg).init_seed(noise)
    phi = o.fields()["phi"]
    import ctypes
    arr = np.ascontiguousarray(phi, dtype=np.float64)
    rc = o.lib.orc_set_fields_ex(o.h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None,
                                 None, None, 4)
    assert rc != 0
