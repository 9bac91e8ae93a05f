"""Host logic of the hybrid loop (no GPU): the judge of a jump."""
import numpy as np
import pytest

from paper_2209_01444_amd.surrogate import judge


def _traj(v0, a):
    """Tip positions of 4 arms moving with velocity v0 + a t (arm-dependent v0)."""
    return lambda t: np.array([v0 * (1 + 0.1 * k) * t + 0.5 * a * t * t for k in range(4)])


@pytest.mark.parametrize("K,L,Lb", [(100, 100, 100), (100, 20, 20), (100, 50, 100), (60, 30, 45)])
def test_judge_is_exact_for_steadily_changing_velocity(K, L, Lb):
    s = _traj(0.01, -2e-6)
    t = 1000
    err, vj, ve = judge((t - Lb, s(t - Lb)), (t, s(t)), (t + K, s(t + K)), (t + K + L, s(t + K + L)))
    assert err < 1e-12
    np.testing.assert_allclose(vj, ve, rtol=1e-12)


def test_judge_flags_a_displacement_error_on_one_arm():
    s = _traj(0.01, 0.0)
    t, K, L = 500, 100, 100
    s1 = s(t + K).copy()
    s1[2] += 0.05 * 0.012 * K  # 5% too far on arm 2 (its velocity is 0.012)
    s2 = s1 + (s(t + K + L) - s(t + K))
    err, vj, ve = judge((t - L, s(t - L)), (t, s(t)), (t + K, s1), (t + K + L, s2))
    assert err == pytest.approx(0.05, rel=1e-9)


def test_judge_rejects_a_still_or_lost_tip():
    s = _traj(0.01, 0.0)
    t, K, L = 500, 100, 100
    err, _, _ = judge((t - L, s(t - L)), (t, s(t)), (t + K, s(t)), (t + K + L, s(t) + s(L) - s(0)))
    assert err == pytest.approx(1.0)
    lost = s(t + K).copy()
    lost[1] = np.nan
    err, _, _ = judge((t - L, s(t - L)), (t, s(t)), (t + K, lost), (t + K + L, s(t + K + L)))
    assert err == float("inf")


def test_bfloat16_packing_rounds_to_nearest_even():
    import numpy as np
    from paper_2209_01444_amd.surrogate import from_bf16_bits, to_bf16_bits
    # halfway cases: 1 + 2^-8 lies between 1 and 1 + 2^-7 (ties to even: 1),
    # 1 + 3 * 2^-8 between 1 + 2^-7 and 1 + 2^-6 (ties to even: 1 + 2^-6)
    x = np.array([1.0, 1 + 2.0**-8, 1 + 3 * 2.0**-8, -2.5, 1e-20, 3.0e38], dtype=np.float32)
    y = from_bf16_bits(to_bf16_bits(x))
    assert y[0] == 1.0 and y[1] == 1.0 and y[2] == np.float32(1 + 2.0**-6) and y[3] == -2.5
    # every bfloat16 value survives the round trip, and the rounding error is at most half a spacing
    r = np.random.default_rng(1).normal(size=4096).astype(np.float32)
    b = to_bf16_bits(r)
    assert np.array_equal(to_bf16_bits(from_bf16_bits(b)), b)
    assert np.all(np.abs(from_bf16_bits(b) - r) <= np.abs(r) * 2.0**-8)


def test_stored_network_matches_the_library_layout():
    """The stored 512^2 network: plain arrays (loads without pickle), one
    bfloat16 weight per 3x3 convolution weight of the library's parameter
    layout, finite values, and the options of the training run."""
    import json
    import os

    import numpy as np
    import pytest
    from paper_2209_01444_amd import surrogate as S
    if not os.path.exists(S.BUNDLE):
        pytest.skip("no stored network")
    z = np.load(S.BUNDLE)
    mask = S.conv_weight_mask()
    assert z["w_bf16"].dtype == np.uint16 and z["w_bf16"].size == mask.sum()
    assert z["rest"].dtype == np.float32 and z["rest"].size == mask.size - mask.sum()
    w = S.from_bf16_bits(z["w_bf16"])
    assert np.all(np.isfinite(w)) and np.all(np.isfinite(z["rest"]))
    for k in ("mean", "std", "rstd", "loss_weights"):
        assert z[k].shape == (5,) and np.all(np.isfinite(z[k]))
    assert np.all(z["std"] > 0) and np.all(z["rstd"] > 0)
    meta = json.loads(str(z["meta"]))
    assert meta["size"] == 512 and meta["K"] == 100 and meta["restart"] in ("continue", "equilibrium")
