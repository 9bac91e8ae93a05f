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
