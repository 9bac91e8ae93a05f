"""Pins of the NumPy U-Net reference: finite differences for every gradient,
adjoint identities for pooling and upsampling, closed forms for the bf16
rounding and the first Adam step."""
import numpy as np
import pytest

from oracle import unet_oracle as U


def _rng():
    return np.random.default_rng(5)


def test_conv3x3_matches_direct_sum():
    rng = _rng()
    x = rng.normal(size=(1, 5, 6, 3))
    W = rng.normal(size=(3, 3, 4, 3))
    b = rng.normal(size=4)
    y = U.conv3x3(x, W, b)
    # direct definition at a few pixels, with zero padding
    for (i, j, o) in [(0, 0, 1), (2, 3, 0), (4, 5, 3)]:
        ref = b[o]
        for ky in range(3):
            for kx in range(3):
                yy, xx = i + ky - 1, j + kx - 1
                if 0 <= yy < 5 and 0 <= xx < 6:
                    ref += x[0, yy, xx] @ W[ky, kx, o]
        assert y[0, i, j, o] == pytest.approx(ref, abs=1e-12)


def test_conv3x3_backward_by_finite_differences():
    rng = _rng()
    x = rng.normal(size=(2, 4, 5, 3))
    W = rng.normal(size=(3, 3, 2, 3))
    b = rng.normal(size=2)
    dy = rng.normal(size=(2, 4, 5, 2))
    dx, dW, db = U.conv3x3_backward(x, W, dy)
    f = lambda x_, W_, b_: float(np.sum(dy * U.conv3x3(x_, W_, b_)))
    eps = 1e-6
    for arr, g, which in ((x, dx, 0), (W, dW, 1), (b, db, 2)):
        d = rng.normal(size=arr.shape)
        args_p = [x, W, b]
        args_m = [x, W, b]
        args_p[which] = arr + eps * d
        args_m[which] = arr - eps * d
        fd = (f(*args_p) - f(*args_m)) / (2 * eps)
        assert fd == pytest.approx(float(np.sum(g * d)), rel=1e-7)


def test_pool_and_upsample_adjoints():
    rng = _rng()
    x = rng.normal(size=(2, 6, 8, 3))
    y = rng.normal(size=(2, 3, 4, 3))
    assert np.sum(U.pool2(x) * y) == pytest.approx(np.sum(x * U.pool2_backward(y)), rel=1e-12)
    assert np.sum(U.up2(y) * x) == pytest.approx(np.sum(y * U.up2_backward(x)), rel=1e-12)
    assert U.pool2(np.ones((1, 4, 4, 1))).ravel().tolist() == [1.0] * 4


def test_unet_gradients_by_finite_differences():
    rng = _rng()
    P = U.init_params(rng, cin=5, cout=5, base=4, head_scale=1.0)
    x = rng.normal(size=(2, 16, 16, 5))
    t = rng.normal(size=(2, 16, 16, 5))

    def loss(P_, x_):
        y, _ = U.forward(P_, x_, base=4)
        return U.mse(y, t)[0]

    y, cache = U.forward(P, x, base=4)
    L, dy = U.mse(y, t)
    G = U.backward(P, cache, dy, base=4)
    eps = 1e-6
    for name in list(P)[::3] + ["x"]:
        arr = x if name == "x" else P[name]
        d = rng.normal(size=arr.shape)
        if name == "x":
            fp, fm = loss(P, x + eps * d), loss(P, x - eps * d)
        else:
            Pp, Pm = dict(P), dict(P)
            Pp[name], Pm[name] = arr + eps * d, arr - eps * d
            fp, fm = loss(Pp, x), loss(Pm, x)
        fd = (fp - fm) / (2 * eps)
        assert fd == pytest.approx(float(np.sum(G[name] * d)), rel=2e-6, abs=1e-12), name


def test_layer_list():
    L = U.layer_shapes()
    assert [l[0] for l in L][:2] == ["enc0a", "enc0b"]
    assert ("dec2a", "conv", 256 + 128, 128) in L
    assert ("dec0a", "conv", 64 + 32, 32) in L
    assert L[-1] == ("head", "conv1", 32, 5)
    flops = 0
    H = 512
    size = {0: H, 1: H // 2, 2: H // 4, 3: H // 8}
    for name, kind, ci, co in L:
        lvl = int(name[3]) if name[0] in "ed" else 0
        flops += 2 * (9 if kind == "conv" else 1) * ci * co * size[lvl] ** 2
    assert 80e9 < flops < 90e9  # about 85 GFLOP per 512^2 forward


def test_bf16_rounding_closed_forms():
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, -2.5, 1.0 + 2**-8 + 2**-20])
    r = U.round_bf16(v)
    # 8 significant bits (ulp 2^-7 at 1): ties go to even, above half rounds up
    assert r.tolist() == [1.0, 1.0, 1.0 + 4 * 2**-8, -2.5, 1.0 + 2**-7]


def test_adam_first_step_is_signed_lr():
    p, m, v = U.adam(np.array([1.0, -2.0]), np.array([0.3, -7.0]), np.zeros(2), np.zeros(2), 1, 0.01)
    np.testing.assert_allclose(p, [1.0 - 0.01, -2.0 + 0.01], rtol=1e-6)


def test_weighted_mse_gradient_by_finite_differences():
    """Per-channel weights: the gradient matches central differences, and
    zero-weight channels get no gradient."""
    rng = np.random.default_rng(8)
    p = rng.normal(size=(2, 3, 4, 5))
    t = rng.normal(size=p.shape)
    w = np.array([1.0, 2.0, 0.5, 0.0, 0.0])
    L, g = U.mse(p, t, w)
    assert L == pytest.approx(np.sum(w * (p - t) ** 2) / p.size, rel=1e-14)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 1), (0, 1, 2, 2), (1, 0, 1, 3)]:
        e = np.zeros_like(p)
        e[idx] = h
        fd = (U.mse(p + e, t, w)[0] - U.mse(p - e, t, w)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-7, abs=1e-12)
    assert np.all(g[..., 3:] == 0)
