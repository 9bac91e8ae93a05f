"""NumPy FP64 reference of the surrogate U-Net (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU surrogate's
kernels; the product never imports it.  Plain definitions: a 3x3 convolution
with zero padding is the sum over the nine shifted copies of the input times
the weight slice of that shift; average pooling, nearest upsampling and
channel concatenation are written out directly; the backward pass is the
chain rule applied to those definitions (checked by finite differences in
tests/test_unet_oracle.py).

Architecture (the surrogate's): 4 levels with 32/64/128/256 channels, two 3x3
convolutions + leaky ReLU per level, 2x2 average pooling down, nearest 2x
upsampling and skip concatenation up, 1x1 head.  Layout NHWC.  Weights of a
3x3 convolution: W[ky, kx, co, ci], bias b[co]; y[n,y,x,co] = b[co] +
sum_{ky,kx,ci} x[n, y+ky-1, x+kx-1, ci] W[ky,kx,co,ci].

`round_bf16` lets the reference round activations to bfloat16 at the same
points as the GPU path (round-to-nearest-even of the FP32 value), so that a
gradient comparison isolates accumulation-order differences.
"""
from __future__ import annotations

import numpy as np

LEAK = 0.1


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) via the FP32 bit pattern."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, W, b):
    n, h, w, ci = x.shape
    xp = np.zeros((n, h + 2, w + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.broadcast_to(b, (n, h, w, W.shape[2])).copy()
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nhwc,oc->nhwo", xp[:, ky:ky + h, kx:kx + w, :], W[ky, kx])
    return y


def conv3x3_backward(x, W, dy):
    """Gradients of sum(dy * conv3x3(x, W, b)) w.r.t. x, W, b."""
    n, h, w, ci = x.shape
    xp = np.zeros((n, h + 2, w + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            dW[ky, kx] = np.einsum("nhwo,nhwc->oc", dy, xp[:, ky:ky + h, kx:kx + w, :])
            dxp[:, ky:ky + h, kx:kx + w, :] += np.einsum("nhwo,oc->nhwc", dy, W[ky, kx])
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dW, db


def leaky(y):
    return np.where(y > 0, y, LEAK * y)


def leaky_backward(out, dout):
    return np.where(out > 0, dout, LEAK * dout)


def pool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dy):
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


LEVELS = (32, 64, 128, 256)


def layer_shapes(cin: int = 5, cout: int = 5, base: int = 32):
    """(name, kind, Cin, Cout) of every layer, in execution order."""
    ch = [base * 2**i for i in range(4)]
    L = []
    c = cin
    for i, co in enumerate(ch):
        L += [(f"enc{i}a", "conv", c, co), (f"enc{i}b", "conv", co, co)]
        c = co
    for i in (2, 1, 0):
        L += [(f"dec{i}a", "conv", c + ch[i], ch[i]), (f"dec{i}b", "conv", ch[i], ch[i])]
        c = ch[i]
    L += [("head", "conv1", c, cout)]
    return L


def init_params(rng, cin=5, cout=5, base=32, head_scale=0.1):
    P = {}
    for name, kind, ci, co in layer_shapes(cin, cout, base):
        if kind == "conv":
            P[name + ".W"] = rng.normal(size=(3, 3, co, ci)) * np.sqrt(2.0 / (9 * ci))
            P[name + ".b"] = np.zeros(co)
        else:
            P[name + ".W"] = rng.normal(size=(co, ci)) * np.sqrt(1.0 / ci) * head_scale
            P[name + ".b"] = np.zeros(co)
    return P


def forward(P, x, base=32, rnd=None):
    """x: (n, h, w, cin).  Returns (prediction (n,h,w,cout), cache).  `rnd`
    (e.g. round_bf16) is applied to every stored activation."""
    r = rnd or (lambda a: a)
    cache = {"x": x}
    ch = [base * 2**i for i in range(4)]
    a = x
    skips = []
    for i in range(4):
        if i > 0:
            a = r(pool2(a))
            cache[f"pool{i}"] = a
        for s in "ab":
            pre = conv3x3(a, P[f"enc{i}{s}.W"], P[f"enc{i}{s}.b"])
            cache[f"enc{i}{s}.in"] = a
            a = r(leaky(pre))
            cache[f"enc{i}{s}.out"] = a
        skips.append(a)
    for i in (2, 1, 0):
        u = r(up2(a))
        a = np.concatenate([u, skips[i]], axis=3)
        cache[f"cat{i}"] = (u.shape[3], skips[i].shape[3])
        for s in "ab":
            pre = conv3x3(a, P[f"dec{i}{s}.W"], P[f"dec{i}{s}.b"])
            cache[f"dec{i}{s}.in"] = a
            a = r(leaky(pre))
            cache[f"dec{i}{s}.out"] = a
    cache["head.in"] = a
    y = np.einsum("nhwc,oc->nhwo", a, P["head.W"]) + P["head.b"]
    return y, cache


def backward(P, cache, dy, base=32, rnd=None):
    """Gradients of sum(dy * forward(P, x)) w.r.t. every parameter.  `rnd`
    (e.g. round_bf16) is applied to every stored activation gradient."""
    r = rnd or (lambda a: a)
    G = {}
    a = cache["head.in"]
    G["head.W"] = np.einsum("nhwo,nhwc->oc", dy, a)
    G["head.b"] = dy.sum(axis=(0, 1, 2))
    da = r(np.einsum("nhwo,oc->nhwc", dy, P["head.W"]))
    dskip = {}
    for i in (0, 1, 2):
        for s in "ba":
            name = f"dec{i}{s}"
            dpre = r(leaky_backward(cache[name + ".out"], da))
            da, G[name + ".W"], G[name + ".b"] = conv3x3_backward(cache[name + ".in"], P[name + ".W"], dpre)
            da = r(da)
        cu, cs = cache[f"cat{i}"]
        dskip[i] = da[..., cu:]
        da = r(up2_backward(da[..., :cu]))
    for i in (3, 2, 1, 0):
        for s in "ba":
            name = f"enc{i}{s}"
            dpre = r(leaky_backward(cache[name + ".out"], da))
            da, G[name + ".W"], G[name + ".b"] = conv3x3_backward(cache[name + ".in"], P[name + ".W"], dpre)
            da = r(da)
        if i > 0:
            # the pooled path adds into the gradient of the level above's skip
            da = r(dskip[i - 1] + pool2_backward(da))
    G["x"] = da
    return G


def mse(pred, target, weights=None):
    """Mean squared error and its gradient w.r.t. pred; optional per-channel
    (last axis) weights w: mean of w_c d^2 over all elements."""
    d = pred - target
    w = np.ones(d.shape[-1]) if weights is None else np.asarray(weights, dtype=np.float64)
    return float(np.mean(w * d * d)), 2.0 * w * d / d.size


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) with bias correction; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
