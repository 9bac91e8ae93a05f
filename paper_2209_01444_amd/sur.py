"""Python binding of libsur.so (include/sur.h): argument marshalling only.

The surrogate's forward, backward and Adam run in the library's HIP kernels
(bf16 matrix-core convolutions); this module allocates the caller-owned
parameter block and workspace with torch and converts arguments.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libsur.so")

LEVEL_CH = (32, 64, 128, 256)
EXPORTS = ("sur_param_count", "sur_param_bytes", "sur_workspace_bytes", "sur_create", "sur_destroy",
           "sur_set_params", "sur_get_params", "sur_get_grads", "sur_get_layer_tensor", "sur_set_normalization",
           "sur_set_loss_weights", "sur_forward",
           "sur_gradients", "sur_train_step", "sur_conv_check", "sur_mfma_check", "sur_last_error")

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2209_01444_amd/build.py`")
    if path == LIB_PATH:
        from paper_2209_01444_amd import build
        build.warn_if_stale(path, build.SUR_DEPS)
    lib = ctypes.CDLL(path)
    vp, fp, i, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_size_t
    sig = {
        "sur_param_count": (sz, []),
        "sur_param_bytes": (sz, []),
        "sur_workspace_bytes": (sz, [i, i, i]),
        "sur_create": (i, [i, i, i, vp, sz, vp, sz, vp, ctypes.POINTER(vp)]),
        "sur_destroy": (i, [vp]),
        "sur_set_params": (i, [vp, fp]),
        "sur_get_params": (i, [vp, fp]),
        "sur_get_grads": (i, [vp, fp]),
        "sur_get_layer_tensor": (i, [vp, ctypes.c_int, ctypes.c_int, fp]),
        "sur_set_normalization": (i, [vp, fp, fp, fp]),
        "sur_set_loss_weights": (i, [vp, fp]),
        "sur_forward": (i, [vp, i, vp, vp]),
        "sur_gradients": (i, [vp, i, vp, vp, fp]),
        "sur_train_step": (i, [vp, i, vp, vp, ctypes.c_float, fp]),
        "sur_conv_check": (i, [i, i, i, i, i, i, fp, fp, fp, fp]),
        "sur_mfma_check": (i, [fp, fp, fp]),
        "sur_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(lib, rc):
    if rc != 0:
        raise RuntimeError(f"sur error {rc}: {lib.sur_last_error().decode()}")


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def layers():
    """(name, Cin, Cin_padded, Cout) of the 3x3 layers in parameter order."""
    out, c = [], 5
    for lv, co in enumerate(LEVEL_CH):
        out += [(f"enc{lv}a", c, (c + 31) // 32 * 32, co), (f"enc{lv}b", co, co, co)]
        c = co
    for lv in (2, 1, 0):
        ci = c + LEVEL_CH[lv]
        out += [(f"dec{lv}a", ci, ci, LEVEL_CH[lv]), (f"dec{lv}b", LEVEL_CH[lv], LEVEL_CH[lv], LEVEL_CH[lv])]
        c = LEVEL_CH[lv]
    return out


def flatten(P: dict) -> np.ndarray:
    """Parameter dictionary {name.W: [3,3,co,ci], name.b: [co], head.W: [5,32],
    head.b: [5]} -> the library's flat FP32 vector (enc0a padded to 32 inputs)."""
    parts = []
    for name, ci, cip, co in layers():
        W = np.zeros((3, 3, co, cip), dtype=np.float32)
        W[..., :ci] = P[name + ".W"]
        parts += [W.ravel(), np.asarray(P[name + ".b"], dtype=np.float32).ravel()]
    parts += [np.asarray(P["head.W"], dtype=np.float32).ravel(), np.asarray(P["head.b"], dtype=np.float32)]
    return np.concatenate(parts)


def unflatten(v: np.ndarray) -> dict:
    P, off = {}, 0
    for name, ci, cip, co in layers():
        n = 9 * co * cip
        P[name + ".W"] = v[off:off + n].reshape(3, 3, co, cip)[..., :ci].astype(np.float64)
        off += n
        P[name + ".b"] = v[off:off + co].astype(np.float64)
        off += co
    P["head.W"] = v[off:off + 160].reshape(5, 32).astype(np.float64)
    P["head.b"] = v[off + 160:off + 165].astype(np.float64)
    return P


class Surrogate:
    """U-Net surrogate for batch B of H x W fields (H, W multiples of 8)."""

    def __init__(self, B: int, H: int, W: int, device: str = "cuda:0", stream=None):
        import torch

        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libsur needs a GPU (no CPU fallback)")
        self.B, self.H, self.W = B, H, W
        self.device = torch.device(device)
        pb = self.lib.sur_param_bytes()
        wb = self.lib.sur_workspace_bytes(B, H, W)
        if wb == 0:
            raise ValueError("B >= 1 and H, W multiples of 8 are required")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.params = torch.zeros(pb, dtype=torch.uint8, device=self.device)
            self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.P = self.lib.sur_param_count()
        self.handle = ctypes.c_void_p()
        _check(self.lib, self.lib.sur_create(B, H, W, ctypes.c_void_p(self.params.data_ptr()), pb,
                                             ctypes.c_void_p(self.work.data_ptr()), wb,
                                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.sur_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.P
        _check(self.lib, self.lib.sur_set_params(self.handle, _fptr(flat)))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.P, dtype=np.float32)
        _check(self.lib, self.lib.sur_get_params(self.handle, _fptr(out)))
        return out

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.P, dtype=np.float32)
        _check(self.lib, self.lib.sur_get_grads(self.handle, _fptr(out)))
        return out

    def layer_tensor(self, k: int, which: int) -> np.ndarray:
        """Stored tensor of conv layer k: which 0 input, 1 output, 2 output
        gradient (NHWC float32, see sur_get_layer_tensor)."""
        name, ci, cip, co = layers()[k]
        level = int(name[3])  # enc{level}a/b, dec{level}a/b
        c = cip if which == 0 else co
        out = np.empty((self.B, self.H >> level, self.W >> level, c), dtype=np.float32)
        _check(self.lib, self.lib.sur_get_layer_tensor(self.handle, int(k), int(which), _fptr(out)))
        return out

    def set_normalization(self, mean, std, rstd):
        m, s, r = (np.ascontiguousarray(a, dtype=np.float32) for a in (mean, std, rstd))
        self.mean, self.std, self.rstd = m.copy(), s.copy(), r.copy()
        _check(self.lib, self.lib.sur_set_normalization(self.handle, _fptr(m), _fptr(s), _fptr(r)))

    def set_loss_weights(self, w5):
        w = np.ascontiguousarray(w5, dtype=np.float32)
        assert w.shape == (5,)
        _check(self.lib, self.lib.sur_set_loss_weights(self.handle, _fptr(w)))
        self.loss_weights = w.copy()

    def _dev(self, t, dtype):
        assert t.is_cuda and t.dtype == dtype and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, x, out=None):
        """x: device float32 [b,5,H,W]; out: device float64 [b,5,H,W] or None."""
        torch = self.torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(self.lib, self.lib.sur_forward(self.handle, x.shape[0], self._dev(x, torch.float32),
                                              None if out is None else self._dev(out, torch.float64)))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def gradients(self, x, y) -> float:
        torch = self.torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        loss = ctypes.c_float()
        _check(self.lib, self.lib.sur_gradients(self.handle, x.shape[0], self._dev(x, torch.float32),
                                                self._dev(y, torch.float32), ctypes.byref(loss)))
        return loss.value

    def train_step(self, x, y, lr: float) -> float:
        torch = self.torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        loss = ctypes.c_float()
        _check(self.lib, self.lib.sur_train_step(self.handle, x.shape[0], self._dev(x, torch.float32),
                                                 self._dev(y, torch.float32), ctypes.c_float(lr),
                                                 ctypes.byref(loss)))
        return loss.value


def conv_check(op: int, X: np.ndarray, Wt: np.ndarray, dY: np.ndarray | None = None) -> np.ndarray:
    """Run one convolution kernel (0 forward, 1 input gradient, 2 weight
    gradient) on host arrays X [B,H,W,Cin], Wt [3,3,Cout,Cin], dY [B,H,W,Cout]."""
    lib = load_library()
    B, H, W, Cin = X.shape
    Cout = Wt.shape[2]
    x = np.ascontiguousarray(X, dtype=np.float32)
    w = np.ascontiguousarray(Wt, dtype=np.float32)
    dy = None if dY is None else np.ascontiguousarray(dY, dtype=np.float32)
    shape = {0: (B, H, W, Cout), 1: (B, H, W, Cin), 2: (3, 3, Cout, Cin)}[op]
    out = np.empty(shape, dtype=np.float32)
    _check(lib, lib.sur_conv_check(op, B, H, W, Cin, Cout, _fptr(x), _fptr(w),
                                   None if dy is None else _fptr(dy), _fptr(out)))
    return out


def mfma_check(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    lib = load_library()
    a = np.ascontiguousarray(A, dtype=np.float32)
    b = np.ascontiguousarray(B, dtype=np.float32)
    d = np.empty((16, 16), dtype=np.float32)
    _check(lib, lib.sur_mfma_check(_fptr(a), _fptr(b), _fptr(d)))
    return d


def layer_work(H: int, W: int, B: int = 1) -> list[dict]:
    """Work of each 3x3 layer of a forward pass at H x W, batch B: flops
    (2 x 9 x Cin_p x Cout per pixel, the padded input channels included, as
    the matrix cores compute them) and the bytes a layer must move at least
    (bf16 input and output activations once, bf16 weights once)."""
    out = []
    for name, ci, cip, co in layers():
        level = int(name[3])
        px = B * (H >> level) * (W >> level)
        out.append({"layer": name, "level": level, "cin": ci, "cout": co, "pixels": px,
                    "flop": 2.0 * 9 * cip * co * px,
                    "bytes": 2.0 * px * (cip + co) + 2.0 * 9 * cip * co})
    return out


def forward_bench(size: int = 512, batch: int = 1, reps: int = 50, seed: int = 5) -> dict:
    """Forward passes of a randomly initialised network (the arithmetic does
    not depend on the weights), timed with HIP events on the network's
    stream."""
    import torch

    rng = np.random.default_rng(seed)
    P = {}
    for name, ci, cip, co in layers():
        P[name + ".W"] = rng.normal(size=(3, 3, co, ci)) * np.sqrt(2.0 / (9 * ci))
        P[name + ".b"] = np.zeros(co)
    P["head.W"] = rng.normal(size=(5, 32)) * 0.01
    P["head.b"] = np.zeros(5)
    net = Surrogate(batch, size, size)
    net.set_params(flatten(P))
    net.set_normalization(np.zeros(5), np.ones(5), np.ones(5))
    x = torch.randn((batch, 5, size, size), dtype=torch.float32, device=net.device)
    out = torch.empty((batch, 5, size, size), dtype=torch.float64, device=net.device)
    for _ in range(3):
        net.forward(x, out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(net.stream)
    for _ in range(reps):
        net.forward(x, out)
    ev[1].record(net.stream)
    ev[1].synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    flop = sum(w["flop"] for w in layer_work(size, size, batch))
    return {"size": size, "batch": batch, "reps": reps, "forward_ms": ms, "conv_flop": flop,
            "TFLOPs": flop / (ms * 1e-3) / 1e12}


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="forward-pass timing of the surrogate U-Net")
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=50)
    a = ap.parse_args()
    print(json.dumps(forward_bench(a.size, a.batch, a.reps)), flush=True)
