"""ctypes binding of the 3-D solver's C ABI (include/dlb3.h, exported by
libdlb.so): argument marshalling only.  Device state lives in a torch
buffer; every step runs in the library's kernels.  There is no CPU
fallback: without the library or a GPU it raises."""
from __future__ import annotations

import ctypes

import numpy as np

from paper_2209_01444_amd import dlb as _dlb

DLB3_OK, DLB3_EINVAL = 0, -1
PRECISION = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
FIELDS = ("phi", "C", "U", "theta", "ux", "uy", "uz", "p")
EXPORTS = ("dlb3_state_bytes", "dlb3_create", "dlb3_destroy", "dlb3_init_seed", "dlb3_set_fields",
           "dlb3_step", "dlb3_get_fields", "dlb3_reduce", "dlb3_last_error")


class Dlb3Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dlb3 error {code}: {msg}")
        self.code = code


class Dlb3Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "nx", "ny", "nz", "walls", "use_t", "h_quintic", "c_init_U", "precision", "grad_iters")] + [
        (n, ctypes.c_double) for n in (
            "W0", "tau0", "eps4", "lambda_", "Mcinf", "k", "D", "alpha", "theta0", "U0", "C0",
            "seed_R", "seed_x", "seed_y", "seed_z", "grad_tol")] + [
        (n, ctypes.c_int32) for n in ("use_ns", "n_sub")] + [(n, ctypes.c_double) for n in ("nu", "rho0")] + [
        ("u0", ctypes.c_double * 3)]


DEFAULTS = dict(nx=24, ny=24, nz=24, walls=0, use_t=1, h_quintic=0, c_init_U=0, precision="f64",
                grad_iters=0, W0=1.0, tau0=20.0, eps4=0.05, lambda_=0.0, Mcinf=0.0, k=0.15, D=0.1,
                alpha=0.1, theta0=0.0, U0=0.0, C0=1.0, seed_R=5.0, seed_x=None, seed_y=None, seed_z=None,
                grad_tol=0.0, use_ns=0, n_sub=1, nu=0.1, rho0=1.0, u0x=0.0, u0y=0.0, u0z=0.0)
_IGNORED = {"name", "steps", "grad_max_iter", "fixed_as"}

_bound = False


def load_library() -> ctypes.CDLL:
    global _bound
    lib = _dlb.load_library()
    if not _bound:
        P, vp, dp = ctypes.POINTER, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        sig = {
            "dlb3_state_bytes": (ctypes.c_size_t, [P(Dlb3Params)]),
            "dlb3_create": (ctypes.c_int, [P(Dlb3Params), vp, ctypes.c_size_t, vp, P(vp)]),
            "dlb3_destroy": (ctypes.c_int, [vp]),
            "dlb3_init_seed": (ctypes.c_int, [vp]),
            "dlb3_set_fields": (ctypes.c_int, [vp, dp, dp, dp, dp, dp, dp]),
            "dlb3_step": (ctypes.c_int, [vp, ctypes.c_int64]),
            "dlb3_get_fields": (ctypes.c_int, [vp, dp]),
            "dlb3_reduce": (ctypes.c_int, [vp, dp]),
            "dlb3_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return lib


def make_params(cfg: dict) -> Dlb3Params:
    c = dict(DEFAULTS)
    for key, val in cfg.items():
        if key in _IGNORED:
            continue
        key = "lambda_" if key == "lambda" else key
        if key not in c:
            raise KeyError(f"unknown parameter {key!r}")
        c[key] = val
    p = Dlb3Params()
    for name in ("nx", "ny", "nz", "walls", "use_t", "h_quintic", "c_init_U", "grad_iters", "use_ns", "n_sub"):
        setattr(p, name, int(c[name]))
    p.nu, p.rho0 = float(c["nu"]), float(c["rho0"])
    p.u0[0], p.u0[1], p.u0[2] = float(c["u0x"]), float(c["u0y"]), float(c["u0z"])
    p.precision = PRECISION[c["precision"]] if isinstance(c["precision"], str) else int(c["precision"])
    for name in ("W0", "tau0", "eps4", "lambda_", "Mcinf", "k", "D", "alpha", "theta0", "U0", "C0", "seed_R",
                 "grad_tol"):
        setattr(p, name, float(c[name]))
    for a, n in (("seed_x", "nx"), ("seed_y", "ny"), ("seed_z", "nz")):
        setattr(p, a, float(c[n] // 2 if c[a] is None else c[a]))
    return p


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Solver3:
    """One 3-D simulation in caller-owned (torch) device memory; fields are
    (nz, ny, nx) arrays."""

    def __init__(self, cfg: dict, device: str = "cuda:0"):
        import torch

        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libdlb needs a GPU (no CPU fallback)")
        self.p = make_params(cfg)
        self.shape = (self.p.nz, self.p.ny, self.p.nx)
        self.device = torch.device(device)
        nbytes = self.lib.dlb3_state_bytes(ctypes.byref(self.p))
        if nbytes == 0:
            raise Dlb3Error(DLB3_EINVAL, self.lib.dlb3_last_error().decode())
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(self.device)
            self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = ctypes.c_void_p()
        self._check(self.lib.dlb3_create(ctypes.byref(self.p), ctypes.c_void_p(self.state.data_ptr()), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)))
        self.step_count = 0

    def _check(self, rc):
        if rc != DLB3_OK:
            raise Dlb3Error(rc, self.lib.dlb3_last_error().decode())

    def __del__(self):
        try:
            if self.handle.value:
                self.lib.dlb3_destroy(self.handle)
                self.handle = ctypes.c_void_p()
        except Exception:
            pass

    def _plane(self, a):
        if a is None:
            return None
        return np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=np.float64).ravel()

    def init_seed(self):
        self._check(self.lib.dlb3_init_seed(self.handle))
        self.step_count = 0
        return self

    def set_fields(self, phi, C=None, theta=None, ux=None, uy=None, uz=None):
        arrs = [self._plane(a) for a in (phi, C, theta, ux, uy, uz)]
        self._check(self.lib.dlb3_set_fields(self.handle, *[_dp(a) for a in arrs]))
        self.step_count = 0
        return self

    def step(self, n: int):
        self._check(self.lib.dlb3_step(self.handle, int(n)))
        self.step_count += int(n)
        return self

    def fields(self) -> dict:
        N = int(np.prod(self.shape))
        out = np.zeros(8 * N)
        self._check(self.lib.dlb3_get_fields(self.handle, _dp(out)))
        return {k: out[i * N:(i + 1) * N].reshape(self.shape) for i, k in enumerate(FIELDS)}

    def reduce(self) -> dict:
        out = np.zeros(10)
        self._check(self.lib.dlb3_reduce(self.handle, _dp(out)))
        return {"sum_C": out[0], "sum_H": out[1], "solid_fraction": out[2], "nonfinite": out[3],
                "tip_s": out[4:10].copy()}
