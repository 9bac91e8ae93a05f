"""ctypes wrapper of the 3-D CPU FP64 oracle (``dlb3_oracle.c``): the
phase-field, solute and heat lattices on D3Q7, no melt flow.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/`` (and by nothing in the
product package).  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdlb3_oracle.so")
SRC = os.path.join(_HERE, "dlb3_oracle.c")
_OVERRIDE = os.environ.get("DLB3_ORACLE_LIB")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
           "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class O3Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in (
        "nx", "ny", "nz", "use_t", "walls", "h_quintic", "c_init_U", "grad_max_iter")] + [
        (n, ctypes.c_double) for n in (
            "W0", "tau0", "eps4", "lambda_", "Mcinf", "k", "D", "alpha", "theta0", "U0", "C0",
            "seed_R", "seed_x", "seed_y", "seed_z", "grad_tol", "fixed_as")] + [
        (n, ctypes.c_int) for n in ("use_ns", "n_sub")] + [(n, ctypes.c_double) for n in (
            "nu", "rho0", "u0x", "u0y", "u0z")]


DEFAULTS = dict(nx=24, ny=24, nz=24, use_t=1, walls=0, h_quintic=0, c_init_U=0, grad_max_iter=100,
                W0=1.0, tau0=20.0, eps4=0.05, lambda_=0.0, Mcinf=0.0, k=0.15, D=0.1, alpha=0.1,
                theta0=0.0, U0=0.0, C0=1.0, seed_R=5.0, seed_x=None, seed_y=None, seed_z=None,
                grad_tol=1e-14, fixed_as=0.0, use_ns=0, n_sub=1, nu=0.1, rho0=1.0, u0x=0.0, u0y=0.0, u0z=0.0)
_GPU_ONLY = {"precision", "name", "steps"}
FIELDS = ("phi", "C", "U", "theta")
FLOW_FIELDS = ("ux", "uy", "uz", "p")

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if _OVERRIDE:
        lib = ctypes.CDLL(_OVERRIDE)
    else:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    d = ctypes.c_double
    lib.o3_create.restype = vp
    lib.o3_create.argtypes = [ctypes.POINTER(O3Params)]
    lib.o3_destroy.argtypes = [vp]
    lib.o3_last_error.restype = ctypes.c_char_p
    lib.o3_init_seed.argtypes = [vp]
    lib.o3_set_fields.argtypes = [vp, dp, dp, dp, dp, dp, dp]
    lib.o3_eq_flow.argtypes = [d, d, d, d, d, dp]
    lib.o3_lambda19.argtypes = [d, dp]
    lib.o3_step.argtypes = [vp, ctypes.c_long]
    lib.o3_get_fields.argtypes = [vp, dp]
    lib.o3_reduce.argtypes = [vp, dp]
    lib.o3_anisotropy.argtypes = [d, d, d, d, dp]
    lib.o3_local_gradient.argtypes = [ctypes.POINTER(O3Params), d, d, d, dp]
    lib.o3_lambda.argtypes = [d, dp]
    lib.o3_step_count.restype = ctypes.c_long
    lib.o3_step_count.argtypes = [vp]
    _lib = lib
    return lib


def make_params(cfg: dict) -> O3Params:
    c = dict(DEFAULTS)
    for key, val in cfg.items():
        if key in _GPU_ONLY:
            continue
        key = "lambda_" if key == "lambda" else key
        if key not in c:
            raise KeyError(f"unknown parameter {key!r}")
        c[key] = val
    for a, n in (("seed_x", "nx"), ("seed_y", "ny"), ("seed_z", "nz")):
        if c[a] is None:
            c[a] = c[n] // 2
    p = O3Params()
    for name, _ in O3Params._fields_:
        setattr(p, name, c[name])
    return p


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def anisotropy(eps4, gx, gy, gz):
    o = np.zeros(4)
    load().o3_anisotropy(eps4, gx, gy, gz, _dptr(o))
    return o


def local_gradient(cfg, m1):
    p = make_params(cfg)
    o = np.zeros(8)
    load().o3_local_gradient(ctypes.byref(p), float(m1[0]), float(m1[1]), float(m1[2]), _dptr(o))
    return o


def eq_flow(rho0, p, ux, uy, uz):
    o = np.zeros(19)
    load().o3_eq_flow(rho0, p, ux, uy, uz, _dptr(o))
    return o


def lam19(s2):
    o = np.zeros(361)
    load().o3_lambda19(s2, _dptr(o))
    return o.reshape(19, 19)


def lam(s1):
    o = np.zeros(49)
    load().o3_lambda(s1, _dptr(o))
    return o.reshape(7, 7)


class Oracle3:
    """One 3-D simulation on the CPU oracle; fields are (nz, ny, nx) arrays."""

    def __init__(self, cfg: dict):
        self.lib = load()
        self.p = make_params(cfg)
        self.shape = (self.p.nz, self.p.ny, self.p.nx)
        self.h = self.lib.o3_create(ctypes.byref(self.p))
        if not self.h:
            raise ValueError(self.lib.o3_last_error().decode())

    def __del__(self):
        try:
            if self.h:
                self.lib.o3_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _plane(self, a):
        if a is None:
            return None
        return np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=np.float64).ravel()

    def init_seed(self):
        self.lib.o3_init_seed(self.h)
        return self

    def set_fields(self, phi, C=None, theta=None, ux=None, uy=None, uz=None):
        arrs = [self._plane(a) for a in (phi, C, theta, ux, uy, uz)]
        self._keep = arrs
        self.lib.o3_set_fields(self.h, *[_dptr(a) for a in arrs])
        return self

    def step(self, n: int):
        self.lib.o3_step(self.h, int(n))
        return self

    @property
    def step_count(self) -> int:
        return int(self.lib.o3_step_count(self.h))

    def fields(self) -> dict:
        N = int(np.prod(self.shape))
        out = np.zeros(8 * N)
        self.lib.o3_get_fields(self.h, _dptr(out))
        return {k: out[i * N:(i + 1) * N].reshape(self.shape) for i, k in enumerate(FIELDS + FLOW_FIELDS)}

    def reduce(self) -> dict:
        out = np.zeros(10)
        self.lib.o3_reduce(self.h, _dptr(out))
        return {"sum_C": out[0], "sum_H": out[1], "solid_fraction": out[2], "nonfinite": out[3],
                "tip_s": out[4:10].copy()}
