"""ctypes wrapper of the CPU FP64 oracle (``dlb_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``; the
product package never imports it.  It shares no code with the GPU library:
the configuration dictionary it accepts is plain data, marshalled here into
the oracle's own parameter struct.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdlb_oracle.so")
SRC = os.path.join(_HERE, "dlb_oracle.c")
# A test may point the wrapper at a deliberately mutated build of the oracle
# (tests/test_oracle_mutations.py) to show that the pins catch the mutation.
_OVERRIDE = os.environ.get("DLB_ORACLE_LIB")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in (
        "nx", "ny", "use_c", "use_t", "use_ns", "walls", "n_sub", "h_quintic", "c_init_U",
        "grad_max_iter", "phi_static", "grad_stencil", "n_sub_t")] + [(n, ctypes.c_double) for n in (
            "W0", "tau0", "eps4", "orient", "lambda_", "Mcinf", "k", "D", "alpha", "nu", "rho0",
            "u_in_x", "u_in_y", "theta0", "U0", "C0", "seed_R", "seed_x", "seed_y", "noise_amp",
            "grad_tol", "fixed_as", "force_x", "force_y", "varphi")]


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
    P = ctypes.POINTER
    d = ctypes.c_double
    dp = P(d)
    vp = ctypes.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [P(OrcParams)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_last_error.restype = ctypes.c_char_p
    lib.orc_init_seed.argtypes = [vp, dp]
    lib.orc_set_fields.argtypes = [vp, dp, dp, dp, dp, dp]
    lib.orc_set_fields_ex.argtypes = [vp, dp, dp, dp, dp, dp, ctypes.c_uint]
    lib.orc_step.argtypes = [vp, ctypes.c_long]
    lib.orc_step_count.restype = ctypes.c_long
    lib.orc_step_count.argtypes = [vp]
    lib.orc_get_fields.argtypes = [vp, dp]
    lib.orc_get_pops.argtypes = [vp, ctypes.c_int, dp]
    lib.orc_reduce.argtypes = [vp, dp]
    lib.orc_m_d2q5.argtypes = [dp]
    lib.orc_m_d2q9.argtypes = [dp]
    lib.orc_lambda_d2q5.argtypes = [d, d, d, dp]
    lib.orc_lambda_d2q9.argtypes = [dp, dp]
    lib.orc_eq_phi.argtypes = [d, dp]
    lib.orc_eq_solute.argtypes = [d, d, d, d, d, dp]
    lib.orc_eq_heat.argtypes = [d, d, ctypes.c_int, d, d, dp]
    lib.orc_eq_flow.argtypes = [d, d, d, d, dp]
    lib.orc_force_flow.argtypes = [d, d, dp]
    lib.orc_force_flow_full.argtypes = [d, d, d, d, d, d, d, dp]
    lib.orc_anisotropy.argtypes = [d, d, d, d, dp]
    lib.orc_local_gradient.argtypes = [P(OrcParams), d, d, dp]
    lib.orc_collide_flow.argtypes = [P(OrcParams), dp, d, dp, dp]
    _lib = lib
    return lib


DEFAULTS = dict(
    nx=64, ny=64, use_c=1, use_t=1, use_ns=0, walls=0, n_sub=1, h_quintic=0, c_init_U=0,
    grad_max_iter=100, phi_static=0, grad_stencil=0, n_sub_t=1, W0=1.0, tau0=20.0, eps4=0.05, orient=0.0, lambda_=0.0, Mcinf=0.0,
    k=0.15, D=0.1, alpha=0.1, nu=0.1, rho0=1.0, u_in=(0.0, 0.0), theta0=0.0, U0=0.0, C0=1.0,
    seed_R=8.0, seed_x=None, seed_y=None, noise_amp=0.0, grad_tol=1e-14, fixed_as=0.0,
    force_x=0.0, force_y=0.0, varphi=0.0,
)

# keys of a workload dictionary that only concern the GPU library
_GPU_ONLY = {"precision", "grad_iters", "flow_fuse", "name", "steps"}


def make_params(cfg: dict) -> OrcParams:
    c = dict(DEFAULTS)
    for key, val in cfg.items():
        if key in _GPU_ONLY:
            continue
        key = "lambda_" if key == "lambda" else key
        if key not in c:
            raise KeyError(f"unknown parameter {key!r}")
        c[key] = val
    if c["seed_x"] is None:
        c["seed_x"] = c["nx"] // 2
    if c["seed_y"] is None:
        c["seed_y"] = c["ny"] // 2
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        if name in ("u_in_x", "u_in_y"):
            continue
        setattr(p, name, c[name])
    p.u_in_x, p.u_in_y = float(c["u_in"][0]), float(c["u_in"][1])
    return p


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


FIELDS = ("phi", "C", "U", "theta", "ux", "uy", "p")
REDUCE_KEYS = ("sum_C", "sum_H", "solid_fraction", "nonfinite", "Fx", "Fy", "torque")


class Oracle:
    """One simulation on the CPU oracle."""

    def __init__(self, cfg: dict):
        self.lib = load()
        self.p = make_params(cfg)
        self.nx, self.ny = self.p.nx, self.p.ny
        self.h = self.lib.orc_create(ctypes.byref(self.p))
        if not self.h:
            raise ValueError(self.lib.orc_last_error().decode())

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _plane(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny * self.nx)
        return a

    def init_seed(self, noise=None):
        n = self._plane(noise)
        rc = self.lib.orc_init_seed(self.h, _dptr(n))
        if rc:
            raise RuntimeError(self.lib.orc_last_error().decode())
        return self

    def set_fields(self, phi, C=None, theta=None, ux=None, uy=None, keep_flow=False,
                   keep_noneq=False):
        """orc_set_fields / orc_set_fields_ex (continuation flags)."""
        arrs = [self._plane(a) for a in (phi, C, theta, ux, uy)]
        flags = (1 if keep_flow else 0) | (2 if keep_noneq else 0)
        rc = self.lib.orc_set_fields_ex(self.h, *[_dptr(a) for a in arrs], flags)
        if rc:
            raise RuntimeError(self.lib.orc_last_error().decode())
        return self

    def step(self, n: int):
        self.lib.orc_step(self.h, int(n))
        return self

    @property
    def step_count(self) -> int:
        return self.lib.orc_step_count(self.h)

    def fields(self) -> dict:
        out = np.empty(7 * self.nx * self.ny)
        self.lib.orc_get_fields(self.h, _dptr(out))
        out = out.reshape(7, self.ny, self.nx)
        return {k: out[i].copy() for i, k in enumerate(FIELDS)}

    def pops(self, lattice: int) -> np.ndarray:
        q = 9 if lattice == 3 else 5
        out = np.empty(q * self.nx * self.ny)
        self.lib.orc_get_pops(self.h, int(lattice), _dptr(out))
        return out.reshape(q, self.ny, self.nx)

    def reduce(self) -> dict:
        out = np.empty(19)
        self.lib.orc_reduce(self.h, _dptr(out))
        r = {k: float(out[i]) for i, k in enumerate(REDUCE_KEYS)}
        r["tip_s"] = out[7:11].copy()
        r["tip_rho"] = out[11:15].copy()
        r["centroid"] = out[15:17].copy()
        r["Fx_solid"], r["Fy_solid"] = float(out[17]), float(out[18])
        return r


# ---- single-node primitives -------------------------------------------------

def _vec(n):
    return np.zeros(n)


def m_d2q5():
    o = _vec(25); load().orc_m_d2q5(_dptr(o)); return o.reshape(5, 5)


def m_d2q9():
    o = _vec(81); load().orc_m_d2q9(_dptr(o)); return o.reshape(9, 9)


def lambda_d2q5(s0, s1, s2):
    o = _vec(25); load().orc_lambda_d2q5(s0, s1, s2, _dptr(o)); return o.reshape(5, 5)


def lambda_d2q9(s9):
    s = np.ascontiguousarray(s9, dtype=np.float64)
    o = _vec(81); load().orc_lambda_d2q9(_dptr(s), _dptr(o)); return o.reshape(9, 9)


def eq_phi(phi):
    o = _vec(5); load().orc_eq_phi(phi, _dptr(o)); return o


def eq_solute(C, phi, U, ux, uy):
    o = _vec(5); load().orc_eq_solute(C, phi, U, ux, uy, _dptr(o)); return o


def eq_heat(theta, phi, ux, uy, h_quintic=0):
    o = _vec(5); load().orc_eq_heat(theta, phi, int(h_quintic), ux, uy, _dptr(o)); return o


def eq_flow(rho0, p, ux, uy):
    o = _vec(9); load().orc_eq_flow(rho0, p, ux, uy, _dptr(o)); return o


def force_flow(Fx, Fy):
    o = _vec(9); load().orc_force_flow(Fx, Fy, _dptr(o)); return o


def force_flow_full(Gx, Gy, Fx, Fy, ux, uy, varphi):
    o = _vec(9); load().orc_force_flow_full(Gx, Gy, Fx, Fy, ux, uy, varphi, _dptr(o)); return o


def anisotropy(eps4, orient, gx, gy):
    o = _vec(3); load().orc_anisotropy(eps4, orient, gx, gy, _dptr(o)); return o


def local_gradient(cfg, m1x, m1y):
    p = make_params(cfg)
    o = _vec(6); load().orc_local_gradient(ctypes.byref(p), m1x, m1y, _dptr(o)); return o


def stencil_gradient(cfg, phi, x, y):
    p = make_params(dict(cfg, nx=phi.shape[1], ny=phi.shape[0]))
    f = np.ascontiguousarray(phi, dtype=np.float64)
    o = _vec(2); load().orc_stencil_gradient(ctypes.byref(p), _dptr(f), int(x), int(y), _dptr(o)); return o


def collide_flow(cfg, h, phi):
    p = make_params(cfg)
    h = np.ascontiguousarray(h, dtype=np.float64)
    post = _vec(9); aux = _vec(4)
    load().orc_collide_flow(ctypes.byref(p), _dptr(h), phi, _dptr(post), _dptr(aux))
    return post, aux
