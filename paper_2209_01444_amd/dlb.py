"""Python binding of libdlb.so (include/dlb.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module
allocates the caller-owned device state with torch, hands the library a
torch stream, and converts arguments.  It fails loudly when the library is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libdlb.so")

DLB_OK, DLB_EINVAL, DLB_ENOMEM, DLB_EHIP, DLB_ENAN, DLB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
# size of the static staging buffer of dlb_get_fields_noalloc (DLB_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 32 << 20
PRECISION = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3, "f32m": 4, "f16sm": 5}
FIELDS = ("phi", "C", "U", "theta", "ux", "uy", "p")


class DlbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dlb error {code}: {msg}")
        self.code = code


class DlbParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "nx", "ny", "use_ns", "bc", "n_sub", "h_quintic", "c_init_U", "precision", "grad_iters",
        "flow_fuse", "phi_static", "isothermal", "grad_stencil", "n_sub_t", "tile_rows")] + [
        (n, ctypes.c_double) for n in (
            "W0", "tau0", "eps4", "orient", "lambda_", "Mcinf", "k", "D", "alpha", "nu", "rho0",
            "u_in_x", "u_in_y", "theta0", "U0", "C0", "seed_R", "seed_x", "seed_y", "noise_amp",
            "grad_tol", "force_x", "force_y", "varphi")]


KEEP_FLOW, KEEP_NONEQ = 1, 2  # continuation flags of dlb_set_fields_ex

EXPORTS = (
    "dlb_state_bytes", "dlb_create", "dlb_destroy", "dlb_init_seed", "dlb_set_fields", "dlb_set_fields_ex", "dlb_step",
    "dlb_step_timed", "dlb_step_count", "dlb_get_fields", "dlb_get_fields_noalloc", "dlb_reduce", "dlb_checkpoint_bytes",
    "dlb_save", "dlb_load", "dlb_copy_state", "dlb_sync", "dlb_equilibria", "dlb_copy_kernel", "dlb_strerror",
    "dlb_last_error", "dlb_batch_state_bytes", "dlb_batch_create", "dlb_batch_destroy",
    "dlb_batch_member", "dlb_batch_step", "dlb_batch_step_count", "dlb_batch_set_config",
    "dlb_batch_get_config", "dlb_batch_set_node_tile", "dlb_batch_get_node_tile", "dlb_batch_autotune",
)

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdlb.so (built in-tree by paper_2209_01444_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2209_01444_amd/build.py`"
                          " (there is no CPU fallback)")
    if path == LIB_PATH:
        from paper_2209_01444_amd import build
        build.warn_if_stale(path, build.DEPS)
    lib = ctypes.CDLL(path)
    P, vp, d, i64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64
    dp = P(d)
    sig = {
        "dlb_state_bytes": (ctypes.c_size_t, [P(DlbParams)]),
        "dlb_create": (ctypes.c_int, [P(DlbParams), vp, ctypes.c_size_t, vp, P(vp)]),
        "dlb_destroy": (ctypes.c_int, [vp]),
        "dlb_init_seed": (ctypes.c_int, [vp, dp]),
        "dlb_set_fields": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.c_int]),
        "dlb_set_fields_ex": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_uint32]),
        "dlb_step": (ctypes.c_int, [vp, i64]),
        "dlb_step_timed": (ctypes.c_int, [vp, i64, dp, dp, P(i64), P(i64)]),
        "dlb_step_count": (i64, [vp]),
        "dlb_get_fields": (ctypes.c_int, [vp, ctypes.c_uint32, vp, ctypes.c_int, ctypes.c_int]),
        "dlb_get_fields_noalloc": (ctypes.c_int, [vp, ctypes.c_uint32, vp, ctypes.c_int]),
        "dlb_reduce": (ctypes.c_int, [vp, dp]),
        "dlb_checkpoint_bytes": (ctypes.c_size_t, [vp]),
        "dlb_save": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "dlb_load": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "dlb_sync": (ctypes.c_int, [vp]),
        "dlb_copy_state": (ctypes.c_int, [vp, vp]),
        "dlb_equilibria": (ctypes.c_int, [i64, dp, dp, ctypes.c_int]),
        "dlb_copy_kernel": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "dlb_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "dlb_last_error": (ctypes.c_char_p, []),
        "dlb_batch_state_bytes": (ctypes.c_size_t, [P(DlbParams), ctypes.c_int]),
        "dlb_batch_create": (ctypes.c_int, [P(DlbParams), ctypes.c_int, vp, ctypes.c_size_t, vp, P(vp)]),
        "dlb_batch_destroy": (ctypes.c_int, [vp]),
        "dlb_batch_member": (vp, [vp, ctypes.c_int]),
        "dlb_batch_step": (ctypes.c_int, [vp, i64]),
        "dlb_batch_step_count": (i64, [vp]),
        "dlb_batch_set_config": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "dlb_batch_get_config": (ctypes.c_int, [vp, P(ctypes.c_int)]),
        "dlb_batch_set_node_tile": (ctypes.c_int, [vp, ctypes.c_int]),
        "dlb_batch_get_node_tile": (ctypes.c_int, [vp]),
        "dlb_batch_autotune": (ctypes.c_int, [vp, ctypes.c_int, dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(lib, rc: int):
    if rc != DLB_OK:
        raise DlbError(rc, lib.dlb_last_error().decode())


DEFAULTS = dict(
    nx=64, ny=64, use_ns=0, walls=0, n_sub=1, h_quintic=0, c_init_U=0, precision="f64",
    grad_iters=0, flow_fuse=0, phi_static=0, grad_stencil=0, n_sub_t=1, tile_rows=0, W0=1.0, tau0=20.0, eps4=0.05, orient=0.0, lambda_=0.0, Mcinf=0.0, k=0.15, D=0.1,
    alpha=0.1, nu=0.1, rho0=1.0, u_in=(0.0, 0.0), theta0=0.0, U0=0.0, C0=1.0, seed_R=8.0,
    seed_x=None, seed_y=None, noise_amp=0.0, grad_tol=0.0, use_c=1, use_t=1,
    force_x=0.0, force_y=0.0, varphi=0.0,
)
_IGNORED = {"name", "steps"}


def make_params(cfg: dict) -> DlbParams:
    c = dict(DEFAULTS)
    for key, val in cfg.items():
        if key in _IGNORED:
            continue
        key = "lambda_" if key == "lambda" else key
        if key not in c:
            raise KeyError(f"unknown parameter {key!r}")
        c[key] = val
    if not c["use_c"]:
        raise ValueError("the GPU solver always runs the solute lattice")
    p = DlbParams()
    p.nx, p.ny = int(c["nx"]), int(c["ny"])
    p.use_ns = int(c["use_ns"])
    p.bc = int(c["walls"])
    p.n_sub = int(c["n_sub"])
    p.h_quintic = int(c["h_quintic"])
    p.c_init_U = int(c["c_init_U"])
    p.precision = PRECISION[c["precision"]] if isinstance(c["precision"], str) else int(c["precision"])
    p.grad_iters = int(c["grad_iters"])
    p.flow_fuse = int(c["flow_fuse"])
    p.phi_static = int(c["phi_static"])
    p.isothermal = 0 if c["use_t"] else 1
    p.grad_stencil = int(c["grad_stencil"])
    p.n_sub_t = int(c["n_sub_t"])
    p.tile_rows = int(c["tile_rows"])
    for name in ("W0", "tau0", "eps4", "orient", "lambda_", "Mcinf", "k", "D", "alpha", "nu", "rho0",
                 "theta0", "U0", "C0", "seed_R", "noise_amp", "grad_tol", "force_x", "force_y", "varphi"):
        setattr(p, name, float(c[name]))
    p.u_in_x, p.u_in_y = float(c["u_in"][0]), float(c["u_in"][1])
    p.seed_x = float(c["nx"] // 2 if c["seed_x"] is None else c["seed_x"])
    p.seed_y = float(c["ny"] // 2 if c["seed_y"] is None else c["seed_y"])
    return p


def _host_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Solver:
    """One lattice Boltzmann simulation in caller-owned (torch) device memory."""

    def __init__(self, cfg: dict, device: str = "cuda:0", stream=None, _member_of=None, _handle=None):
        import torch

        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libdlb needs a GPU (no CPU fallback)")
        self.cfg = dict(cfg)
        self.p = make_params(cfg)
        self.nx, self.ny = self.p.nx, self.p.ny
        self.device = torch.device(device)
        if _member_of is not None:  # borrowed view of a batch member
            self._owner = _member_of
            self.stream = _member_of.stream
            self.handle = ctypes.c_void_p(_handle)
            self._borrowed = True
            return
        self._borrowed = False
        nbytes = self.lib.dlb_state_bytes(ctypes.byref(self.p))
        if nbytes == 0:
            raise DlbError(DLB_EINVAL, self.lib.dlb_last_error().decode())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = ctypes.c_void_p()
        _check(self.lib, self.lib.dlb_create(ctypes.byref(self.p), ctypes.c_void_p(self.state.data_ptr()),
                                             nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(self.handle)))

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_borrowed", False):
            return
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.dlb_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _plane(self, a):
        if a is None:
            return None
        return np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny * self.nx)

    def init_seed(self, noise=None):
        n = self._plane(noise)
        _check(self.lib, self.lib.dlb_init_seed(self.handle, None if n is None else
                                                n.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return self

    def set_fields(self, phi, C=None, theta=None, ux=None, uy=None, keep_flow=False,
                   keep_noneq=False):
        """Host numpy arrays or device torch tensors (float64, ny x nx);
        keep_flow / keep_noneq select the continuation flags of
        dlb_set_fields_ex."""
        arrs = (phi, C, theta, ux, uy)
        flags = (KEEP_FLOW if keep_flow else 0) | (KEEP_NONEQ if keep_noneq else 0)
        if any(self.torch.is_tensor(a) for a in arrs if a is not None):
            keep = [None if a is None else a.to(self.device, self.torch.float64).contiguous()
                    for a in arrs]
            ptrs = [None if a is None else ctypes.c_void_p(a.data_ptr()) for a in keep]
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
            _check(self.lib, self.lib.dlb_set_fields_ex(self.handle, *ptrs, 1, flags))
            self.stream.synchronize()
            return self
        keep = [self._plane(a) for a in arrs]
        _check(self.lib, self.lib.dlb_set_fields_ex(self.handle, *[_host_ptr(a) for a in keep], 0, flags))
        return self

    def step(self, n: int):
        _check(self.lib, self.lib.dlb_step(self.handle, int(n)))
        return self

    def step_timed(self, n: int) -> dict:
        a, b = ctypes.c_double(), ctypes.c_double()
        la, lb = ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib, self.lib.dlb_step_timed(self.handle, int(n), ctypes.byref(a), ctypes.byref(b),
                                                 ctypes.byref(la), ctypes.byref(lb)))
        return dict(ms_pct=a.value, ms_flow=b.value, launches_pct=la.value, launches_flow=lb.value)

    def sync(self):
        _check(self.lib, self.lib.dlb_sync(self.handle))

    @property
    def step_count(self) -> int:
        return int(self.lib.dlb_step_count(self.handle))

    # -- observation ------------------------------------------------------
    def fields(self, names=FIELDS) -> dict:
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS.index(nm)
        sel = [f for f in FIELDS if mask & (1 << FIELDS.index(f))]
        out = np.empty((len(sel), self.ny, self.nx), dtype=np.float64)
        _check(self.lib, self.lib.dlb_get_fields(self.handle, mask, out.ctypes.data_as(ctypes.c_void_p),
                                                 0, 0))
        return {f: out[i] for i, f in enumerate(sel)}

    def fields_noalloc(self, names=FIELDS, f32: bool = False) -> dict:
        """As fields(), through dlb_get_fields_noalloc (a static device
        staging buffer, no device allocation)."""
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS.index(nm)
        sel = [f for f in FIELDS if mask & (1 << FIELDS.index(f))]
        out = np.empty((len(sel), self.ny, self.nx), dtype=np.float32 if f32 else np.float64)
        _check(self.lib, self.lib.dlb_get_fields_noalloc(self.handle, mask, out.ctypes.data_as(ctypes.c_void_p),
                                                         int(f32)))
        return {f: out[i] for i, f in enumerate(sel)}

    def fields_device(self, names=FIELDS, f32: bool = True):
        """Selected fields as a (n_fields, ny, nx) torch tensor on the device."""
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS.index(nm)
        n = bin(mask).count("1")
        dt = self.torch.float32 if f32 else self.torch.float64
        with self.torch.cuda.device(self.device):
            out = self.torch.empty((n, self.ny, self.nx), dtype=dt, device=self.device)
        _check(self.lib, self.lib.dlb_get_fields(self.handle, mask, ctypes.c_void_p(out.data_ptr()), 1,
                                                 int(f32)))
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def reduce(self, allow_nonfinite: bool = False) -> dict:
        out = np.empty(19)
        rc = self.lib.dlb_reduce(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if rc != DLB_OK and not (rc == DLB_ENAN and allow_nonfinite):
            _check(self.lib, rc)
        keys = ("sum_C", "sum_H", "solid_fraction", "nonfinite", "Fx", "Fy", "torque")
        r = {k: float(out[i]) for i, k in enumerate(keys)}
        r["tip_s"] = out[7:11].copy()
        r["tip_rho"] = out[11:15].copy()
        r["centroid"] = out[15:17].copy()
        r["Fx_solid"], r["Fy_solid"] = float(out[17]), float(out[18])
        r["code"] = rc
        return r

    # -- checkpoint -------------------------------------------------------
    def save(self) -> bytes:
        n = self.lib.dlb_checkpoint_bytes(self.handle)
        buf = ctypes.create_string_buffer(n)
        _check(self.lib, self.lib.dlb_save(self.handle, ctypes.cast(buf, ctypes.c_void_p), n))
        return buf.raw

    def copy_from(self, other: "Solver"):
        """Device-to-device copy of another solver's state (same parameters)."""
        _check(self.lib, self.lib.dlb_copy_state(self.handle, other.handle))
        return self

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.lib, self.lib.dlb_load(self.handle, ctypes.cast(buf, ctypes.c_void_p), len(blob)))
        return self


class Batch:
    """Independent solvers stepped in lockstep by one launch per kernel
    class over a (seed, tile) work list (see dlb_batch_* in include/dlb.h)."""

    def __init__(self, cfgs: list[dict], device: str = "cuda:0"):
        import torch

        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libdlb needs a GPU (no CPU fallback)")
        self.cfgs = [dict(c) for c in cfgs]
        n = len(cfgs)
        self.params = (DlbParams * n)(*[make_params(c) for c in cfgs])
        nbytes = self.lib.dlb_batch_state_bytes(self.params, n)
        if nbytes == 0:
            raise DlbError(DLB_EINVAL, self.lib.dlb_last_error().decode())
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(self.device)
            self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = ctypes.c_void_p()
        _check(self.lib, self.lib.dlb_batch_create(self.params, n, ctypes.c_void_p(self.state.data_ptr()),
                                                   nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                                   ctypes.byref(self.handle)))
        self.members = [Solver(c, device, _member_of=self, _handle=self.lib.dlb_batch_member(self.handle, i))
                        for i, c in enumerate(cfgs)]

    @property
    def nodes(self) -> int:
        return sum(c["nx"] * c["ny"] for c in self.cfgs)

    def step(self, n: int):
        _check(self.lib, self.lib.dlb_batch_step(self.handle, int(n)))
        return self

    def sync(self):
        self.stream.synchronize()

    @property
    def step_count(self) -> int:
        return int(self.lib.dlb_batch_step_count(self.handle))

    def set_config(self, fuse: int, bpc_node: int, bpc_tb: int):
        _check(self.lib, self.lib.dlb_batch_set_config(self.handle, fuse, bpc_node, bpc_tb))

    def config(self) -> tuple:
        out = (ctypes.c_int * 3)()
        _check(self.lib, self.lib.dlb_batch_get_config(self.handle, out))
        return tuple(out)

    def set_node_tile(self, width: int):
        """Node tile of the batched node kernels: width x 256/width nodes."""
        _check(self.lib, self.lib.dlb_batch_set_node_tile(self.handle, int(width)))

    @property
    def node_tile(self) -> int:
        w = int(self.lib.dlb_batch_get_node_tile(self.handle))
        if w < 0:
            _check(self.lib, w)
        return w

    def autotune(self, trial_steps: int = 20) -> float:
        """Pick the fastest launch configuration (consumes the state)."""
        ms = ctypes.c_double()
        _check(self.lib, self.lib.dlb_batch_autotune(self.handle, int(trial_steps), ctypes.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.dlb_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def equilibria(macros: np.ndarray, h_quintic: int = 0) -> np.ndarray:
    """FP64 device equilibria for rows (phi, C, U, theta, ux, uy, p, rho0)."""
    lib = load_library()
    m = np.ascontiguousarray(macros, dtype=np.float64)
    out = np.empty((m.shape[0], 24))
    _check(lib, lib.dlb_equilibria(m.shape[0], m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(h_quintic)))
    return out
