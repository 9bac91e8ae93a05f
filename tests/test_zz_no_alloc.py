"""dlb_get_fields_noalloc, the field read for callers that cannot allocate
device memory, against dlb_get_fields (which stages through hipMalloc): both
run the same field kernel, so the values must be identical, call after call,
while the static staging buffer keeps the previous call's contents."""
import ctypes

import numpy as np
import pytest

from paper_2209_01444_amd import workloads as W

pytestmark = pytest.mark.gpu
FIELDS = ("phi", "C", "U", "theta", "ux", "uy", "p")


@pytest.fixture(scope="module")
def dlb():
    from paper_2209_01444_amd import dlb as mod
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mod.load_library()
    return mod


def _read(solver, entry, mask, f32):
    n = bin(mask).count("1")
    out = np.full((n, solver.ny, solver.nx), np.nan, dtype=np.float32 if f32 else np.float64)
    ptr = out.ctypes.data_as(ctypes.c_void_p)
    if entry == "noalloc":
        rc = solver.lib.dlb_get_fields_noalloc(solver.handle, mask, ptr, int(f32))
    else:
        rc = solver.lib.dlb_get_fields(solver.handle, mask, ptr, 0, int(f32))
    assert rc == 0, solver.lib.dlb_last_error().decode()
    return out


def test_noalloc_read_matches_get_fields_on_consecutive_calls(dlb):
    print("case: no-alloc field read, 96x80 channel f32 (7 fields, FP32 out), then 40x32 FP64 (3 fields)",
          flush=True)
    cfg, noise = W.thermosolutal_flow(96, 80, seed=2, precision="f32")
    big = dlb.Solver(cfg).init_seed(noise).step(30)
    small_cfg = dict(W.pure_diffusion_128("f64"), nx=40, ny=32, seed_x=20.0, seed_y=16.0, seed_R=5.0)
    small = dlb.Solver(small_cfg).init_seed().step(10)
    cases = [(big, 0x7F, True), (small, 0b1011, False), (big, 0b0110001, False)]
    for solver, mask, f32 in cases:
        a = _read(solver, "noalloc", mask, f32)
        b = _read(solver, "alloc", mask, f32)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), f"{solver.nx}x{solver.ny} mask {mask:#x}"
    # the binding method gives the same named fields
    got = small.fields_noalloc(("phi", "C", "theta"))
    ref = small.fields(("phi", "C", "theta"))
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


def test_noalloc_read_rejects_a_selection_beyond_its_buffer(dlb):
    print("case: no-alloc field read size limit, 1024x1024", flush=True)
    cfg, noise = W.thermosolutal_flow(1024, 1024, seed=2, precision="f32")
    s = dlb.Solver(cfg).init_seed(noise)
    limit = dlb.NOALLOC_SCRATCH_BYTES
    assert 7 * 1024 * 1024 * 8 > limit >= 7 * 1024 * 1024 * 4
    out = np.empty((7, 1024, 1024))
    rc = s.lib.dlb_get_fields_noalloc(s.handle, 0x7F, out.ctypes.data_as(ctypes.c_void_p), 0)
    assert rc == dlb.DLB_EINVAL
    assert b"staging buffer" in s.lib.dlb_last_error()
    # all seven fields in FP32 fit, and match the allocating read
    a = _read(s, "noalloc", 0x7F, True)
    b = _read(s, "alloc", 0x7F, True)
    assert np.array_equal(a, b)
