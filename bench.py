"""Benchmark: coupled four-lattice main steps of the diffuse-interface MRT
lattice Boltzmann method on one MI355X.

One step = one main step of the whole hot path: the phi/C/theta kernel plus
N_sub = 15 flow sub-steps, over the 1024^2 thermosolutal-with-flow workload
(FP32), inputs resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
  python bench.py --calibrate-copy   # plain copy kernel for counter scaling
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lattice.h", "kernels.h", "dlb.hip"):
        with open(os.path.join(ROOT, "paper_2209_01444_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(cfg: dict) -> dict:
    """Bytes each kernel must move per node (each state word read once and
    written once; neighbour reuse assumed perfect)."""
    sb = {"f64": 8, "f32": 4, "f32m": 4, "f16s": 2, "bf16s": 2}[cfg["precision"]]
    cb = 8 if cfg["precision"] == "f64" else 4  # history planes
    ns = bool(cfg.get("use_ns"))
    # k_pct: 15 populations in + out, 8 flow populations in (velocity),
    # history in + out (phi, Q and, with flow, C u, H u)
    hist = 6 if ns else 2
    pct = 30 * sb + (8 * sb if ns else 0) + 2 * hist * cb
    # k_flow: 9 populations in + out, frozen phi in
    flow = 18 * sb + cb
    return {"pct": pct, "flow": flow, "step": pct + (cfg["n_sub"] * flow if ns else 0)}


# VALU issue rate of the chip: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64
# vector instruction per SIMD every 4 cycles
PEAK_VALU_INSTS_PER_S = 256 * 4 * 2.4e9 / 4


def _profile_record(kind: str, kernel: str, workload: str) -> dict | None:
    """A committed counter summary, only if it was taken on the current
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def traffic_from_profiles(kernel: str, workload: str) -> float | None:
    """Counter-measured HBM bytes per launch (FETCH_SIZE and WRITE_SIZE,
    copy-calibrated)."""
    rec = _profile_record("traffic", kernel, workload)
    return rec.get("bytes_per_launch") if rec else None


def valu_from_profiles(kernel: str, workload: str) -> float | None:
    """Counter-measured wave-level VALU instructions per launch
    (SQ_INSTS_VALU)."""
    rec = _profile_record("valu", kernel, workload)
    return rec.get("valu_insts_per_launch") if rec else None


def cpu_baseline(cfg, noise, budget_s: float = 12.0) -> dict:
    from oracle import oracle as orc

    o = orc.Oracle(cfg).init_seed(noise)
    o.step(1)
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    nodes = cfg["nx"] * cfg["ny"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": nodes * steps / el / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} main steps of the same {cfg['nx']}x{cfg['ny']} workload "
                      f"(FP64 oracle, OpenMP), {el:.1f} s"}


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 5):
    import ctypes

    import torch

    from paper_2209_01444_amd import dlb

    lib = dlb.load_library()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(reps):
        rc = lib.dlb_copy_kernel(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                 nbytes, ctypes.c_void_p(st))
        assert rc == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lib.dlb_copy_kernel(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                            ctypes.c_void_p(st))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"copy_bytes": nbytes, "reps": reps,
                      "copy_GBs": 2 * nbytes * reps / el / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--flow-fuse", type=int, default=0, help="flow sub-steps per launch (0: library default)")
    ap.add_argument("--timed-launch-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--grad-stencil", action="store_true",
                    help="stencil-gradient ablation of the local scheme (not the method's default)")
    ap.add_argument("--n-sub-t", type=int, default=1,
                    help="heat sub-steps per main step (multi-time-scaling variant; the method's default is 1)")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver has no multi-GPU "
              "path, it measures one GPU's share of the workload", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch

    from paper_2209_01444_amd import dlb, workloads

    cfg, noise = workloads.thermosolutal_flow(args.size, args.size, seed=2, precision=args.precision)
    cfg["flow_fuse"] = args.flow_fuse
    cfg["grad_stencil"] = int(args.grad_stencil)
    cfg["n_sub_t"] = args.n_sub_t
    solver = dlb.Solver(cfg).init_seed(noise)
    nodes = cfg["nx"] * cfg["ny"]

    solver.step(args.warmup)
    solver.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(args.steps)
    solver.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    mlups = nodes * args.steps / el / 1e6
    ms_per_step = el / args.steps * 1e3

    # per-kernel durations from HIP events on the solver's stream
    tk = solver.step_timed(args.timed_launch_steps)
    ab = algorithmic_bytes(cfg)
    flow_ms = tk["ms_flow"] / max(tk["launches_flow"], 1)
    pct_ms = tk["ms_pct"] / max(tk["launches_pct"], 1)
    # a fused launch advances several flow sub-steps: count its algorithmic
    # bytes as that many sub-steps of 76 B/node (FP32)
    subs_per_launch = cfg["n_sub"] * tk["launches_pct"] / max(tk["launches_flow"], 1)
    flow_bytes = ab["flow"] * nodes * subs_per_launch
    achieved = flow_bytes / (flow_ms * 1e-3) / 1e9
    wl = f"thermosolutal_flow_{cfg['nx']}x{cfg['ny']}_{cfg['precision']}"
    # FP32 arithmetic fuses with the wave-row tile kernel, FP64 arithmetic with the LDS tile kernel
    fused_name = "k_flow_tb" if cfg["precision"] in ("f64", "f32m") else "k_flow_tbw"
    valu = valu_from_profiles(fused_name if subs_per_launch > 1 else "k_flow", wl)
    red = solver.reduce(allow_nonfinite=True)

    line = {
        "metric": "coupled-lattice MLUPS",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfg["precision"],
        "data": "synthetic",
        "config": {"workload": wl, "nx": cfg["nx"], "ny": cfg["ny"], "n_sub": cfg["n_sub"],
                   "lattices": "phi D2Q5 + C D2Q5 + theta D2Q5 + flow D2Q9",
                   "algorithmic_bytes_per_node_step": ab["step"], "parallelism": "single GPU",
                   "grad_phi": "stencil (ablation)" if args.grad_stencil else "local (Sec. 3.1)",
                   "heat_sub_steps": args.n_sub_t},
        "roofline": {
            "bound": "hbm",
            "kernel": f"{fused_name} (fused flow sub-steps)" if subs_per_launch > 1 else "k_flow (flow sub-step)",
            "substeps_per_launch": subs_per_launch,
            "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic_from_profiles(fused_name if subs_per_launch > 1 else "k_flow", wl),
            "avg_launch_ms": round(flow_ms, 5), "bytes_per_launch": flow_bytes,
            "valu_issue_frac": (None if valu is None
                                else round(valu / (flow_ms * 1e-3) / PEAK_VALU_INSTS_PER_S, 4)),
        },
        "kernels": {
            "k_pct": {"avg_ms": round(pct_ms, 5), "GBs": round(ab["pct"] * nodes / (pct_ms * 1e-3) / 1e9, 1)},
            "flow_launch": {"avg_ms": round(flow_ms, 5), "GBs": round(achieved, 1),
                            "substeps": subs_per_launch},
            "whole_step_algorithmic_GBs": round(ab["step"] * nodes / (ms_per_step * 1e-3) / 1e9, 1),
        },
        "state": {"step": solver.step_count, "solid_fraction": red["solid_fraction"],
                  "nonfinite": red["nonfinite"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, noise)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
