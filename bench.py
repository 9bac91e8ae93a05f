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
    """Hash of the files holding the device code of the profiled kernels
    (k_pct and the fused flow launch), which counter records must match."""
    h = hashlib.sha256()
    for f in ("lattice.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2209_01444_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(cfg: dict) -> dict:
    """Bytes each kernel must move per node (each state word read once and
    written once; neighbour reuse assumed perfect)."""
    sb = {"f64": 8, "f32": 4, "f32m": 4, "f16s": 2, "bf16s": 2, "f16sm": 2}[cfg["precision"]]
    sc = 4 if cfg["precision"] == "f16sm" else sb  # solute and heat populations
    cb = 8 if cfg["precision"] == "f64" else 4  # history planes
    ns = bool(cfg.get("use_ns"))
    # k_pct: 15 populations in + out, 8 flow populations in (velocity),
    # history in + out (phi, Q and, with flow, C u, H u)
    hist = 6 if ns else 2
    pct = 10 * sb + 20 * sc + (8 * sb if ns else 0) + 2 * hist * cb
    # k_flow: 9 populations in + out, frozen phi in
    flow = 18 * sb + cb
    return {"pct": pct, "flow": flow, "step": pct + (cfg["n_sub"] * flow if ns else 0)}


# VALU issue rate of the chip: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64
# vector instruction per SIMD every 4 cycles
PEAK_VALU_INSTS_PER_S = 256 * 4 * 2.4e9 / 4
# Vector arithmetic peak without packed FP32 (kept out of the build): 256 CUs
# x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz = 78.6 TFLOP/s, which is
# also the FP64 vector peak.  (Packed FP32 doubles it to the published 157.3.)
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Flops of one D2Q9 flow node and sub-step as the collision computes it
# (moments, velocity and pressure, relaxation, inverse transform; an FMA
# counts 2): 70.  The streaming moves data only.
FLOW_FLOP_PER_NODE_SUBSTEP = 70


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


def measure(cfg: dict, noise, steps: int, warmup: int, timed_launch_steps: int) -> dict:
    """Whole-step rate and per-kernel launch times (HIP events on the
    solver's stream) of one workload, inputs resident in HBM."""
    import torch

    from paper_2209_01444_amd import dlb

    solver = dlb.Solver(cfg).init_seed(noise)
    nodes = cfg["nx"] * cfg["ny"]
    solver.step(warmup)
    solver.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(steps)
    solver.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tk = solver.step_timed(timed_launch_steps)
    red = solver.reduce(allow_nonfinite=True)
    out = {"solver": solver, "nodes": nodes, "elapsed": el, "mlups": nodes * steps / el / 1e6,
           "ms_per_step": el / steps * 1e3, "tk": tk, "reduce": red}
    out["step_count"] = solver.step_count
    return out


def kernel_rooflines(cfg: dict, m: dict, wl: str | None = None) -> dict:
    """Per-kernel figures of one measurement: the phi/C/theta kernel against
    the HBM peak (its algorithmic bytes), the flow launch against the vector
    arithmetic peak when it fuses several sub-steps (its data stays on chip
    between them), else against the HBM peak."""
    ab = algorithmic_bytes(cfg)
    tk, nodes = m["tk"], m["nodes"]
    flow_ms = tk["ms_flow"] / max(tk["launches_flow"], 1)
    pct_ms = tk["ms_pct"] / max(tk["launches_pct"], 1)
    subs = cfg["n_sub"] * tk["launches_pct"] / max(tk["launches_flow"], 1)
    pct_gbs = ab["pct"] * nodes / (pct_ms * 1e-3) / 1e9
    flow = {"avg_ms": round(flow_ms, 5), "substeps": subs}
    # bytes a flow launch must move at least: its populations and phi in, its populations out
    flow_min_bytes = ab["flow"] * nodes
    flow["hbm_min_bytes"] = flow_min_bytes
    flow["hbm_min_frac"] = round(flow_min_bytes / (flow_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    flops = FLOW_FLOP_PER_NODE_SUBSTEP * nodes * subs
    flow["flop"] = flops
    flow["TFLOPs"] = round(flops / (flow_ms * 1e-3) / 1e12, 3)
    flow["alu_frac"] = round(flops / (flow_ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS, 4)
    pct = {"avg_ms": round(pct_ms, 5), "GBs": round(pct_gbs, 1), "hbm_frac": round(pct_gbs / PEAK_HBM_GBS, 4),
           "bytes": ab["pct"] * nodes}
    if wl:
        # counter records (profiles/) taken on the current kernel sources, else null
        pct["traffic"] = traffic_from_profiles("k_pct", wl)
        pct["traffic_GBs"] = None if pct["traffic"] is None else round(pct["traffic"] / (pct_ms * 1e-3) / 1e9, 1)
        # counter records exist for the wave-row fused kernel and the one-sub-step kernel
        kf = ("k_flow" if subs == 1 else
              "k_flow_tbw" if cfg["precision"] not in ("f64", "f32m") else None)
        flow["traffic"] = traffic_from_profiles(kf, wl) if kf else None
        valu = valu_from_profiles(kf, wl) if kf else None
        flow["valu_issue_frac"] = None if valu is None else round(valu / (flow_ms * 1e-3) / PEAK_VALU_INSTS_PER_S, 4)
    return {"k_pct": pct,
            "flow_launch": flow,
            "whole_step_algorithmic_GBs": round(ab["step"] * nodes / (m["ms_per_step"] * 1e-3) / 1e9, 1)}


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


def surrogate_leg() -> dict:
    """Third part of the metric: time to main step 10000 of the hybrid loop
    (K = 100 network jumps, L = 100 lattice Boltzmann steps after each, the
    2% tip-velocity check with fallback) with the stored 512^2 network,
    against plain lattice Boltzmann, on the seed held out of its training;
    and the same with L = 50."""
    from paper_2209_01444_amd import surrogate

    if not os.path.exists(surrogate.BUNDLE):
        return {"skipped": f"no trained network at {os.path.relpath(surrogate.BUNDLE, ROOT)}"}
    def one(L):
        r = surrogate.speedup_check(L=L)
        return {"value": round(r["speedup"], 3), "tip_velocity_rel_err": round(r["tip_v_rel_err"], 5),
                "accepted": r["accepted"], "jumps": r["jumps"], "plain_s": round(r["plain_seconds"], 4),
                "hybrid_s": round(r["hybrid_seconds"], 4), "L": L}

    main = one(100)
    return {"metric": "surrogate time-to-solution speedup", **main, "bound": 0.02, "size": 512, "K": 100,
            "T": 10000, "network": os.path.relpath(surrogate.BUNDLE, ROOT),
            # a shorter lattice Boltzmann window after each jump: faster, closer to the bound
            "L50": one(50)}


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
    ap.add_argument("--hbm-size", type=int, default=4096,
                    help="also measure the workload at this grid size, whose state does not fit the "
                         "last-level cache (0: skip)")
    ap.add_argument("--hbm-steps", type=int, default=100)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate leg (hybrid loop with the stored network against plain LB)")
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
    m = measure(cfg, noise, args.steps, args.warmup, args.timed_launch_steps)
    wl = f"thermosolutal_flow_{cfg['nx']}x{cfg['ny']}_{cfg['precision']}"
    kr = kernel_rooflines(cfg, m, wl)
    ab = algorithmic_bytes(cfg)
    nodes = m["nodes"]
    fl = kr["flow_launch"]
    subs_per_launch = fl["substeps"]
    # FP32 arithmetic fuses with the wave-row tile kernel, FP64 arithmetic with the LDS tile kernel
    fused_name = "k_flow_tbw" if cfg["precision"] not in ("f64", "f32m") else "k_flow_tb"
    kname = fused_name if subs_per_launch > 1 else "k_flow"
    traffic = traffic_from_profiles(kname, wl)
    valu = valu_from_profiles(kname, wl)
    if subs_per_launch > 1:
        # several sub-steps per launch: the populations stay on chip between
        # them, so the launch is bound by vector arithmetic issue, not by HBM
        roof = {"bound": "alu", "kernel": f"{kname} (fused flow sub-steps)",
                "achieved": fl["TFLOPs"], "peak": round(PEAK_VALU_TFLOPS, 2), "unit": "TFLOP/s",
                "frac": fl["alu_frac"], "traffic": traffic,
                "flop_per_launch": fl["flop"], "flop_per_node_substep": FLOW_FLOP_PER_NODE_SUBSTEP,
                "peak_note": "non-packed vector FMA rate, 256 CU x 64 lanes x 2 x 2.4 GHz",
                "valu_issue_frac": (None if valu is None
                                    else round(valu / (fl["avg_ms"] * 1e-3) / PEAK_VALU_INSTS_PER_S, 4)),
                "hbm_min_bytes_per_launch": fl["hbm_min_bytes"], "hbm_min_frac": fl["hbm_min_frac"]}
    else:
        gbs = fl["hbm_min_bytes"] / (fl["avg_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_flow (one flow sub-step)", "achieved": round(gbs, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                "traffic": traffic, "bytes_per_launch": fl["hbm_min_bytes"]}
    roof.update({"substeps_per_launch": subs_per_launch, "avg_launch_ms": fl["avg_ms"]})
    red = m["reduce"]
    pct_arith = {"f64": "f64", "f32": "f64", "f32m": "f64", "f16s": "f32", "bf16s": "f32",
                 "f16sm": "f64"}[cfg["precision"]]
    flow_arith = {"f64": "f64", "f32": "f32", "f32m": "f64", "f16s": "f32", "bf16s": "f32",
                  "f16sm": "f32"}[cfg["precision"]]

    line = {
        "metric": "coupled-lattice MLUPS",
        "value": round(m["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": flow_arith if flow_arith == pct_arith else f"{flow_arith}/{pct_arith}",
        "data": "synthetic",
        "config": {"workload": wl, "nx": cfg["nx"], "ny": cfg["ny"], "n_sub": cfg["n_sub"],
                   "lattices": "phi D2Q5 + C D2Q5 + theta D2Q5 + flow D2Q9",
                   "storage": cfg["precision"],
                   "arithmetic": {"flow sub-steps": flow_arith, "phi/C/theta step": pct_arith,
                                  "reductions": "f64"},
                   "algorithmic_bytes_per_node_step": ab["step"], "parallelism": "single GPU",
                   "grad_phi": "stencil (ablation)" if args.grad_stencil else "local (Sec. 3.1)",
                   "heat_sub_steps": args.n_sub_t},
        "roofline": roof,
        "kernels": kr,
        "state": {"step": m["step_count"], "solid_fraction": red["solid_fraction"],
                  "nonfinite": red["nonfinite"]},
    }
    m["solver"].close()
    del m
    if args.hbm_size and args.hbm_size != args.size:
        # the same workload on a grid whose state is far larger than the
        # 256 MB last-level cache: every launch streams from HBM
        c2, n2 = workloads.thermosolutal_flow(args.hbm_size, args.hbm_size, seed=2, precision=args.precision)
        c2["flow_fuse"] = args.flow_fuse
        c2["grad_stencil"] = int(args.grad_stencil)
        c2["n_sub_t"] = args.n_sub_t
        m2 = measure(c2, n2, args.hbm_steps, max(2, args.warmup // 4), max(2, args.timed_launch_steps // 4))
        wl2 = f"thermosolutal_flow_{args.hbm_size}x{args.hbm_size}_{c2['precision']}"
        line["hbm_resident"] = {"workload": wl2,
                                "MLUPS": round(m2["mlups"], 2), "ms_per_step": round(m2["ms_per_step"], 5),
                                "steps": args.hbm_steps, "state_bytes": int(m2["solver"].state.numel()),
                                "kernels": kernel_rooflines(c2, m2, wl2)}
        m2["solver"].close()
    if not args.no_surrogate:
        try:
            line["surrogate"] = surrogate_leg()
        except Exception as e:  # the lattice figures above still stand; say what failed
            line["surrogate"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, noise)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
