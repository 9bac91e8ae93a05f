"""Host-side checks of bench.py: algorithmic byte counts, the single-GPU
guard and the readers of the committed counter summaries."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_node_step():
    # FP32 with flow: k_pct moves 15 populations in and out, reads 8 moving
    # flow populations and reads and writes 6 history planes; each of the
    # 15 flow sub-steps moves 9 populations in and out and reads phi
    cfg = {"precision": "f32", "use_ns": 1, "n_sub": 15}
    ab = bench.algorithmic_bytes(cfg)
    assert ab["pct"] == 30 * 4 + 8 * 4 + 2 * 6 * 4
    assert ab["flow"] == 18 * 4 + 4
    assert ab["step"] == 1340
    # 16-bit storage halves the population bytes, history stays FP32
    ab16 = bench.algorithmic_bytes(dict(cfg, precision="f16s"))
    assert ab16["flow"] == 18 * 2 + 4 and ab16["pct"] == 30 * 2 + 8 * 2 + 48
    # mixed 16-bit storage: phi and flow populations 2 B, solute and heat 4 B
    abm = bench.algorithmic_bytes(dict(cfg, precision="f16sm"))
    assert abm["pct"] == 10 * 2 + 20 * 4 + 8 * 2 + 48 and abm["flow"] == ab16["flow"]
    # no flow: 15 populations and 2 history planes
    ab0 = bench.algorithmic_bytes({"precision": "f64", "use_ns": 0, "n_sub": 1})
    assert ab0["step"] == ab0["pct"] == 30 * 8 + 2 * 2 * 8


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_valu_issue_peak():
    # 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction
    assert bench.PEAK_VALU_INSTS_PER_S == pytest.approx(614.4e9)


def test_counter_records_follow_the_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernel_source_hash()
    (prof / "traffic_kx_wl.json").write_text(json.dumps({"source_hash": h, "bytes_per_launch": 123.0}))
    (prof / "valu_kx_wl.json").write_text(json.dumps({"source_hash": h, "valu_insts_per_launch": 7}))
    (prof / "traffic_ky_wl.json").write_text(json.dumps({"source_hash": "stale", "bytes_per_launch": 1.0}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.traffic_from_profiles("kx", "wl") == 123.0
    assert bench.valu_from_profiles("kx", "wl") == 7
    assert bench.traffic_from_profiles("ky", "wl") is None  # taken on other sources
    assert bench.valu_from_profiles("kz", "wl") is None     # absent


def test_vector_peak_and_kernel_rooflines():
    # non-packed vector FMA: 256 CUs x 64 lanes x 2 flops x 2.4 GHz
    assert bench.PEAK_VALU_TFLOPS == pytest.approx(78.6432)
    cfg = {"precision": "f32", "use_ns": 1, "n_sub": 15}
    nodes = 1 << 20
    # one main step = one phi/C/theta launch (0.04 ms) + 3 fused flow launches (0.02 ms each)
    m = {"nodes": nodes, "ms_per_step": 0.1,
         "tk": {"ms_pct": 0.4, "ms_flow": 0.6, "launches_pct": 10, "launches_flow": 30}}
    kr = bench.kernel_rooflines(cfg, m)
    fl = kr["flow_launch"]
    assert fl["substeps"] == 5
    assert fl["flop"] == bench.FLOW_FLOP_PER_NODE_SUBSTEP * nodes * 5
    assert fl["TFLOPs"] == pytest.approx(fl["flop"] / 0.02e-3 / 1e12, rel=1e-3)
    assert fl["alu_frac"] == pytest.approx(fl["TFLOPs"] / bench.PEAK_VALU_TFLOPS, rel=1e-3)
    # a fused launch must still read and write its populations once
    assert fl["hbm_min_bytes"] == 76 * nodes
    assert kr["k_pct"]["GBs"] == pytest.approx(200 * nodes / 0.04e-3 / 1e9, rel=1e-3)
    assert 0 < kr["k_pct"]["hbm_frac"] <= 1 and 0 < fl["alu_frac"] <= 1


def test_surrogate_leg_without_a_stored_network(monkeypatch, tmp_path):
    """The bench's surrogate object says what is missing instead of failing
    when the package holds no trained network."""
    import bench
    from paper_2209_01444_amd import surrogate
    monkeypatch.setattr(surrogate, "BUNDLE", str(tmp_path / "none.npz"))
    out = bench.surrogate_leg()
    assert set(out) == {"skipped"} and "none.npz" in out["skipped"]
