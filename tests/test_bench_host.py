"""Host-side behaviour of bench.py that needs no GPU: the one-GPU rule, the
missing-GPU exit, and the rule that HBM traffic is reported only for the
kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          env=env, capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_a_multi_rank_launch_is_refused():
    r = _run([], {"WORLD_SIZE": "2", "RANK": "0", "LOCAL_RANK": "0"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_no_gpu_exits_without_a_result_line():
    import torch
    if torch.cuda.is_available():
        return
    r = _run(["--steps", "1", "--warmup", "0"])
    assert r.returncode == 1
    assert "needs a GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": "abc", "bytes_per_launch": 1234}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("abc") == 1234
    assert bench.load_traffic("abd") is None
    f.write_text("not json")
    assert bench.load_traffic("abc") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.load_traffic("abc") is None


def test_source_hash_covers_every_listed_file():
    h = bench._src_hash(bench.POWERMAP_SOURCES)
    assert len(h) == 16 and int(h, 16) >= 0
    for f in bench.POWERMAP_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f
    assert bench._src_hash(bench.POWERMAP_SOURCES[:-1]) != h


def test_algorithmic_slots_per_term():
    # the synthesis count, plus the VALU contraction of the K <= 2 FP32 kernel,
    # plus the hi/lo split of the split-precision maps
    assert bench.alg_slots_per_term(8) == bench.SYNTH_SLOTS == 23
    assert bench.alg_slots_per_term(1) == 27
    assert bench.alg_slots_per_term(2) == 31
    assert bench.alg_slots_per_term(32, "f16x3") == bench.alg_slots_per_term(8, "bf16x3") == 27
    assert bench.mfma_flops_per_term(32, "f16x3") == 768
    assert bench.mfma_flops_per_term(32, "f32") == 256


def test_hall_roofline_fields():
    r = bench.hall_roofline(32, 2048 * 2048, 1024, "f16x3", 5.0, "abc", None)
    assert r["bound"] == "alu" and r["unit"] == "T VALU lane-slots/s"
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    # 27 slots x 4.29e9 terms in 5 ms
    assert abs(r["achieved"] - 27 * 2048 * 2048 * 1024 / 5e-3 / 1e12) < 1e-2
    assert r["floor_ms"] > 0 and r["mfma"]["flops_per_term"] == 768


def test_host_info():
    h = bench.host_info()
    assert h["nproc"] >= 1


def test_batched_bytes_per_room():
    # one room of K = 16 users and M = 256 antennas: NLoS draws and positions
    # read, W, p_m, SINR_k, R_sum, l21 and info written
    import bench
    per = 16 * 256 * 8 + 256 * 24 + 16 * 24 + 16 * 256 * 8 + 256 * 8 + 16 * 8 + 8 + 8 + 4
    assert bench.batched_bytes(1, 16, 256) == per == 74260
    assert bench.batched_bytes(1024, 16, 256, want_W=False) == 1024 * (per - 16 * 256 * 8)
