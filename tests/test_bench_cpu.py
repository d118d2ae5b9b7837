"""Host-side logic of bench.py (no GPU): the one-GPU contract, the algorithmic
traffic model of the roofline line, and the lookup of the committed HBM
counter summary, which must go null once a kernel's sources change."""

import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_model_at_the_headline_shape():
    b = _bench()
    F, T, M, N, K = 513, 3000, 8, 5, 32
    km = b.kernel_model(F, T, M, N, K, 4)
    FT = F * T
    assert km["vpass"]["bytes"] == FT * M * 8 == 98_496_000  # complex64 X, read once
    assert km["wpass"]["bytes"] == km["hpass"]["bytes"] == km["gpass"]["bytes"] == FT * M * 4
    assert km["proj"]["bytes"] == FT * M * (8 + 4)  # X in, x~ out
    assert all(v["bound"] == "hbm" for v in km.values())
    # the FP64 path moves twice the bytes
    km64 = b.kernel_model(F, T, M, N, K, 8)
    assert all(km64[k]["bytes"] == 2 * km[k]["bytes"] for k in km)


def test_measured_traffic_follows_the_source_digest(tmp_path, monkeypatch):
    b = _bench()
    path = os.path.join(ROOT, "profiles", "hbm_traffic_fp32_m8_513x3000.json")
    with open(path) as f:
        t = json.load(f)
    e = t["kernels"]["vpass/bf16"]
    expect = (e["fetch_kib"] * t["fetch_scale"] + e["write_kib"] * t["write_scale"]) * 1024.0
    if e["sources_sha256"] == b.kernel_sources_digest("vpass"):
        assert b.measured_traffic("vpass", "bf16") == expect
    else:  # the kernel changed since the counters were taken
        assert b.measured_traffic("vpass", "bf16") is None
    assert b.measured_traffic("vpass", "no-such-path") is None
    # a changed source must void the figure
    monkeypatch.setattr(b, "kernel_sources_digest", lambda k: "0" * 64)
    assert b.measured_traffic("vpass", "bf16") is None
