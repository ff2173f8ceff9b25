"""The committed measurement records agree with the sources and with each other (no GPU needed).

  * every HBM-traffic record was taken with the kernel sources as they are now (sha256), so bench.py
    reports its traffic; a changed source makes measured_traffic return None;
  * the default bench record carries the traffic of its roofline kernel's record, and no figure in a
    bench record that is a fraction of a peak exceeds 1;
  * the roofline's achieved rate is its algorithmic work per launch over its average launch time.
"""
import json
import os
import shutil

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


@pytest.mark.parametrize("key", sorted(bench.TRAFFIC_RECORDS))
def test_traffic_records_match_the_sources(key):
    name, files = bench.TRAFFIC_RECORDS[key]
    rec = json.load(open(os.path.join(PROFILES, name)))
    assert rec["source_sha256"] == bench.source_sha(files), name
    assert rec["mode"] == key[1] and rec["product"] == key[2]
    t = bench.measured_traffic(rec["frequencies"], rec["workload"], key[0], key[1], key[2])
    assert t == rec["traffic_bytes_per_launch"] and t > rec["algorithmic_bytes_per_launch"]


def test_changed_source_voids_the_traffic(tmp_path, monkeypatch):
    key = ("fp32_3m", "tile_grad", "gemm_line")
    name, files = bench.TRAFFIC_RECORDS[key]
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "profiles"), root / "profiles")
    shutil.copytree(os.path.join(ROOT, "paper_2412_14973_amd", "csrc"), root / "paper_2412_14973_amd" / "csrc")
    monkeypatch.setattr(bench, "ROOT", str(root))
    rec = json.load(open(os.path.join(PROFILES, name)))
    args = (rec["frequencies"], rec["workload"]) + key
    assert bench.measured_traffic(*args) == rec["traffic_bytes_per_launch"]
    with open(root / "paper_2412_14973_amd" / "csrc" / files[0], "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic(*args) is None
    assert bench.measured_traffic(rec["frequencies"] + 1, rec["workload"], *key) is None


def _fractions(obj, path=""):
    if isinstance(obj, dict):
        for k, v in obj.items():
            yield from _fractions(v, f"{path}.{k}")
            if (k == "frac" or k.startswith("frac_")) and isinstance(v, (int, float)):
                yield f"{path}.{k}", v
    elif isinstance(obj, list):
        for i, v in enumerate(obj):
            yield from _fractions(v, f"{path}[{i}]")


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(PROFILES) if f.startswith("bench_") and f.endswith(".json")))
def test_bench_records_have_no_fraction_above_one(name):
    rec = json.load(open(os.path.join(PROFILES, name)))
    fr = list(_fractions(rec))
    assert fr, name
    for where, v in fr:
        assert 0.0 <= v <= 1.0, (name, where, v)


def test_default_record_roofline_is_consistent():
    rec = json.load(open(os.path.join(PROFILES, "bench_fp32_3m_batched_nr1024.json")))
    r = rec["roofline"]
    assert rec["metric"] == "TLR-MDD grad iters/s" and rec["n_gpus"] == 1 and rec["config"]["frequencies"] == 64
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9
    name, _ = bench.TRAFFIC_RECORDS[("fp32_3m", "tile_grad", "gemm_line")]
    tr = json.load(open(os.path.join(PROFILES, name)))
    assert r["traffic"] == tr["traffic_bytes_per_launch"]
    assert r["algorithmic_bytes"] == tr["algorithmic_bytes_per_launch"]
    k = rec["kernels"]["gemm_line"]
    # executed flops per launch over the launch time (the instrumented step's table) agree with the
    # timed steps' rate within the launch-to-launch spread
    assert abs(k["tflops"] - r["achieved"]) / r["achieved"] < 0.05
    cb = rec["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and 0 < cb["value"] < rec["value"]
