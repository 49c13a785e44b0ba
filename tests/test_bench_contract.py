"""bench.py's contract on a host without a GPU: more than one GPU is refused
with a message, a missing GPU ends with a message and exit status 2, and the
HBM traffic record is only reported for the product-kernel sources it was
measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_missing_gpu_ends_with_status_2():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the bench would run")
    r = run("--steps", "1", "--warmup", "0", "--no-cpu-baseline", "--no-extra")
    assert r.returncode == 2
    assert "needs a GPU" in r.stderr


def test_traffic_record_is_keyed_by_the_kernel_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["k_cgemm_f64_c2"]
    # a record keyed by another source hash is not reported
    fake_root = tmp_path
    (fake_root / "profiles").mkdir()
    stale = dict(rec, source_sha256_16="0" * 16)
    (fake_root / "profiles" / "traffic.json").write_text(json.dumps({"k_cgemm_f64_c2": stale}))
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    monkeypatch.setattr(bench, "gemm_source_hash", lambda: "f" * 16)
    assert bench.load_traffic("k_cgemm_f64_c2") is None
    # the same record under the current hash is
    fresh = dict(rec, source_sha256_16="f" * 16)
    (fake_root / "profiles" / "traffic.json").write_text(json.dumps({"k_cgemm_f64_c2": fresh}))
    assert bench.load_traffic("k_cgemm_f64_c2") == rec["hbm_bytes_per_launch"]
