"""Host-side checks of bench.py's command line (no device needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_extras_list_names_every_block():
    assert set(bench.EXTRAS) == {"transforms", "second_projection", "forms", "csr", "serving", "accuracy"}


@pytest.mark.parametrize("r,l,s", [(10, 20, 128), (50, 60, 256), (200, 210, 1024), (500, 510, 2048), (900, 910, 4096)])
def test_sweep_parameters(r, l, s):
    # k = r, l = r + 10, s the power of two at or above 4 l
    assert bench.sweep_params(r, 5000) == dict(k=r, l=l, s=s)


def test_headline_workload_is_the_dense_invsq_matrix():
    w = bench.WORKLOADS["dense_16384x8192_invsq"]
    assert (w["m"], w["n"], w["k"], w["l"], w["s"], w["precision"]) == (16384, 8192, 200, 210, 2048, "f64")


def test_measured_traffic_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    """The roofline's traffic comes from the committed counter summary only
    while the kernel source hashes as it did when the counters were taken."""
    import hashlib
    import json
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    rec = {"kern": {"kernel": "k", "source": "k.hip", "bytes_per_launch": 1234,
                    "source_sha256": hashlib.sha256(b"kernel v1\n").hexdigest()}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    assert bench.measured_traffic("kern") == 1234
    assert bench.measured_traffic("other") is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("kern") is None
