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
