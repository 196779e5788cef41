"""The parameter ranges of the problem statement (Section 1: any target rank
with l <= min(m, n)) and of the sparse embedding's width, against the oracle:

* s above the LDS-resident transform (s in 16384 .. 65536): dense A takes the
  explicit projection (Omega^T = S^T diag(d) T R formed n x l, Y = A Omega^T on
  the FP64 GEMM), CSR A reads its cos table from global memory; both
  transforms, FP64 and FP32 storage;
* l up to 1024 (the largest rank of Section 4.1's sweep is 900, l = 910):
  the Cholesky panel's LDS form at l > 544, the CSR kernels at 12 and 16
  outputs per lane;

on inputs with sigma_i = 1/i and rank >= l; pivots bit-exact, Y and the
factors to parity.py's bar (every column whose predicted rounding allows)."""
import numpy as np
import pytest
import torch

import paper_1601_04280_amd as rlu
import synth
from parity import compare_factors, rel_fro, screened_factor, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("s,transform,dtype", [
    (16384, "fourier", torch.float64), (65536, "fourier", torch.float64),
    (32768, "hadamard", torch.float64), (16384, "fourier", torch.float32),
])
def test_wide_s_dense(s, transform, dtype):
    m, n, k, l = 700, 1500, 30, 40
    A = synth.lowrank_dense(m, n, 1.0 / np.arange(1, 101), 1700 + s // 1024)
    if dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    seed, o = screened_factor(A, k, l, s, 1, transform=transform)
    flags = rlu.RLU_FLAG_HADAMARD if transform == "hadamard" else 0
    g = rlu.factor(to_dev(A).to(dtype), k=k, l=l, s=s, seed=seed, flags=flags, keep_intermediates=True)
    compare_factors(A, g, o)
    # the sketch alone, and twice (the explicit route sums in a fixed order)
    Ad = to_dev(A).to(dtype)
    y1 = rlu.sketch(Ad, k=k, l=l, s=s, seed=seed, flags=flags)
    y2 = rlu.sketch(Ad, k=k, l=l, s=s, seed=seed, flags=flags)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    assert rel_fro(y1.cpu().numpy(), o.Y) <= 1e-10


@pytest.mark.parametrize("s,transform", [(65536, "fourier"), (16384, "hadamard")])
def test_wide_s_csr(s, transform):
    m, n, k, l = 3000, 5000, 20, 30
    rp, col, val = synth.random_csr(m, n, 0.01, 1800 + s // 1024, plant_rank=40, plant_rows=600, plant_scale=1e3)
    csr_host = (rp, col, val, m, n)
    seed, o = screened_factor(None, k, l, s, 1, csr=csr_host, transform=transform)
    flags = rlu.RLU_FLAG_HADAMARD if transform == "hadamard" else 0
    csr = (to_dev(rp), to_dev(col), to_dev(val), m, n)
    g = rlu.factor(csr=csr, k=k, l=l, s=s, seed=seed, flags=flags, keep_intermediates=True)
    compare_factors(float(np.linalg.norm(val)), g, o)


@pytest.mark.parametrize("l", [600, 910, 1024])
def test_large_l_dense(l):
    m, n, s = 3000, 2000, 2048 if l < 1024 else 4096
    A = synth.lowrank_dense(m, n, 1.0 / np.arange(1, 1201), 1900 + l)
    seed, o = screened_factor(A, l - 10, l, s, 1)
    g = rlu.factor(to_dev(A), k=l - 10, l=l, s=s, seed=seed, keep_intermediates=True)
    compare_factors(A, g, o)


@pytest.mark.parametrize("l", [700, 1000])
def test_large_l_csr(l):
    m, n, s = 6000, 3000, 2048
    rp, col, val = synth.random_csr(m, n, 0.05, 2000 + l)
    csr_host = (rp, col, val, m, n)
    seed, o = screened_factor(None, l - 10, l, s, 1, csr=csr_host)
    csr = (to_dev(rp), to_dev(col), to_dev(val), m, n)
    g = rlu.factor(csr=csr, k=l - 10, l=l, s=s, seed=seed, keep_intermediates=True)
    compare_factors(float(np.linalg.norm(val)), g, o)


def test_out_of_range_rejected():
    A = to_dev(synth.lowrank_dense(2000, 1500, 1.0 / np.arange(1, 101), 3))
    for kw in [dict(k=10, l=1025, s=2048), dict(k=10, l=20, s=131072), dict(k=10, l=20, s=3000)]:
        with pytest.raises(rlu.RluError) as ei:
            rlu.factor(A, seed=1, **kw)
        assert ei.value.status == rlu.RLU_ERR_INVALID_ARG
