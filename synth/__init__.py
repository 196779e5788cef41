"""Seeded synthetic inputs for the randomized LU path.

This module only builds input matrices: it holds none of the decomposition's
arithmetic (no sketch, no pivoting, no least squares), so the CPU oracle and
the GPU path can both consume what it makes without sharing method code.

Workload shapes follow the paper's experiments, which are themselves
synthetic (Section 4: matrices given by their singular values with random
singular vectors), and the dense / sparse cost split of Section 3.1:

* ``lowrank_dense``   -- A = U diag(sigma) V^T (+ i.i.d. Gaussian noise), with
  U, V the Q factors of Householder QRs of N(0,1) matrices, column signs
  fixed so that diag(R) > 0.
* ``random_csr``      -- CSR with Binomial per-row counts, distinct uniform
  column positions, N(0,1) values, and an optional low-rank component added
  on the existing pattern of a subset of rows.

Everything is seeded; numpy's PCG64 for CPU generation, torch's generator
for device generation of the large matrices (QR of a 16384 x 8192 Gaussian is
too slow on a CPU for a benchmark set-up).
"""
from __future__ import annotations

import math

import numpy as np

DATA_SEED_BASE = 160104280


def orthonormal_gaussian(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Q factor (rows x cols) of the reduced QR of an N(0,1) matrix, diag(R) > 0."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn


def lowrank_dense(m: int, n: int, sigma, seed: int, noise: float = 0.0,
                  dtype=np.float64) -> np.ndarray:
    """Row-major dense A = U diag(sigma) V^T + noise * N(0,1), on the CPU."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.shape[0]
    rng = np.random.default_rng(seed)
    u = orthonormal_gaussian(rng, m, r)
    v = orthonormal_gaussian(rng, n, r)
    a = (u * sigma) @ v.T
    if noise:
        a += noise * rng.standard_normal((m, n))
    return np.ascontiguousarray(a.astype(dtype))


def lowrank_dense_torch(m: int, n: int, sigma, seed: int, noise: float = 0.0,
                        dtype=None, device="cuda"):
    """Same construction as ``lowrank_dense`` generated with torch on ``device``.

    The values differ from the numpy version (different generator); the
    distribution and the spectrum are the same.
    """
    import torch
    if dtype is None:
        dtype = torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    sigma_t = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    r = sigma_t.shape[0]

    def orth(rows, cols):
        g = torch.randn(rows, cols, generator=gen, device=device, dtype=torch.float64)
        q, rr = torch.linalg.qr(g, mode="reduced")
        d = torch.sign(torch.diagonal(rr))
        d[d == 0] = 1.0
        return q * d

    u = orth(m, r)
    v = orth(n, r)
    a = (u * sigma_t) @ v.T.contiguous()
    del u, v
    if noise:
        a += noise * torch.randn(m, n, generator=gen, device=device, dtype=torch.float64)
    return a.to(dtype).contiguous()


def random_csr(m: int, n: int, density: float, seed: int,
               plant_rank: int = 0, plant_rows: int = 0,
               plant_scale: float = 1e5, plant_decay: float = 0.95):
    """CSR matrix (row_ptr int32, col int32, val float64).

    Per-row counts ~ Binomial(n, density); columns uniform without repeats,
    sorted ascending; values N(0,1).  With ``plant_rank`` > 0, the entries of
    ``plant_rows`` rows (chosen without replacement) get the matching entries
    of U diag(s) V^T added, U and V orthonormal Gaussian, s_i = scale *
    decay^(i-1); the sparsity pattern (and nnz) is unchanged.
    """
    rng = np.random.default_rng(seed)
    counts = rng.binomial(n, density, size=m).astype(np.int64)
    total = int(counts.sum())
    rows = np.repeat(np.arange(m, dtype=np.int64), counts)
    cols = rng.integers(0, n, size=total, dtype=np.int64)
    key = np.unique(rows * n + cols)          # sorted, distinct per row
    rows = key // n
    cols = key - rows * n
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    vals = rng.standard_normal(key.shape[0])
    if plant_rank > 0 and plant_rows > 0:
        prow = np.sort(rng.choice(m, size=plant_rows, replace=False))
        u = orthonormal_gaussian(rng, plant_rows, plant_rank)
        v = orthonormal_gaussian(rng, n, plant_rank)
        s = plant_scale * plant_decay ** np.arange(plant_rank)
        us = u * s
        for blk in range(0, plant_rows, 1024):
            rr = prow[blk:blk + 1024]
            for t, i in enumerate(rr):
                a, b = row_ptr[i], row_ptr[i + 1]
                vals[a:b] += v[cols[a:b]] @ us[blk + t]
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 indexing")
    return (row_ptr.astype(np.int32), cols.astype(np.int32), vals)


def csr_to_dense(row_ptr, col, val, m: int, n: int) -> np.ndarray:
    a = np.zeros((m, n))
    for i in range(m):
        a[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    return a


# ---------------------------------------------------------------------------
# Named workloads (sizes and spectra of the benchmark configurations)
# ---------------------------------------------------------------------------

def spectrum_geometric(r: int) -> np.ndarray:
    """sigma_i = 2^-(i-1), i = 1..r."""
    return 2.0 ** (-np.arange(r, dtype=np.float64))


def spectrum_inverse_square(count: int) -> np.ndarray:
    """sigma_i = i^-2, i = 1..count."""
    i = np.arange(1, count + 1, dtype=np.float64)
    return i ** -2.0


def spectrum_exp(count: int, scale: float = 100.0) -> np.ndarray:
    """sigma_i = exp(-i/scale), i = 1..count."""
    i = np.arange(1, count + 1, dtype=np.float64)
    return np.exp(-i / scale)


def spectrum_step_exp(n: int, r: int, lo: float = 10.0, hi: float = 200.0) -> np.ndarray:
    """Section 4.1: sigma_1..r = 1, then n - r values decaying exponentially
    from e^-lo to e^-hi (exponents evenly spaced)."""
    return np.concatenate([np.ones(r), np.exp(-np.linspace(lo, hi, n - r))])


def spectrum_exp_range(n: int, hi: float = 100.0) -> np.ndarray:
    """Section 4.2: n values decaying exponentially from 1 to e^-hi
    (exponents evenly spaced)."""
    return np.exp(-np.linspace(0.0, hi, n))


WORKLOADS = {
    # name: (m, n, k, l, s)
    "dense_1024x512_geometric": (1024, 512, 20, 30, 256),
    "dense_16384x8192_invsq": (16384, 8192, 200, 210, 2048),
    "csr_200000x100000_planted": (200000, 100000, 100, 110, 4096),
    "dense_32768x16384_exp_fp32": (32768, 16384, 500, 520, 4096),
}


def small_dense(seed: int = DATA_SEED_BASE):
    """1024 x 512, r = 20, sigma_i = 2^-(i-1), plus N(0, 1e-20) noise."""
    return lowrank_dense(1024, 512, spectrum_geometric(20), seed, noise=1e-10)


def invsq_dense_torch(m=16384, n=8192, seed=DATA_SEED_BASE + 1, device="cuda"):
    """Full spectrum sigma_i = i^-2 over min(m, n) singular values (no noise)."""
    return lowrank_dense_torch(m, n, spectrum_inverse_square(min(m, n)), seed,
                               device=device)


def exp_dense_fp32_torch(m=32768, n=16384, r_gen=2000, seed=DATA_SEED_BASE + 3,
                         device="cuda"):
    """sigma_i = exp(-i/100), i <= r_gen, stored as float32 (round to nearest)."""
    import torch
    return lowrank_dense_torch(m, n, spectrum_exp(r_gen), seed, dtype=torch.float32,
                               device=device)


def planted_csr(m=200000, n=100000, seed=DATA_SEED_BASE + 2):
    """0.1% density, rank-50 plant on 5% of the rows."""
    return random_csr(m, n, 1e-3, seed, plant_rank=50, plant_rows=m // 20)


def serving_shapes(count: int, seed: int):
    """Request shapes for the serving mix: m, n log-uniform, k uniform.

    m in [512, 8192], n in [256, 4096], k in {16, 32, 64, 128, 256},
    l = k + 10, s = min(2^floor(log2 n), 8k); when k + 10 > min(s, n, m) the
    rank drops to the largest listed value that fits.  The precision class is
    Bernoulli(0.3) for the reduced-precision form.
    """
    rng = np.random.default_rng(seed)
    out = []
    ks = [16, 32, 64, 128, 256]
    for _ in range(count):
        m = int(round(math.exp(rng.uniform(math.log(512), math.log(8192)))))
        n = int(round(math.exp(rng.uniform(math.log(256), math.log(4096)))))
        k = int(ks[rng.integers(0, len(ks))])
        while True:
            s = min(1 << int(math.floor(math.log2(n))), 8 * k)
            if k + 10 <= min(s, n, m):
                break
            k = max(x for x in ks if x < k)
        prec = "bf16" if rng.random() < 0.3 else "f64"
        out.append({"m": m, "n": n, "k": k, "l": k + 10, "s": s, "precision": prec})
    return out
