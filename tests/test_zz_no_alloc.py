"""rlu_sketch_noalloc (the sketch of Algorithm 1 steps 1-2 from the library's
fixed per-device scratch array, no workspace argument) against rlu_sketch on
the same inputs, through the C ABI: two calls in a row, the second on a
smaller problem, so that the second reuses the scratch the first left behind.

The two entry points run the same kernels; the dense sketch sums its buckets
with LDS atomics, whose order may differ run to run, so Y is held to the
sketch's parity bar (1e-10 relative, Frobenius) and, for the CSR input (a
fixed-order per-row evaluation), bit for bit.  A problem whose codes do not
fit the scratch is rejected with RLU_ERR_NO_MEMORY before anything runs."""
import numpy as np
import pytest
import torch

import paper_1601_04280_amd as rlu
import synth
from oracle import rlu as R

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def test_noalloc_matches_workspace_entry_point_twice():
    ctx = rlu.Context(0)
    try:
        cases = [  # m, n, k, l, s, seed; the second is smaller than the first
            (6000, 3000, 40, 50, 1024, 11),
            (700, 400, 20, 30, 256, 12),
        ]
        for m, n, k, l, s, seed in cases:
            A = torch.from_numpy(synth.lowrank_dense(m, n, synth.spectrum_geometric(20), seed, noise=1e-10)).to(DEV)
            Yw = rlu.sketch(A, k=k, l=l, s=s, seed=seed, ctx=ctx)
            Yn = torch.full((m, l), float("nan"), dtype=torch.float64, device=DEV)
            rlu.sketch_noalloc(A, k=k, l=l, s=s, seed=seed, ctx=ctx, Y=Yn)
            torch.cuda.synchronize()
            assert torch.isfinite(Yn).all()
            assert rel(Yn, Yw) <= 1e-10, (m, n, rel(Yn, Yw))
            # and the oracle's sketch of the same matrix
            Yo = R.sketch_y(A.cpu().numpy(), R.Params(k, l, s, seed))
            assert np.linalg.norm(Yn.cpu().numpy() - Yo) <= 1e-10 * np.linalg.norm(Yo)
    finally:
        ctx.close()


def test_noalloc_csr_bit_identical_twice():
    ctx = rlu.Context(0)
    try:
        for m, n, density, l, s, seed in [(5000, 8000, 0.01, 60, 512, 3), (900, 1200, 0.02, 20, 128, 4)]:
            rp, col, val = synth.random_csr(m, n, density, seed)
            csr = (torch.from_numpy(rp).to(DEV), torch.from_numpy(col).to(DEV), torch.from_numpy(val).to(DEV), m, n)
            Yw = rlu.sketch(csr=csr, k=l, l=l, s=s, seed=seed, ctx=ctx)
            Yn = rlu.sketch_noalloc(csr=csr, k=l, l=l, s=s, seed=seed, ctx=ctx)
            torch.cuda.synchronize()
            assert torch.equal(Yn, Yw)
    finally:
        ctx.close()


def test_noalloc_rejects_problems_above_its_scratch():
    ctx = rlu.Context(0)
    try:
        n = ((8 << 20) // 4) + 1024        # the column codes alone exceed it
        A = torch.zeros(2, n, dtype=torch.float32, device=DEV)
        with pytest.raises(rlu.RluError) as ei:
            rlu.sketch_noalloc(A, k=1, l=1, s=2, seed=1, ctx=ctx)
        assert ei.value.status == rlu.RLU_ERR_NO_MEMORY
        # the context still works afterwards
        B = torch.from_numpy(synth.lowrank_dense(300, 200, synth.spectrum_geometric(20), 5, noise=1e-10)).to(DEV)
        Yw = rlu.sketch(B, k=10, l=20, s=64, seed=2, ctx=ctx)
        Yn = rlu.sketch_noalloc(B, k=10, l=20, s=64, seed=2, ctx=ctx)
        torch.cuda.synchronize()
        assert rel(Yn, Yw) <= 1e-10
    finally:
        ctx.close()
