"""GPU checks of the reduced-precision forms of the least-squares contraction
(BF16 with one refinement step, FP32 single pass) against the FP64 oracle.

The forms change only W = Lhat^T A, so the sketch and the row-pivoted LU of
Y are the FP64 path's and their pivots match the oracle's exactly on inputs
whose Y pivots are well separated.  The factors themselves are judged
through the relative residual r = ||LU - PAQ||_F / ||A||_F, which must be
within 1e-3 relative of the oracle's r where the forms are meant to be used
(A a rank-l approximation away from rounding level: r >> 2^-16).

Why the bar holds: LU - PAQ splits into the part of PA outside Im L_y
(unchanged by the contraction) and L_y (B~ - B) inside it, so a contraction
error moves r^2 by ||L_y (B~ - B)||^2 / ||A||^2 (Pythagoras).  After one
refinement step ||L_y (B~ - B)|| is about 2^-8 ||R|| with R = A - Lhat X0,
i.e. r moves by ~ (2^-8 ||R|| / ||A||)^2 / (2 r^2), far below 1e-3 r.
"""
import numpy as np
import pytest
import torch

import paper_1601_04280_amd as rlu
import synth
from oracle import rlu as R
from oracle import lu as OL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel_res(A, L, U, pr, pc):
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.norm(L @ U - A[np.ix_(pr, pc)]) / np.linalg.norm(A)


def screened_y(A64, k, l, s, seed):
    """Seed whose row pivots (the ones every form shares) are well separated."""
    for sd in range(seed, seed + 20):
        p = R.Params(k, l, s, sd)
        Y = R.sketch_y(A64, p)
        _, Uy, _, _, zero, gap = OL.gepp(Y)
        d = np.abs(np.diag(Uy))
        if zero == 0 and gap >= 1e-5 and d[0] / d.min() <= 1e9:
            return sd, R.rlu(A64, p)
    raise RuntimeError("no screened seed")


def check_structure(g, m, n, l):
    L, U = g.L.cpu().numpy(), g.U.cpu().numpy()
    pr, pc = g.perm_r.cpu().numpy(), g.perm_c.cpu().numpy()
    assert sorted(pr.tolist()) == list(range(m)) and sorted(pc.tolist()) == list(range(n))
    np.testing.assert_array_equal(np.diag(L[:l]), 1.0)
    assert np.all(np.triu(L[:l], 1) == 0) and np.all(np.tril(U, -1) == 0)
    return L, U, pr, pc


DECAY_CASES = [
    # m, n, k, l, s, storage, spectrum scale, generating rank
    # (sigma_l / sigma_1 ~ e^-5: oracle residuals ~2e-2, far above 2^-16)
    (2000, 1000, 100, 110, 512, np.float32, 22.0, 600),
    (1500, 700, 50, 60, 256, np.float64, 12.0, 500),
    (4100, 300, 20, 45, 64, np.float32, 9.0, 300),         # split-K W0 GEMM, ragged tiles
    (333, 2500, 30, 33, 128, np.float64, 7.0, 333),        # wide, ragged
]


@pytest.mark.parametrize("precision", ["bf16", "f32"])
@pytest.mark.parametrize("m,n,k,l,s,dtype,scale,rgen", DECAY_CASES)
def test_residual_matches_oracle(precision, m, n, k, l, s, dtype, scale, rgen):
    A = synth.lowrank_dense(m, n, synth.spectrum_exp(rgen, scale), m + n, dtype=dtype)
    A64 = A.astype(np.float64)
    seed, o = screened_y(A64, k, l, s, 1)
    g = rlu.factor(to_dev(A), k=k, l=l, s=s, seed=seed, precision=precision)
    assert g.info_dict()["status"] == 0
    np.testing.assert_array_equal(g.perm_r.cpu().numpy(), o.perm_r)
    np.testing.assert_array_equal(g.ipiv_r.cpu().numpy(), o.ipiv_r)
    L, U, pr, pc = check_structure(g, m, n, l)
    r_g = rel_res(A64, L, U, pr, pc)
    r_o = rel_res(A64, o.L, o.U, o.perm_r, o.perm_c)
    print(f"{precision} {m}x{n} l={l}: residual {r_g:.6e} oracle {r_o:.6e} rel.diff {abs(r_g - r_o) / r_o:.2e}")
    assert abs(r_g - r_o) <= 1e-3 * r_o


def test_exp_spectrum_l520_quarter_size():
    """sigma_i = exp(-i/100), l = 520, s = 4096 on an 8192 x 4096 FP32 matrix
    (a quarter of the 32768 x 16384 precision workload)."""
    m, n, k, l, s = 8192, 4096, 500, 520, 4096
    A = synth.lowrank_dense(m, n, synth.spectrum_exp(2000), 99, dtype=np.float32)
    A64 = A.astype(np.float64)
    o = R.rlu(A64, R.Params(k, l, s, 7))
    r_o = rel_res(A64, o.L, o.U, o.perm_r, o.perm_c)
    for precision in ("bf16", "f32", "f64"):
        g = rlu.factor(to_dev(A), k=k, l=l, s=s, seed=7, precision=precision)
        assert g.info_dict()["status"] == 0
        L, U, pr, pc = check_structure(g, m, n, l)
        r_g = rel_res(A64, L, U, pr, pc)
        print(f"{precision}: residual {r_g:.6e} oracle {r_o:.6e} rel.diff {abs(r_g - r_o) / r_o:.2e}")
        assert abs(r_g - r_o) <= 1e-3 * r_o


def test_bf16_refinement_reduces_error():
    """The refined B is much closer to the exact product than one BF16 pass."""
    m, n, k, l, s = 3000, 1500, 100, 110, 512
    A = synth.lowrank_dense(m, n, synth.spectrum_exp(800, 22.0), 5, dtype=np.float32)
    A64 = A.astype(np.float64)
    seed, o = screened_y(A64, k, l, s, 3)
    g = rlu.factor(to_dev(A), k=k, l=l, s=s, seed=seed, precision="bf16", keep_intermediates=True)
    Bg = g.B.cpu().numpy()
    err_ref = np.linalg.norm(Bg - o.B) / np.linalg.norm(o.B)
    # one BF16 pass with FP32 accumulation, from the oracle's Lhat, in torch
    Lhat = np.empty_like(o.Ly)
    Lhat[o.perm_r] = o.Ly
    Lb = torch.from_numpy(Lhat).to(DEV).to(torch.bfloat16).float()
    Ab = torch.from_numpy(A).to(DEV).to(torch.bfloat16).float()
    W0 = (Lb.T.contiguous() @ Ab).double().cpu().numpy()
    B0 = np.linalg.solve(Lhat.T @ Lhat, W0)
    err_one = np.linalg.norm(B0 - o.B) / np.linalg.norm(o.B)
    print(f"B error: one pass {err_one:.3e}, refined {err_ref:.3e}")
    assert err_ref <= err_one / 8


def test_bf16_near_exact_input_error_reported():
    """On the 1024 x 512 geometric-spectrum input (residual at the 1e-10 noise
    level) one step cannot reach FP64 residuals; it lands near (2^-8)^2 of ||A||."""
    A = synth.small_dense()
    g = rlu.factor(to_dev(A), k=20, l=30, s=256, seed=1, precision="bf16")
    L, U, pr, pc = check_structure(g, 1024, 512, 30)
    r = rel_res(A, L, U, pr, pc)
    print(f"bf16 residual on the geometric-spectrum input: {r:.3e}")
    assert r <= 1e-4
    g = rlu.factor(to_dev(A), k=20, l=30, s=256, seed=1, precision="f32")
    L, U, pr, pc = check_structure(g, 1024, 512, 30)
    r = rel_res(A, L, U, pr, pc)
    print(f"f32 residual on the geometric-spectrum input: {r:.3e}")
    assert r <= 1e-5


def test_reduced_precision_rejected_for_csr():
    row_ptr, col, val = synth.random_csr(100, 80, 0.05, 1)
    csr = (to_dev(row_ptr), to_dev(col), to_dev(val), 100, 80)
    with pytest.raises(rlu.RluError):
        rlu.factor(csr=csr, k=4, l=8, s=16, seed=1, precision="bf16")
