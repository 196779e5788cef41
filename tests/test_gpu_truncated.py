"""The truncated (rank-k) form, RLU_FLAG_TRUNCATE, against the oracle: the
problem statement of Section 1 asks for L of m x k and U of k x n; the
l-column sketch Y is reduced to k columns by column pivoting (oracle:
colsel.pivoted_cholesky_order, pinned to LAPACK's pivoted QR) and steps 3-7
run on them.

Checked: the chosen columns (ysel) bit-exact, on inputs whose selection
gaps are screened like the LU pivots; P, Q bit-exact; Y (m x l), L (m x k),
U (k x n), B (k x n) to parity.py's bar; the residual equal to the distance
of A from the span of the chosen columns (the Theorem 3.1 identity for Y_k),
formed on the device; every form of the contraction and CSR input."""
import numpy as np
import pytest
import torch

import paper_1601_04280_amd as rlu
import synth
from oracle import colsel
from oracle import rlu as R
from parity import compare_factors, rel_fro, screened, to_dev

pytestmark = pytest.mark.gpu
TR = rlu.RLU_FLAG_TRUNCATE


def screened_truncated(A, k, l, s, seed=1, tries=20, csr=None, **kw):
    """The first seed whose pivots and column choices are robust to rounding:
    the LU pivots screened as in parity.py, every selection step's top-two
    gap of the remaining squared norms >= 1e-5, and the k-th chosen column's
    remaining norm r_kk >= 1e-6 r_00: the squared norms are formed by
    subtraction from the Gram diagonal, so far below (u ||Y||^2) they are
    rounding and their order is not determined by the input."""
    for sd in range(seed, seed + tries):
        o = R.rlu(A, R.Params(k, l, s, sd, truncate=True, **kw), csr=csr)
        _, rdiag, _, _ = colsel.pivoted_cholesky_order(o.Y, k)
        if screened(o) and o.min_gap_sel >= 1e-5 and rdiag[-1] >= 1e-6 * rdiag[0]:
            return sd, o
    raise RuntimeError("no screened seed")


def check(g, o, a_fro, sample=None):
    np.testing.assert_array_equal(g.ysel.cpu().numpy(), o.ysel)
    compare_factors(a_fro, g, o, sample=sample)
    assert g.info_dict()["zero_pivots_sel"] == 0


@pytest.mark.parametrize("m,n,k,l,s,spec", [
    (2000, 1200, 20, 40, 256, "geometric"),
    (3000, 2500, 100, 120, 1024, "invsq"),
    (1500, 900, 7, 64, 128, "geometric"),
    (900, 700, 30, 30, 64, "inverse"),          # k = l: a reordering of all columns
])
def test_dense_truncated(m, n, k, l, s, spec):
    sig = {"geometric": synth.spectrum_geometric(40), "invsq": 1.0 / np.arange(1, 801) ** 2,
           "inverse": 1.0 / np.arange(1, 701)}[spec]
    A = synth.lowrank_dense(m, n, sig, 3100 + k, noise=1e-10 if spec == "geometric" else 0.0)
    seed, o = screened_truncated(A, k, l, s)
    g = rlu.factor(to_dev(A), k=k, l=l, s=s, seed=seed, flags=TR, keep_intermediates=True)
    assert g.L.shape == (m, k) and g.U.shape == (k, n) and g.Y.shape == (m, l)
    check(g, o, A)
    # residual = distance of A from span(Y[:, ysel]) (Theorem 3.1 with Y_k)
    Ad = to_dev(A)
    res = torch.linalg.norm(g.L @ g.U - Ad[g.perm_r.long()][:, g.perm_c.long()]).item()
    Q, _ = torch.linalg.qr(g.Y[:, g.ysel.long()])
    proj = torch.linalg.norm(Ad - Q @ (Q.T @ Ad)).item()
    assert abs(res - proj) <= 1e-9 * np.linalg.norm(A)


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_truncated_reduced_forms(precision):
    m, n, k, l, s = 4000, 2000, 60, 90, 512
    A = synth.lowrank_dense(m, n, synth.spectrum_exp(2000, 15.0), 3200)
    seed, o = screened_truncated(A, k, l, s)
    g = rlu.factor(to_dev(A), k=k, l=l, s=s, seed=seed, flags=TR, precision=precision, keep_intermediates=True)
    np.testing.assert_array_equal(g.ysel.cpu().numpy(), o.ysel)
    np.testing.assert_array_equal(g.perm_r.cpu().numpy(), o.perm_r)
    L, U = g.L.cpu().numpy(), g.U.cpu().numpy()
    pr, pc = g.perm_r.cpu().numpy(), g.perm_c.cpu().numpy()
    r_g = np.linalg.norm(L @ U - A[np.ix_(pr, pc)])
    r_o = R.residual_fro(A, o.L, o.U, o.perm_r, o.perm_c)
    assert abs(r_g - r_o) <= 1e-3 * r_o, (r_g, r_o)


def test_truncated_csr_and_second_projection():
    m, n, k, l, s = 8000, 5000, 25, 50, 512
    rp, col, val = synth.random_csr(m, n, 0.01, 3300, plant_rank=40, plant_rows=800, plant_scale=1e3)
    csr_host = (rp, col, val, m, n)
    seed, o = screened_truncated(None, k, l, s, csr=csr_host)
    csr = (to_dev(rp), to_dev(col), to_dev(val), m, n)
    g = rlu.factor(csr=csr, k=k, l=l, s=s, seed=seed, flags=TR, keep_intermediates=True)
    check(g, o, float(np.linalg.norm(val)))
    # the second projection on the k chosen columns (k2 >= l)
    A = synth.lowrank_dense(3000, 2000, synth.spectrum_geometric(40), 3301, noise=1e-10)
    seed, o = screened_truncated(A, 20, 40, 256, k2=160, l2=512)
    g = rlu.factor(to_dev(A), k=20, l=40, s=256, seed=seed, flags=TR, k2=160, l2=512, keep_intermediates=True)
    np.testing.assert_array_equal(g.ysel.cpu().numpy(), o.ysel)
    compare_factors(A, g, o, tol=1e-8)


def test_truncated_deterministic_and_served():
    A = to_dev(synth.lowrank_dense(2500, 1500, synth.spectrum_geometric(40), 3400, noise=1e-10))
    fl = TR | rlu.RLU_FLAG_DETERMINISTIC
    a = rlu.factor(A, k=16, l=32, s=256, seed=4, flags=fl, keep_intermediates=True)
    a2 = rlu.factor(A, k=16, l=32, s=256, seed=4, flags=fl, keep_intermediates=True)
    with rlu.Server(hbm_budget_bytes=1 << 30, max_inflight=2) as srv:
        b = srv.wait(srv.submit(A, k=16, l=32, s=256, seed=4, flags=fl, keep_intermediates=True))
    torch.cuda.synchronize()
    for key in ["L", "U", "perm_r", "perm_c", "ysel", "Y", "B"]:
        assert torch.equal(getattr(a, key), getattr(a2, key)), key
    # served on a partition of the device: its own GEMM splits, so the parity bar
    for key in ["perm_r", "perm_c", "ysel"]:
        assert torch.equal(getattr(a, key), getattr(b, key)), key
    for key in ["L", "U", "B"]:
        x, y = getattr(b, key), getattr(a, key)
        assert (torch.linalg.norm(x - y) / torch.linalg.norm(y)).item() <= 1e-10, key
