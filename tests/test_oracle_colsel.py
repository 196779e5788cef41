"""Pins of the column selection of the truncated (rank-k) output
(oracle/colsel.py) and of the truncated pipeline, against what does not
depend on the oracle's code:

* LAPACK's column-pivoted QR (dgeqp3, through scipy.linalg.qr with
  pivoting): the same first k columns, and r_jj = |R_jj|;
* closed forms: orthogonal columns are taken by decreasing norm with
  r_jj = the norms; a column in the span of earlier choices is never taken
  before the columns outside it; exactly dependent columns give zero steps;
* the truncated pipeline: ||L U - P A Q||_F equals the distance of A from
  the span of the k chosen columns of Y (the Theorem 3.1 identity with Y_k
  in place of Y), is at least Delta_k (rank-k factors, Eckart-Young), and
  with the oversampled sketch is on average below the error of a k-column
  sketch (the purpose of the truncated form)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import colsel
from oracle import rlu as R


def lapack_order(Y, k):
    Q, Rm, piv = sla.qr(Y, mode="economic", pivoting=True)
    return piv[:k], np.abs(np.diag(Rm))[:k]


@pytest.mark.parametrize("m,l,k,seed", [(200, 30, 20, 1), (500, 60, 60, 2), (90, 12, 5, 3), (1000, 210, 200, 4)])
def test_matches_lapack_pivoted_qr(m, l, k, seed):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((m, l)) * np.exp(rng.uniform(-3, 3, size=l))   # columns of varied scale
    Y = Y @ np.triu(rng.standard_normal((l, l)) * 0.2 + np.eye(l))        # and correlated
    sel, rdiag, zero, gap = colsel.pivoted_cholesky_order(Y, k)
    assert gap >= 1e-6, "input not screened"
    piv, rabs = lapack_order(Y, k)
    np.testing.assert_array_equal(sel, piv)
    np.testing.assert_allclose(rdiag, rabs, rtol=1e-9)
    assert zero == 0


def test_orthogonal_columns_by_decreasing_norm():
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((300, 40)))
    norms = rng.permutation(np.arange(1, 41, dtype=float))
    sel, rdiag, zero, _ = colsel.pivoted_cholesky_order(Q * norms, 40)
    np.testing.assert_array_equal(sel, np.argsort(-norms, kind="stable"))
    np.testing.assert_allclose(rdiag, np.sort(norms)[::-1], rtol=1e-12)


def test_span_and_dependent_columns():
    rng = np.random.default_rng(6)
    a, b, c = rng.standard_normal((3, 100))
    # columns: a, 3a (parallel), b + 0.1 c, 2b (almost parallel to column 2), c
    Y = np.stack([a, 3 * a, b + 0.1 * c, 2 * b, 0.5 * c], axis=1)
    sel, rdiag, zero, _ = colsel.pivoted_cholesky_order(Y, 5)
    # 3a (largest), then 2b (largest part outside a), then 0.5c (b + 0.1c has
    # only 0.1c left); a and b + 0.1c then lie in the span: near-zero steps
    np.testing.assert_array_equal(sel[:3], [1, 3, 4])
    assert rdiag[3] < 1e-6 * rdiag[0] and rdiag[4] < 1e-6 * rdiag[0]
    # exactly dependent: a rank-2 matrix of 4 columns has two zero steps
    Z = np.stack([a, b, a + b, a - b], axis=1)
    sel, rdiag, zero, _ = colsel.pivoted_cholesky_order(Z, 4)
    assert np.all(rdiag[2:] <= 1e-7 * rdiag[0])


def test_truncated_pipeline_identity_and_bounds():
    m, n, r = 600, 400, 25
    A = synth.lowrank_dense(m, n, 0.7 ** np.arange(r), 11, noise=1e-9)
    sv = np.linalg.svd(A, compute_uv=False)
    k, l, s = 12, 24, 128
    o = R.rlu(A, R.Params(k, l, s, 3, truncate=True))
    assert o.L.shape == (m, k) and o.U.shape == (k, n)
    assert np.allclose(np.triu(o.L[:k], 1), 0) and np.allclose(np.diag(o.L), 1)
    assert np.allclose(np.tril(o.U[:, :k], -1), 0)
    err = R.residual_fro(A, o.L, o.U, o.perm_r, o.perm_c)
    Qk, _ = np.linalg.qr(o.Y[:, o.ysel])
    proj = np.linalg.norm(A - Qk @ (Qk.T @ A))
    assert abs(err - proj) <= 1e-9 * np.linalg.norm(A)
    assert err >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-12)
    assert o.Y.shape == (m, l)                                       # Y is the full m x l sketch
    assert len(set(o.ysel.tolist())) == k


def test_oversampling_is_kept():
    """Over 20 seeds, rank-k factors from an l = 2k sketch are on average
    closer to A than those from a k-column sketch (same k, same A)."""
    m, n = 500, 300
    A = synth.lowrank_dense(m, n, 0.8 ** np.arange(60), 12, noise=1e-8)
    k = 10
    e_trunc = [R.residual_fro(A, *_f(R.rlu(A, R.Params(k, 2 * k, 64, sd, truncate=True)))) for sd in range(20)]
    e_plain = [R.residual_fro(A, *_f(R.rlu(A, R.Params(k, k, 64, sd)))) for sd in range(20)]
    assert np.mean(e_trunc) < 0.8 * np.mean(e_plain), (np.mean(e_trunc), np.mean(e_plain))


def _f(o):
    return o.L, o.U, o.perm_r, o.perm_c


def test_truncated_pipeline_factors_the_chosen_columns_in_pivot_order():
    """Steps 3-7 run on Y_k = the chosen columns of Y in the order column
    pivoting chose them: P Y_k = L_y U_y holds for that order."""
    A = synth.lowrank_dense(400, 300, 0.8 ** np.arange(80), 6, noise=1e-6)
    o = R.rlu(A, R.Params(12, 40, 64, 2, truncate=True))
    assert np.any(np.diff(o.ysel) < 0), "selection happens to be sorted: order not exercised"
    Yk = o.Y[:, o.ysel]
    np.testing.assert_allclose(o.Ly @ o.Uy, Yk[o.perm_r], rtol=0, atol=1e-12 * np.abs(Yk).max())


def test_selection_gap_hand_value():
    """Orthogonal columns of norms 2, 4, 3: the candidates' d are 16, 9, 4
    at step 0 (gap 7/16) and 9, 4 at step 1 (gap 5/9); the screening gap is
    the smaller, relative to the top candidate."""
    Y = np.zeros((5, 3))
    Y[0, 0], Y[1, 1], Y[2, 2] = 2.0, 4.0, 3.0
    sel, rdiag, zero, gap = colsel.pivoted_cholesky_order(Y, 2)
    assert sel.tolist() == [1, 2]
    assert gap == pytest.approx(7.0 / 16.0, abs=1e-15)
