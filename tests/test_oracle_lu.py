"""Pins of the oracle's pivoted LUs (Algorithm 1 steps 3 and 6)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import lu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "hand_worked.json")) as f:
        return json.load(f)


def _lapack_perm(piv, m):
    perm = np.arange(m)
    for j, p in enumerate(piv):
        perm[[j, p]] = perm[[p, j]]
    return perm


def test_gepp_hand_worked():
    g = _golden()["gepp"]
    L, U, perm, ipiv, zp, _ = lu.gepp(np.array(g["Y"], float))
    np.testing.assert_array_equal(perm, g["perm"])
    np.testing.assert_array_equal(ipiv, g["ipiv"])
    np.testing.assert_allclose(L, g["L"], rtol=1e-15)
    np.testing.assert_allclose(U, g["U"], rtol=1e-15)
    assert zp == 0


def test_colpiv_hand_worked():
    g = _golden()["colpiv"]
    Lt, U, perm, ipiv, zp, _ = lu.colpiv_lu(np.array(g["B"], float))
    np.testing.assert_array_equal(perm, g["perm"])
    np.testing.assert_array_equal(ipiv, g["ipiv"])
    np.testing.assert_allclose(Lt, g["Lt"], rtol=1e-15)
    np.testing.assert_allclose(U, g["U"], rtol=1e-14)


@pytest.mark.parametrize("m,l,seed", [(10, 3, 0), (200, 30, 1), (1000, 64, 2), (64, 64, 3)])
def test_gepp_matches_lapack(m, l, seed):
    y = np.random.default_rng(seed).standard_normal((m, l))
    L, U, perm, ipiv, zp, gap = lu.gepp(y)
    lu_, piv = sla.lu_factor(y)
    np.testing.assert_array_equal(ipiv, piv)
    np.testing.assert_array_equal(perm, _lapack_perm(piv, m))
    np.testing.assert_allclose(np.triu(lu_[:l]), U, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.tril(lu_, -1)[:, :l] + np.eye(m, l), L, rtol=1e-12, atol=1e-12)
    assert np.abs(L).max() <= 1.0
    eps = np.finfo(float).eps
    assert np.linalg.norm(y[perm] - L @ U) <= 10 * m * eps * np.linalg.norm(y)


@pytest.mark.parametrize("l,n,seed", [(3, 10, 0), (30, 200, 1), (64, 1000, 2)])
def test_colpiv_matches_lapack_on_transpose(l, n, seed):
    b = np.random.default_rng(seed).standard_normal((l, n))
    Lt, U, perm, ipiv, zp, gap = lu.colpiv_lu(b)
    # dgetrf on B^T: Q^T B^T = L' U'  =>  Lt = U'^T diag(U')^-1, U = diag(U') L'^T
    lu_, piv = sla.lu_factor(b.T)
    np.testing.assert_array_equal(ipiv, piv)
    np.testing.assert_array_equal(perm, _lapack_perm(piv, n))
    Up = np.triu(lu_[:l])
    Lp = np.tril(lu_, -1)[:, :l] + np.eye(n, l)
    dg = np.diag(Up)
    np.testing.assert_allclose(Lt, Up.T / dg, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(U, dg[:, None] * Lp.T, rtol=1e-11, atol=1e-11)
    # the pivot is the largest entry of its row of U
    assert np.all(np.abs(U) <= np.abs(np.diag(U))[:, None] * (1 + 1e-15))
    assert np.allclose(np.tril(U, -1), 0)


def test_gepp_ties_take_first_position():
    y = np.array([[1.0, 2.0], [-3.0, 1.0], [3.0, 5.0], [2.0, 0.0]])
    L, U, perm, ipiv, _, gap = lu.gepp(y)
    _, piv = sla.lu_factor(y)
    assert ipiv[0] == 1
    np.testing.assert_array_equal(ipiv, piv)
    assert gap == 0.0


def test_zero_pivot_rule():
    y = np.random.default_rng(0).standard_normal((8, 4))
    y[:, 1] = y[:, 0]                 # Schur column 1 is exactly zero after step 0
    L, U, perm, ipiv, zp, _ = lu.gepp(y)
    assert zp == 1
    assert ipiv[1] == 1
    assert U[1, 1] == 0.0
    np.testing.assert_array_equal(L[2:, 1], 0.0)
    np.testing.assert_allclose(y[perm], L @ U, atol=1e-14)
    b = y.T.copy()
    Lt, Ub, permc, ipivc, zpb, _ = lu.colpiv_lu(b)
    assert zpb == 1 and ipivc[1] == 1
    assert np.all(Ub[1] == 0.0) and np.all(Lt[2:, 1] == 0.0)
    # A zero pivot row cannot eliminate the entries below it in its column:
    # the zero-pivot rule drops exactly those (column 1, rows 2..), and
    # nothing else.
    resid = b[:, permc] - Lt @ Ub
    mask = np.ones_like(resid, dtype=bool)
    mask[2:, 1] = False
    np.testing.assert_allclose(resid[mask], 0.0, atol=1e-14)


def test_nonfinite_raises():
    y = np.ones((4, 2))
    y[2, 0] = np.nan
    with pytest.raises(FloatingPointError):
        lu.gepp(y)
    with pytest.raises(FloatingPointError):
        lu.colpiv_lu(y.T.copy())


def test_pivot_gap_hand_values():
    """The screening gap is the smallest (top - second) / top over the
    steps.  Y: step 0 sees |4|, |3|, 0 (gap 1/4), step 1 sees 2, 1 (gap 1/2).
    B: step 0 sees |4|, |3|, 0 in row 0 (1/4); row 1 is untouched by the
    elimination (multiplier 0) and step 1 sees 2, 1 (1/2)."""
    Y = np.array([[4.0, 0.0], [3.0, 2.0], [0.0, 1.0]])
    assert lu.gepp(Y)[5] == pytest.approx(0.25, abs=1e-15)
    B = np.array([[4.0, 3.0, 0.0], [0.0, 2.0, 1.0]])
    assert lu.colpiv_lu(B)[5] == pytest.approx(0.25, abs=1e-15)
    # the step-1 gap alone, when step 0's is wider
    assert lu.gepp(np.array([[4.0, 0.0], [1.0, 2.0], [0.0, 1.0]]))[5] == pytest.approx(0.5, abs=1e-15)
    assert lu.colpiv_lu(np.array([[4.0, 1.0, 0.0], [0.0, 2.0, 1.0]]))[5] == pytest.approx(0.5, abs=1e-15)
