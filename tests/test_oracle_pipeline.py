"""Pins of the oracle end to end: Corollary 3.2, Theorem 3.1, Theorem 3.3."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import lstsq, rlu as R


def test_lstsq_matches_library():
    rng = np.random.default_rng(0)
    Lhat = rng.standard_normal((300, 20))
    A = rng.standard_normal((300, 70))
    B = lstsq.lstsq_product(Lhat, A)
    ref = np.linalg.lstsq(Lhat, A, rcond=None)[0]
    np.testing.assert_allclose(B, ref, rtol=1e-11, atol=1e-11)
    Bs = lstsq.lstsq_product(Lhat, sp.csr_matrix(A))
    np.testing.assert_allclose(Bs, ref, rtol=1e-11, atol=1e-11)


def _tiny(seed, m=120, n=80, r=12, decay=0.5, noise=1e-6):
    sig = decay ** np.arange(r)
    return synth.lowrank_dense(m, n, sig, seed, noise=noise)


def _structure(res, m, n, l):
    L, U = res.L, res.U
    assert L.shape == (m, l) and U.shape == (l, n)
    np.testing.assert_allclose(np.diag(L[:l]), 1.0, rtol=1e-12)
    assert np.all(np.triu(L[:l], 1) == 0)
    assert np.all(np.tril(U, -1) == 0)
    assert sorted(res.perm_r.tolist()) == list(range(m))
    assert sorted(res.perm_c.tolist()) == list(range(n))
    assert np.all(np.abs(U) <= np.abs(np.diag(U))[:, None] * (1 + 1e-15))


def test_structure_and_identity_with_range_projection():
    # LU - PAQ = -(I - L_y L_y^+) P A Q and Im L_y = Im Y (Corollary 3.2 via Theorem 3.1):
    # ||LU - PAQ||_F equals ||A - Q_Y Q_Y^T A||_F.
    A = synth.small_dense()
    p = R.Params(20, 30, 256, 1)
    res = R.rlu(A, p)
    _structure(res, 1024, 512, 30)
    assert res.zero_pivots_y == 0
    qy, _ = np.linalg.qr(res.Y)
    proj = np.linalg.norm(A - qy @ (qy.T @ A))
    got = R.residual_fro(A, res.L, res.U, res.perm_r, res.perm_c)
    # The residual here is ~1.2e-7 ||A||, so the rounding of the two sides
    # (~1e-16 ||A|| each) bounds their agreement near 1e-9 relative; measured 2e-11.
    assert got == pytest.approx(proj, rel=1e-9)
    # Eckart-Young lower bound: rank(LU) <= l
    assert got >= R.tail_norm(A, 30) * (1 - 1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_identity_with_range_projection_large_residual(seed):
    # A residual of order ||A|| leaves nothing for rounding to cancel: the
    # identity holds to a few ulps.
    A = synth.lowrank_dense(300, 200, 0.7 ** np.arange(40), seed, noise=1e-3)
    res = R.rlu(A, R.Params(10, 16, 64, seed + 1))
    qy, _ = np.linalg.qr(res.Y)
    proj = np.linalg.norm(A - qy @ (qy.T @ A))
    got = R.residual_fro(A, res.L, res.U, res.perm_r, res.perm_c)
    assert got == pytest.approx(proj, rel=1e-12)


def test_tail_norm_hand_values():
    # Delta_k = sqrt(sum_{i > k} sigma_i^2) for a matrix of known singular
    # values 5, 4, 3, 2, 1: a signed, permuted diagonal inside a 7 x 6 zero matrix
    A = np.zeros((7, 6))
    for r, c, v in [(2, 4, -3.0), (0, 1, 5.0), (6, 0, 1.0), (3, 5, -4.0), (5, 2, 2.0)]:
        A[r, c] = v
    want = {0: np.sqrt(55.0), 1: np.sqrt(30.0), 2: np.sqrt(14.0), 3: np.sqrt(5.0), 4: 1.0, 5: 0.0}
    for k, v in want.items():
        assert R.tail_norm(A, k) == pytest.approx(v, rel=1e-14, abs=1e-14), k
    # without the empty column every singular value is nonzero (the last
    # one, 1, is in every tail but the empty one)
    A5 = np.delete(A, 3, axis=1)
    for k, v in want.items():
        assert R.tail_norm(A5, k) == pytest.approx(v, rel=1e-14, abs=1e-14), k


def test_rank_exact_input_is_reproduced():
    A = synth.lowrank_dense(400, 300, np.linspace(1.0, 0.1, 15), 3)
    res = R.rlu(A, R.Params(15, 20, 64, 7))
    assert R.residual_fro(A, res.L, res.U, res.perm_r, res.perm_c) <= 1e-12 * np.linalg.norm(A)


def test_error_bound_against_tail_norm():
    # Theorem 3.3 / Corollary 3.2: ||LU - PAQ||_F <= C Delta_k on most draws
    ratios = []
    for seed in range(100):
        A = _tiny(seed)
        res = R.rlu(A, R.Params(8, 16, 64, seed + 1))
        ratios.append(R.residual_fro(A, res.L, res.U, res.perm_r, res.perm_c) / R.tail_norm(A, 8))
    ratios = np.array(ratios)
    assert np.mean(ratios <= 10.0) >= 0.95
    assert ratios.min() >= R.tail_norm(_tiny(0), 16) / R.tail_norm(_tiny(0), 8) * 0.5


def test_csr_and_dense_agree():
    row_ptr, col, val = synth.random_csr(300, 200, 0.05, 4, plant_rank=5, plant_rows=30,
                                         plant_scale=50.0)
    A = synth.csr_to_dense(row_ptr, col, val, 300, 200)
    p = R.Params(10, 16, 64, 3)
    rd = R.rlu(A, p)
    rc = R.rlu(None, p, csr=(row_ptr, col, val, 300, 200))
    np.testing.assert_array_equal(rd.perm_r, rc.perm_r)
    np.testing.assert_array_equal(rd.perm_c, rc.perm_c)
    np.testing.assert_allclose(rc.L, rd.L, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(rc.U, rd.U, rtol=1e-9, atol=1e-9 * np.abs(rd.U).max())


def test_factors_reassemble_steps():
    A = _tiny(5)
    res = R.rlu(A, R.Params(8, 16, 64, 9))
    # L = L_y L~ and B Q = L~ U
    np.testing.assert_allclose(res.L, res.Ly @ res.Lt, atol=1e-14)
    np.testing.assert_allclose(res.B[:, res.perm_c], res.Lt @ res.U, atol=1e-12 * np.abs(res.B).max())
    # P Y = L_y U_y
    np.testing.assert_allclose(res.Y[res.perm_r], res.Ly @ res.Uy, atol=1e-13 * np.abs(res.Y).max())


@pytest.mark.parametrize("bad", [dict(k=0, l=4, s=8), dict(k=5, l=4, s=8), dict(k=2, l=9, s=8),
                                 dict(k=2, l=4, s=12), dict(k=2, l=70, s=128)])
def test_invalid_params(bad):
    with pytest.raises(ValueError):
        R.check_params(60, 50, R.Params(seed=1, **bad))


def test_rank_exact_input_is_reproduced_with_hadamard():
    A = synth.lowrank_dense(400, 300, np.linspace(1.0, 0.1, 15), 3)
    res = R.rlu(A, R.Params(15, 20, 64, 7, "hadamard"))
    assert R.residual_fro(A, res.L, res.U, res.perm_r, res.perm_c) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("section", ["4.1", "4.2"])
def test_section4_spectra_error_between_tail_norms(section):
    # Section 4's matrices (singular values given, vectors random): the
    # rank-l factorization's error lies between Delta_l (Eckart-Young) and a
    # small multiple of Delta_r (Theorem 3.3).
    n, r = 400, 20
    sig = synth.spectrum_step_exp(n, r) if section == "4.1" else synth.spectrum_exp_range(n)
    A = synth.lowrank_dense(n, n, sig, 11)
    p = R.Params(r, r + 10, 128, 5)
    res = R.rlu(A, p)
    err = R.residual_fro(A, res.L, res.U, res.perm_r, res.perm_c)
    d_r = np.sqrt(np.sum(sig[r:] ** 2))
    d_l = np.sqrt(np.sum(sig[r + 10:] ** 2))
    assert d_l * (1 - 1e-9) <= err <= 10 * d_r
