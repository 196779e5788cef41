"""Pins of the oracle's second projection (Algorithm 1 steps 4-5, Theorem 3.3).

B = (Omega_2 L_y)^+ Omega_2 P A with Omega_2 = Pi_2 S_2 (k_2 x m).
"""
import numpy as np
import pytest

import synth
from oracle import lstsq, rng, rlu as R
from test_oracle_sketch import explicit_real_dft, explicit_sem


def _omega2_explicit(m, h2, sgn2, d2, sel2, l2, transform):
    """Omega_2 = R^T T D S_2 (k_2 x m) with every operator an explicit matrix."""
    T = explicit_real_dft(l2)
    if transform == "hadamard":
        b = np.arange(l2)
        T = np.array([[(-1.0) ** bin(x & y).count("1") for y in b] for x in b]) / np.sqrt(l2)
    return T[sel2] @ np.diag(d2) @ explicit_sem(h2, sgn2, l2)


@pytest.mark.parametrize("transform", ["fourier", "hadamard"])
def test_second_projection_brute_force(transform):
    g = np.random.default_rng(11)
    m, n, l, l2, k2 = 90, 40, 6, 32, 20
    Ly = np.tril(g.standard_normal((m, l)), -1)
    Ly[np.arange(l), np.arange(l)] = 1.0
    PA = g.standard_normal((m, n))
    h2, sgn2 = rng.sem_hash(5, m, l2, stream=rng.STREAM_SEM2)
    d2 = rng.srft_signs(5, l2, stream=rng.STREAM_SIGNS2)
    sel2 = rng.srft_select(5, l2, k2, stream=rng.STREAM_SELECT2)
    om = _omega2_explicit(m, h2, sgn2, d2, sel2, l2, transform)
    X, M, Z = lstsq.sketched_lstsq_product(Ly, PA, h2, sgn2, d2, sel2, l2, transform)
    np.testing.assert_allclose(M, om @ Ly, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Z, om @ PA, rtol=1e-12, atol=1e-12)
    ref = np.linalg.lstsq(om @ Ly, om @ PA, rcond=None)[0]
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-10)


def test_orthogonal_omega2_gives_the_exact_product():
    # With S_2 a signed permutation (l_2 = m) and every SRFT coordinate kept
    # (k_2 = l_2), Omega_2 is orthogonal, so (Omega_2 L)^+ Omega_2 = L^+ and
    # the sketched product equals the exact one for any A.
    g = np.random.default_rng(3)
    m, n, l = 64, 30, 9
    Ly = g.standard_normal((m, l))
    PA = g.standard_normal((m, n))
    h2 = g.permutation(m)
    sgn2 = g.choice([-1, 1], m)
    d2 = g.choice([-1, 1], m)
    sel2 = g.permutation(m)
    X, _, _ = lstsq.sketched_lstsq_product(Ly, PA, h2, sgn2, d2, sel2, m)
    np.testing.assert_allclose(X, np.linalg.lstsq(Ly, PA, rcond=None)[0], rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("transform", ["fourier", "hadamard"])
def test_rank_exact_input_is_reproduced(transform):
    # P A = L_y X exactly, so Omega_2 P A = (Omega_2 L_y) X and the
    # least-squares solve returns X itself: the same B as the exact product.
    A = synth.lowrank_dense(400, 300, np.linspace(1.0, 0.1, 15), 3)
    ex = R.rlu(A, R.Params(15, 20, 64, 7, transform))
    sk = R.rlu(A, R.Params(15, 20, 64, 7, transform, k2=48, l2=128))
    assert R.residual_fro(A, sk.L, sk.U, sk.perm_r, sk.perm_c) <= 1e-12 * np.linalg.norm(A)
    np.testing.assert_array_equal(sk.perm_r, ex.perm_r)
    np.testing.assert_allclose(sk.B, ex.B, rtol=1e-9, atol=1e-9 * np.abs(ex.B).max())


def test_sketched_residual_is_bounded_by_the_exact_one():
    # LU - PAQ = (L_y X - P A) Q, and the exact product minimises ||L_y X - P A||_F,
    # so the sketched residual is never below it; Theorem 3.3's argument bounds
    # it by a constant times the exact one (checked on most draws).
    ratios = []
    for seed in range(40):
        A = synth.lowrank_dense(150, 90, 0.5 ** np.arange(12), seed, noise=1e-6)
        ex = R.rlu(A, R.Params(8, 16, 64, seed + 1))
        sk = R.rlu(A, R.Params(8, 16, 64, seed + 1, k2=64, l2=128))
        r_ex = R.residual_fro(A, ex.L, ex.U, ex.perm_r, ex.perm_c)
        r_sk = R.residual_fro(A, sk.L, sk.U, sk.perm_r, sk.perm_c)
        assert r_sk >= r_ex * (1 - 1e-9)
        ratios.append(r_sk / r_ex)
    assert np.mean(np.array(ratios) <= 2.0) >= 0.95


def test_structure_with_second_projection():
    A = synth.small_dense()
    res = R.rlu(A, R.Params(20, 30, 256, 1, k2=96, l2=512))
    m, n, l = 1024, 512, 30
    assert res.L.shape == (m, l) and res.U.shape == (l, n)
    np.testing.assert_allclose(np.diag(res.L[:l]), 1.0, rtol=1e-12)
    assert np.all(np.triu(res.L[:l], 1) == 0) and np.all(np.tril(res.U, -1) == 0)
    assert sorted(res.perm_r.tolist()) == list(range(m))
    assert sorted(res.perm_c.tolist()) == list(range(n))
    assert res.extra["M"].shape == (96, l) and res.extra["Z"].shape == (96, n)


@pytest.mark.parametrize("bad", [dict(k2=10, l2=64), dict(k2=80, l2=64), dict(k2=40, l2=96),
                                 dict(k2=40, l2=0)])
def test_invalid_second_projection_params(bad):
    with pytest.raises(ValueError):
        R.check_params(600, 500, R.Params(8, 16, 64, 1, **bad))


def test_streams_of_the_two_projections_differ():
    h1, _ = rng.sem_hash(9, 2000, 256)
    h2, _ = rng.sem_hash(9, 2000, 256, stream=rng.STREAM_SEM2)
    assert np.mean(h1 == h2) < 0.02


def test_second_projection_csr_and_dense_agree():
    import scipy.sparse as sp
    a = synth.lowrank_dense(300, 200, 0.7 ** np.arange(60), 4, noise=1e-3)
    a[np.abs(a) < 2e-3] = 0.0           # a sparse pattern
    c = sp.csr_matrix(a)
    p = R.Params(8, 16, 64, 3, k2=48, l2=128)
    d = R.rlu(a, p)
    s = R.rlu(None, p, csr=(c.indptr, c.indices, c.data, 300, 200))
    np.testing.assert_array_equal(d.perm_r, s.perm_r)
    np.testing.assert_array_equal(d.perm_c, s.perm_c)
    np.testing.assert_allclose(s.B, d.B, rtol=1e-10, atol=1e-12)


def test_pipeline_draws_omega2_independently_of_omega1():
    """Algorithm 1 step 4 draws Omega_2 afresh: at equal sizes (m = n,
    l2 = s) the pipeline's Omega_2 parameters must not repeat Omega_1's."""
    p = R.Params(8, 16, 256, 5, k2=64, l2=256)
    h, sgn, d, sel = R.sketch_params(2000, p)
    h2, sgn2, d2, sel2 = R.omega2_params(2000, p)
    assert np.mean(h == h2) < 0.02                 # about 1/256 by chance
    assert np.mean(sgn == sgn2) < 0.6              # about 1/2 by chance
    assert np.mean(d == d2) < 0.65
    assert len(set(sel[:16]) & set(sel2[:16])) < 8
