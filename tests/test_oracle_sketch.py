"""Pins of the oracle's sketch: SEM (Section 2.2) and SRFT transform (2.1)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import rng, sketch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "hand_worked.json")) as f:
        return json.load(f)


def explicit_sem(h, sgn, s):
    """Dense S (s x n): S[h(j), j] = sgn(j)."""
    n = len(h)
    S = np.zeros((s, n))
    S[h, np.arange(n)] = sgn
    return S


def explicit_real_dft(s):
    """Rows = the orthonormal real functionals, written from the DFT definition."""
    b = np.arange(s)
    T = np.empty((s, s))
    T[0] = 1.0 / np.sqrt(s)
    T[s // 2] = np.cos(np.pi * b) / np.sqrt(s)
    for f in range(1, s // 2):
        T[f] = np.sqrt(2.0 / s) * np.cos(2 * np.pi * f * b / s)
        T[s - f] = -np.sqrt(2.0 / s) * np.sin(2 * np.pi * f * b / s)
    return T  # c = T @ z


def test_sem_hand_worked():
    g = _golden()["sem"]
    y0 = sketch.sem_apply_dense(np.array(g["A"], float), np.array(g["h"]), np.array(g["sgn"]), g["s"])
    np.testing.assert_array_equal(y0, np.array(g["Y0"], float))


def test_fourier_pack_hand_worked():
    g = _golden()["fourier_pack"]
    z = np.array(g["z"], float)
    c = sketch.real_fourier_pack(np.fft.fft(z)[None, :], len(z))[0]
    np.testing.assert_allclose(c, g["c"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n,s", [(64, 8), (300, 32), (1000, 256)])
def test_sem_frobenius_norm(n, s):
    # Lemma 2.3: ||S||_F = sqrt(n)
    h, sgn = rng.sem_hash(9, n, s)
    S = explicit_sem(h, sgn, s)
    assert np.sum(S * S) == n


@pytest.mark.parametrize("n,s", [(40, 8), (200, 16)])
def test_sem_spectrum_is_sqrt_bucket_counts(n, s):
    # Lemma 2.5 and Remark 2.6: singular values are sqrt(kappa_i)
    h, sgn = rng.sem_hash(4, n, s)
    sv = np.linalg.svd(explicit_sem(h, sgn, s), compute_uv=False)
    kappa = np.sort(np.bincount(h, minlength=s))[::-1]
    np.testing.assert_allclose(sv, np.sqrt(kappa), rtol=1e-13, atol=1e-13)


def test_sem_max_load_matches_balls_into_bins():
    # Theorem 2.4 (asymptotic): mean max bucket load close to C(n,k)^2
    for ratio, s in [(2, 256), (4, 256)]:
        n = ratio * s
        loads = [np.bincount(rng.sem_hash(seed, n, s)[0], minlength=s).max() for seed in range(40)]
        c2 = n / s + np.sqrt(2 * (n / s) * np.log(s))
        assert abs(np.mean(loads) - c2) / c2 < 0.15


@pytest.mark.parametrize("m,n,s", [(5, 40, 8), (17, 100, 32)])
def test_sem_apply_brute_force(m, n, s):
    a = np.random.default_rng(1).standard_normal((m, n))
    h, sgn = rng.sem_hash(2, n, s)
    ref = a @ explicit_sem(h, sgn, s).T
    np.testing.assert_allclose(sketch.sem_apply_dense(a, h, sgn, s), ref, rtol=1e-13, atol=1e-13)
    csr = sp.csr_matrix(a)
    y0 = sketch.sem_apply_csr(csr.indptr, csr.indices, csr.data, m, n, h, sgn, s)
    np.testing.assert_allclose(y0, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("s", [4, 16, 64])
def test_real_transform_orthonormal_and_matches_dft(s):
    T = explicit_real_dft(s)
    np.testing.assert_allclose(T @ T.T, np.eye(s), atol=1e-14)
    z = np.random.default_rng(s).standard_normal((3, s))
    c = sketch.real_fourier_pack(np.fft.fft(z, axis=1), s)
    np.testing.assert_allclose(c, z @ T.T, atol=1e-13)


@pytest.mark.parametrize("m,n,s,l", [(6, 50, 16, 5), (20, 300, 64, 12)])
def test_sketch_brute_force(m, n, s, l):
    # Y = A S^T diag(d) T^T R with every operator an explicit matrix
    a = np.random.default_rng(5).standard_normal((m, n))
    seed = 21
    h, sgn = rng.sem_hash(seed, n, s)
    d = rng.srft_signs(seed, s)
    sel = rng.srft_select(seed, s, l)
    R = np.zeros((s, l))
    R[sel, np.arange(l)] = 1.0
    omega_t = explicit_sem(h, sgn, s).T @ np.diag(d) @ explicit_real_dft(s).T @ R
    y = sketch.sketch_dense(a, h, sgn, d, sel, s)
    np.testing.assert_allclose(y, a @ omega_t, rtol=1e-12, atol=1e-12)
    csr = sp.csr_matrix(a)
    yc = sketch.sketch_csr(csr.indptr, csr.indices, csr.data, m, n, h, sgn, d, sel, s)
    np.testing.assert_allclose(yc, a @ omega_t, rtol=1e-12, atol=1e-12)


def test_srft_embedding_theorem():
    # Theorem 2.2: for orthonormal U (s x r) and k >= 4[sqrt r + sqrt(8 log(r s))]^2 log r,
    # sigma(sqrt(s/k) * Pi^T U) lies in [0.40, 1.48] w.h.p.  r = 2, s = 256 -> k >= 199.
    s, r, k = 256, 2, 220
    assert 4 * (np.sqrt(r) + np.sqrt(8 * np.log(r * s))) ** 2 * np.log(r) <= k
    T = explicit_real_dft(s)
    ok = 0
    for seed in range(40):
        U = synth.orthonormal_gaussian(np.random.default_rng(seed), s, r)
        d = rng.srft_signs(seed, s)
        sel = rng.srft_select(seed, s, k)
        M = np.sqrt(s / k) * (T[sel] @ (d[:, None] * U))
        sv = np.linalg.svd(M, compute_uv=False)
        ok += (sv.min() >= 0.40) and (sv.max() <= 1.48)
    assert ok >= 36


# ---- the Walsh-Hadamard form of the transform (the paper's Section 4 choice)

@pytest.mark.parametrize("s", [1, 2, 4, 16, 256, 2048])
def test_hadamard_matches_sylvester_construction(s):
    import scipy.linalg as sl
    H = sketch.hadamard_columns(s, np.arange(s))
    np.testing.assert_array_equal(H, sl.hadamard(s))         # Sylvester order
    np.testing.assert_array_equal(H @ H.T, s * np.eye(s))      # H H^T = s I
    cols = np.array([s - 1, 0, s // 2]) if s > 1 else np.array([0])
    np.testing.assert_array_equal(sketch.hadamard_columns(s, cols), sl.hadamard(s)[:, cols])


def test_hadamard_transform_hand_worked():
    # s = 2: z = Y0 diag(d) = [3, -1]; z H_2 / sqrt 2 = [2, 4] / sqrt 2; sel = (1, 0)
    y = sketch.fjl_apply(np.array([[3.0, 1.0]]), np.array([1.0, -1.0]), np.array([1, 0]), "hadamard")
    np.testing.assert_allclose(y, [[4.0 / np.sqrt(2.0), 2.0 / np.sqrt(2.0)]], rtol=0, atol=1e-15)


@pytest.mark.parametrize("s", [8, 128])
def test_hadamard_transform_orthonormal(s):
    # every coordinate kept: an orthogonal transform keeps the row norms
    y0 = np.random.default_rng(s).standard_normal((5, s))
    d = rng.srft_signs(3, s)
    y = sketch.fjl_apply(y0, d, np.arange(s), "hadamard")
    np.testing.assert_allclose(np.linalg.norm(y, axis=1), np.linalg.norm(y0, axis=1), rtol=1e-13)


@pytest.mark.parametrize("m,n,s,l", [(6, 50, 16, 5), (20, 300, 64, 12)])
def test_hadamard_sketch_brute_force(m, n, s, l):
    # Y = A S^T diag(d) (H / sqrt s) R with every operator an explicit matrix
    import scipy.linalg as sl
    a = np.random.default_rng(6).standard_normal((m, n))
    seed = 22
    h, sgn = rng.sem_hash(seed, n, s)
    d = rng.srft_signs(seed, s)
    sel = rng.srft_select(seed, s, l)
    R = np.zeros((s, l))
    R[sel, np.arange(l)] = 1.0
    omega_t = explicit_sem(h, sgn, s).T @ np.diag(d) @ (sl.hadamard(s) / np.sqrt(s)) @ R
    y = sketch.sketch_dense(a, h, sgn, d, sel, s, "hadamard")
    np.testing.assert_allclose(y, a @ omega_t, rtol=1e-12, atol=1e-12)
    csr = sp.csr_matrix(a)
    yc = sketch.sketch_csr(csr.indptr, csr.indices, csr.data, m, n, h, sgn, d, sel, s, "hadamard")
    np.testing.assert_allclose(yc, a @ omega_t, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("transform", ["fourier", "hadamard"])
def test_csr_sketch_spans_row_chunks(transform):
    """The CSR sketch of a matrix with more rows than one processing chunk
    (5000) equals the sketch of the same matrix held dense."""
    rs = np.random.default_rng(12)
    a = sp.random(5000, 300, density=0.02, format="csr", random_state=rs,
                  data_rvs=lambda k: rs.standard_normal(k))
    h, sgn = rng.sem_hash(4, 300, 64)
    d = rng.srft_signs(4, 64)
    sel = rng.srft_select(4, 64, 20)
    got = sketch.sketch_csr(a.indptr, a.indices, a.data, 5000, 300, h, sgn, d, sel, 64, transform)
    want = sketch.sketch_dense(a.toarray(), h, sgn, d, sel, 64, transform)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
