"""The two projections of Algorithm 1, steps 1-2 (Section 3), plain FP64.

* ``sem_apply``  -- Y0 = A S^T with S = Phi D the sparse embedding matrix of
  Section 2.2 (one nonzero, +-1, per column of S; column j of A is added with
  sign sgn(j) into bucket h(j)).
* ``fjl_apply``  -- Y = Y0 diag(d) T R: the SRFT of Section 2.1 in its real
  form.  d is a +-1 diagonal; T is the length-s DFT (kernel e^{-2 pi i f b / s},
  1/sqrt(s) normalisation, Section 2.1) re-expressed on an orthonormal real
  basis; R keeps the l coordinates listed in ``sel``, in that order.

The real basis (the paper's experiments also use a real transform, Section 4)
packs the spectrum X of a real vector z as
    c_0 = X_0 / sqrt(s),  c_{s/2} = X_{s/2} / sqrt(s),
    c_f = sqrt(2) Re X_f / sqrt(s),  c_{s-f} = sqrt(2) Im X_f / sqrt(s)
for 1 <= f < s/2.  These s functionals are orthonormal, so T is orthogonal.

With ``transform="hadamard"`` T is instead the normalised Walsh-Hadamard
matrix H_s / sqrt(s) in Sylvester order, H[b, c] = (-1)^popcount(b & c): the
subsampled randomized Hadamard transform, the real transform of the paper's
own experiments (Section 4).  d, sel and the sparse embedding are the same.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

ROW_CHUNK = 4096


def sem_apply_dense(A: np.ndarray, h: np.ndarray, sgn: np.ndarray, s: int) -> np.ndarray:
    """Y0[i, h(j)] += sgn(j) * A[i, j] for every j, taken in ascending order."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    y0 = np.zeros((m, s))
    for j in range(n):
        y0[:, h[j]] += sgn[j] * A[:, j]
    return y0


def sem_apply_csr(row_ptr, col, val, m: int, n: int, h, sgn, s: int) -> np.ndarray:
    """Y0 = A S^T for CSR A, by a library sparse product with the explicit S."""
    a = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)),
                      shape=(m, n))
    st = sp.csr_matrix((np.asarray(sgn, dtype=np.float64), (np.arange(n), np.asarray(h))),
                       shape=(n, s))
    return np.asarray((a @ st).todense())


def real_fourier_pack(X: np.ndarray, s: int) -> np.ndarray:
    """Orthonormal real coordinates c (last axis, length s) from a spectrum X."""
    c = np.empty(X.shape[:-1] + (s,))
    half = s // 2
    rs = 1.0 / np.sqrt(s)
    c[..., 0] = X[..., 0].real * rs
    c[..., half] = X[..., half].real * rs
    f = np.arange(1, half)
    c[..., f] = np.sqrt(2.0) * X[..., f].real * rs
    c[..., s - f] = np.sqrt(2.0) * X[..., f].imag * rs
    return c


def hadamard_columns(s: int, cols: np.ndarray) -> np.ndarray:
    """Columns ``cols`` of the Sylvester-order Hadamard matrix of order s,
    from the definition H[b, c] = (-1)^popcount(b & c)."""
    b = np.arange(s, dtype=np.int64)[:, None]
    c = np.asarray(cols, dtype=np.int64)[None, :]
    x = b & c
    parity = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        parity ^= x & 1
        x = x >> 1
    return np.where(parity == 1, -1.0, 1.0)


def fjl_apply(Y0: np.ndarray, d: np.ndarray, sel: np.ndarray, transform: str = "fourier") -> np.ndarray:
    """Y = (Y0 diag(d)) T R, one row at a time (rows are independent)."""
    m, s = Y0.shape
    y = np.empty((m, len(sel)))
    if transform == "hadamard":
        Hs = hadamard_columns(s, sel) / np.sqrt(s)   # T R: the kept columns of H_s / sqrt(s)
    elif transform != "fourier":
        raise ValueError(f"unknown transform {transform!r}")
    for a in range(0, m, ROW_CHUNK):
        z = Y0[a:a + ROW_CHUNK] * d
        if transform == "hadamard":
            y[a:a + ROW_CHUNK] = z @ Hs
        else:
            X = np.fft.fft(z, axis=1)
            y[a:a + ROW_CHUNK] = real_fourier_pack(X, s)[:, sel]
    return y


def sketch_dense(A, h, sgn, d, sel, s, transform="fourier"):
    """Algorithm 1 step 2 for dense A: Y = A Omega_1^T (m x l)."""
    out = np.empty((A.shape[0], len(sel)))
    for a in range(0, A.shape[0], ROW_CHUNK):
        y0 = sem_apply_dense(A[a:a + ROW_CHUNK], h, sgn, s)
        out[a:a + ROW_CHUNK] = fjl_apply(y0, d, sel, transform)
    return out


def sketch_csr(row_ptr, col, val, m, n, h, sgn, d, sel, s, transform="fourier"):
    """Algorithm 1 step 2 for CSR A (cost proportional to nnz, Theorem 2.9)."""
    out = np.empty((m, len(sel)))
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    for a in range(0, m, ROW_CHUNK):
        b = min(m, a + ROW_CHUNK)
        lo, hi = row_ptr[a], row_ptr[b]
        y0 = sem_apply_csr(row_ptr[a:b + 1] - lo, col[lo:hi], val[lo:hi], b - a, n, h, sgn, s)
        out[a:b] = fjl_apply(y0, d, sel, transform)
    return out


def sketch_rows_dense(A_rows, h, sgn, d, sel, s, transform="fourier"):
    """Y for a subset of rows (rows are independent); used for sampled checks."""
    return fjl_apply(sem_apply_dense(A_rows, h, sgn, s), d, sel, transform)
