"""Least-squares product of Algorithm 1: exact form (Corollary 3.2) and the
paper's own sketched form (Algorithm 1 steps 4-6).

Algorithm 1 steps 4-6 approximate L_y^+ P A through a second projection;
the exact product B = L_y^+ P A is the quantity that Corollary 3.2 bounds
(||PA - L_y L_y^+ PA||_F < (1 + eps) Delta_r).  Since P is a permutation,
L_y^+ P = (P^T L_y)^+, so with Lhat = P^T L_y (rows back in A's order)
B = Lhat^+ A.

The oracle forms it by Householder QR (LAPACK dgeqrf via numpy.linalg.qr):
Lhat = Q R, B = R^{-1} (Q^T A).  This is deliberately a different route from
normal equations so that it checks them independently.

The sketched form follows Algorithm 1 steps 4-5 as printed: a second
projection Omega_2 = Pi_2 S_2 (k_2 x m; S_2 an l_2 x m SEM, Pi_2 a k_2 x l_2
SRFT, built exactly like Omega_1 but over the m rows), then
X = (Omega_2 L_y)^+ (Omega_2 P A), a k_2 x l least-squares problem solved
by the same Householder QR.  Omega_2 acts on the rows of P A and L_y in
pivoted order (row i of P A is row perm_r[i] of A).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import sketch as sk


def unpermute_rows(L: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Lhat = P^T L: row i of L belongs to row perm[i] of A."""
    Lhat = np.empty_like(L)
    Lhat[perm] = L
    return Lhat


def lstsq_product(Lhat: np.ndarray, A) -> np.ndarray:
    """B = Lhat^+ A for dense A (m x n) or a scipy sparse A."""
    Q, R = np.linalg.qr(Lhat, mode="reduced")
    if sp.issparse(A):
        QtA = np.asarray((A.T @ Q).T)
    else:
        QtA = Q.T @ np.asarray(A, dtype=np.float64)
    return sla.solve_triangular(R, QtA, lower=False)


def omega2_apply(X, h2, sgn2, d2, sel2, l2: int, transform: str = "fourier") -> np.ndarray:
    """Omega_2 X for X with m rows (k_2 x cols): the column-wise form of the
    sketch of steps 1-2, since (Omega_2 X)^T = X^T Omega_2^T.  X dense, or
    scipy sparse (then the CSR sketch of X^T)."""
    if sp.issparse(X):
        xt = sp.csr_matrix(X.T)
        cols, rows = xt.shape
        return sk.sketch_csr(xt.indptr, xt.indices, xt.data, cols, rows, h2, sgn2, d2, sel2, l2, transform).T
    X = np.asarray(X, dtype=np.float64)
    return sk.sketch_dense(np.ascontiguousarray(X.T), h2, sgn2, d2, sel2, l2, transform).T


def sketched_lstsq_product(Ly: np.ndarray, PA: np.ndarray, h2, sgn2, d2, sel2, l2: int,
                           transform: str = "fourier"):
    """Algorithm 1 steps 4-5: X = (Omega_2 L_y)^+ Omega_2 P A.

    Ly: m x l in pivoted row order; PA: m x n (dense or scipy sparse), the
    rows of A in that order.
    Returns X (l x n) and the two sketches M = Omega_2 L_y, Z = Omega_2 P A.
    """
    M = omega2_apply(Ly, h2, sgn2, d2, sel2, l2, transform)
    Z = omega2_apply(PA, h2, sgn2, d2, sel2, l2, transform)
    return lstsq_product(M, Z), M, Z
