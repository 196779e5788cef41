"""Least-squares product of Algorithm 1, exact form (Corollary 3.2).

Algorithm 1 steps 4-6 approximate L_y^+ P A through a second projection;
the exact product B = L_y^+ P A is the quantity that Corollary 3.2 bounds
(||PA - L_y L_y^+ PA||_F < (1 + eps) Delta_r).  Since P is a permutation,
L_y^+ P = (P^T L_y)^+, so with Lhat = P^T L_y (rows back in A's order)
B = Lhat^+ A.

The oracle forms it by Householder QR (LAPACK dgeqrf via numpy.linalg.qr):
Lhat = Q R, B = R^{-1} (Q^T A).  This is deliberately a different route from
normal equations so that it checks them independently.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


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
