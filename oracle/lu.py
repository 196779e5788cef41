"""The two pivoted LU factorizations of Algorithm 1 (Section 3), textbook form.

* ``gepp``       -- step 3: P Y = L_y U_y, Gaussian elimination with partial
  (row) pivoting, right-looking, one column at a time (Golub & Van Loan,
  Matrix Computations, Alg. 3.4.1).
* ``colpiv_lu``  -- step 6: B Q = L~ U, "LU with right partial pivoting",
  read as pivoting on columns: at step j the pivot is the entry of largest
  magnitude in the current row j; L~ is unit lower triangular.

Conventions where the paper is silent:
* ties: the candidate at the smallest current position wins, and the pivot
  exchanges position j with the pivot's position (LAPACK ipiv semantics);
* zero pivot (the whole candidate row / column is zero): no exchange, the
  multipliers of that step are zero, the U diagonal entry is zero, and a
  counter is incremented;
* a non-finite value reaching a pivot search raises FloatingPointError.

Each factorization also reports the smallest relative gap between the
largest and second-largest candidate magnitudes over all steps, used to
screen inputs whose pivot choices are not robust to rounding.
"""
from __future__ import annotations

import numpy as np


def _pivot(vals: np.ndarray):
    """Index of the first maximum of |vals|, and the top-two relative gap."""
    mag = np.abs(vals)
    if not np.all(np.isfinite(mag)):
        raise FloatingPointError("non-finite value in pivot search")
    p = int(np.argmax(mag))
    top = mag[p]
    if mag.shape[0] > 1 and top > 0:
        rest = np.delete(mag, p)
        gap = (top - rest.max()) / top
    else:
        gap = np.inf
    return p, top, gap


def gepp(Y: np.ndarray):
    """Row-pivoted LU of a tall m x l matrix (m >= l).

    Returns (L, U, perm, ipiv, zero_pivots, min_gap) with
    Y[perm, :] = L @ U, L m x l unit lower trapezoidal, U l x l upper,
    ipiv[j] = the position exchanged with position j at step j.
    """
    W = np.array(Y, dtype=np.float64, copy=True)
    m, l = W.shape
    if m < l:
        raise ValueError("gepp expects m >= l")
    perm = np.arange(m)
    ipiv = np.empty(l, dtype=np.int64)
    zero_pivots, min_gap = 0, np.inf
    for j in range(l):
        off, top, gap = _pivot(W[j:, j])
        p = j + off
        min_gap = min(min_gap, gap)
        ipiv[j] = p
        if p != j:
            W[[j, p], :] = W[[p, j], :]
            perm[[j, p]] = perm[[p, j]]
        if top == 0.0:
            zero_pivots += 1
            W[j + 1:, j] = 0.0
            continue
        W[j + 1:, j] = W[j + 1:, j] / W[j, j]
        W[j + 1:, j + 1:] -= np.outer(W[j + 1:, j], W[j, j + 1:])
    L = np.tril(W[:, :l], -1)
    L[np.arange(l), np.arange(l)] = 1.0
    U = np.triu(W[:l, :l])
    return L, U, perm, ipiv, zero_pivots, min_gap


def colpiv_lu(B: np.ndarray):
    """Column-pivoted LU of a wide l x n matrix (n >= l).

    Returns (Lt, U, perm, ipiv, zero_pivots, min_gap) with
    B[:, perm] = Lt @ U, Lt l x l unit lower, U l x n upper trapezoidal.
    """
    W = np.array(B, dtype=np.float64, copy=True)
    l, n = W.shape
    if n < l:
        raise ValueError("colpiv_lu expects n >= l")
    perm = np.arange(n)
    ipiv = np.empty(l, dtype=np.int64)
    Lt = np.eye(l)
    zero_pivots, min_gap = 0, np.inf
    for j in range(l):
        off, top, gap = _pivot(W[j, j:])
        c = j + off
        min_gap = min(min_gap, gap)
        ipiv[j] = c
        if c != j:
            W[:, [j, c]] = W[:, [c, j]]
            perm[[j, c]] = perm[[c, j]]
        if top == 0.0:
            zero_pivots += 1
            continue
        Lt[j + 1:, j] = W[j + 1:, j] / W[j, j]
        W[j + 1:, j + 1:] -= np.outer(Lt[j + 1:, j], W[j, j + 1:])
        W[j + 1:, j] = 0.0
    U = np.triu(W)
    return Lt, U, perm, ipiv, zero_pivots, min_gap
