"""Column selection of the rank-k (truncated) output, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 (Section 3) returns factors of the sketch's width: L is m x k_1,
U is k_1 x n, in the paper's notation, with the error bounded by Delta_r for a
target rank r < k_1.  The problem statement of Section 1 asks for L of m x k
and U of k x n.  To return rank-k factors from an oversampled sketch Y
(m x l, l > k) without wasting the oversampling, k columns of Y are chosen
first and steps 3-7 run on them.  The columns are chosen by column pivoting
(Businger & Golub 1965; Golub & Van Loan, Matrix Computations, Alg. 5.4.1):
at step j the column whose component orthogonal to the columns already
chosen is largest is taken.  Here that greedy rule is written on the Gram
matrix G = Y^T Y as pivoted Cholesky, which makes the same choices in exact
arithmetic:

    d_i = G[i, i];  for j = 0 .. k-1:
        p = the remaining column with the largest d (ties: smallest current
            position; position j and p are exchanged, LAPACK-style);
        r_jj = sqrt(d_p);
        r_ji = (G[p, i] - sum_{t<j} r_tp r_ti) / r_jj  for every remaining i;
        d_i -= r_ji^2.

r_jj is the norm of column p's part orthogonal to the earlier choices (the
|R_jj| of a column-pivoted QR).  A step whose largest d is <= 0 (the
remaining columns already lie in the span of the chosen ones) still takes
its candidate by the same rule, sets r_jj = 0 and is counted, as a zero
pivot.
"""
from __future__ import annotations

import numpy as np


def pivoted_cholesky_order(Y: np.ndarray, k: int):
    """First k columns of Y in column-pivoting order.

    Returns (sel, rdiag, zero_steps, min_gap): sel[j] is the column of Y
    chosen at step j, rdiag[j] = r_jj, zero_steps the number of steps with
    no positive candidate, min_gap the smallest top-two relative gap of the
    candidates' d over the steps (for screening inputs)."""
    Y = np.asarray(Y, dtype=np.float64)
    l = Y.shape[1]
    if not 1 <= k <= l:
        raise ValueError("need 1 <= k <= l")
    G = Y.T @ Y
    order = np.arange(l)
    d = np.diag(G).copy()
    R = np.zeros((k, l))
    rdiag = np.zeros(k)
    zero_steps, min_gap = 0, np.inf
    for j in range(k):
        cand = d[order[j:]]
        off = int(np.argmax(cand))
        top = cand[off]
        if cand.shape[0] > 1 and top > 0:
            rest = np.delete(cand, off)
            min_gap = min(min_gap, (top - rest.max()) / top)
        p = j + off
        order[j], order[p] = order[p], order[j]
        piv = order[j]
        rest_cols = order[j + 1:]
        if top <= 0:
            zero_steps += 1
            continue                              # r_jj = 0, row j of R stays 0
        rjj = np.sqrt(top)
        rdiag[j] = rjj
        R[j, piv] = rjj
        R[j, rest_cols] = (G[piv, rest_cols] - R[:j, piv] @ R[:j, rest_cols]) / rjj
        d[rest_cols] -= R[j, rest_cols] ** 2
    return order[:k].copy(), rdiag, zero_steps, min_gap
