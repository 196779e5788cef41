"""Algorithm 1 (Section 3) end to end: with the exact least-squares product
(k2 = 0), or with the second projection Omega_2 of steps 4-5 (k2 > 0).

Outputs follow the problem statement of Section 1 and the output line of
Algorithm 1: permutations P (rows) and Q (columns), L (m x l, unit lower
trapezoidal) and U (l x n, upper trapezoidal) with P A Q ~ L U.

Permutations are index vectors: (PA)[i, :] = A[perm_r[i], :] and
(AQ)[:, j] = A[:, perm_c[j]].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import rng, lu, lstsq, colsel
from . import sketch as sk


@dataclass
class Params:
    k: int
    l: int
    s: int
    seed: int
    transform: str = "fourier"   # or "hadamard": the FJL's T (see sketch.py)
    k2: int = 0                  # rows of Omega_2 (0: exact least-squares product)
    l2: int = 0                  # SEM width of Omega_2 (a power of two, k2 <= l2)
    truncate: bool = False       # rank-k output: k columns of Y by column pivoting (colsel.py)


@dataclass
class Result:
    L: np.ndarray
    U: np.ndarray
    perm_r: np.ndarray
    perm_c: np.ndarray
    ipiv_r: np.ndarray
    ipiv_c: np.ndarray
    Y: np.ndarray
    Ly: np.ndarray
    Uy: np.ndarray
    B: np.ndarray
    Lt: np.ndarray
    zero_pivots_y: int = 0
    zero_pivots_b: int = 0
    min_gap_y: float = np.inf
    min_gap_b: float = np.inf
    ysel: np.ndarray = None      # truncated form: the columns of Y kept, in pivot order
    min_gap_sel: float = np.inf
    extra: dict = field(default_factory=dict)


def check_params(m: int, n: int, p: Params):
    """Validity of one projection: 1 <= k <= l <= min(m, n), l <= s, s = 2^b."""
    if m < 1 or n < 1:
        raise ValueError("empty matrix")
    if not (1 <= p.k <= p.l <= min(m, n)):
        raise ValueError("need 1 <= k <= l <= min(m, n)")
    if p.s < 2 or p.s & (p.s - 1) or p.s > 65536:
        raise ValueError("s must be a power of two in [2, 65536]")
    if p.l > p.s:
        raise ValueError("need l <= s")
    if p.k2 or p.l2:
        # Algorithm 1's input line orders k_1 < l_1 < k_2 < l_2; only what the
        # least-squares step needs (Omega_2 L_y of full column rank possible)
        # and a power-of-two transform are required here.
        if not (p.l <= p.k2 <= p.l2):
            raise ValueError("need l <= k2 <= l2")
        if p.l2 < 2 or p.l2 & (p.l2 - 1) or p.l2 > 65536:
            raise ValueError("l2 must be a power of two in [2, 65536]")


def sketch_params(n: int, p: Params):
    h, sgn = rng.sem_hash(p.seed, n, p.s)
    d = rng.srft_signs(p.seed, p.s)
    sel = rng.srft_select(p.seed, p.s, p.l)
    return h, sgn, d, sel


def omega2_params(m: int, p: Params):
    """Random parameters of Omega_2 (Algorithm 1 step 4), streams 4-6."""
    h2, sgn2 = rng.sem_hash(p.seed, m, p.l2, stream=rng.STREAM_SEM2)
    d2 = rng.srft_signs(p.seed, p.l2, stream=rng.STREAM_SIGNS2)
    sel2 = rng.srft_select(p.seed, p.l2, p.k2, stream=rng.STREAM_SELECT2)
    return h2, sgn2, d2, sel2


def sketch_y(A, p: Params, csr=None):
    """Algorithm 1 steps 1-2: Y = A Omega_1^T."""
    if csr is not None:
        row_ptr, col, val, m, n = csr
        check_params(m, n, p)
        h, sgn, d, sel = sketch_params(n, p)
        return sk.sketch_csr(row_ptr, col, val, m, n, h, sgn, d, sel, p.s, p.transform)
    A = np.asarray(A, dtype=np.float64)
    check_params(*A.shape, p)
    h, sgn, d, sel = sketch_params(A.shape[1], p)
    return sk.sketch_dense(A, h, sgn, d, sel, p.s, p.transform)


def rlu(A, p: Params, csr=None) -> Result:
    """Algorithm 1 with B = L_y^+ P A exactly (Corollary 3.2's product) when
    p.k2 == 0, else with B = (Omega_2 L_y)^+ Omega_2 P A (steps 4-5).

    With ``p.truncate`` the factors have rank k (the problem statement of
    Section 1: L m x k, U k x n): k columns of the sketch Y, chosen by column
    pivoting (``colsel``), take Y's place from step 3 on.

    ``A`` is a dense array, or None with ``csr = (row_ptr, col, val, m, n)``.
    """
    if csr is not None:
        row_ptr, col, val, m, n = csr
        Aop = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col),
                             np.asarray(row_ptr)), shape=(m, n))
    else:
        Aop = np.asarray(A, dtype=np.float64)
    Y = sketch_y(Aop if csr is None else None, p, csr=csr)          # steps 1-2
    ysel, gsel, Yk = None, np.inf, Y
    if p.truncate:                                                # rank-k output
        ysel, _, _, gsel = colsel.pivoted_cholesky_order(Y, p.k)
        Yk = Y[:, ysel]
    Ly, Uy, perm_r, ipiv_r, zy, gy = lu.gepp(Yk)                  # step 3
    extra = {}
    if p.k2:                                                      # steps 4-5 (sketched)
        h2, sgn2, d2, sel2 = omega2_params(Aop.shape[0], p)
        B, M, Z = lstsq.sketched_lstsq_product(Ly, Aop[perm_r], h2, sgn2, d2, sel2, p.l2, p.transform)
        extra = {"M": M, "Z": Z}
    else:
        Lhat = lstsq.unpermute_rows(Ly, perm_r)
        B = lstsq.lstsq_product(Lhat, Aop)                        # steps 5-6 (exact)
    Lt, U, perm_c, ipiv_c, zb, gb = lu.colpiv_lu(B)               # step 6
    L = Ly @ Lt                                                   # step 7
    return Result(L=L, U=U, perm_r=perm_r, perm_c=perm_c, ipiv_r=ipiv_r,
                  ipiv_c=ipiv_c, Y=Y, Ly=Ly, Uy=Uy, B=B, Lt=Lt,
                  zero_pivots_y=zy, zero_pivots_b=zb, min_gap_y=gy, min_gap_b=gb, ysel=ysel,
                  min_gap_sel=gsel, extra=extra)


def residual_fro(A, L, U, perm_r, perm_c) -> float:
    """||L U - P A Q||_F for dense A."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(L @ U - A[np.ix_(perm_r, perm_c)]))


def tail_norm(A, k: int) -> float:
    """Delta_k(A) = sqrt(sum_{i > k} sigma_i^2) (Section 1), by full SVD."""
    sv = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(np.sqrt(np.sum(sv[k:] ** 2)))
