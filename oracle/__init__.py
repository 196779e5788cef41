"""Plain FP64 CPU oracle of the sparse-projection randomized LU.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s CPU-baseline leg may import this package.  The GPU library
never calls into it, and it shares no code with the GPU path: the two
implement the same published definitions independently.

It follows Algorithm 1 (Section 3) of Aizenbud, Shabat & Averbuch,
"Randomized LU decomposition using sparse projections", with the exact
least-squares product of Corollary 3.2 by default, or the paper's second
projection Omega_2 (steps 4-5) when asked for:

1. parameters of the SEM (Section 2.2) and of the SRFT (Section 2.1) from a
   seed, by a counter-based generator (``rng``);
2. Y0 = A S^T, the sparse embedding (``sketch.sem_apply``);
3. Y  = Y0 diag(d) T R, the FFT transform with sub-sampling
   (``sketch.fjl_apply``);
4. P Y = L_y U_y, LU with partial (row) pivoting (``lu.gepp``);
5. B  = L_y^+ P A via Householder QR (``lstsq.lstsq_product``), or
   B = (Omega_2 L_y)^+ Omega_2 P A (``lstsq.sketched_lstsq_product``);
6. B Q = L~ U, LU with column pivoting (``lu.colpiv_lu``);
7. L  = L_y L~ (``rlu.rlu``);

and, for factors of rank k below the sketch's width, the column selection
of Y by column pivoting (``colsel``) ahead of step 4.

Every function cites the passage it follows.  Pins: ``tests/test_oracle_*``.
"""
from . import rng, sketch, lu, lstsq, colsel, rlu  # noqa: F401
