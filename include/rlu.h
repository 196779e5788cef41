/*
 * rlu.h -- C ABI of the MI355X (gfx950) sparse-projection randomized LU.
 *
 * Method: Aizenbud, Shabat & Averbuch, "Randomized LU decomposition using
 * sparse projections" (arXiv 1601.04280).  Given A (m x n), the library
 * returns permutations P, Q, a unit lower trapezoidal L (m x l) and an upper
 * trapezoidal U (l x n) with P A Q ~ L U (problem statement, Section 1;
 * output line of Algorithm 1).  The steps (Algorithm 1, Section 3):
 *
 *   1. draw a sparse embedding S (SEM, Section 2.2: bucket h(j) in [0, s)
 *      and sign sgn(j) per column j) and an SRFT (Section 2.1: +-1 diagonal
 *      d, length-s Fourier transform on an orthonormal real basis, l
 *      selected coordinates sel);
 *   2. Y = A S^T diag(d) T R  (m x l), one streaming pass over A;
 *   3. P Y = L_y U_y, LU with partial (row) pivoting;
 *   4. B = L_y^+ P A, the exact least-squares product bounded by
 *      Corollary 3.2 (by default), or the paper's own steps 4-5 when
 *      rlu_params.k2 > 0: a second projection Omega_2 = Pi_2 S_2 (k2 x m,
 *      built like the first over the m rows of P A, with SEM width l2) and
 *      B = (Omega_2 L_y)^+ Omega_2 P A through the normal equations;
 *   5. B Q = L~ U, LU with column ("right partial") pivoting;
 *   6. L = L_y L~.
 *
 * Conventions (where the paper is silent):
 *   - Pivot ties go to the smallest current position; a pivot exchanges
 *     position j with the pivot's position (LAPACK ipiv semantics).
 *   - A zero pivot (all candidates exactly 0) performs no exchange, sets the
 *     step's multipliers to 0 and the U diagonal entry to 0, and is counted
 *     in rlu_info; it is not an error.
 *   - No truncation: L is m x l and U is l x n; k is the target rank of the
 *     error reference Delta_k and only needs 1 <= k <= l.
 *   - Permutations are index vectors: (PA)[i,:] = A[perm_r[i],:] and
 *     (AQ)[:,j] = A[:,perm_c[j]].
 *   - The random parameters come from a counter-based rule: mix64 is the
 *     SplitMix64 output function (Steele, Lea & Flood 2014), gamma =
 *     0x9E3779B97F4A7C15, stream key K_t = mix64(seed + t*gamma) for t = 1
 *     (SEM), 2 (d), 3 (selection), draw r_t(i) = mix64(K_t + (i+1)*gamma);
 *     Omega_2 uses t = 4, 5, 6 for the same three, with l2 and k2 in place
 *     of s and l and the pivoted row position i in place of the column j;
 *     h(j) = r_1(j) >> (64 - log2 s), sgn(j) = 1 - 2*(r_1(j) & 1),
 *     d_b = 1 - 2*(r_2(b) >> 63), sel by a partial Fisher-Yates shuffle of
 *     [0, s) with j = i + mulhi64(r_3(i), s - i).
 *   - The real transform packs the DFT X of a real row z (kernel
 *     e^{-2 pi i f b / s}) as c_0 = X_0/sqrt(s), c_{s/2} = X_{s/2}/sqrt(s),
 *     c_f = sqrt(2) Re X_f / sqrt(s), c_{s-f} = sqrt(2) Im X_f / sqrt(s)
 *     for 0 < f < s/2; Y[i, q] = c[sel[q]] of row i.
 *
 * Memory and streams.  Every matrix and vector pointer below is a DEVICE
 * pointer on the context's device, except where a comment says "host".  All
 * compute calls are asynchronous and ordered on the given stream (a
 * hipStream_t passed as void*; NULL is the null stream).  The caller owns A,
 * every output and the workspace; the library never frees caller memory and
 * allocates nothing inside rlu_sketch / rlu_factor.  Dense matrices are row
 * major with a leading dimension (elements between consecutive rows).
 *
 * Errors.  Every call returns rlu_status; nothing throws across the ABI and
 * rlu_last_error() describes the last failure of the calling thread.
 * Arguments are validated before anything is enqueued (the library never
 * clamps).  Conditions found on the device (a non-finite value reaching a
 * pivot search, a device-wide barrier that timed out) are written to the
 * rlu_info record and are visible once the stream has been synchronised.
 */
#ifndef RLU_H_
#define RLU_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RLU_OK = 0,
  RLU_ERR_INVALID_ARG = 1,   /* bad shape, parameter or pointer               */
  RLU_ERR_NO_MEMORY = 2,     /* workspace too small / request over budget     */
  RLU_ERR_DEVICE = 3,        /* HIP runtime error or device-side time-out     */
  RLU_ERR_NUMERIC = 4,       /* non-finite value reached a pivot search       */
  RLU_ERR_AGAIN = 5,         /* serving: request still in flight              */
  RLU_ERR_UNKNOWN_TICKET = 6 /* serving: no such ticket                       */
} rlu_status;

typedef enum { RLU_DENSE_ROW_MAJOR = 0, RLU_CSR = 1 } rlu_layout;
typedef enum { RLU_F64 = 0, RLU_F32 = 1 } rlu_dtype; /* storage type of A's values */

/* Arithmetic of the least-squares contraction W = L^T A (step 4 above).
 * Pivot searches, the Gram matrix, its Cholesky factor and the l x l solves
 * are FP64 in every form.  The reduced forms apply to dense A only.
 * BF16_REFINED: W0 = bf16(L)^T bf16(A), X0 = G^-1 W0, R = A - L X0 (L X0 from
 * hi/lo BF16 splits, good to ~2^-16), B = X0 + G^-1 bf16(L)^T bf16(R). */
typedef enum {
  RLU_PREC_F64 = 0,          /* FP64 MFMA                                           */
  RLU_PREC_F32 = 1,          /* FP32 operands and accumulation, single pass         */
  RLU_PREC_BF16_REFINED = 2  /* BF16 operands, FP32 accumulation, one refinement    */
} rlu_precision;

typedef struct {
  int64_t m, n;             /* rows, columns (>= 1); at most 524288 each for
                             * rlu_factor: each LU holds its rows in registers
                             * (256 blocks x 256 threads x 8 rows)              */
  int32_t layout;           /* rlu_layout                                          */
  int32_t dtype;            /* rlu_dtype (CSR: RLU_F64 only)                       */
  const void *values;       /* dense: m x n row major; CSR: nnz values             */
  int64_t ld;               /* dense: leading dimension >= n                       */
  const int32_t *row_ptr;   /* CSR: m + 1 offsets, row_ptr[0] = 0, row_ptr[m] = nnz */
  const int32_t *col_idx;   /* CSR: nnz column indices in [0, n); CSR n <= 2^29    */
  int64_t nnz;              /* CSR: number of stored entries                       */
} rlu_matrix;

typedef struct {
  int32_t k;                /* target rank of the error reference, 1 <= k <= l      */
  int32_t l;                /* sketch columns = rank of the factors,
                             * l <= min(m, n, 1024)                                 */
  int32_t s;                /* SEM width: a power of two in [2, 65536], s >= l.
                             * Up to 8192 the transform runs on each row's s
                             * buckets in LDS; above, the projection is formed
                             * explicitly (n x l FP64 in the workspace) and
                             * Y = A Omega^T runs on the FP64 GEMM (dense A), or
                             * the cos table is read from global memory (CSR A) */
  int32_t precision;        /* rlu_precision                                        */
  uint64_t seed;            /* seed of the random parameters                        */
  uint32_t flags;           /* RLU_FLAG_* bits                                      */
  int32_t k2;               /* rows of the second projection Omega_2 of Algorithm 1
                             * steps 4-5; 0 (with l2 = 0): B is the exact product
                             * L_y^+ P A of Corollary 3.2.  Else l <= k2 <= l2,
                             * k2 <= 1024, RLU_PREC_F64 only                      */
  int32_t l2;               /* SEM width of Omega_2: a power of two in [2, 8192]   */
  uint32_t reserved;        /* must be 0                                            */
} rlu_params;

/* flags */
#define RLU_FLAG_VALIDATE 1u  /* CSR: also check on the device (async) that row_ptr never
                                 * decreases; counted in info.bad_index.  Column indices and
                                 * row_ptr[0] = 0, row_ptr[m] = nnz are always checked. */
#define RLU_FLAG_TIMING 2u    /* record HIP events around each stage (rlu_stage_times) */
#define RLU_FLAG_EXCLUSIVE 4u /* the caller guarantees that no other work runs on the device
                               * while this call's kernels run.  The LU panel kernels, whose
                               * blocks wait for each other, are then ordinary launches (on an
                               * otherwise idle device every block is resident at once) rather
                               * than cooperative launches, which guarantee co-residency under
                               * any load but leave the device idle for about 11 us on each
                               * side of every panel (8 panels at l = 210).  If other work does
                               * keep some blocks from starting, the exchange gives up after
                               * 2 s and the call reports RLU_ERR_DEVICE with info.timeouts > 0;
                               * it does not hang.  Not accepted for served requests: the
                               * serving loop launches their panels this way by itself, under
                               * its admission rule (rlu_serve_start). */
#define RLU_FLAG_HADAMARD 16u  /* the sketch's transform T is the Walsh-Hadamard matrix
                                * H_s / sqrt(s) in Sylvester order, H[b][c] = (-1)^popcount(b & c)
                                * (the subsampled randomized Hadamard transform of Section 4),
                                * instead of the orthonormal real Fourier transform; the
                                * signs, the selection and the sparse embedding are the same */
#define RLU_FLAG_DETERMINISTIC 32u /* bitwise-reproducible results: every sum the call forms is
                                    * taken in an order fixed by the inputs alone, so two calls
                                    * with the same A and parameters give identical bits (on the
                                    * same device and library build).  The dense sketch adds each
                                    * bucket's columns in ascending column order (the order of the
                                    * SEM's definition, Section 2.2) from bucket-sorted tables built
                                    * per call (workspace grows by about 4 n + 4 (s + 1) n / C bytes,
                                    * C = min(s, 8192)); the sparse contraction sorts each column's
                                    * entries of its CSC copy by row; the second projection sums
                                    * each bucket's rows in position order.  Slower than the default
                                    * atomic accumulation, whose results agree with these to
                                    * rounding; the pivots are the same on screened inputs. */
#define RLU_FLAG_TRUNCATE 64u /* factors of rank k instead of l (the problem statement of
                              * Section 1: L m x k, U k x n).  The sketch Y keeps its l
                              * columns; k of them are chosen by column pivoting (the first
                              * k pivots of Y's column-pivoted QR, Businger & Golub 1965,
                              * taken as pivoted Cholesky of Y^T Y), and steps 3-6 run on
                              * those k columns, so every output sized by l above (L, U,
                              * U_y, B, ipiv_r, ipiv_c) is sized by k instead; Y stays
                              * m x l.  Keeps the oversampling: the k columns are the ones
                              * that best span Y's range greedily, where truncating L_y to
                              * its first k columns would equal a k-column sketch. */
#define RLU_FLAG_TIMING_CONTRACT 8u /* events around the contraction stage only (one stage
                                     * boundary instead of nine; rlu_stage_times reports the
                                     * other stages as 0 for such calls) */

/* Stages reported by rlu_stage_times, in order. */
enum {
  RLU_STAGE_PARAMS = 0,      /* random parameters (step 1)                        */
  RLU_STAGE_SKETCH = 1,      /* Y = A Omega^T (step 2)                            */
  RLU_STAGE_LU_Y = 2,        /* row-pivoted LU of Y (step 3)                      */
  RLU_STAGE_CONTRACT = 3,    /* W = Lhat^T A (step 4, the dominant product); with
                              * k2 > 0, Z = Omega_2 P A and W = M^T Z instead     */
  RLU_STAGE_GRAM = 4,        /* G = Lhat^T Lhat; with k2 > 0, M = Omega_2 L_y and
                              * G = M^T M                                         */
  RLU_STAGE_CHOL = 5,        /* inverse Cholesky factor of G and G^{-1}            */
  RLU_STAGE_SOLVE = 6,       /* B^T = W^T G^{-1} (or the refined reduced form)     */
  RLU_STAGE_LU_B = 7,        /* column-pivoted LU of B (step 5)                   */
  RLU_STAGE_ASSEMBLE = 8,    /* L~, U and L = L_y L~ (step 6)                     */
  RLU_NUM_STAGES = 9
};

/* Device-side record of one factorization (8-byte aligned); the call that
 * fills it clears it first, on its stream. */
typedef struct {
  int32_t status;           /* rlu_status of the device work (RLU_OK when fine)     */
  int32_t zero_pivots_y;    /* zero pivots in the row-pivoted LU of Y               */
  int32_t zero_pivots_b;    /* zero pivots in the column-pivoted LU of B            */
  int32_t nonfinite;        /* non-finite values seen by a pivot search             */
  int32_t timeouts;         /* device-wide barriers that gave up (then status != 0) */
  int32_t bad_index;        /* CSR: entries with a column index out of range, plus
                               row_ptr violations (then status = INVALID_ARG)       */
  int32_t zero_pivots_sel;  /* RLU_FLAG_TRUNCATE: column-selection steps whose
                               remaining columns had no positive norm left          */
  int32_t reserved;
  /* Pivot screening.  At step j of a pivoted LU the candidates are the
   * entries of the current column (step 3) or row (step 5); the step's
   * relative gap is (|c_1| - |c_2|) / |c_1| for its two largest candidate
   * magnitudes, i.e. 1 - max |multiplier| over the candidates that lost.
   * min_gap_y / min_gap_b are the smallest gap over the steps of the two LUs
   * (steps with a single candidate or a zero pivot are skipped; +inf when no
   * step counts).  A small gap means that rounding could change the pivot. */
  double min_gap_y;
  double min_gap_b;         /* +inf from rlu_tall_lu (no column-pivoted LU)       */
} rlu_info;

typedef struct {
  double *L;  int64_t ldl;  /* m x l, unit lower trapezoidal (row order of PA)      */
  double *U;  int64_t ldu;  /* l x n, upper trapezoidal (column order of AQ)        */
  int32_t *perm_r;          /* m entries                                            */
  int32_t *perm_c;          /* n entries                                            */
  int32_t *ipiv_r;          /* optional (NULL): l row exchanges of step 3           */
  int32_t *ipiv_c;          /* optional (NULL): l column exchanges of step 5        */
  double *Y;  int64_t ldy;  /* optional (NULL): the sketch Y, m x l                 */
  double *Uy;               /* optional (NULL): U_y, l x l, leading dimension l     */
  double *B;                /* optional (NULL): B = L_y^+ P A (k2 > 0: the sketched
                             * product of steps 4-5), l x n, ld n                  */
  int32_t *ysel;            /* optional (NULL), RLU_FLAG_TRUNCATE only: the k columns
                             * of Y kept, in the order chosen                       */
  rlu_info *info;           /* required: device record, see rlu_info                */
} rlu_factors;

typedef struct rlu_ctx rlu_ctx;

/* Context on HIP device `device` (made current by every call that uses it).
 * Owns no large buffers.  One context may be used from one thread at a time. */
rlu_status rlu_create(int device, rlu_ctx **ctx);
rlu_status rlu_destroy(rlu_ctx *ctx);

/* Bytes of workspace rlu_sketch / rlu_factor need for this problem (host
 * out-parameter).  The workspace must be 256-byte aligned device memory. */
rlu_status rlu_workspace_size(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p,
                              size_t *bytes);

/* The random parameters of Algorithm 1 step 1 exactly as the compute calls
 * draw them: h[n] (int32 buckets), sgn[n] (int8 +-1), d[s] (int8 +-1),
 * sel[l] (int32).  Any output may be NULL.  For bit-exact checks. */
rlu_status rlu_sketch_params(const rlu_params *p, int64_t n, int32_t *h, int8_t *sgn,
                             int8_t *d, int32_t *sel, void *stream);

/* Algorithm 1 steps 1-2: Y = A Omega_1^T (m x l, row major, ldy >= l). */
rlu_status rlu_sketch(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, double *Y,
                      int64_t ldy, void *ws, size_t ws_bytes, void *stream);

/* rlu_sketch without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same validation, kernels and result as rlu_sketch;
 * the scratch (control words, column codes, selection, twiddles) lives in a
 * fixed device array of RLU_SKETCH_NOALLOC_MAX_BYTES per device, held from
 * the first rlu_create on that device until the process ends.  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * RLU_ERR_NO_MEMORY when the problem needs more scratch than that (the codes
 * take 4 n bytes, the twiddles 16 s: n up to about two million columns).
 * Every call on a device shares its array and rewrites what it uses, so
 * calls that overlap on one device (different streams, threads or contexts)
 * race; serialise them. */
#define RLU_SKETCH_NOALLOC_MAX_BYTES ((size_t)8 << 20)
rlu_status rlu_sketch_noalloc(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, double *Y,
                              int64_t ldy, void *stream);

/* The whole decomposition (steps 1-6 above); see rlu_factors for outputs. */
rlu_status rlu_factor(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p,
                      const rlu_factors *out, void *ws, size_t ws_bytes, void *stream);

/* Row-pivoted LU of a tall matrix alone (Algorithm 1 step 3): X (rows x cols,
 * row major, ldx >= cols, rows >= cols) is left unchanged; Lhat receives the
 * multipliers in X's own row order (Lhat = P^T L, rows x cols, ld cols), U the
 * cols x cols upper factor, perm[rows] and ipiv[cols] the pivoting.  info
 * counts zero pivots in zero_pivots_y. */
rlu_status rlu_tall_lu(rlu_ctx *ctx, const double *X, int64_t rows, int64_t cols, int64_t ldx,
                       double *Lhat, double *U, int32_t *perm, int32_t *ipiv, rlu_info *info,
                       void *ws, size_t ws_bytes, void *stream);
rlu_status rlu_tall_lu_workspace_size(rlu_ctx *ctx, int64_t rows, int64_t cols, size_t *bytes);

/* Per-stage device milliseconds (HIP events at each stage's start and end)
 * summed over every rlu_factor call made with RLU_FLAG_TIMING (all stages) or
 * RLU_FLAG_TIMING_CONTRACT (the contraction only; 0 for its other stages) on
 * this context since the previous rlu_stage_times call (which waits for those
 * events and then clears them).  For a sparse A, or a contraction of at least 1e11
 * multiply-adds (m n l), the Gram and Cholesky stages run on a second stream
 * beside the contraction: their intervals then overlap it, and the stage
 * times add up to more than the call.
 * ms: host array of RLU_NUM_STAGES floats; calls: host out-param, number of
 * timed calls. */
rlu_status rlu_stage_times(rlu_ctx *ctx, float *ms, int *calls);

/* ---- serving: continuous batching of independent decompositions -------- */

/* Start the request loop: at most `max_inflight` requests on the device at
 * once, their workspaces carved from one pool of `hbm_budget_bytes` that the
 * library allocates here (freed by rlu_serve_stop).  Served requests launch
 * their LU panels as ordinary launches, not cooperative ones: a request is
 * admitted only while the panel blocks of all running requests, its own
 * included, number at most one per compute unit, so every waiting block's
 * siblings can be placed.  Other work on the device from outside the loop
 * can still hold compute units; the exchange's bounded wait then ends the
 * request with RLU_ERR_DEVICE (info.timeouts > 0) instead of hanging. */
rlu_status rlu_serve_start(rlu_ctx *ctx, size_t hbm_budget_bytes, int max_inflight);

/* Queue one decomposition; returns at once with a ticket (host out-param).
 * A and every output buffer must stay valid until rlu_poll returns a
 * terminal status for the ticket.  RLU_ERR_NO_MEMORY if the request alone
 * exceeds the pool. */
rlu_status rlu_submit(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p,
                      const rlu_factors *out, uint64_t *ticket);

/* RLU_OK when the ticket's results are complete, RLU_ERR_AGAIN while it is
 * pending, or the ticket's own error.  A terminal status retires the ticket. */
rlu_status rlu_poll(rlu_ctx *ctx, uint64_t ticket);

/* Counters of the serving loop (host out-param, 8 words): [0] 1 when the
 * loop has one slot, whose requests run one at a time (each request's stages
 * as one HIP graph),
 * [1] compute units the requests are planned for, [2] requests launched as
 * graphs, [3] of those, graphs updated in place, [4] graphs instantiated,
 * [5] requests enqueued directly because capture or instantiation failed,
 * [6..7] 0. */
rlu_status rlu_serve_stats(rlu_ctx *ctx, uint64_t *stats);

/* Wait for all admitted requests, then stop and free the pool. */
rlu_status rlu_serve_stop(rlu_ctx *ctx);

/* Message of the calling thread's last failed call ("" if none). */
const char *rlu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RLU_H_ */
