// Host-side internals of the library: launchers and small helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <string>
#include <vector>

#include "rlu.h"

namespace rlu {

inline int ilog2_exact(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int kMaxS = 65536;           // SEM width s: the codes keep 16 bits of bucket
constexpr int kLdsMaxS = 8192;         // LDS-resident transform: 16 s bytes per block; wider
                                       // s takes the explicit-projection route
constexpr int kMaxL2 = 8192;           // SEM width of Omega_2 (its transform is LDS-resident)
constexpr int kMaxL = 1024;            // sketch width l: the Cholesky panel (l x 17 doubles) and the
                                       // triangular inverse's column (l doubles) live in LDS, the CSR
                                       // kernels hold 16 outputs per lane, column selection one
                                       // column per thread
// Column selection of the truncated form: ysel[0..k) from G = Y^T Y (l x l);
// Rt: l x k doubles of scratch
hipError_t launch_colsel(int l, int k, const double *G, double *Rt, int32_t *ysel, rlu_info *info, hipStream_t st);
hipError_t launch_gather_cols(int64_t m, int k, const double *Y, int64_t ldy, const int32_t *ysel, double *Yk,
                              hipStream_t st);
constexpr int kSketchThreads = 256;

// ---- parameters -----------------------------------------------------------
void launch_sem_codes(int64_t n, int s, uint64_t seed, uint32_t *code, int32_t *h, int8_t *sgn,
                      hipStream_t st);
// second: the streams of Omega_2 (else Omega_1)
void launch_srft_params(int s, int l, uint64_t seed, int8_t *d, int32_t *sel, double2 *twf,
                        double2 *twp, hipStream_t st, bool second = false);
// Omega_2 (Algorithm 1 step 4): bucket lists of its SEM over m positions
// (start: l2 + 1 offsets into list; list: position | sign bit 31) and the
// transform step's codes (code2: l2 entries); `ordered`: each list sorted by
// position
hipError_t launch_omega2_lists(int64_t m, int l2, uint64_t seed, int32_t *start, uint32_t *list,
                               uint32_t *code2, bool ordered, hipStream_t st);
// Codes of Omega_2's SEM by row of A: code_row[perm[p]] = h_2(p) with bit 31
// set when sgn_2(p) d_2(h_2(p)) = -1 (p < m, the pivoted position)
hipError_t launch_omega2_rowcodes(int64_t m, int l2, uint64_t seed, const int32_t *perm, uint32_t *code_row,
                                  hipStream_t st);
// Z0T (ncols x l2, ldz) = (S_2 P X)^T for X with m rows (row i of P X is
// row perm[i] of X); dtype RLU_F64 or RLU_F32.  `ordered` (with ordered
// lists): every bucket summed in list order, the same on every run
hipError_t launch_omega2_gather(int64_t ncols, const void *X, int dtype, int64_t ldx, const int32_t *perm,
                                const int32_t *start, const uint32_t *list, int l2, double *Z0T, int64_t ldz,
                                bool ordered, hipStream_t st);

// ---- sketch -----------------------------------------------------------------
struct SketchPlan {
  int grid;  // blocks of the dense sketch
};
// row_counter: one word, zero on entry (rows are handed out through it).
// hadamard: the transform is H_s / sqrt(s) (Sylvester order) instead of the
// orthonormal real Fourier transform
hipError_t launch_sketch_dense(int64_t m, int64_t n, const void *A, int dtype, int64_t lda, int s,
                               int l, const uint32_t *code, const int32_t *sel,
                               const double2 *twf, const double2 *twp, double *Y, int64_t ldy,
                               uint32_t *row_counter, int num_cu, bool hadamard, hipStream_t st);
// gctab: for s > kLdsMaxS, the cos table in global memory (launch_cos_table),
// else nullptr (the kernel builds it in LDS from twp)
hipError_t launch_sketch_csr(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col,
                             const double *val, int64_t nnz, int s, int l, const uint32_t *code,
                             const int32_t *sel, const double2 *twp, const double *gctab, double *Y,
                             int64_t ldy, int32_t *bad_index, int num_cu, bool hadamard, hipStream_t st);
hipError_t launch_csr_check(const rlu_matrix *A, int validate_rows, rlu_info *info, hipStream_t st);
// (with m and l: also room for the contraction's copy of Lhat with rows
// padded to whole 128-byte lines)
size_t csc_scratch_bytes(int64_t n, int64_t nnz, int64_t m = 0, int l = 0);
// CSC copy of CSR A in `scratch` (csc_scratch_bytes): column pointers (n + 1),
// row indices and values; entries of a column in no particular order, or by
// ascending row when `sorted`
struct CscView {
  const int32_t *colptr;
  const int32_t *crow;
  const double *cval;
};
hipError_t build_csc(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                     int64_t nnz, void *scratch, int num_cu, bool sorted, hipStream_t st, CscView *out);
// W^T (n x l) = A^T Lhat for CSR A, through a CSC copy built in `scratch`
hipError_t contraction_csr(int64_t m, int64_t n, int l, const int32_t *row_ptr, const int32_t *col,
                           const double *val, int64_t nnz, const double *Lhat, double *Wt, void *scratch,
                           int num_cu, bool sorted, hipStream_t st);
// Explicit projection for s > kLdsMaxS: OmT (n x l, row major) with
// OmT[j, q] = (folded sign of j) T[h(j), sel[q]], then Y = A OmT on the GEMM.
// ctab: cos(2 pi k / s) for k < s (launch_cos_table), unused by the Hadamard form.
hipError_t launch_cos_table(int s, const double2 *twp, double *ctab, hipStream_t st);
hipError_t launch_explicit_projection(int64_t n, int s, int l, const uint32_t *code, const int32_t *sel,
                                      const double *ctab, bool hadamard, double *OmT, hipStream_t st);
// Bucket-ordered dense sketch (RLU_FLAG_DETERMINISTIC): every bucket sum in
// ascending column order.  `tables`: ordered_tables_bytes(n, s) of workspace.
size_t ordered_tables_bytes(int64_t n, int s);
hipError_t launch_sketch_ordered(int64_t m, int64_t n, const void *A, int dtype, int64_t lda, int s, int l,
                                 const uint32_t *code, const int32_t *sel, const double2 *twf, const double2 *twp,
                                 void *tables, double *Y, int64_t ldy, int num_cu, bool hadamard, hipStream_t st);

// ---- tall pivoted LU (cooperative) ---------------------------------------------
struct GeppPlan {
  int G;         // blocks (co-resident)
  int R;         // rows per block
  int nb;        // panel width
  int slot_stride;
  size_t lds;    // dynamic LDS bytes
  bool multi;    // more than one panel
};
struct DevCaps {
  int device;
  int num_cu;
  size_t max_lds;  // dynamic LDS bytes a block may use
};
bool plan_gepp(int64_t rows, int cols, const DevCaps &caps, GeppPlan *plan, std::string *why);
size_t gepp_workspace_bytes(int64_t rows, int cols, const GeppPlan &plan);
// X: rows x cols (ldx), left unchanged.  The exchange slots, positions and
// (for more than one panel) a working copy of X live in `ws`
// (gepp_workspace_bytes); abort_flag is a zeroed word shared by the launches
// of one call.  exclusive: the panel kernels are ordinary launches (the
// caller guarantees an otherwise idle device), else cooperative ones.
// x_scratch: X is the library's own scratch and may be overwritten (the
// trailing updates then run in place, without the working copy).
hipError_t launch_gepp(int64_t rows, int cols, const double *X, int64_t ldx, double *Lhat, double *U,
                       int32_t *perm, int32_t *ipiv, void *ws, int32_t *abort_flag, rlu_info *info,
                       int which, const GeppPlan &plan, bool exclusive, bool x_scratch, hipStream_t st);

// ---- GEMM on MFMA ----------------------------------------------------------------
// C (M x N, ldc, FP64) = alpha * op(A) * op(B) + beta * C, or split-K partials.
// compute = RLU_F64: FP64 operands and MFMA.  compute = RLU_F32: B is FP32,
// op(A) (transposed only) is rounded to FP32, FP32 MFMA and accumulation.
struct GemmArgs {
  int64_t M, N, K;
  const void *A; int64_t lda; int a_dtype; bool trans_a; const int32_t *gather;
  const void *B; int64_t ldb; bool trans_b;
  double *C; int64_t ldc;
  double alpha, beta;
  int compute;
  // B is lower triangular (B[k][j] = 0 for k < j): a column tile starting
  // at n0 sums from k = n0 only, and the tiles are narrow so that few of
  // their K steps are spent on B's zero part
  bool b_lower;
};
// Plain (no split): writes C directly.
hipError_t gemm_f64(const GemmArgs &g, hipStream_t st);
// Split-K: partials into `parts` (splits x M x N), then reduced into C
// (C = alpha * sum + beta * C).  Returns the scratch bytes needed when
// parts == nullptr (no launch).
size_t gemm_f64_splitk_scratch(int64_t M, int64_t N, int splits);
hipError_t gemm_f64_splitk(const GemmArgs &g, int splits, double *parts, hipStream_t st);
int choose_splits(int64_t M, int64_t N, int64_t K, int num_cu);

// ---- reduced-precision contraction ------------------------------------------------
// Scratch offsets (bytes, relative to the form's scratch base) and shapes.
struct PrecPlan {
  int precision;
  int lp;              // l rounded up to 32: row stride of the BF16 operands
  int64_t mp;          // m rounded up to 64: row stride of Lhat^T and R^T
  int64_t np_rows;     // rows of Lhat^T (l rounded up to 128)
  int wm, wn;          // BF16 GEMM tile (32 wm x 32 wn)
  int splits;          // K splits of that GEMM
  int64_t Kc;          // K extent of one split
  size_t lhi, llo, lht, xhi, xlo, r, parts, lf;
  size_t total;
};
bool plan_precision(int64_t m, int64_t n, int l, int precision, int num_cu, PrecPlan *pp);
// W^T (n x l) = A^T Lhat in the plan's precision (BF16: the first pass W0^T).
// FP32 uses `parts64` (splits_w partials of n x l doubles) when splits_w > 1.
hipError_t precision_contract(const PrecPlan &pp, const rlu_matrix *A, const double *Lhat, int l, double *Wt,
                              double *parts64, int splits_w, void *scratch, hipStream_t st);
// BF16 only: B^T = X0^T + dW^T G^{-1} from W0^T (overwritten) and G^{-1}.
hipError_t precision_refine(const PrecPlan &pp, const rlu_matrix *A, int l, double *Wt, const double *Ginv,
                            double *Bt, void *scratch, hipStream_t st);

// ---- small dense FP64 pieces ---------------------------------------------------------
// In place: G (l x l, ld l, SPD) -> Linv = inverse of the Cholesky factor
// (G = L L^T), written to Linv (l x l, lower, zeros above).
hipError_t launch_chol_inv(int l, double *G, double *Linv, double *dinv_scratch, rlu_info *info,
                           hipStream_t st);
size_t chol_scratch_bytes(int l);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st);
hipError_t launch_ltilde(int l, const double *Up, double *Lt, hipStream_t st);
hipError_t launch_assemble_u(int l, int64_t n, const double *Up, const double *Lphat,
                             const int32_t *perm_c, double *U, int64_t ldu, hipStream_t st);
hipError_t launch_transpose(int64_t rows, int64_t cols, const double *in, int64_t ldin, double *out,
                            int64_t ldout, hipStream_t st);
hipError_t launch_copy_rows(int64_t rows, int64_t cols, const double *in, int64_t ldin,
                            double *out, int64_t ldout, hipStream_t st);
hipError_t launch_finalize(rlu_info *info, const int32_t *abort_flag, hipStream_t st);
// *out = the smallest top-two relative pivot gap of a finished tall LU
// (Lhat rows x l in X's row order, U l x l, perm its row order); maxbits:
// l words of scratch
hipError_t launch_pivot_gap(int64_t rows, int l, const double *Lhat, const int32_t *perm, const double *U,
                            unsigned long long *maxbits, double *out, hipStream_t st);
hipError_t launch_store_f64(double *p, double v, hipStream_t st);

// ---- context, errors, validation ---------------------------------------------------
struct ServeState;
// HIP events (start, end) of every stage for calls made with RLU_FLAG_TIMING.
// Stages on the auxiliary stream overlap the contraction.
struct StageTimer {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Call {
    std::array<hipEvent_t, 2 * RLU_NUM_STAGES> ev;
    uint32_t mask;  // stages recorded
  };
  std::vector<Call> calls;
};
// A second stream per caller stream: the Gram matrix, its Cholesky factor and
// G^{-1} depend only on Lhat and run there while the contraction runs on the
// caller's stream (fork and join through the two events).
struct AuxStream {
  hipStream_t main = nullptr, aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
struct rlu_ctx_impl {
  DevCaps caps{};
  void *scratch = nullptr;  // this device's copy of the no-allocation scratch array
  ServeState *serve = nullptr;
  StageTimer timer;
  std::mutex aux_mu;
  std::vector<AuxStream> aux;
};
rlu_status fail(rlu_status st, const char *fmt, ...);
rlu_status hip_fail(hipError_t e, const char *what);
rlu_status validate_matrix(const rlu_matrix *A);
rlu_status validate_params(const rlu_matrix *A, const rlu_params *p);
rlu_status validate_factors(const rlu_matrix *A, const rlu_params *p, const rlu_factors *out);
void serve_shutdown(rlu_ctx_impl &cx);

// ---- the decomposition's stage sequence ------------------------------------------
struct FactorPlan {
  int64_t m, n;
  int l, s;
  GeppPlan py, pb;
  int splits_w, splits_g;
  int splits_i, splits_b;  // G^{-1} = L^{-T} L^{-1} (in parts_g) and B^T = W^T G^{-1} (in parts)
  PrecPlan pp;
  int k2 = 0, l2 = 0;  // second projection (k2 > 0), else the exact product
  // offsets (bytes) into the workspace
  size_t ctl, code, sel, twf, twp, Y, slots, csc, Lhat, Uy, Wt, parts, parts_g, Gm, Linv, Dinv, Ginv, Bt,
      Lph, Up, Lt, prec, gaps, ordt, ctabg, omt;
  // truncated form: Y^T Y and its split partials, R of the selection, the
  // selection (when the caller passes none) and the k chosen columns of Y
  int ls = 0;        // sketch width (p->l); l above is the factors' rank
  int splits_y = 1;
  size_t Gy, parts_y, Rsel, ysel, Yk;
  // second projection: bucket lists and transform parameters of Omega_2,
  // (S_2 P A)^T, (Omega_2 P A)^T, Z = Omega_2 P A, and the same three for L_y
  size_t o2start, o2list, o2code, o2sel, o2twf, o2twp, Z0T, ZT, Zs, M0T, MT, Ms;
  size_t o2rowcode;  // CSR A: Omega_2's codes by row of A
  size_t total;
  size_t sketch_total;
};
rlu_status plan_factor(const DevCaps &caps, const rlu_matrix *A, const rlu_params *p, FactorPlan *fp);
// Where one decomposition runs when it is not the context's own call: the
// compute units it may use (num_cu of them, planned with these caps), its
// auxiliary stream, whether its LU panels may be ordinary launches (every
// block resident because nothing else runs on those compute units), and
// whether stages may overlap on the auxiliary stream.
struct ExecEnv {
  DevCaps caps;
  AuxStream ax;
  bool exclusive = false;
  bool overlap = true;
};
// Enqueue every stage of one decomposition on `st` (arguments validated);
// env == nullptr: the context's device, caps and per-stream auxiliary stream.
rlu_status factor_enqueue(rlu_ctx_impl &cx, const rlu_matrix *A, const rlu_params *p, const rlu_factors *out,
                          void *ws, const FactorPlan &fp, hipStream_t st, const ExecEnv *env);

}  // namespace rlu
