// C ABI of the library: contexts, argument validation, workspace planning
// and the stage sequence of Algorithm 1 (see include/rlu.h).
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

static thread_local std::string g_last_error;

rlu_status fail(rlu_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}
rlu_status hip_fail(hipError_t e, const char *what) {
  (void)hipGetLastError();  // a rejected launch must not surface in the caller's next HIP call
  return fail(RLU_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void sketch_dense_set_attrs();
void sketch_csr_set_attrs();

constexpr int kMaxK2 = 1024;  // rows of Omega_2: the transform kernels' output limit

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
static bool deterministic(const rlu_params *p) { return (p->flags & RLU_FLAG_DETERMINISTIC) != 0; }
static bool truncated(const rlu_params *p) { return (p->flags & RLU_FLAG_TRUNCATE) != 0; }
// rank of the factors: k columns of Y kept with RLU_FLAG_TRUNCATE, else all l
static int factor_rank(const rlu_params *p) { return truncated(p) ? p->k : p->l; }

rlu_status validate_matrix(const rlu_matrix *A) {
  if (!A) return fail(RLU_ERR_INVALID_ARG, "A is NULL");
  if (A->m < 1 || A->n < 1) return fail(RLU_ERR_INVALID_ARG, "m and n must be >= 1 (m=%lld n=%lld)", (long long)A->m, (long long)A->n);
  if (A->m > INT32_MAX || A->n > INT32_MAX) return fail(RLU_ERR_INVALID_ARG, "m and n must fit int32 indices");
  if (!A->values && !(A->layout == RLU_CSR && A->nnz == 0)) return fail(RLU_ERR_INVALID_ARG, "A->values is NULL");
  if (A->layout == RLU_DENSE_ROW_MAJOR) {
    if (A->dtype != RLU_F64 && A->dtype != RLU_F32) return fail(RLU_ERR_INVALID_ARG, "dense dtype must be RLU_F64 or RLU_F32");
    if (A->ld < A->n) return fail(RLU_ERR_INVALID_ARG, "ld (%lld) < n (%lld)", (long long)A->ld, (long long)A->n);
  } else if (A->layout == RLU_CSR) {
    if (A->dtype != RLU_F64) return fail(RLU_ERR_INVALID_ARG, "CSR values must be RLU_F64");
    if (!A->row_ptr) return fail(RLU_ERR_INVALID_ARG, "CSR row_ptr is NULL");
    if (!A->col_idx && A->nnz > 0) return fail(RLU_ERR_INVALID_ARG, "CSR col_idx is NULL");
    if (A->nnz < 0 || A->nnz > INT32_MAX) return fail(RLU_ERR_INVALID_ARG, "CSR nnz out of range");
    if (A->n > ((int64_t)1 << 29)) return fail(RLU_ERR_INVALID_ARG, "CSR n must be at most 2^29");
  } else {
    return fail(RLU_ERR_INVALID_ARG, "unknown layout %d", A->layout);
  }
  return RLU_OK;
}

rlu_status validate_params(const rlu_matrix *A, const rlu_params *p) {
  if (!p) return fail(RLU_ERR_INVALID_ARG, "params is NULL");
  if (p->reserved != 0) return fail(RLU_ERR_INVALID_ARG, "params.reserved must be 0");
  if (p->s < 2 || p->s > kMaxS || !is_pow2(p->s)) return fail(RLU_ERR_INVALID_ARG, "s (%d) must be a power of two in [2, %d]", p->s, kMaxS);
  if (p->l < 1 || p->l > p->s) return fail(RLU_ERR_INVALID_ARG, "need 1 <= l <= s (l=%d s=%d)", p->l, p->s);
  if (p->k < 1 || p->k > p->l) return fail(RLU_ERR_INVALID_ARG, "need 1 <= k <= l (k=%d l=%d)", p->k, p->l);
  if (A) {
    if (p->l > A->m || p->l > A->n) return fail(RLU_ERR_INVALID_ARG, "need l <= min(m, n) (l=%d m=%lld n=%lld)", p->l, (long long)A->m, (long long)A->n);
    if (A->layout == RLU_CSR && p->precision != RLU_PREC_F64)
      return fail(RLU_ERR_INVALID_ARG, "the reduced-precision forms apply to dense A only");
  }
  if (p->l > kMaxL) return fail(RLU_ERR_INVALID_ARG, "l (%d) exceeds the supported maximum %d", p->l, kMaxL);
  if (p->precision < RLU_PREC_F64 || p->precision > RLU_PREC_BF16_REFINED) return fail(RLU_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  if (p->flags & ~(RLU_FLAG_VALIDATE | RLU_FLAG_TIMING | RLU_FLAG_EXCLUSIVE | RLU_FLAG_TIMING_CONTRACT |
                   RLU_FLAG_HADAMARD | RLU_FLAG_DETERMINISTIC | RLU_FLAG_TRUNCATE)) return fail(RLU_ERR_INVALID_ARG, "unknown flag bits 0x%x", p->flags);
  if (p->k2 != 0 || p->l2 != 0) {  // the second projection of steps 4-5
    if (p->l2 < 2 || p->l2 > kMaxL2 || !is_pow2(p->l2))
      return fail(RLU_ERR_INVALID_ARG, "l2 (%d) must be a power of two in [2, %d]", p->l2, kMaxL2);
    if (p->k2 < p->l || p->k2 > p->l2 || p->k2 > kMaxK2)
      return fail(RLU_ERR_INVALID_ARG, "need l <= k2 <= min(l2, %d) (l=%d k2=%d l2=%d)", kMaxK2, p->l, p->k2, p->l2);
    if (p->precision != RLU_PREC_F64)
      return fail(RLU_ERR_INVALID_ARG, "the second projection is built for RLU_PREC_F64 only");
    if (A && A->m > INT32_MAX) return fail(RLU_ERR_INVALID_ARG, "the second projection needs m < 2^31");
  }
  return RLU_OK;
}

rlu_status validate_factors(const rlu_matrix *A, const rlu_params *p, const rlu_factors *out) {
  if (!out) return fail(RLU_ERR_INVALID_ARG, "factors is NULL");
  if (!out->L || !out->U || !out->perm_r || !out->perm_c) return fail(RLU_ERR_INVALID_ARG, "L, U, perm_r and perm_c are required");
  if (!out->info) return fail(RLU_ERR_INVALID_ARG, "info (device record) is required");
  if (out->ldl < factor_rank(p))
    return fail(RLU_ERR_INVALID_ARG, "ldl (%lld) < the factors' rank (%d)", (long long)out->ldl, factor_rank(p));
  if (out->ysel && !truncated(p)) return fail(RLU_ERR_INVALID_ARG, "ysel is an output of RLU_FLAG_TRUNCATE only");
  if (out->ldu < A->n) return fail(RLU_ERR_INVALID_ARG, "ldu (%lld) < n (%lld)", (long long)out->ldu, (long long)A->n);
  if (out->Y && out->ldy < p->l) return fail(RLU_ERR_INVALID_ARG, "ldy (%lld) < l (%d)", (long long)out->ldy, p->l);
  if ((reinterpret_cast<uintptr_t>(out->info) & 7)) return fail(RLU_ERR_INVALID_ARG, "info must be 8-byte aligned");
  return RLU_OK;
}

// ---------------------------------------------------------------------------
// workspace plan
// ---------------------------------------------------------------------------
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  }
};

// control words: [1] abort flag of the cooperative launches
constexpr int kCtlWords = 64;


static void plan_sketch_part(Carver &cv, FactorPlan &fp, const rlu_matrix *A, const rlu_params *p) {
  const int64_t n = A->n;
  const int l = p->l, s = p->s;
  fp.ctl = cv.take(kCtlWords * 4);
  fp.code = cv.take((size_t)n * 4);
  fp.sel = cv.take((size_t)l * 4);
  fp.twf = cv.take((size_t)std::max(1, s / 2) * 16);
  fp.twp = cv.take((size_t)std::max(1, s / 2) * 16);
  const bool dense = A->layout == RLU_DENSE_ROW_MAJOR, wide = s > kLdsMaxS;
  // bucket-ordered tables of the deterministic dense sketch (the explicit
  // projection of wide s sums in a fixed order already)
  fp.ordt = cv.take(deterministic(p) && dense && !wide ? ordered_tables_bytes(n, s) : 0);
  // wide s: the cos table in global memory, and the explicit n x l projection
  fp.ctabg = cv.take(wide && !(p->flags & RLU_FLAG_HADAMARD) ? (size_t)s * 8 : 0);
  fp.omt = cv.take(wide && dense ? (size_t)n * l * 8 : 0);
}

rlu_status plan_factor(const DevCaps &caps, const rlu_matrix *A, const rlu_params *p, FactorPlan *fp) {
  std::string why;
  fp->m = A->m;
  fp->n = A->n;
  fp->ls = p->l;
  fp->l = factor_rank(p);  // k with RLU_FLAG_TRUNCATE, else l
  fp->s = p->s;
  const int64_t m = A->m, n = A->n;
  const int l = fp->l, ls = fp->ls;
  if (!plan_gepp(m, l, caps, &fp->py, &why)) return fail(RLU_ERR_INVALID_ARG, "row-pivoted LU: %s", why.c_str());
  if (!plan_gepp(n, l, caps, &fp->pb, &why)) return fail(RLU_ERR_INVALID_ARG, "column-pivoted LU: %s", why.c_str());
  fp->k2 = p->k2;
  fp->l2 = p->l2;
  const bool second = p->k2 > 0;
  const int64_t kc = second ? p->k2 : m;  // depth of the contraction and of the Gram matrix
  fp->splits_w = choose_splits(n, l, kc, caps.num_cu);
  fp->splits_g = choose_splits(l, l, kc, caps.num_cu);
  fp->splits_i = choose_splits(l, l, l, caps.num_cu);
  fp->splits_b = choose_splits(n, l, l, caps.num_cu);
  Carver cv;
  plan_sketch_part(cv, *fp, A, p);
  fp->sketch_total = cv.off;
  fp->Y = cv.take((size_t)m * ls * 8);
  const bool trunc = truncated(p);
  fp->splits_y = trunc ? choose_splits(ls, ls, m, caps.num_cu) : 1;
  fp->Gy = cv.take(trunc ? (size_t)ls * ls * 8 : 0);
  fp->parts_y = cv.take(trunc ? gemm_f64_splitk_scratch(ls, ls, fp->splits_y) : 0);
  fp->Rsel = cv.take(trunc ? (size_t)ls * l * 8 : 0);
  fp->ysel = cv.take(trunc ? (size_t)l * 4 : 0);
  fp->Yk = cv.take(trunc ? (size_t)m * l * 8 : 0);
  fp->slots = cv.take(std::max(gepp_workspace_bytes(m, l, fp->py), gepp_workspace_bytes(n, l, fp->pb)));
  fp->Lhat = cv.take((size_t)m * l * 8);
  fp->Uy = cv.take((size_t)l * l * 8);
  fp->Wt = cv.take((size_t)n * l * 8);
  // parts: the contraction's partials, later B^T's; parts_g: the Gram
  // matrix's (it runs beside the contraction), later G^{-1}'s
  fp->parts = cv.take(gemm_f64_splitk_scratch(n, l, std::max(fp->splits_w, fp->splits_b)));
  fp->parts_g = cv.take(gemm_f64_splitk_scratch(l, l, std::max(fp->splits_g, fp->splits_i)));
  fp->Gm = cv.take((size_t)l * l * 8);
  fp->Linv = cv.take((size_t)l * l * 8);
  fp->Dinv = cv.take(chol_scratch_bytes(l));
  fp->Ginv = cv.take((size_t)l * l * 8);
  fp->Bt = cv.take((size_t)n * l * 8);
  fp->Lph = cv.take((size_t)n * l * 8);
  fp->Up = cv.take((size_t)l * l * 8);
  fp->Lt = cv.take((size_t)l * l * 8);
  fp->gaps = cv.take((size_t)2 * l * 8);
  fp->csc = cv.take(A->layout == RLU_CSR ? csc_scratch_bytes(n, A->nnz, m, l) : 0);
  fp->pp = PrecPlan{};
  if (A->layout == RLU_DENSE_ROW_MAJOR && p->precision != RLU_PREC_F64 &&
      !plan_precision(m, n, l, p->precision, caps.num_cu, &fp->pp))
    return fail(RLU_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  fp->prec = cv.take(fp->pp.total);
  const size_t k2 = second ? (size_t)p->k2 : 0, l2 = second ? (size_t)p->l2 : 0;
  fp->o2start = cv.take(second ? (l2 + 1) * 4 : 0);
  fp->o2list = cv.take(second ? (size_t)m * 4 : 0);
  fp->o2code = cv.take(l2 * 4);
  fp->o2sel = cv.take(k2 * 4);
  fp->o2twf = cv.take(second ? std::max<size_t>(1, l2 / 2) * 16 : 0);
  fp->o2twp = cv.take(second ? std::max<size_t>(1, l2 / 2) * 16 : 0);
  fp->o2rowcode = cv.take(second && A->layout == RLU_CSR ? (size_t)m * 4 : 0);
  fp->Z0T = cv.take(A->layout == RLU_CSR ? 0 : (size_t)n * l2 * 8);
  fp->ZT = cv.take((size_t)n * k2 * 8);
  fp->Zs = cv.take(k2 * (size_t)n * 8);
  fp->M0T = cv.take((size_t)l * l2 * 8);
  fp->MT = cv.take((size_t)l * k2 * 8);
  fp->Ms = cv.take(k2 * l * 8);
  fp->total = cv.off;
  return RLU_OK;
}

template <typename T>
static T *at(void *ws, size_t off) { return reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + off); }

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------
static rlu_status run_params(const FactorPlan &fp, const rlu_params *p, void *ws, hipStream_t st) {
  launch_sem_codes(fp.n, p->s, p->seed, at<uint32_t>(ws, fp.code), nullptr, nullptr, st);
  launch_srft_params(p->s, p->l, p->seed, nullptr, at<int32_t>(ws, fp.sel), at<double2>(ws, fp.twf),
                     at<double2>(ws, fp.twp), st);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RLU_OK : hip_fail(e, "parameter kernels");
}

// Omega_2's parameters (step 4): bucket lists, codes, selection, twiddles.
// They depend on nothing but the seed and the shape.
static rlu_status run_params2(const FactorPlan &fp, const rlu_params *p, void *ws, hipStream_t st) {
  hipError_t e = launch_omega2_lists(fp.m, fp.l2, p->seed, at<int32_t>(ws, fp.o2start), at<uint32_t>(ws, fp.o2list),
                                     at<uint32_t>(ws, fp.o2code), deterministic(p), st);
  if (e != hipSuccess) return hip_fail(e, "second projection lists");
  launch_srft_params(fp.l2, fp.k2, p->seed, nullptr, at<int32_t>(ws, fp.o2sel), at<double2>(ws, fp.o2twf),
                     at<double2>(ws, fp.o2twp), st, true);
  e = hipGetLastError();
  return e == hipSuccess ? RLU_OK : hip_fail(e, "second projection parameters");
}


static rlu_status run_sketch(const DevCaps &caps, const FactorPlan &fp, const rlu_matrix *A,
                             const rlu_params *p, double *Y, int64_t ldy, void *ws, rlu_info *info,
                             hipStream_t st) {
  hipError_t e;
  const bool hadamard = (p->flags & RLU_FLAG_HADAMARD) != 0;
  const bool wide = p->s > kLdsMaxS;
  double *gctab = nullptr;
  if (wide && !hadamard) {
    gctab = at<double>(ws, fp.ctabg);
    if ((e = launch_cos_table(p->s, at<double2>(ws, fp.twp), gctab, st)) != hipSuccess) return hip_fail(e, "cos table");
  }
  if (A->layout == RLU_DENSE_ROW_MAJOR && wide) {
    // the row's s buckets do not fit in LDS: Y = A Omega^T with Omega^T explicit
    double *OmT = at<double>(ws, fp.omt);
    e = launch_explicit_projection(A->n, p->s, p->l, at<uint32_t>(ws, fp.code), at<int32_t>(ws, fp.sel), gctab,
                                   hadamard, OmT, st);
    if (e != hipSuccess) return hip_fail(e, "explicit projection");
    GemmArgs g{};
    g.M = A->m; g.N = p->l; g.K = A->n;
    g.A = A->values; g.lda = A->ld; g.a_dtype = A->dtype; g.trans_a = false;
    g.B = OmT; g.ldb = p->l;
    g.C = Y; g.ldc = ldy; g.alpha = 1.0; g.beta = 0.0;
    e = gemm_f64(g, st);
  } else if (A->layout == RLU_DENSE_ROW_MAJOR && deterministic(p)) {
    e = launch_sketch_ordered(A->m, A->n, A->values, A->dtype, A->ld, p->s, p->l, at<uint32_t>(ws, fp.code),
                              at<int32_t>(ws, fp.sel), at<double2>(ws, fp.twf), at<double2>(ws, fp.twp),
                              at<void>(ws, fp.ordt), Y, ldy, caps.num_cu, (p->flags & RLU_FLAG_HADAMARD) != 0,
                              st);
  } else if (A->layout == RLU_DENSE_ROW_MAJOR) {
    e = launch_sketch_dense(A->m, A->n, A->values, A->dtype, A->ld, p->s, p->l, at<uint32_t>(ws, fp.code),
                            at<int32_t>(ws, fp.sel), at<double2>(ws, fp.twf), at<double2>(ws, fp.twp),
                            Y, ldy, at<uint32_t>(ws, fp.ctl) + 3, caps.num_cu, (p->flags & RLU_FLAG_HADAMARD) != 0, st);
  } else {
    if (info) {
      e = launch_csr_check(A, (p->flags & RLU_FLAG_VALIDATE) != 0, info, st);
      if (e != hipSuccess) return hip_fail(e, "CSR check");
    }
    e = launch_sketch_csr(A->m, A->n, A->row_ptr, A->col_idx, (const double *)A->values, A->nnz, p->s, p->l,
                          at<uint32_t>(ws, fp.code), at<int32_t>(ws, fp.sel), at<double2>(ws, fp.twp),
                          gctab, Y, ldy, info ? &info->bad_index : at<int32_t>(ws, fp.ctl) + 2,
                          caps.num_cu, hadamard, st);
  }
  return e == hipSuccess ? RLU_OK : hip_fail(e, "sketch kernel");
}

// Omega_2 X for X with m rows (ncols columns), Algorithm 1 steps 4-5:
// (S_2 P X)^T into Z0T, the transform down its columns as the row sketch of
// Z0T (identity SEM, d_2 in the codes) into ZT, then Zs = Omega_2 P X
// (k2 x ncols, ld ncols).
static rlu_status omega2_apply(const DevCaps &caps, const FactorPlan &fp, const void *X, int dtype, int64_t ldx,
                               int64_t ncols, const int32_t *perm, double *Z0T, double *ZT, double *Zs,
                               uint32_t *row_counter, bool hadamard, bool ordered, void *ws, hipStream_t st) {
  hipError_t e = launch_omega2_gather(ncols, X, dtype, ldx, perm, at<int32_t>(ws, fp.o2start),
                                      at<uint32_t>(ws, fp.o2list), fp.l2, Z0T, fp.l2, ordered, st);
  if (e != hipSuccess) return hip_fail(e, "second projection: sparse embedding");
  e = launch_sketch_dense(ncols, fp.l2, Z0T, RLU_F64, fp.l2, fp.l2, fp.k2, at<uint32_t>(ws, fp.o2code),
                          at<int32_t>(ws, fp.o2sel), at<double2>(ws, fp.o2twf), at<double2>(ws, fp.o2twp), ZT, fp.k2,
                          row_counter, caps.num_cu, hadamard, st);
  if (e != hipSuccess) return hip_fail(e, "second projection: transform");
  if ((e = launch_transpose(ncols, fp.k2, ZT, fp.k2, Zs, ncols, st)) != hipSuccess)
    return hip_fail(e, "second projection: transpose");
  return RLU_OK;
}

// Start / end events of the recorded stages of one timed call (no-ops when
// timing is off): every stage, or the contraction only.
struct StageMarks {
  std::array<hipEvent_t, 2 * RLU_NUM_STAGES> ev{};
  uint32_t mask = 0;  // bit i: stage i recorded
  void begin(int i, hipStream_t s) {
    if (mask >> i & 1) hipEventRecord(ev[2 * i], s);
  }
  void end(int i, hipStream_t s) {
    if (mask >> i & 1) hipEventRecord(ev[2 * i + 1], s);
  }
};

static rlu_status begin_timing(rlu_ctx_impl &cx, StageMarks &sm, uint32_t mask) {
  StageTimer &t = cx.timer;
  while (t.pool.size() < t.used + 2 * RLU_NUM_STAGES) {
    // timing only (read after the caller synchronises): no system-scope
    // fence, i.e. no cache write-back and invalidation at each stage boundary
    hipEvent_t e;
    hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (err != hipSuccess) return hip_fail(err, "hipEventCreateWithFlags");
    t.pool.push_back(e);
  }
  for (int i = 0; i < 2 * RLU_NUM_STAGES; ++i) sm.ev[i] = t.pool[t.used + i];
  t.used += 2 * RLU_NUM_STAGES;
  t.calls.push_back({sm.ev, mask});
  sm.mask = mask;
  return RLU_OK;
}

// The auxiliary stream paired with `st` (created on first use).
static rlu_status aux_for(rlu_ctx_impl &cx, hipStream_t st, AuxStream *out) {
  std::lock_guard<std::mutex> g(cx.aux_mu);
  for (const AuxStream &a : cx.aux)
    if (a.main == st) {
      *out = a;
      return RLU_OK;
    }
  AuxStream a;
  a.main = st;
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&a.aux, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "auxiliary stream");
  if ((e = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&a.join, hipEventDisableTiming)) != hipSuccess) {
    if (a.fork) hipEventDestroy(a.fork);
    hipStreamDestroy(a.aux);
    return hip_fail(e, "auxiliary events");
  }
  cx.aux.push_back(a);
  *out = a;
  return RLU_OK;
}

void destroy_aux_streams(rlu_ctx_impl &cx) {
  std::lock_guard<std::mutex> g(cx.aux_mu);
  for (AuxStream &a : cx.aux) {
    hipStreamSynchronize(a.aux);
    hipEventDestroy(a.fork);
    hipEventDestroy(a.join);
    hipStreamDestroy(a.aux);
  }
  cx.aux.clear();
}

rlu_status factor_enqueue(rlu_ctx_impl &cx, const rlu_matrix *A, const rlu_params *p,
                          const rlu_factors *out, void *ws, const FactorPlan &fp, hipStream_t st,
                          const ExecEnv *env) {
  const DevCaps &caps = env ? env->caps : cx.caps;
  const int64_t m = A->m, n = A->n;
  const int l = fp.l;  // rank of the factors (k with RLU_FLAG_TRUNCATE); the sketch has fp.ls columns
  hipError_t e;
  StageMarks sm;
  if (p->flags & (RLU_FLAG_TIMING | RLU_FLAG_TIMING_CONTRACT)) {
    const uint32_t mask = (p->flags & RLU_FLAG_TIMING) ? (1u << RLU_NUM_STAGES) - 1 : 1u << RLU_STAGE_CONTRACT;
    rlu_status ts = begin_timing(cx, sm, mask);
    if (ts != RLU_OK) return ts;
  }
  AuxStream ax;
  rlu_status rs = RLU_OK;
  if (env) ax = env->ax;
  else if ((rs = aux_for(cx, st, &ax)) != RLU_OK) return rs;
  sm.begin(RLU_STAGE_PARAMS, st);
  rlu_info *info = out->info;
  uint32_t *ctl = at<uint32_t>(ws, fp.ctl);
  int32_t *abort_flag = reinterpret_cast<int32_t *>(ctl + 1);

  if ((e = launch_fill_u32(ctl, 0u, kCtlWords, st)) != hipSuccess) return hip_fail(e, "fill");
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(info), 0u, sizeof(rlu_info) / 4, st)) != hipSuccess)
    return hip_fail(e, "fill");
  if ((rs = run_params(fp, p, ws, st)) != RLU_OK) return rs;
  const bool second = fp.k2 > 0;
  sm.end(RLU_STAGE_PARAMS, st);

  double *Y = out->Y ? out->Y : at<double>(ws, fp.Y);
  int64_t ldy = out->Y ? out->ldy : fp.ls;
  sm.begin(RLU_STAGE_SKETCH, st);
  if ((rs = run_sketch(caps, fp, A, p, Y, ldy, ws, info, st)) != RLU_OK) return rs;
  if (truncated(p)) {
    // rank-k factors: k columns of Y by column pivoting (the first k pivots of
    // Y's column-pivoted QR, as pivoted Cholesky of Y^T Y); steps 3-6 then run
    // on those columns
    double *Gy = at<double>(ws, fp.Gy);
    GemmArgs g{};
    g.M = fp.ls; g.N = fp.ls; g.K = m;
    g.A = Y; g.lda = ldy; g.a_dtype = RLU_F64; g.trans_a = true;
    g.B = Y; g.ldb = ldy;
    g.C = Gy; g.ldc = fp.ls; g.alpha = 1.0; g.beta = 0.0;
    if ((e = gemm_f64_splitk(g, fp.splits_y, at<double>(ws, fp.parts_y), st)) != hipSuccess)
      return hip_fail(e, "Gram matrix of Y");
    int32_t *ysel = out->ysel ? out->ysel : at<int32_t>(ws, fp.ysel);
    if ((e = launch_colsel(fp.ls, l, Gy, at<double>(ws, fp.Rsel), ysel, info, st)) != hipSuccess)
      return hip_fail(e, "column selection");
    double *Yk = at<double>(ws, fp.Yk);
    if ((e = launch_gather_cols(m, l, Y, ldy, ysel, Yk, st)) != hipSuccess) return hip_fail(e, "column gather");
    Y = Yk;
    ldy = l;
  }
  sm.end(RLU_STAGE_SKETCH, st);
  if (second) {  // Omega_2's parameters on the auxiliary stream, beside step 3 (whose
                 // panels leave most CUs idle); the streaming sketch would share its CUs
    if ((e = hipEventRecord(ax.fork, st)) != hipSuccess || (e = hipStreamWaitEvent(ax.aux, ax.fork, 0)) != hipSuccess)
      return hip_fail(e, "fork");
    if ((rs = run_params2(fp, p, ws, ax.aux)) != RLU_OK) return rs;
    if ((e = hipEventRecord(ax.join, ax.aux)) != hipSuccess) return hip_fail(e, "join");
  }

  // Step 3: P Y = L_y U_y (rows of L_y kept in A's order: Lhat = P^T L_y)
  double *Lhat = at<double>(ws, fp.Lhat);
  double *Uy = out->Uy ? out->Uy : at<double>(ws, fp.Uy);
  sm.begin(RLU_STAGE_LU_Y, st);
  const bool exclusive = (p->flags & RLU_FLAG_EXCLUSIVE) != 0 || (env && env->exclusive);
  // Y is not read again: when it is the library's scratch (no Y output, or
  // the gathered columns of the rank-k form), the LU's updates run in it
  const bool y_scratch = out->Y == nullptr || truncated(p);
  e = launch_gepp(m, l, Y, ldy, Lhat, Uy, out->perm_r, out->ipiv_r, at<void>(ws, fp.slots), abort_flag, info,
                  0, fp.py, exclusive, y_scratch, st);
  if (e != hipSuccess) return hip_fail(e, "row-pivoted LU launch");
  sm.end(RLU_STAGE_LU_Y, st);

  // Step 4: G = Lhat^T Lhat, its inverse Cholesky factor and G^{-1}, and the
  // contraction W^T = A^T Lhat (n x l).  When the contraction is long enough
  // to run in several rounds of blocks, the G chain runs on the auxiliary
  // stream beside it; a one-round contraction holds every CU and would only
  // delay the chain (and one of its own blocks), so then the chain runs first.
  //
  // With the second projection (steps 4-5), M = Omega_2 L_y and G = M^T M
  // come first, on the caller's stream: Z's pass over A holds every CU, and
  // M's short launches queued beside it would wait for them.  The Cholesky
  // chain after G is latency-bound and runs on the auxiliary stream beside
  // Z's pass and W^T = Z^T M; B^T = W^T G^{-1} then ends both forms alike.
  const bool hadamard = (p->flags & RLU_FLAG_HADAMARD) != 0;
  const bool det = deterministic(p);
  const bool overlap = (!env || env->overlap) &&
                       (second || A->layout == RLU_CSR || (double)m * (double)n * (double)l >= 1e11);
  hipStream_t gs = overlap ? ax.aux : st;
  // The Gram matrix first, on the caller's stream, with the second projection
  // (see above) and with the BF16 form, whose contraction is short enough that
  // a Gram product starved beside it would put the Cholesky chain on the
  // critical path; otherwise it runs beside the contraction as well.
  const bool gram_first = second || (overlap && p->precision == RLU_PREC_BF16_REFINED);
  hipStream_t gram_st = gram_first ? st : gs;  // stream of the Gram stage
  double *Ms = at<double>(ws, fp.Ms);
  if (second && (e = hipStreamWaitEvent(st, ax.join, 0)) != hipSuccess) return hip_fail(e, "join");  // parameters
  if (overlap && !gram_first) {
    if ((e = hipEventRecord(ax.fork, st)) != hipSuccess || (e = hipStreamWaitEvent(ax.aux, ax.fork, 0)) != hipSuccess)
      return hip_fail(e, "fork");
  }
  sm.begin(RLU_STAGE_GRAM, gram_st);
  if (second) {  // M = Omega_2 L_y = Omega_2 P Lhat
    rs = omega2_apply(caps, fp, Lhat, RLU_F64, l, l, out->perm_r, at<double>(ws, fp.M0T), at<double>(ws, fp.MT), Ms,
                      ctl + 4, hadamard, det, ws, gram_st);
    if (rs != RLU_OK) return rs;
  }
  {
    GemmArgs g{};
    g.M = l; g.N = l; g.K = second ? fp.k2 : m;
    g.A = second ? Ms : Lhat; g.lda = l; g.a_dtype = RLU_F64; g.trans_a = true;
    g.B = second ? Ms : Lhat; g.ldb = l;
    g.C = at<double>(ws, fp.Gm); g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    e = gemm_f64_splitk(g, fp.splits_g, at<double>(ws, fp.parts_g), gram_st);
    if (e != hipSuccess) return hip_fail(e, "Gram matrix");
  }
  sm.end(RLU_STAGE_GRAM, gram_st);
  if (overlap && gram_first) {
    if ((e = hipEventRecord(ax.fork, st)) != hipSuccess || (e = hipStreamWaitEvent(ax.aux, ax.fork, 0)) != hipSuccess)
      return hip_fail(e, "fork");
  }
  sm.begin(RLU_STAGE_CHOL, gs);
  if ((e = launch_chol_inv(l, at<double>(ws, fp.Gm), at<double>(ws, fp.Linv), at<double>(ws, fp.Dinv), info, gs)) != hipSuccess)
    return hip_fail(e, "Cholesky");
  {  // G^{-1} = Linv^T Linv
    GemmArgs g{};
    g.M = l; g.N = l; g.K = l;
    g.A = at<double>(ws, fp.Linv); g.lda = l; g.a_dtype = RLU_F64; g.trans_a = true;
    g.B = at<double>(ws, fp.Linv); g.ldb = l; g.b_lower = true;  // Linv is lower triangular
    g.C = at<double>(ws, fp.Ginv); g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    if ((e = gemm_f64_splitk(g, fp.splits_i, at<double>(ws, fp.parts_g), gs)) != hipSuccess)
      return hip_fail(e, "inverse Gram");
  }
  sm.end(RLU_STAGE_CHOL, gs);
  if (overlap && (e = hipEventRecord(ax.join, ax.aux)) != hipSuccess) return hip_fail(e, "join");

  double *Wt = at<double>(ws, fp.Wt);
  sm.begin(RLU_STAGE_CONTRACT, st);
  if (second && A->layout == RLU_CSR) {
    // Z^T = (Omega_2 P A)^T = A^T (Omega_2 P)^T: the CSR sketch of A^T, held
    // as a CSC copy of A, with Omega_2's codes by row of A
    CscView cs;
    if ((e = build_csc(m, n, A->row_ptr, A->col_idx, (const double *)A->values, A->nnz, at<void>(ws, fp.csc),
                       caps.num_cu, det, st, &cs)) != hipSuccess)
      return hip_fail(e, "CSC copy");
    uint32_t *rowcode = at<uint32_t>(ws, fp.o2rowcode);
    if ((e = launch_omega2_rowcodes(m, fp.l2, p->seed, out->perm_r, rowcode, st)) != hipSuccess)
      return hip_fail(e, "second projection codes");
    e = launch_sketch_csr(n, m, cs.colptr, cs.crow, cs.cval, A->nnz, fp.l2, fp.k2, rowcode, at<int32_t>(ws, fp.o2sel),
                          at<double2>(ws, fp.o2twp), nullptr, at<double>(ws, fp.ZT), fp.k2,
                          reinterpret_cast<int32_t *>(ctl + 6), caps.num_cu, hadamard, st);
    if (e != hipSuccess) return hip_fail(e, "second projection: sparse sketch");
    if ((e = launch_transpose(n, fp.k2, at<double>(ws, fp.ZT), fp.k2, at<double>(ws, fp.Zs), n, st)) != hipSuccess)
      return hip_fail(e, "second projection: transpose");
  } else if (second) {  // Z = Omega_2 P A
    rs = omega2_apply(caps, fp, A->values, A->dtype, A->ld, n, out->perm_r, at<double>(ws, fp.Z0T),
                      at<double>(ws, fp.ZT), at<double>(ws, fp.Zs), ctl + 5, hadamard, det, ws, st);
    if (rs != RLU_OK) return rs;
  } else if (A->layout == RLU_CSR) {
    e = contraction_csr(m, n, l, A->row_ptr, A->col_idx, (const double *)A->values, A->nnz, Lhat, Wt,
                        at<void>(ws, fp.csc), caps.num_cu, det, st);
    if (e != hipSuccess) return hip_fail(e, "sparse contraction");
  } else if (p->precision == RLU_PREC_F64) {
    GemmArgs g{};
    g.M = n; g.N = l; g.K = m;
    g.A = A->values; g.lda = A->ld; g.a_dtype = A->dtype; g.trans_a = true;
    g.B = Lhat; g.ldb = l;
    g.C = Wt; g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    e = gemm_f64_splitk(g, fp.splits_w, at<double>(ws, fp.parts), st);
    if (e != hipSuccess) return hip_fail(e, "contraction");
  } else {
    e = precision_contract(fp.pp, A, Lhat, l, Wt, at<double>(ws, fp.parts), fp.splits_w, at<void>(ws, fp.prec), st);
    if (e != hipSuccess) return hip_fail(e, "reduced-precision contraction");
  }
  if (second) {  // W^T = Z^T M (n x l): the normal equations' right-hand side
    GemmArgs g{};
    g.M = n; g.N = l; g.K = fp.k2;
    g.A = at<double>(ws, fp.Zs); g.lda = n; g.a_dtype = RLU_F64; g.trans_a = true;
    g.B = Ms; g.ldb = l;
    g.C = Wt; g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    if ((e = gemm_f64_splitk(g, fp.splits_w, at<double>(ws, fp.parts), st)) != hipSuccess)
      return hip_fail(e, "Z^T M");
  }
  sm.end(RLU_STAGE_CONTRACT, st);
  if (overlap && (e = hipStreamWaitEvent(st, ax.join, 0)) != hipSuccess) return hip_fail(e, "join");
  sm.begin(RLU_STAGE_SOLVE, st);
  if (A->layout == RLU_DENSE_ROW_MAJOR && p->precision == RLU_PREC_BF16_REFINED) {
    // one refinement step of the BF16 contraction; writes Bt
    e = precision_refine(fp.pp, A, l, Wt, at<double>(ws, fp.Ginv), at<double>(ws, fp.Bt), at<void>(ws, fp.prec), st);
    if (e != hipSuccess) return hip_fail(e, "refinement");
  } else {  // B^T = W^T G^{-1}; with k2 > 0, ((Omega_2 L_y)^+ Omega_2 P A)^T
    GemmArgs g{};
    g.M = n; g.N = l; g.K = l;
    g.A = Wt; g.lda = l; g.a_dtype = RLU_F64; g.trans_a = false;
    g.B = at<double>(ws, fp.Ginv); g.ldb = l;
    g.C = at<double>(ws, fp.Bt); g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    if ((e = gemm_f64_splitk(g, fp.splits_b, at<double>(ws, fp.parts), st)) != hipSuccess)
      return hip_fail(e, "least-squares product");
  }
  sm.end(RLU_STAGE_SOLVE, st);
  double *Bt = at<double>(ws, fp.Bt);
  if (out->B) {
    if ((e = launch_transpose(n, l, Bt, l, out->B, n, st)) != hipSuccess) return hip_fail(e, "transpose");
  }

  // Step 5: B Q = L~ U through the row-pivoted LU of B^T
  double *Lph = at<double>(ws, fp.Lph), *Up = at<double>(ws, fp.Up), *Lt = at<double>(ws, fp.Lt);
  sm.begin(RLU_STAGE_LU_B, st);
  e = launch_gepp(n, l, Bt, l, Lph, Up, out->perm_c, out->ipiv_c, at<void>(ws, fp.slots), abort_flag, info, 1,
                  fp.pb, exclusive, true, st);
  if (e != hipSuccess) return hip_fail(e, "column-pivoted LU launch");
  sm.end(RLU_STAGE_LU_B, st);
  sm.begin(RLU_STAGE_ASSEMBLE, st);
  if ((e = launch_ltilde(l, Up, Lt, st)) != hipSuccess) return hip_fail(e, "L~");
  if ((e = launch_assemble_u(l, n, Up, Lph, out->perm_c, out->U, out->ldu, st)) != hipSuccess)
    return hip_fail(e, "U");

  // Step 6: L = L_y L~ = (P Lhat) L~
  {
    GemmArgs g{};
    g.M = m; g.N = l; g.K = l;
    g.A = Lhat; g.lda = l; g.a_dtype = RLU_F64; g.trans_a = false; g.gather = out->perm_r;
    g.B = Lt; g.ldb = l; g.b_lower = true;  // L~ is unit lower triangular
    g.C = out->L; g.ldc = out->ldl; g.alpha = 1.0; g.beta = 0.0;
    if ((e = gemm_f64(g, st)) != hipSuccess) return hip_fail(e, "L = L_y L~");
  }
  // pivot screening of both LUs (rlu_info.min_gap_y / min_gap_b)
  unsigned long long *gaps = at<unsigned long long>(ws, fp.gaps);
  if ((e = launch_pivot_gap(m, l, Lhat, out->perm_r, Uy, gaps, &info->min_gap_y, st)) != hipSuccess ||
      (e = launch_pivot_gap(n, l, Lph, out->perm_c, Up, gaps + l, &info->min_gap_b, st)) != hipSuccess)
    return hip_fail(e, "pivot gaps");
  if ((e = launch_finalize(info, abort_flag, st)) != hipSuccess) return hip_fail(e, "finalize");
  sm.end(RLU_STAGE_ASSEMBLE, st);
  return RLU_OK;
}

// ---------------------------------------------------------------------------
// rlu_sketch and its no-allocation form
// ---------------------------------------------------------------------------
// Scratch of rlu_sketch_noalloc: a file-scope device array, one copy per
// device, alive until the process ends.  Host code never passes its name to a
// kernel (on the host that name is a stand-in, not a device address): the
// address comes from hipGetSymbolAddress, taken once per device with that
// device current (rlu_create), and is kept in every context of the device.
constexpr size_t kScratchBytes = RLU_SKETCH_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;  // by device

static rlu_status scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return RLU_OK;
}

// Validation, the workspace check and the launches of Algorithm 1 steps 1-2.
// Everything the kernels need beyond A and Y lives in ws (control words, the
// column codes, the selection and the twiddles), cleared or rewritten by the
// call itself, so a workspace may be reused by calls that do not overlap.
static rlu_status sketch_call(rlu_ctx_impl &cx, const rlu_matrix *A, const rlu_params *p, double *Y, int64_t ldy,
                              void *ws, size_t ws_bytes, bool noalloc, void *stream) {
  rlu_status st = validate_matrix(A);
  if (st != RLU_OK) return st;
  if ((st = validate_params(A, p)) != RLU_OK) return st;
  if (!Y) return fail(RLU_ERR_INVALID_ARG, "Y is NULL");
  if (ldy < p->l) return fail(RLU_ERR_INVALID_ARG, "ldy (%lld) < l (%d)", (long long)ldy, p->l);
  FactorPlan fp;
  Carver cv;
  plan_sketch_part(cv, fp, A, p);
  fp.n = A->n;
  fp.m = A->m;
  if (noalloc && cv.off > ws_bytes)
    return fail(RLU_ERR_NO_MEMORY,
                "rlu_sketch_noalloc: this problem needs %zu bytes of scratch, above the fixed %zu (use rlu_sketch "
                "with a workspace)", cv.off, ws_bytes);
  if (!ws || ws_bytes < cv.off || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(RLU_ERR_NO_MEMORY, "workspace must be 256-byte aligned and hold %zu bytes", cv.off);
  hipError_t e = hipSetDevice(cx.caps.device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((e = launch_fill_u32(at<uint32_t>(ws, fp.ctl), 0u, kCtlWords, s)) != hipSuccess) return hip_fail(e, "fill");
  if ((st = run_params(fp, p, ws, s)) != RLU_OK) return st;
  return run_sketch(cx.caps, fp, A, p, Y, ldy, ws, nullptr, s);
}

}  // namespace rlu

using namespace rlu;

// ---------------------------------------------------------------------------
// exported C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *rlu_last_error(void) { return g_last_error.c_str(); }

rlu_status rlu_create(int device, rlu_ctx **ctx) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx out-pointer is NULL");
  *ctx = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count) return fail(RLU_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, count);
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(RLU_ERR_DEVICE, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
  int coop = 0;
  hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device);
  if (!coop) return fail(RLU_ERR_DEVICE, "device %d does not support cooperative launches", device);
  rlu_ctx_impl *c = new (std::nothrow) rlu_ctx_impl();
  if (!c) return fail(RLU_ERR_NO_MEMORY, "host allocation failed");
  c->caps.device = device;
  c->caps.num_cu = prop.multiProcessorCount;
  c->caps.max_lds = prop.sharedMemPerBlockOptin ? prop.sharedMemPerBlockOptin : prop.sharedMemPerBlock;
  rlu_status sst = scratch_address(device, &c->scratch);  // with `device` current
  if (sst != RLU_OK) {
    delete c;
    return sst;
  }
  sketch_dense_set_attrs();
  sketch_csr_set_attrs();
  *ctx = reinterpret_cast<rlu_ctx *>(c);
  return RLU_OK;
}

rlu_status rlu_destroy(rlu_ctx *ctx) {
  if (!ctx) return RLU_OK;
  rlu_ctx_impl *c = reinterpret_cast<rlu_ctx_impl *>(ctx);
  serve_shutdown(*c);
  destroy_aux_streams(*c);
  for (hipEvent_t e : c->timer.pool) hipEventDestroy(e);
  delete c;
  return RLU_OK;
}

rlu_status rlu_workspace_size(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, size_t *bytes) {
  if (!ctx || !bytes) return fail(RLU_ERR_INVALID_ARG, "NULL argument");
  rlu_status st = validate_matrix(A);
  if (st != RLU_OK) return st;
  if ((st = validate_params(A, p)) != RLU_OK) return st;
  FactorPlan fp;
  if ((st = plan_factor(reinterpret_cast<rlu_ctx_impl *>(ctx)->caps, A, p, &fp)) != RLU_OK) return st;
  *bytes = fp.total;
  return RLU_OK;
}

rlu_status rlu_sketch_params(const rlu_params *p, int64_t n, int32_t *h, int8_t *sgn, int8_t *d,
                             int32_t *sel, void *stream) {
  rlu_status st = validate_params(nullptr, p);
  if (st != RLU_OK) return st;
  if (n < 1) return fail(RLU_ERR_INVALID_ARG, "n must be >= 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (h || sgn) launch_sem_codes(n, p->s, p->seed, nullptr, h, sgn, s);
  if (d || sel) launch_srft_params(p->s, p->l, p->seed, d, sel, nullptr, nullptr, s);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RLU_OK : hip_fail(e, "parameter kernels");
}

rlu_status rlu_sketch(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, double *Y, int64_t ldy,
                      void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  return sketch_call(*reinterpret_cast<rlu_ctx_impl *>(ctx), A, p, Y, ldy, ws, ws_bytes, false, stream);
}

rlu_status rlu_sketch_noalloc(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, double *Y, int64_t ldy,
                              void *stream) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  if (!cx.scratch) return fail(RLU_ERR_DEVICE, "the context has no scratch address");
  return sketch_call(cx, A, p, Y, ldy, cx.scratch, kScratchBytes, true, stream);
}

rlu_status rlu_factor(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, const rlu_factors *out,
                      void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  rlu_status st = validate_matrix(A);
  if (st != RLU_OK) return st;
  if ((st = validate_params(A, p)) != RLU_OK) return st;
  if ((st = validate_factors(A, p, out)) != RLU_OK) return st;
  FactorPlan fp;
  if ((st = plan_factor(cx.caps, A, p, &fp)) != RLU_OK) return st;
  if (!ws || ws_bytes < fp.total || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(RLU_ERR_NO_MEMORY, "workspace must be 256-byte aligned and hold %zu bytes", fp.total);
  hipError_t e = hipSetDevice(cx.caps.device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return factor_enqueue(cx, A, p, out, ws, fp, reinterpret_cast<hipStream_t>(stream), nullptr);
}

rlu_status rlu_stage_times(rlu_ctx *ctx, float *ms, int *calls) {
  if (!ctx || !ms) return fail(RLU_ERR_INVALID_ARG, "NULL argument");
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  for (int i = 0; i < RLU_NUM_STAGES; ++i) ms[i] = 0.f;
  StageTimer &t = cx.timer;
  for (auto &call : t.calls) {
    const auto &ev = call.ev;
    for (int i = 0; i < RLU_NUM_STAGES; ++i) {
      if (!(call.mask >> i & 1)) continue;
      hipError_t e = hipEventSynchronize(ev[2 * i + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
      float v = 0.f;
      if ((e = hipEventElapsedTime(&v, ev[2 * i], ev[2 * i + 1])) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      ms[i] += v;
    }
  }
  if (calls) *calls = (int)t.calls.size();
  t.calls.clear();
  t.used = 0;
  return RLU_OK;
}

rlu_status rlu_tall_lu_workspace_size(rlu_ctx *ctx, int64_t rows, int64_t cols, size_t *bytes) {
  if (!ctx || !bytes) return fail(RLU_ERR_INVALID_ARG, "NULL argument");
  if (cols < 1 || rows < cols || cols > kMaxL || rows > INT32_MAX)
    return fail(RLU_ERR_INVALID_ARG, "need 1 <= cols <= rows, cols <= %d", kMaxL);
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  GeppPlan gp;
  std::string why;
  if (!plan_gepp(rows, (int)cols, cx.caps, &gp, &why)) return fail(RLU_ERR_INVALID_ARG, "%s", why.c_str());
  Carver cv;
  cv.take(kCtlWords * 4);
  cv.take(gepp_workspace_bytes(rows, (int)cols, gp));
  cv.take((size_t)cols * 8);
  *bytes = cv.off;
  return RLU_OK;
}

rlu_status rlu_tall_lu(rlu_ctx *ctx, const double *X, int64_t rows, int64_t cols, int64_t ldx, double *Lhat,
                       double *U, int32_t *perm, int32_t *ipiv, rlu_info *info, void *ws, size_t ws_bytes,
                       void *stream) {
  size_t need = 0;
  rlu_status st = rlu_tall_lu_workspace_size(ctx, rows, cols, &need);
  if (st != RLU_OK) return st;
  if (!X || !Lhat || !U || !perm || !info) return fail(RLU_ERR_INVALID_ARG, "NULL matrix argument");
  if (reinterpret_cast<uintptr_t>(info) & 7) return fail(RLU_ERR_INVALID_ARG, "info must be 8-byte aligned");
  if (ldx < cols) return fail(RLU_ERR_INVALID_ARG, "ldx < cols");
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(RLU_ERR_NO_MEMORY, "workspace must be 256-byte aligned and hold %zu bytes", need);
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  GeppPlan gp;
  std::string why;
  plan_gepp(rows, (int)cols, cx.caps, &gp, &why);
  Carver cv;
  const size_t o_ctl = cv.take(kCtlWords * 4);
  const size_t o_slots = cv.take(gepp_workspace_bytes(rows, (int)cols, gp));
  const size_t o_gaps = cv.take((size_t)cols * 8);
  hipError_t e = hipSetDevice(cx.caps.device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint32_t *ctl = at<uint32_t>(ws, o_ctl);
  if ((e = launch_fill_u32(ctl, 0u, kCtlWords, s)) != hipSuccess) return hip_fail(e, "fill");
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(info), 0u, sizeof(rlu_info) / 4, s)) != hipSuccess)
    return hip_fail(e, "fill");
  e = launch_gepp(rows, (int)cols, X, ldx, Lhat, U, perm, ipiv, at<void>(ws, o_slots),
                  reinterpret_cast<int32_t *>(ctl + 1), info, 0, gp, false, false, s);
  if (e != hipSuccess) return hip_fail(e, "tall LU launch");
  if ((e = launch_pivot_gap(rows, (int)cols, Lhat, perm, U, at<unsigned long long>(ws, o_gaps), &info->min_gap_y,
                            s)) != hipSuccess ||
      (e = launch_store_f64(&info->min_gap_b, __builtin_inf(), s)) != hipSuccess)
    return hip_fail(e, "pivot gaps");
  if ((e = launch_finalize(info, reinterpret_cast<int32_t *>(ctl + 1), s)) != hipSuccess) return hip_fail(e, "finalize");
  return RLU_OK;
}

}  // extern "C"
