// C ABI of the DEANN query path: argument validation, workspace layout and
// kernel launches.  No allocation, no stream synchronisation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/deann.h"
#include "common.h"
#include "kernels.h"

using namespace deann;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(DEANN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Per-thread event pairs around the dense tile kernels (measurement only).
constexpr int kTimingSites = 2;   // 0: kde_exact tiles, 1: kde_exact_backward tiles
struct KernelTimer {
  int cap = 0;
  int used[kTimingSites] = {0, 0};
  hipEvent_t* ev[kTimingSites] = {nullptr, nullptr};   // [cap][2] per site
};
thread_local KernelTimer g_timer;

void timer_release() {
  for (int s = 0; s < kTimingSites; ++s) {
    if (g_timer.ev[s])
      for (int i = 0; i < 2 * g_timer.cap; ++i)
        if (g_timer.ev[s][i]) (void)hipEventDestroy(g_timer.ev[s][i]);
    delete[] g_timer.ev[s];
    g_timer.ev[s] = nullptr;
    g_timer.used[s] = 0;
  }
  g_timer.cap = 0;
}

TimingHook timer_hook(int site) {
  TimingHook th;
  if (g_timer.cap > 0 && g_timer.used[site] < g_timer.cap) {
    const int i = g_timer.used[site]++;
    th.start = g_timer.ev[site][2 * i];
    th.stop = g_timer.ev[site][2 * i + 1];
  }
  return th;
}

constexpr int64_t kAlign = 256;
constexpr int64_t kMaxK = 496;             // k limit of the candidate-list kernels (K1 <= 512)
constexpr int64_t kCenterRows = 2048;      // row slices of the column-mean reduction
constexpr int64_t kSortCap = 4096;         // second-pass candidate capacity per query

int64_t elem_bytes(int prec) { return prec == DEANN_FP32 ? 4 : 2; }

int64_t padded_d(int64_t d, int prec) {
  const int64_t per = CHUNK_BYTES / elem_bytes(prec);
  return round_up(d, per);
}

// Bump allocator over the caller's workspace (or a null base for sizing).
struct Carve {
  char* base;
  int64_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(int64_t count) {
    off = round_up(off, kAlign);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * (int64_t)sizeof(T);
    return p;
  }
};

// Prepared operands shared by every tile sweep.
struct Prep {
  float* c;
  double* cpart;
  char* Xs;
  double* xnorm;
  float *xknorm, *xerr;
  char* Ys;
  double* ynorm;
  float *yknorm, *yerr;
  uint32_t* err_max;
  int64_t dp, np, qp;
};

Prep carve_prep(Carve& cv, int64_t n, int64_t q, int64_t d, int prec) {
  Prep p{};
  p.dp = padded_d(d, prec);
  p.np = round_up(n, BN);
  p.qp = round_up(q, BQ);
  const int64_t es = elem_bytes(prec);
  p.c = cv.take<float>(d);
  p.cpart = cv.take<double>(kCenterRows * d);
  p.Xs = cv.take<char>(p.np * p.dp * es);
  p.xnorm = cv.take<double>(p.np);
  p.xknorm = cv.take<float>(p.np);
  p.xerr = cv.take<float>(p.np);
  p.Ys = cv.take<char>(p.qp * p.dp * es);
  p.ynorm = cv.take<double>(p.qp);
  p.yknorm = cv.take<float>(p.qp);
  p.yerr = cv.take<float>(p.qp);
  p.err_max = cv.take<uint32_t>(2);
  return p;
}

// Relative slack of the lower-bound keys: twice the worst-case FP32 dot-product
// error gamma_d plus the roundings of norms and of the key arithmetic.
double key_scale(int64_t dp) {
  const double u = std::ldexp(1.0, -24);
  const double gamma = (double)dp * u / (1.0 - (double)dp * u);
  return 2.0 * gamma + 16.0 * u;
}

int64_t choose_splits(int64_t qtiles, int64_t ntiles, int64_t target) {
  int64_t s = target / (qtiles > 0 ? qtiles : 1);
  if (s < 1) s = 1;
  if (s > ntiles) s = ntiles;
  return s;
}

TileProblem make_problem(const Prep& p, int64_t n, int64_t q, int prec, int64_t splits_target) {
  TileProblem t{};
  t.Ys = p.Ys;
  t.Xs = p.Xs;
  t.ld_bytes = p.dp * elem_bytes(prec);
  t.nchunks = (int)(t.ld_bytes / CHUNK_BYTES);
  t.ynorm = p.ynorm;
  t.xnorm = p.xnorm;
  t.yknorm = p.yknorm;
  t.xknorm = p.xknorm;
  t.n = n;
  t.q = q;
  t.np = p.np;
  t.qp = p.qp;
  t.qtiles = p.qp / BQ;
  t.ntiles = p.np / BN;
  t.splits = choose_splits(t.qtiles, t.ntiles, splits_target);
  // engines that re-read the query tile per data tile group 4 splits per
  // query-tile sweep (L2 reuse of both operands); the 16-bit engines for rows
  // of at most 256 bytes hold the query tile in LDS or registers
  const bool resident_query = prec != DEANN_FP32 && t.ld_bytes <= 2 * CHUNK_BYTES;
  t.map = make_tile_map(t.qtiles, t.splits, resident_query ? 1 : 4);
  return t;
}

hipError_t run_prep(const Prep& p, const float* X, int64_t n, const float* Y, int64_t q,
                    int64_t d, int prec, hipStream_t s) {
  const int64_t R = n < kCenterRows ? n : kCenterRows;
  hipError_t e = launch_center(X, n, d, p.cpart, R, p.c, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(p.err_max, 2, 0u, s)) != hipSuccess) return e;
  const double a = key_scale(p.dp);
  e = launch_prep_rows_prec(prec, X, n, p.np, d, p.dp, p.c, a, p.Xs, p.xnorm, p.xknorm, p.xerr,
                            p.err_max, s);
  if (e != hipSuccess) return e;
  return launch_prep_rows_prec(prec, Y, q, p.qp, d, p.dp, p.c, a, p.Ys, p.ynorm, p.yknorm, p.yerr,
                               p.err_max + 1, s);
}

bool bad_prec(int prec) { return prec != DEANN_FP32 && prec != DEANN_BF16 && prec != DEANN_FP16; }
bool bad_kernel(int k) { return k != DEANN_GAUSSIAN && k != DEANN_EXPONENTIAL; }

int check_common(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                 int kernel) {
  if (n < 1) return fail(DEANN_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
  if (d < 1) return fail(DEANN_EINVAL, "d must be >= 1 (got %lld)", (long long)d);
  if (q < 0) return fail(DEANN_EINVAL, "q must be >= 0 (got %lld)", (long long)q);
  if (n >= (int64_t)1 << 31) return fail(DEANN_EINVAL, "n must be < 2^31");
  if (q >= (int64_t)1 << 31) return fail(DEANN_EINVAL, "q must be < 2^31");
  if (!(std::isfinite(h) && h > 0.0)) return fail(DEANN_EINVAL, "h must be finite and > 0");
  if (bad_kernel(kernel)) return fail(DEANN_EINVAL, "unknown kernel %d", kernel);
  if (!X) return fail(DEANN_EINVAL, "X is NULL");
  if (q > 0 && !Y) return fail(DEANN_EINVAL, "Y is NULL");
  return DEANN_OK;
}

// ---- per-path workspace plans -------------------------------------------------
constexpr int64_t kKdeSplitTarget = 4096;
constexpr int64_t kKnnSplitTarget = 512;     // selection scan: about one wave of workgroups
constexpr int64_t kCollectSplitTarget = 4096;  // candidate and collect passes

struct KdePlan {
  Prep prep;
  double* partial;
  int64_t bytes;
};

KdePlan plan_kde(void* ws, int64_t n, int64_t q, int64_t d, int prec) {
  Carve cv(ws);
  KdePlan k{};
  k.prep = carve_prep(cv, n, q, d, prec);
  const int64_t qtiles = k.prep.qp / BQ, ntiles = k.prep.np / BN;
  const int64_t splits = choose_splits(qtiles, ntiles, kKdeSplitTarget);
  k.partial = cv.take<double>(splits * k.prep.qp);
  k.bytes = cv.off + kAlign;
  return k;
}

int64_t knn_K1(int64_t k) {
  int64_t v = k + 16;
  if (v < 64) v = 64;
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

struct DeannPlan {
  Prep prep;
  KnnBuffers kb;
  int32_t* nn_internal;
  int64_t bytes;
};

DeannPlan plan_deann(void* ws, int64_t n, int64_t q, int64_t d, int64_t k, int prec) {
  Carve cv(ws);
  DeannPlan P{};
  P.prep = carve_prep(cv, n, q, d, prec);
  const int64_t qtiles = P.prep.qp / BQ, ntiles = P.prep.np / BN;
  const int64_t splits = choose_splits(qtiles, ntiles, kKnnSplitTarget);
  KnnBuffers& b = P.kb;
  b.K1 = knn_K1(k);
  // a list must hold K1 kept entries plus one tile (BN) of new ones
  b.cap1 = 256;
  while (b.cap1 < 2 * b.K1 + BN) b.cap1 <<= 1;
  // list scan (FP32) or one candidate per cell of the collect geometry (16-bit)
  const int64_t splits_c = choose_splits(qtiles, ntiles, kCollectSplitTarget);
  const int64_t lists = prec == DEANN_FP32 ? splits * b.cap1 : splits_c * 32;
  b.cand = cv.take<uint64_t>(P.prep.qp * lists);
  b.cand_cnt = cv.take<int32_t>((splits > splits_c ? splits : splits_c) * P.prep.qp);
  P.nn_internal = cv.take<int32_t>(q * (k > 0 ? k : 1));
  b.z1 = cv.take<double>(q > 0 ? q : 1);
  b.thr2 = cv.take<float>(q > 0 ? q : 1);
  b.flags = cv.take<int32_t>(qtiles > 0 ? qtiles : 1);
  b.cap2 = kSortCap;
  b.cand2 = cv.take<uint64_t>(q * b.cap2);
  b.cand2_cnt = cv.take<int32_t>(q > 0 ? q : 1);
  b.status = cv.take<int32_t>(q > 0 ? q : 1);
  b.yerr = P.prep.yerr;
  b.xerr_max = P.prep.err_max;
  P.bytes = cv.off + kAlign;
  return P;
}

struct KdeBwdPlan {
  Prep prep;
  double* gy_part;
  double* gh_part;   // gh, rw, ks [splits][qp] each, then per-query [q]
  int64_t bytes;
};

KdeBwdPlan plan_kde_bwd(void* ws, int64_t n, int64_t q, int64_t d) {
  Carve cv(ws);
  KdeBwdPlan P{};
  P.prep = carve_prep(cv, n, q, d, DEANN_FP32);
  const int64_t qtiles = P.prep.qp / BQ, ntiles = P.prep.np / BN;
  const int64_t splits = choose_splits(qtiles, ntiles, kKdeSplitTarget);
  P.gy_part = cv.take<double>(splits * P.prep.qp * P.prep.dp);
  P.gh_part = cv.take<double>(3 * splits * P.prep.qp + (q > 0 ? q : 1));
  P.bytes = cv.off + kAlign;
  return P;
}

// Align the caller's workspace pointer.
void* align_ws(void* ws) {
  const uintptr_t v = reinterpret_cast<uintptr_t>(ws);
  return reinterpret_cast<void*>((v + kAlign - 1) / kAlign * kAlign);
}

}  // namespace

extern "C" {

const char* deann_last_error(void) { return g_last_error.c_str(); }

int deann_kernel_timing(int capacity) {
  if (capacity < 0 || capacity > 4096)
    return fail(DEANN_EINVAL, "timing capacity must be in [0, 4096] (got %d)", capacity);
  timer_release();
  if (capacity == 0) return DEANN_OK;
  for (int s = 0; s < kTimingSites; ++s) {
    g_timer.ev[s] = new hipEvent_t[2 * capacity]();
    g_timer.cap = capacity;
    for (int i = 0; i < 2 * capacity; ++i) {
      const hipError_t e = hipEventCreate(&g_timer.ev[s][i]);
      if (e != hipSuccess) {
        g_timer.ev[s][i] = nullptr;
        timer_release();
        return hip_fail(e, "hipEventCreate");
      }
    }
  }
  return DEANN_OK;
}

int deann_kernel_times(int site, float* ms, int max_count) {
  if (site < 0 || site >= kTimingSites || (!ms && max_count > 0) || max_count < 0) {
    fail(DEANN_EINVAL, "bad timing site or buffer");
    return -1;
  }
  const int n = g_timer.used[site] < max_count ? g_timer.used[site] : max_count;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(g_timer.ev[site][2 * i + 1]);
    if (e == hipSuccess)
      e = hipEventElapsedTime(&ms[i], g_timer.ev[site][2 * i], g_timer.ev[site][2 * i + 1]);
    if (e != hipSuccess) {
      hip_fail(e, "kernel timing");
      return -1;
    }
  }
  g_timer.used[site] = 0;
  return n;
}

size_t kde_exact_workspace(int64_t n, int64_t q, int64_t d, int precision) {
  if (n < 1 || d < 1 || q < 0 || bad_prec(precision)) return 0;
  return (size_t)plan_kde(nullptr, n, q, d, precision).bytes;
}

int kde_exact(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
              int kernel, int precision, double* out, void* ws, size_t ws_bytes, void* stream) {
  int st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (bad_prec(precision)) return fail(DEANN_EINVAL, "unknown precision %d", precision);
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_kde(nullptr, n, q, d, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  KdePlan P = plan_kde(align_ws(ws), n, q, d, precision);
  hipError_t e = run_prep(P.prep, X, n, Y, q, d, precision, s);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tp = make_problem(P.prep, n, q, precision, kKdeSplitTarget);
  e = launch_kde_exact(precision, tp, kernel, h, P.partial, out, s, timer_hook(0));
  if (e != hipSuccess) return hip_fail(e, "kde_exact");
  return DEANN_OK;
}

size_t deann_query_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                             int precision) {
  (void)m;
  if (n < 1 || d < 1 || q < 0 || k < 0 || k > n || bad_prec(precision)) return 0;
  return (size_t)plan_deann(nullptr, n, q, d, k, precision).bytes;
}

}  // extern "C"

static int deann_query_impl(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                            double h, int kernel, int64_t k, int64_t m, uint64_t seed,
                            uint64_t query_offset, uint64_t word2, int permuted, uint64_t start,
                            int precision, double* out, int32_t* nn_idx, int32_t* sample_idx,
                            void* ws, size_t ws_bytes, void* stream) {
  int st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (bad_prec(precision)) return fail(DEANN_EINVAL, "unknown precision %d", precision);
  if (k < 0 || k > n) return fail(DEANN_EINVAL, "k must be in [0, n] (got %lld)", (long long)k);
  if (m < 0) return fail(DEANN_EINVAL, "m must be >= 0 (got %lld)", (long long)m);
  if (k > kMaxK && k != n)
    return fail(DEANN_EUNSUPPORTED, "k = %lld: supported are k <= %lld and k = n", (long long)k,
                (long long)kMaxK);
  if (d > 4096) return fail(DEANN_EUNSUPPORTED, "d > 4096 is not supported by deann_query");
  if (permuted && k < n && m > n - k)
    return fail(DEANN_EINVAL, "permuted sampling needs m <= n - k (got m = %lld)", (long long)m);
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_deann(nullptr, n, q, d, k, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeannPlan P = plan_deann(align_ws(ws), n, q, d, k, precision);
  P.kb.nn_work = nn_idx ? nn_idx : P.nn_internal;
  hipError_t e;
  if (k == n) {
    e = launch_knn_all(X, Y, n, q, d, h, kernel, P.kb.nn_work, P.kb.z1, s);
    if (e != hipSuccess) return hip_fail(e, "all-points sum");
  } else if (k > 0) {
    e = run_prep(P.prep, X, n, Y, q, d, precision, s);
    if (e != hipSuccess) return hip_fail(e, "prep");
    TileProblem tp = make_problem(P.prep, n, q, precision, kKnnSplitTarget);
    TileProblem tc = make_problem(P.prep, n, q, precision, kCollectSplitTarget);
    e = launch_knn(precision, tp, tc, P.kb, X, Y, d, k, h, kernel, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "knn");
  }
  e = launch_sample(X, Y, n, q, d, h, kernel, k, m, seed, query_offset, word2, permuted, start,
                    P.kb.nn_work, P.kb.z1, out, sample_idx, s);
  if (e != hipSuccess) return hip_fail(e, "sample");
  return DEANN_OK;
}

extern "C" {

int deann_query(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                int kernel, int64_t k, int64_t m, uint64_t seed, uint64_t query_offset,
                uint64_t word2, int precision, double* out, int32_t* nn_idx, int32_t* sample_idx,
                void* ws, size_t ws_bytes, void* stream) {
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, query_offset, word2, 0, 0,
                          precision, out, nn_idx, sample_idx, ws, ws_bytes, stream);
}

size_t deann_query_permuted_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                                      int precision) {
  return deann_query_workspace(n, q, d, k, m, precision);
}

int deann_query_permuted(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                         double h, int kernel, int64_t k, int64_t m, uint64_t seed,
                         uint64_t start, int precision, double* out, int32_t* nn_idx,
                         int32_t* sample_idx, void* ws, size_t ws_bytes, void* stream) {
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, 0, 0, 1, start, precision, out,
                          nn_idx, sample_idx, ws, ws_bytes, stream);
}

size_t deann_query_backward_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m) {
  (void)n; (void)d; (void)k; (void)m;
  if (q < 0) return 0;
  return (size_t)(round_up((q > 0 ? q : 1) * 8, kAlign) + kAlign);
}

int deann_query_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                         double h, int kernel, int64_t k, int64_t m, const int32_t* nn_idx,
                         const int32_t* sample_idx, const double* grad_out, float* grad_Y,
                         double* grad_h, void* ws, size_t ws_bytes, void* stream) {
  int st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (k < 0 || k > n) return fail(DEANN_EINVAL, "k must be in [0, n]");
  if (m < 0) return fail(DEANN_EINVAL, "m must be >= 0");
  if (d > 2048) return fail(DEANN_EUNSUPPORTED, "d > 2048 is not supported by the backward");
  if (q == 0) {
    if (grad_h) return fail(DEANN_EUNSUPPORTED, "grad_h with q = 0: nothing to write into");
    return DEANN_OK;
  }
  if (k > 0 && !nn_idx) return fail(DEANN_EINVAL, "nn_idx is NULL");
  if (m > 0 && k < n && !sample_idx) return fail(DEANN_EINVAL, "sample_idx is NULL");
  if (!grad_out) return fail(DEANN_EINVAL, "grad_out is NULL");
  const int64_t need = (int64_t)deann_query_backward_workspace(n, q, d, k, m);
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* gh_part = static_cast<double*>(align_ws(ws));
  hipError_t e = launch_deann_backward(X, Y, n, q, d, h, kernel, k, m, nn_idx, sample_idx,
                                       grad_out, grad_Y, gh_part, grad_h, s);
  if (e != hipSuccess) return hip_fail(e, "deann backward");
  return DEANN_OK;
}

size_t kde_exact_backward_workspace(int64_t n, int64_t q, int64_t d) {
  if (n < 1 || d < 1 || q < 0) return 0;
  return (size_t)plan_kde_bwd(nullptr, n, q, d).bytes;
}

int kde_exact_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                       int kernel, const double* grad_out, float* grad_Y, double* grad_h,
                       void* ws, size_t ws_bytes, void* stream) {
  int st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (d > 128) return fail(DEANN_EUNSUPPORTED, "kde_exact_backward supports d <= 128");
  if (q == 0) return DEANN_OK;
  if (!grad_out) return fail(DEANN_EINVAL, "grad_out is NULL");
  const int64_t need = plan_kde_bwd(nullptr, n, q, d).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  KdeBwdPlan P = plan_kde_bwd(align_ws(ws), n, q, d);
  hipError_t e = run_prep(P.prep, X, n, Y, q, d, DEANN_FP32, s);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tp = make_problem(P.prep, n, q, DEANN_FP32, kKdeSplitTarget);
  // one 8-wave workgroup per CU: the query tiles of the split-major order
  // already fit the L2 next to the shared data tiles
  tp.map = make_tile_map(tp.qtiles, tp.splits, 1);
  e = launch_kde_backward(tp, Y, d, h, kernel, grad_out, P.gy_part, P.gh_part, grad_Y, grad_h, s,
                          timer_hook(1));
  if (e != hipSuccess) return hip_fail(e, "kde backward");
  return DEANN_OK;
}

int mean_shift_update(const float* Y, const float* grad_Y, const double* density, int64_t q,
                      int64_t d, double h, float* Y_out, void* stream) {
  if (q < 0 || d < 1) return fail(DEANN_EINVAL, "need q >= 0 and d >= 1");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(DEANN_EINVAL, "h must be finite and > 0");
  if (q == 0) return DEANN_OK;
  if (!Y || !grad_Y || !density || !Y_out) return fail(DEANN_EINVAL, "NULL array");
  const hipError_t e = launch_mean_shift_update(Y, grad_Y, density, q, d, h, Y_out,
                                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mean shift update");
  return DEANN_OK;
}

size_t kde_exact_with_grad_workspace(int64_t n, int64_t q, int64_t d) {
  return kde_exact_backward_workspace(n, q, d);
}

int kde_exact_with_grad(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                        int kernel, double* out, float* grad_Y, double* grad_h, void* ws,
                        size_t ws_bytes, void* stream) {
  int st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (d > 128) return fail(DEANN_EUNSUPPORTED, "kde_exact_with_grad supports d <= 128");
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_kde_bwd(nullptr, n, q, d).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  KdeBwdPlan P = plan_kde_bwd(align_ws(ws), n, q, d);
  hipError_t e = run_prep(P.prep, X, n, Y, q, d, DEANN_FP32, s);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tp = make_problem(P.prep, n, q, DEANN_FP32, kKdeSplitTarget);
  tp.map = make_tile_map(tp.qtiles, tp.splits, 1);
  e = launch_kde_backward(tp, Y, d, h, kernel, nullptr, P.gy_part, P.gh_part, grad_Y, nullptr, s,
                          timer_hook(1), out, grad_h);
  if (e != hipSuccess) return hip_fail(e, "kde value and gradient");
  return DEANN_OK;
}

}  // extern "C"
