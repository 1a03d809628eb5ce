// C ABI of the DEANN query path: argument validation, workspace layout and
// kernel launches.  No allocation, no stream synchronisation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/deann.h"
#include "common.h"
#include "kernels.h"

using namespace deann;

namespace {

thread_local std::string g_last_error;

deann_status fail(deann_status status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
deann_status fail(deann_status status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

deann_status hip_fail(hipError_t e, const char* what) {
  return fail(DEANN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Per-thread event pairs around the dense tile kernels (measurement only).
// 0: kde_exact tiles, 1: kde_exact_backward / kde_exact_with_grad tiles, 2: kde_hybrid tiles
constexpr int kTimingSites = 3;
struct KernelTimer {
  int cap = 0;
  int used[kTimingSites] = {0, 0, 0};
  hipEvent_t* ev[kTimingSites] = {nullptr, nullptr, nullptr};   // [cap][2] per site
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
constexpr int64_t kSortCapMax = 4096;      // second-pass candidate capacity per query (workspace)

deann_options default_options() {
  deann_options o{};
  o.rel_tol = 1e-5;
  o.value_floor = 1e-16;
  o.knn_slack = 16;
  o.knn_cap2 = kSortCapMax;
  o.center = 1;
  o.knn_seed_stride = 4;
  return o;
}

// Options of the calls made on this thread (deann_set_options).
thread_local deann_options g_opt = default_options();

// Device counters of the last call on this thread, for deann_last_stats: the
// exact KDE's list length of re-evaluated queries, the k-NN status per query.
struct LastCall {
  const int32_t* refined = nullptr;
  const int32_t* knn_status = nullptr;
  int64_t knn_q = 0;
};
thread_local LastCall g_last;

void record_last(const int32_t* refined, const int32_t* knn_status, int64_t q) {
  g_last.refined = refined;
  g_last.knn_status = knn_status;
  g_last.knn_q = knn_status ? q : 0;
}
constexpr int64_t kMaxK = 496;             // k limit of the candidate-list kernels (K1 <= 512)
constexpr int64_t kCenterRows = 2048;      // row slices of the column-mean reduction

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
  p.err_max = cv.take<uint32_t>(3);   // rounding bounds of X and Y, largest data norm
  return p;
}

// Relative slack of the lower-bound keys: twice the worst-case FP32 dot-product
// error gamma_d plus the roundings of norms and of the key arithmetic.
double key_scale(int64_t dp) {
  const double u = std::ldexp(1.0, -24);
  const double gamma = (double)dp * u / (1.0 - (double)dp * u);
  return 2.0 * gamma + 16.0 * u;
}

// Data splits per query tile for a sweep of `target` workgroups, at most 512:
// a batch of one query tile still fills the GPU (two workgroups per CU), and
// the per-query reductions over the splits stay short.
int64_t choose_splits(int64_t qtiles, int64_t ntiles, int64_t target) {
  constexpr int64_t kMaxSplits = 512;
  int64_t s = target / (qtiles > 0 ? qtiles : 1);
  if (s > kMaxSplits) s = kMaxSplits;
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
  // 4 splits per query-tile sweep (L2 reuse of both operands; also for the
  // 16-bit engines that hold the query tile in LDS or registers, whose data
  // tiles are then shared in L2 as well: 5% faster than split-major there)
  t.map = make_tile_map(t.qtiles, t.splits, 4);
  t.tstride = 1;
  return t;
}

// The data half of the preparation: centre, bounds (err_max[1], the queries'
// bound, is left 0), the data rows in the scan type with their norms.
hipError_t run_prep_x(const Prep& p, const float* X, int64_t n, int64_t d, int prec,
                      hipStream_t s) {
  const int64_t R = n < kCenterRows ? n : kCenterRows;
  hipError_t e = g_opt.center ? launch_center(X, n, d, p.cpart, R, p.c, s)
                              : launch_fill_u32(reinterpret_cast<uint32_t*>(p.c), d, 0u, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(p.err_max, 3, 0u, s)) != hipSuccess) return e;
  const double a = key_scale(p.dp);
  e = launch_prep_rows_prec(prec, X, n, p.np, d, p.dp, p.c, a, p.Xs, p.xnorm, p.xknorm, p.xerr,
                            p.err_max, s);
  if (e != hipSuccess) return e;
  return launch_max_u32(p.xknorm, n, p.err_max + 2, s);
}

hipError_t run_prep_y(const Prep& p, const float* Y, int64_t q, int64_t d, int prec,
                      hipStream_t s) {
  return launch_prep_rows_prec(prec, Y, q, p.qp, d, p.dp, p.c, key_scale(p.dp), p.Ys, p.ynorm,
                               p.yknorm, p.yerr, p.err_max + 1, s);
}

hipError_t run_prep(const Prep& p, const float* X, int64_t n, const float* Y, int64_t q,
                    int64_t d, int prec, hipStream_t s) {
  hipError_t e = run_prep_x(p, X, n, d, prec, s);
  if (e != hipSuccess) return e;
  return run_prep_y(p, Y, q, d, prec, s);
}

// Prepared data set (deann_prepare), caller-owned device memory: the data half
// of a Prep -- centre c[d], bounds err_max[3], centring partials, rows
// Xs[np][dp] in the scan type, xnorm[np], xknorm[np], xerr[np].
Prep carve_prepared(void* base, int64_t n, int64_t d, int prec, int64_t* bytes) {
  Carve cv(base);
  Prep p{};
  p.dp = padded_d(d, prec);
  p.np = round_up(n, BN);
  p.c = cv.take<float>(d);
  p.err_max = cv.take<uint32_t>(3);
  p.cpart = cv.take<double>(kCenterRows * d);
  p.Xs = cv.take<char>(p.np * p.dp * elem_bytes(prec));
  p.xnorm = cv.take<double>(p.np);
  p.xknorm = cv.take<float>(p.np);
  p.xerr = cv.take<float>(p.np);
  if (bytes) *bytes = cv.off + kAlign;
  return p;
}

// A call's preparation from a prepared data set: the data rows are read where
// they are; centre and bounds are copied into the call's workspace (the
// queries' bound is formed there); then the queries are prepared.
hipError_t run_prep_prepared(Prep& p, const Prep& h, const float* Y, int64_t q, int64_t d,
                             int prec, hipStream_t s) {
  p.Xs = h.Xs;
  p.xnorm = h.xnorm;
  p.xknorm = h.xknorm;
  p.xerr = h.xerr;
  hipError_t e = launch_copy_u32(reinterpret_cast<uint32_t*>(p.c),
                                 reinterpret_cast<const uint32_t*>(h.c), d, s);
  if (e != hipSuccess) return e;
  if ((e = launch_copy_u32(p.err_max, h.err_max, 3, s)) != hipSuccess) return e;
  return run_prep_y(p, Y, q, d, prec, s);
}

bool bad_prec(int prec) { return prec != DEANN_FP32 && prec != DEANN_BF16 && prec != DEANN_FP16; }
bool bad_kernel(int k) { return k != DEANN_GAUSSIAN && k != DEANN_EXPONENTIAL; }

deann_status check_common(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
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

// Exact adjoint / value + gradient: each (query tile, split) workgroup writes
// per-split FP64 gradient partials (qp x dp doubles per split), so it takes
// about five rounds of resident workgroups (one 8-wave workgroup per CU, two
// for rows of 64 floats) instead of the forward's 4096, each sweeping a longer
// range of data tiles: about a third of the partial traffic.
int64_t bwd_split_target(int64_t dp) { return (dp == 64 ? 512 : 256) * 5; }
constexpr int64_t kKnnSplitTarget = 512;     // selection scan: about one wave of workgroups
constexpr int64_t kCollectSplitTarget = 4096;  // candidate and collect passes
constexpr int64_t kIvfPartTarget = 512;        // inverted-file sweep parts: 2 per CU

// Certificate of the float32-operand sweeps (see cert.hip): queries whose
// bounded relative error exceeds the rel_tol option are re-evaluated exactly,
// unless their value is certainly below the value_floor option (by default
// 1e-16: the paper reports no relative error for KDE values under 1e-16).

struct CertBuf {
  float2* part;      // [splits][qp]
  float* pn;         // [splits][qp] (the generic float32 tile kernel's per-pair norm sums)
  float* pk;         // [splits][qp] (its split engine's sums of K N)
  int32_t* ids;      // [q]
  int32_t* count;    // [1]
};

CertBuf carve_cert(Carve& cv, int64_t splits, int64_t qp, int64_t q) {
  CertBuf c{};
  c.part = cv.take<float2>(splits * qp);
  c.pn = cv.take<float>(splits * qp);
  c.pk = cv.take<float>(splits * qp);
  c.ids = cv.take<int32_t>(q > 0 ? q : 1);
  c.count = cv.take<int32_t>(1);
  return c;
}

// cd: roundings of one dot product (its accumulation length); split: the
// distance product comes from three-part bfloat16 operands
CertArgs cert_args(const CertBuf& c, const Prep& p, int64_t cd, bool split = false) {
  CertArgs a{};
  a.sys = split ? 2.0 : 0.0;
  a.part = c.part;
  a.xnmax = p.err_max + 2;
  a.a_scale = key_scale(p.dp);
  a.cd = (int)cd;
  a.tau = g_opt.rel_tol;
  a.floor = g_opt.value_floor;
  a.fb_ids = c.ids;
  a.fb_count = c.count;
  a.pn = c.pn;   // dropped by the launches whose sweep does not write it
  a.pk = c.pk;
  return a;
}

struct KdePlan {
  Prep prep;
  double* partial;
  char *Xsp, *Ysp;   // three-part bfloat16 rows (DEANN_FP32_SPLIT)
  int64_t dps;
  CertBuf cert;      // float32 operands only
  double* fb_part;   // [direct_splits(n)][q]
  int64_t bytes;
};

KdePlan plan_kde(void* ws, int64_t n, int64_t q, int64_t d, int prec) {
  Carve cv(ws);
  KdePlan k{};
  const bool split = prec == DEANN_FP32_SPLIT;
  k.prep = carve_prep(cv, n, q, d, split ? DEANN_FP32 : prec);
  if (split) {
    k.dps = round_up(d, 64);
    k.Xsp = cv.take<char>(k.prep.np * 3 * k.dps * 2);
    k.Ysp = cv.take<char>(k.prep.qp * 3 * k.dps * 2);
  }
  const int64_t qtiles = k.prep.qp / BQ, ntiles = k.prep.np / BN;
  const int64_t splits = choose_splits(qtiles, ntiles, kKdeSplitTarget);
  k.partial = cv.take<double>(splits * k.prep.qp);
  if (prec == DEANN_FP32 || split) {
    k.cert = carve_cert(cv, splits, k.prep.qp, q);
    k.fb_part = cv.take<double>(direct_splits(n) * (q > 0 ? q : 1));
  }
  k.bytes = cv.off + kAlign;
  return k;
}

int64_t knn_K1(int64_t k) {
  int64_t v = k + g_opt.knn_slack;
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
  b.cand2 = cv.take<uint64_t>(q * kSortCapMax);
  b.cap2 = g_opt.knn_cap2;   // row stride of cand2 as well: within the carved rows
  b.cand2_cnt = cv.take<int32_t>(q > 0 ? q : 1);
  b.status = cv.take<int32_t>(q > 0 ? q : 1);
  b.yerr = P.prep.yerr;
  b.xerr_max = P.prep.err_max;
  b.seed_stride = g_opt.knn_seed_stride;
  P.bytes = cv.off + kAlign;
  return P;
}

// Near/far form: the k-NN plan (its prepared 16-bit operands also feed the
// tile sweep), then the sweep's partials and the neighbour-pair CSR.
struct HybPlan {
  DeannPlan dn;
  double* partial;
  int32_t *cnt, *off, *tot;
  uint16_t* hits;
  int64_t bytes;
};

HybPlan plan_hybrid(void* ws, int64_t n, int64_t q, int64_t d, int64_t k, int prec) {
  HybPlan H{};
  H.dn = plan_deann(ws, n, q, d, k, prec);
  const int64_t head = round_up(H.dn.bytes, kAlign);
  Carve cv(ws ? static_cast<char*>(ws) + head : nullptr);
  const int64_t qtiles = H.dn.prep.qp / BQ, ntiles = H.dn.prep.np / BN;
  const int64_t splits = choose_splits(qtiles, ntiles, kKdeSplitTarget);
  H.partial = cv.take<double>(splits * H.dn.prep.qp);
  const int64_t keys = qtiles * ntiles;
  H.cnt = cv.take<int32_t>(keys);
  H.off = cv.take<int32_t>(keys + 1);
  H.tot = cv.take<int32_t>(scan_blocks(keys));
  H.hits = cv.take<uint16_t>(k > 0 && k < n ? q * k : 1);
  H.bytes = head + cv.off + kAlign;
  return H;
}

bool bad_hyb_prec(int p) { return p != DEANN_BF16 && p != DEANN_FP16; }

// DEANN with the gradient of every estimate: the k-NN plan, then the
// per-query d/dh terms and room for the draws (used when the caller passes no
// sample_idx and the shape takes the sampler followed by the adjoint).
struct DeannGradPlan {
  DeannPlan dn;
  double* gh_part;
  int32_t* samp;
  int64_t bytes;
};

DeannGradPlan plan_deann_grad(void* ws, int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                              int prec) {
  DeannGradPlan G{};
  G.dn = plan_deann(ws, n, q, d, k, prec);
  const int64_t head = round_up(G.dn.bytes, kAlign);
  Carve cv(ws ? static_cast<char*>(ws) + head : nullptr);
  G.gh_part = cv.take<double>(q > 0 ? q : 1);
  G.samp = cv.take<int32_t>(q * m > 0 ? q * m : 1);
  G.bytes = head + cv.off + kAlign;
  return G;
}

struct KdeBwdPlan {
  Prep prep;
  double* gy_part;
  double* gh_part;   // gh, rw, ks [splits][qp] each, then per-query [q]
  char *Xsp, *Ysp;   // three-part bfloat16 rows (DEANN_FP32_SPLIT)
  int64_t dps;
  CertBuf cert;
  int64_t bytes;
};

KdeBwdPlan plan_kde_bwd(void* ws, int64_t n, int64_t q, int64_t d, int precision) {
  Carve cv(ws);
  KdeBwdPlan P{};
  P.prep = carve_prep(cv, n, q, d, DEANN_FP32);
  const int64_t qtiles = P.prep.qp / BQ, ntiles = P.prep.np / BN;
  const int64_t splits = choose_splits(qtiles, ntiles, bwd_split_target(P.prep.dp));
  P.gy_part = cv.take<double>(splits * P.prep.qp * P.prep.dp);
  P.gh_part = cv.take<double>(3 * splits * P.prep.qp + (q > 0 ? q : 1));
  if (precision == DEANN_FP32_SPLIT) {
    P.dps = round_up(d, 64);
    P.Xsp = cv.take<char>(P.prep.np * 3 * P.dps * 2);
    P.Ysp = cv.take<char>(P.prep.qp * 3 * P.dps * 2);
  }
  P.cert = carve_cert(cv, splits, P.prep.qp, q);
  P.bytes = cv.off + kAlign;
  return P;
}

bool bad_exact_grad_prec(int p) { return p != DEANN_FP32 && p != DEANN_FP32_SPLIT; }

// Float32 prep (and for DEANN_FP32_SPLIT the bfloat16 parts) of the exact
// gradient paths; returns the split rows to use (X null: float32).
// `pre`: a prepared float32 data set, or null to prepare X here.
hipError_t prep_exact_grad(KdeBwdPlan& P, const float* X, int64_t n, const float* Y,
                           int64_t q, int64_t d, int precision, SplitRows& sp, hipStream_t s,
                           const Prep* pre = nullptr) {
  hipError_t e = pre ? run_prep_prepared(P.prep, *pre, Y, q, d, DEANN_FP32, s)
                     : run_prep(P.prep, X, n, Y, q, d, DEANN_FP32, s);
  if (e != hipSuccess || precision != DEANN_FP32_SPLIT) return e;
  e = launch_split_rows(reinterpret_cast<const float*>(P.prep.Xs), P.prep.np, P.prep.dp, P.dps,
                        P.Xsp, s);
  if (e == hipSuccess)
    e = launch_split_rows(reinterpret_cast<const float*>(P.prep.Ys), P.prep.qp, P.prep.dp, P.dps,
                          P.Ysp, s);
  sp.X = P.Xsp;
  sp.Y = P.Ysp;
  sp.dps = P.dps;
  return e;
}

// Align the caller's workspace pointer.
void* align_ws(void* ws) {
  const uintptr_t v = reinterpret_cast<uintptr_t>(ws);
  return reinterpret_cast<void*>((v + kAlign - 1) / kAlign * kAlign);
}

}  // namespace

extern "C" {

const char* deann_last_error(void) { return g_last_error.c_str(); }

void deann_default_options(deann_options* o) {
  if (o) *o = default_options();
}

deann_status deann_get_options(deann_options* o) {
  if (!o) return fail(DEANN_EINVAL, "options pointer is NULL");
  *o = g_opt;
  return DEANN_OK;
}

deann_status deann_set_options(const deann_options* o) {
  if (!o) return fail(DEANN_EINVAL, "options pointer is NULL");
  if (!(o->rel_tol >= 1e-7 && o->rel_tol <= 1.0))
    return fail(DEANN_EINVAL, "rel_tol must be in [1e-7, 1]");
  if (!(o->value_floor >= 0.0 && std::isfinite(o->value_floor)))
    return fail(DEANN_EINVAL, "value_floor must be finite and >= 0");
  if (o->knn_slack < 0 || o->knn_slack > 512)
    return fail(DEANN_EINVAL, "knn_slack must be in [0, 512]");
  if (o->knn_cap2 < 1 || o->knn_cap2 > kSortCapMax)
    return fail(DEANN_EINVAL, "knn_cap2 must be in [1, %lld]", (long long)kSortCapMax);
  if (o->center != 0 && o->center != 1) return fail(DEANN_EINVAL, "center must be 0 or 1");
  if (o->knn_seed_stride < 1 || o->knn_seed_stride > 64)
    return fail(DEANN_EINVAL, "knn_seed_stride must be in [1, 64]");
  g_opt = *o;
  return DEANN_OK;
}

deann_status deann_last_stats(deann_stats* st, void* stream) {
  if (!st) return fail(DEANN_EINVAL, "stats pointer is NULL");
  st->exact_refined = -1;
  st->knn_second_pass = -1;
  st->knn_exhaustive = -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (g_last.refined) {
    int32_t c = 0;
    e = hipMemcpy(&c, g_last.refined, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "stats copy");
    st->exact_refined = c;
  }
  if (g_last.knn_status && g_last.knn_q > 0) {
    std::vector<int32_t> v((size_t)g_last.knn_q);
    e = hipMemcpy(v.data(), g_last.knn_status, v.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "stats copy");
    int64_t a = 0, b = 0;
    for (int32_t x : v) {   // final states: 0 first pass, 4 second pass, 5 exhaustive scan
      a += x == 4 || x == 5;
      b += x == 5;
    }
    st->knn_second_pass = a;
    st->knn_exhaustive = b;
  }
  return DEANN_OK;
}

deann_status deann_kernel_timing(int capacity) {
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

size_t kde_exact_workspace(int64_t n, int64_t q, int64_t d, deann_precision precision) {
  if (n < 1 || d < 1 || q < 0 || (bad_prec(precision) && precision != DEANN_FP32_SPLIT)) return 0;
  return (size_t)plan_kde(nullptr, n, q, d, precision).bytes;
}

}  // extern "C"

// Size check of a prepared data set for (n, d, prec); DEANN_OK when it holds.
static deann_status check_prepared(const void* prepared, size_t prepared_bytes, int64_t n,
                                   int64_t d, int prec) {
  int64_t need = 0;
  carve_prepared(nullptr, n, d, prec, &need);
  if (!prepared) return fail(DEANN_EINVAL, "prepared is NULL");
  if ((int64_t)prepared_bytes < need)
    return fail(DEANN_EWORKSPACE, "a prepared data set of %lld bytes is needed for n = %lld, "
                "d = %lld in this precision", (long long)need, (long long)n, (long long)d);
  return DEANN_OK;
}

static Prep prepared_of(const void* prepared, int64_t n, int64_t d, int prec) {
  return carve_prepared(align_ws(const_cast<void*>(prepared)), n, d, prec, nullptr);
}

static deann_status kde_exact_impl(const void* prepared, size_t prepared_bytes, const float* X,
                                   int64_t n, const float* Y, int64_t q, int64_t d, double h,
                                   int kernel, int precision, double* out, void* ws,
                                   size_t ws_bytes, void* stream) {
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  const bool split = precision == DEANN_FP32_SPLIT;
  if (bad_prec(precision) && !split) return fail(DEANN_EINVAL, "unknown precision %d", precision);
  const int prep_prec = split ? DEANN_FP32 : precision;
  if (prepared && (st = check_prepared(prepared, prepared_bytes, n, d, prep_prec)) != DEANN_OK)
    return st;
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_kde(nullptr, n, q, d, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  KdePlan P = plan_kde(align_ws(ws), n, q, d, precision);
  record_last(P.cert.count, nullptr, q);   // null for 16-bit operands
  hipError_t e = prepared ? run_prep_prepared(P.prep, prepared_of(prepared, n, d, prep_prec), Y,
                                              q, d, prep_prec, s)
                          : run_prep(P.prep, X, n, Y, q, d, prep_prec, s);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tp = make_problem(P.prep, n, q, prep_prec, kKdeSplitTarget);
  if (split) {
    e = launch_split_rows(reinterpret_cast<const float*>(P.prep.Xs), P.prep.np, P.prep.dp, P.dps,
                          P.Xsp, s);
    if (e == hipSuccess)
      e = launch_split_rows(reinterpret_cast<const float*>(P.prep.Ys), P.prep.qp, P.prep.dp,
                            P.dps, P.Ysp, s);
    if (e == hipSuccess)
      e = launch_kde_exact_split(tp, P.Xsp, P.Ysp, P.dps, kernel, h, P.partial, out, s,
                                 timer_hook(0), cert_args(P.cert, P.prep, P.dps + 4, true), X, Y, d,
                                 P.fb_part);
  } else {
    const CertArgs ca = precision == DEANN_FP32 ? cert_args(P.cert, P.prep, P.prep.dp) : CertArgs{};
    e = launch_kde_exact(precision, tp, kernel, h, P.partial, out, s, timer_hook(0), ca, X, Y, d,
                         P.fb_part);
  }
  if (e != hipSuccess) return hip_fail(e, "kde_exact");
  return DEANN_OK;
}

extern "C" {

deann_status kde_exact(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
              deann_kernel kernel, deann_precision precision, double* out, void* ws, size_t ws_bytes, void* stream) {
  return kde_exact_impl(nullptr, 0, X, n, Y, q, d, h, kernel, precision, out, ws, ws_bytes,
                        stream);
}

size_t deann_prepared_bytes(int64_t n, int64_t d, deann_precision precision) {
  if (n < 1 || d < 1 || bad_prec(precision)) return 0;
  int64_t need = 0;
  carve_prepared(nullptr, n, d, precision, &need);
  return (size_t)need;
}

deann_status deann_prepare(const float* X, int64_t n, int64_t d, deann_precision precision,
                           void* prepared, size_t prepared_bytes, void* stream) {
  if (n < 1) return fail(DEANN_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
  if (d < 1) return fail(DEANN_EINVAL, "d must be >= 1 (got %lld)", (long long)d);
  if (n >= (int64_t)1 << 31) return fail(DEANN_EINVAL, "n must be < 2^31");
  if (!X) return fail(DEANN_EINVAL, "X is NULL");
  if (bad_prec(precision)) return fail(DEANN_EINVAL, "unknown precision %d", precision);
  deann_status st = check_prepared(prepared, prepared_bytes, n, d, precision);
  if (st != DEANN_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = run_prep_x(prepared_of(prepared, n, d, precision), X, n, d, precision, s);
  if (e != hipSuccess) return hip_fail(e, "prepare");
  return DEANN_OK;
}

deann_status kde_exact_prepared(const void* prepared, size_t prepared_bytes, const float* X,
                                int64_t n, const float* Y, int64_t q, int64_t d, double h,
                                deann_kernel kernel, deann_precision precision, double* out,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!prepared) return fail(DEANN_EINVAL, "prepared is NULL");
  return kde_exact_impl(prepared, prepared_bytes, X, n, Y, q, d, h, kernel, precision, out, ws,
                        ws_bytes, stream);
}

size_t deann_query_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                             deann_precision precision) {
  (void)m;
  if (n < 1 || d < 1 || q < 0 || k < 0 || k > n || bad_prec(precision)) return 0;
  return (size_t)plan_deann(nullptr, n, q, d, k, precision).bytes;
}

}  // extern "C"

// Layout of the permuted index (Algorithm 2's preprocessing, caller-owned):
// pi[n] and inv[n] int32, then the permuted rows [n][d] float32 at a 256-byte
// boundary.
static int64_t perm_index_bytes(int64_t n, int64_t d) {
  return round_up(2 * n * 4, kAlign) + n * d * 4 + kAlign;
}

static PermIndex carve_perm_index(void* index, int64_t n) {
  char* base = static_cast<char*>(align_ws(index));
  PermIndex p;
  p.pi = reinterpret_cast<const int32_t*>(base);
  p.inv = p.pi + n;
  p.Xp = reinterpret_cast<const float*>(base + round_up(2 * n * 4, kAlign));
  return p;
}

// grad (deann_query_with_grad only): also d out_j / d y_j into grad->Y and
// d out_j / d h into grad->h[j] (each may be NULL), plain sampling.
struct DeannGradOut {
  float* Y;
  double* h;
};

static deann_status deann_query_impl(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                            double h, int kernel, int64_t k, int64_t m, uint64_t seed,
                            uint64_t query_offset, uint64_t word2, int permuted, uint64_t start,
                            int precision, double* out, int32_t* nn_idx, int32_t* sample_idx,
                            void* ws, size_t ws_bytes, void* stream,
                            const PermIndex* pidx = nullptr, const DeannGradOut* grad = nullptr,
                            const void* prepared = nullptr, size_t prepared_bytes = 0) {
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (bad_prec(precision)) return fail(DEANN_EINVAL, "unknown precision %d", precision);
  if (prepared && (st = check_prepared(prepared, prepared_bytes, n, d, precision)) != DEANN_OK)
    return st;
  if (k < 0 || k > n) return fail(DEANN_EINVAL, "k must be in [0, n] (got %lld)", (long long)k);
  if (m < 0) return fail(DEANN_EINVAL, "m must be >= 0 (got %lld)", (long long)m);
  if (k > kMaxK && k != n)
    return fail(DEANN_EUNSUPPORTED, "k = %lld: supported are k <= %lld and k = n", (long long)k,
                (long long)kMaxK);
  if (k > 0 && k < n && knn_K1(k) > 512)
    return fail(DEANN_EUNSUPPORTED, "k + knn_slack = %lld exceeds the 512 candidates of a list",
                (long long)(k + g_opt.knn_slack));
  if (d > 4096) return fail(DEANN_EUNSUPPORTED, "d > 4096 is not supported by deann_query");
  if (grad && d > 2048)
    return fail(DEANN_EUNSUPPORTED, "d > 2048 is not supported by the gradient");
  if (permuted && k < n && m > n - k)
    return fail(DEANN_EINVAL, "permuted sampling needs m <= n - k (got m = %lld)", (long long)m);
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = grad ? plan_deann_grad(nullptr, n, q, d, k, m, precision).bytes
                            : plan_deann(nullptr, n, q, d, k, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeannGradPlan G = grad ? plan_deann_grad(align_ws(ws), n, q, d, k, m, precision)
                               : DeannGradPlan{};
  DeannPlan P = grad ? G.dn : plan_deann(align_ws(ws), n, q, d, k, precision);
  P.kb.nn_work = nn_idx ? nn_idx : P.nn_internal;
  record_last(nullptr, (k > 0 && k < n) ? P.kb.status : nullptr, q);
  hipError_t e;
  if (k == n) {
    e = launch_knn_all(X, Y, n, q, d, h, kernel, P.kb.nn_work, P.kb.z1, s);
    if (e != hipSuccess) return hip_fail(e, "all-points sum");
  } else if (k > 0) {
    e = prepared ? run_prep_prepared(P.prep, prepared_of(prepared, n, d, precision), Y, q, d,
                                     precision, s)
                 : run_prep(P.prep, X, n, Y, q, d, precision, s);
    if (e != hipSuccess) return hip_fail(e, "prep");
    TileProblem tp = make_problem(P.prep, n, q, precision, kKnnSplitTarget);
    TileProblem tc = make_problem(P.prep, n, q, precision, kCollectSplitTarget);
    e = launch_knn(precision, tp, tc, P.kb, X, Y, d, k, h, kernel, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "knn");
  }
  if (grad) {
    e = launch_deann_value_grad(X, Y, n, q, d, h, kernel, k, m, seed, query_offset, word2,
                                P.kb.nn_work, P.kb.z1, out, sample_idx ? sample_idx : G.samp,
                                grad->Y, grad->h ? grad->h : G.gh_part, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "value and gradient");
    return DEANN_OK;
  }
  e = launch_sample(X, Y, n, q, d, h, kernel, k, m, seed, query_offset, word2, permuted, start,
                    P.kb.nn_work, P.kb.z1, out, sample_idx, s, pidx);
  if (e != hipSuccess) return hip_fail(e, "sample");
  return DEANN_OK;
}

extern "C" {

deann_status deann_query(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                deann_kernel kernel, int64_t k, int64_t m, uint64_t seed, uint64_t query_offset,
                uint64_t word2, deann_precision precision, double* out, int32_t* nn_idx, int32_t* sample_idx,
                void* ws, size_t ws_bytes, void* stream) {
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, query_offset, word2, 0, 0,
                          precision, out, nn_idx, sample_idx, ws, ws_bytes, stream);
}

size_t deann_query_with_grad_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                                       deann_precision precision) {
  if (n < 1 || d < 1 || q < 0 || k < 0 || k > n || m < 0 || bad_prec(precision)) return 0;
  return (size_t)plan_deann_grad(nullptr, n, q, d, k, m, precision).bytes;
}

deann_status deann_query_with_grad(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                                   double h, deann_kernel kernel, int64_t k, int64_t m,
                                   uint64_t seed, uint64_t query_offset, uint64_t word2,
                                   deann_precision precision, double* out, float* grad_Y,
                                   double* grad_h, int32_t* nn_idx, int32_t* sample_idx, void* ws,
                                   size_t ws_bytes, void* stream) {
  const DeannGradOut g{grad_Y, grad_h};
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, query_offset, word2, 0, 0,
                          precision, out, nn_idx, sample_idx, ws, ws_bytes, stream, nullptr, &g);
}

deann_status deann_query_prepared(const void* prepared, size_t prepared_bytes, const float* X,
                                  int64_t n, const float* Y, int64_t q, int64_t d, double h,
                                  deann_kernel kernel, int64_t k, int64_t m, uint64_t seed,
                                  uint64_t query_offset, uint64_t word2,
                                  deann_precision precision, double* out, int32_t* nn_idx,
                                  int32_t* sample_idx, void* ws, size_t ws_bytes, void* stream) {
  if (!prepared) return fail(DEANN_EINVAL, "prepared is NULL");
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, query_offset, word2, 0, 0,
                          precision, out, nn_idx, sample_idx, ws, ws_bytes, stream, nullptr,
                          nullptr, prepared, prepared_bytes);
}

deann_status deann_query_with_grad_prepared(const void* prepared, size_t prepared_bytes,
                                            const float* X, int64_t n, const float* Y, int64_t q,
                                            int64_t d, double h, deann_kernel kernel, int64_t k,
                                            int64_t m, uint64_t seed, uint64_t query_offset,
                                            uint64_t word2, deann_precision precision,
                                            double* out, float* grad_Y, double* grad_h,
                                            int32_t* nn_idx, int32_t* sample_idx, void* ws,
                                            size_t ws_bytes, void* stream) {
  if (!prepared) return fail(DEANN_EINVAL, "prepared is NULL");
  const DeannGradOut g{grad_Y, grad_h};
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, query_offset, word2, 0, 0,
                          precision, out, nn_idx, sample_idx, ws, ws_bytes, stream, nullptr, &g,
                          prepared, prepared_bytes);
}

size_t deann_query_permuted_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                                      deann_precision precision) {
  return deann_query_workspace(n, q, d, k, m, precision);
}

deann_status deann_query_permuted(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                         double h, deann_kernel kernel, int64_t k, int64_t m, uint64_t seed,
                         uint64_t start, deann_precision precision, double* out, int32_t* nn_idx,
                         int32_t* sample_idx, void* ws, size_t ws_bytes, void* stream) {
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, seed, 0, 0, 1, start, precision, out,
                          nn_idx, sample_idx, ws, ws_bytes, stream);
}

size_t deann_perm_index_bytes(int64_t n, int64_t d) {
  if (n < 1 || d < 1 || n >= ((int64_t)1 << 31)) return 0;
  return (size_t)perm_index_bytes(n, d);
}

deann_status deann_perm_index_create(const float* X, int64_t n, int64_t d, uint64_t seed,
                                     void* index, size_t index_bytes, void* stream) {
  if (n < 1 || d < 1) return fail(DEANN_EINVAL, "need n >= 1 and d >= 1");
  if (n >= ((int64_t)1 << 31)) return fail(DEANN_EINVAL, "n must be < 2^31");
  if (!X) return fail(DEANN_EINVAL, "X is NULL");
  if (!index || (int64_t)index_bytes < perm_index_bytes(n, d))
    return fail(DEANN_EWORKSPACE, "index of %lld bytes needed", (long long)perm_index_bytes(n, d));
  const PermIndex p = carve_perm_index(index, n);
  const hipError_t e = launch_perm_index(X, n, d, seed, p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "permuted index");
  return DEANN_OK;
}

deann_status deann_query_permuted_index(const float* X, int64_t n, const float* Y, int64_t q,
                                        int64_t d, double h, deann_kernel kernel, int64_t k,
                                        int64_t m, const void* index, size_t index_bytes,
                                        uint64_t start, deann_precision precision, double* out,
                                        int32_t* nn_idx, int32_t* sample_idx, void* ws,
                                        size_t ws_bytes, void* stream) {
  if (n >= 1 && d >= 1 && (!index || (int64_t)index_bytes < perm_index_bytes(n, d)))
    return fail(DEANN_EINVAL, "index of %lld bytes needed (deann_perm_index_bytes)",
                (long long)perm_index_bytes(n, d));
  const PermIndex p = carve_perm_index(const_cast<void*>(index), n);
  // the seed only keys the permutation, which the index already holds
  return deann_query_impl(X, n, Y, q, d, h, kernel, k, m, 0, 0, 0, 1, start, precision, out,
                          nn_idx, sample_idx, ws, ws_bytes, stream, &p);
}

size_t deann_query_backward_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m) {
  (void)n; (void)d; (void)k; (void)m;
  if (q < 0) return 0;
  return (size_t)(round_up((q > 0 ? q : 1) * 8, kAlign) + kAlign);
}

}  // extern "C"

// Argument checks shared by both adjoint entry points of deann_query; returns
// DEANN_OK with *noop set when q = 0 leaves nothing to do.
static deann_status check_deann_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                                double h, int kernel, int64_t k, int64_t m, const int32_t* nn_idx,
                                const int32_t* sample_idx, const double* grad_out, double* grad_h,
                                bool* noop) {
  *noop = false;
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (k < 0 || k > n) return fail(DEANN_EINVAL, "k must be in [0, n]");
  if (m < 0) return fail(DEANN_EINVAL, "m must be >= 0");
  if (d > 2048) return fail(DEANN_EUNSUPPORTED, "d > 2048 is not supported by the backward");
  if (q == 0) {
    if (grad_h) return fail(DEANN_EUNSUPPORTED, "grad_h with q = 0: nothing to write into");
    *noop = true;
    return DEANN_OK;
  }
  if (k > 0 && !nn_idx) return fail(DEANN_EINVAL, "nn_idx is NULL");
  if (m > 0 && k < n && !sample_idx) return fail(DEANN_EINVAL, "sample_idx is NULL");
  if (!grad_out) return fail(DEANN_EINVAL, "grad_out is NULL");
  return DEANN_OK;
}

// Scratch of deann_query_backward_noalloc: the per-query dK/dh terms that the
// workspace holds otherwise.  Each device holds its own copy of the array; in
// host code its name is only a stand-in, so its device address is looked up
// once per device (hipGetSymbolAddress with that device current) and only that
// address is ever handed to a kernel.
static __device__ __align__(256) double scratch[DEANN_NOALLOC_MAX_Q];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device that `stream` runs on, which must
// be the current device.
deann_status scratch_address(hipStream_t stream, double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (stream) {
    int sdev = 0;
    e = hipStreamGetDevice(stream, &sdev);
    if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    if (sdev != dev)
      return fail(DEANN_EINVAL, "stream is on device %d but device %d is current", sdev, dev);
  }
  if (dev < 0 || dev >= kMaxDevices)
    return fail(DEANN_EUNSUPPORTED, "device ordinal %d is beyond %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return DEANN_OK;
}
}  // namespace

extern "C" {

deann_status deann_query_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                         double h, deann_kernel kernel, int64_t k, int64_t m, const int32_t* nn_idx,
                         const int32_t* sample_idx, const double* grad_out, float* grad_Y,
                         double* grad_h, void* ws, size_t ws_bytes, void* stream) {
  bool noop = false;
  deann_status st = check_deann_backward(X, n, Y, q, d, h, kernel, k, m, nn_idx, sample_idx, grad_out,
                                grad_h, &noop);
  if (st != DEANN_OK || noop) return st;
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

deann_status deann_query_backward_noalloc(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                                 double h, deann_kernel kernel, int64_t k, int64_t m,
                                 const int32_t* nn_idx, const int32_t* sample_idx,
                                 const double* grad_out, float* grad_Y, double* grad_h,
                                 void* stream) {
  bool noop = false;
  deann_status st = check_deann_backward(X, n, Y, q, d, h, kernel, k, m, nn_idx, sample_idx, grad_out,
                                grad_h, &noop);
  if (st != DEANN_OK || noop) return st;
  if (q > DEANN_NOALLOC_MAX_Q)
    return fail(DEANN_EUNSUPPORTED, "q = %lld exceeds the %d queries of the library's scratch",
                (long long)q, DEANN_NOALLOC_MAX_Q);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* gh_part = nullptr;
  if ((st = scratch_address(s, &gh_part)) != DEANN_OK) return st;
  // every query's entry is written before the h sum reads it: nothing to clear
  hipError_t e = launch_deann_backward(X, Y, n, q, d, h, kernel, k, m, nn_idx, sample_idx,
                                       grad_out, grad_Y, gh_part, grad_h, s);
  if (e != hipSuccess) return hip_fail(e, "deann backward");
  return DEANN_OK;
}

size_t kde_exact_backward_workspace(int64_t n, int64_t q, int64_t d, deann_precision precision) {
  if (n < 1 || d < 1 || q < 0 || bad_exact_grad_prec(precision)) return 0;
  return (size_t)plan_kde_bwd(nullptr, n, q, d, precision).bytes;
}

}  // extern "C"

static deann_status kde_exact_backward_impl(const void* prepared, size_t prepared_bytes,
                                            const float* X, int64_t n, const float* Y, int64_t q,
                                            int64_t d, double h, int kernel, int precision,
                                            const double* grad_out, float* grad_Y, double* grad_h,
                                            void* ws, size_t ws_bytes, void* stream) {
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (bad_exact_grad_prec(precision))
    return fail(DEANN_EINVAL, "precision must be DEANN_FP32 or DEANN_FP32_SPLIT");
  if (d > 128) return fail(DEANN_EUNSUPPORTED, "kde_exact_backward supports d <= 128");
  if (prepared && (st = check_prepared(prepared, prepared_bytes, n, d, DEANN_FP32)) != DEANN_OK)
    return st;
  if (q == 0) return DEANN_OK;
  if (!grad_out) return fail(DEANN_EINVAL, "grad_out is NULL");
  const int64_t need = plan_kde_bwd(nullptr, n, q, d, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  KdeBwdPlan P = plan_kde_bwd(align_ws(ws), n, q, d, precision);
  record_last(P.cert.count, nullptr, q);
  SplitRows sp;
  const Prep pre = prepared ? prepared_of(prepared, n, d, DEANN_FP32) : Prep{};
  hipError_t e = prep_exact_grad(P, X, n, Y, q, d, precision, sp, s, prepared ? &pre : nullptr);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tp = make_problem(P.prep, n, q, DEANN_FP32, bwd_split_target(P.prep.dp));
  // one 8-wave workgroup per CU: the query tiles of the split-major order
  // already fit the L2 next to the shared data tiles
  tp.map = make_tile_map(tp.qtiles, tp.splits, 1);
  e = launch_kde_backward(tp, X, Y, d, h, kernel, grad_out, P.gy_part, P.gh_part, grad_Y, grad_h,
                          s, timer_hook(1), nullptr, nullptr, sp,
                          cert_args(P.cert, P.prep, sp.X ? P.dps + 4 : P.prep.dp, sp.X != nullptr));
  if (e != hipSuccess) return hip_fail(e, "kde backward");
  return DEANN_OK;
}

extern "C" {

deann_status kde_exact_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                       deann_kernel kernel, deann_precision precision, const double* grad_out, float* grad_Y,
                       double* grad_h, void* ws, size_t ws_bytes, void* stream) {
  return kde_exact_backward_impl(nullptr, 0, X, n, Y, q, d, h, kernel, precision, grad_out,
                                 grad_Y, grad_h, ws, ws_bytes, stream);
}

deann_status kde_exact_backward_prepared(const void* prepared, size_t prepared_bytes,
                                         const float* X, int64_t n, const float* Y, int64_t q,
                                         int64_t d, double h, deann_kernel kernel,
                                         deann_precision precision, const double* grad_out,
                                         float* grad_Y, double* grad_h, void* ws,
                                         size_t ws_bytes, void* stream) {
  if (!prepared) return fail(DEANN_EINVAL, "prepared is NULL");
  return kde_exact_backward_impl(prepared, prepared_bytes, X, n, Y, q, d, h, kernel, precision,
                                 grad_out, grad_Y, grad_h, ws, ws_bytes, stream);
}

deann_status mean_shift_update(const float* Y, const float* grad_Y, const double* density, int64_t q,
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

size_t kde_hybrid_workspace(int64_t n, int64_t q, int64_t d, int64_t k, deann_precision precision) {
  if (n < 1 || d < 1 || q < 0 || k < 0 || k > n || bad_hyb_prec(precision)) return 0;
  return (size_t)plan_hybrid(nullptr, n, q, d, k, precision).bytes;
}

deann_status kde_hybrid(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
               deann_kernel kernel, int64_t k, deann_precision precision, const int32_t* nn_in, double* out,
               int32_t* nn_idx, void* ws, size_t ws_bytes, void* stream) {
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (bad_hyb_prec(precision))
    return fail(DEANN_EINVAL, "kde_hybrid takes DEANN_BF16 or DEANN_FP16 (got %d)", precision);
  if (k < 0 || k > n) return fail(DEANN_EINVAL, "k must be in [0, n] (got %lld)", (long long)k);
  if (!nn_in && k > kMaxK && k != n)
    return fail(DEANN_EUNSUPPORTED, "k = %lld: supported are k <= %lld and k = n", (long long)k,
                (long long)kMaxK);
  if (!nn_in && k > 0 && k < n && knn_K1(k) > 512)
    return fail(DEANN_EUNSUPPORTED, "k + knn_slack = %lld exceeds the 512 candidates of a list",
                (long long)(k + g_opt.knn_slack));
  if (k > 0 && d > 4096)
    return fail(DEANN_EUNSUPPORTED, "d > 4096 is not supported by kde_hybrid with k > 0");
  if (k > 0 && k < n && q * k >= ((int64_t)1 << 31))
    return fail(DEANN_EUNSUPPORTED, "q * k must be < 2^31");
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_hybrid(nullptr, n, q, d, k, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HybPlan H = plan_hybrid(align_ws(ws), n, q, d, k, precision);
  record_last(nullptr, (!nn_in && k > 0 && k < n) ? H.dn.kb.status : nullptr, q);
  hipError_t e;
  if (k == n) {   // every row is near: the exact FP64 sum
    if (nn_in) {
      e = launch_knn_list_sum(X, Y, n, q, d, h, kernel, nn_in, k, H.dn.kb.z1, s);
      if (e == hipSuccess && nn_idx)
        e = hipMemcpyAsync(nn_idx, nn_in, (size_t)(q * k) * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s);
    } else {
      e = launch_knn_all(X, Y, n, q, d, h, kernel, nn_idx ? nn_idx : H.dn.nn_internal,
                         H.dn.kb.z1, s);
    }
    if (e == hipSuccess)
      e = launch_sample(X, Y, n, q, d, h, kernel, k, 0, 0, 0, 0, 0, 0, nullptr, H.dn.kb.z1, out,
                        nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "kde_hybrid (k = n)");
    return DEANN_OK;
  }
  e = run_prep(H.dn.prep, X, n, Y, q, d, precision, s);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tk = make_problem(H.dn.prep, n, q, precision, kKdeSplitTarget);
  if (k == 0) {   // nothing is near: the 16-bit sweep of kde_exact
    e = launch_kde_exact(precision, tk, kernel, h, H.partial, out, s, timer_hook(2), CertArgs{},
                         X, Y, d, nullptr);
    if (e != hipSuccess) return hip_fail(e, "kde_hybrid (k = 0)");
    return DEANN_OK;
  }
  const int32_t* nn_use = nn_in;
  if (nn_in) {
    e = launch_knn_list_sum(X, Y, n, q, d, h, kernel, nn_in, k, H.dn.kb.z1, s);
    if (e == hipSuccess && nn_idx)
      e = hipMemcpyAsync(nn_idx, nn_in, (size_t)(q * k) * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "neighbour sum");
  } else {
    H.dn.kb.nn_work = nn_idx ? nn_idx : H.dn.nn_internal;
    TileProblem tp = make_problem(H.dn.prep, n, q, precision, kKnnSplitTarget);
    TileProblem tc = make_problem(H.dn.prep, n, q, precision, kCollectSplitTarget);
    e = launch_knn(precision, tp, tc, H.dn.kb, X, Y, d, k, h, kernel, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "knn");
    nn_use = H.dn.kb.nn_work;
  }
  e = launch_hybrid_hits(nn_use, q, k, n, tk.qtiles, tk.ntiles, H.cnt, H.off, H.tot, H.hits, s);
  if (e != hipSuccess) return hip_fail(e, "neighbour pairs");
  e = launch_kde_hybrid(precision, tk, kernel, h, H.off, H.hits, H.dn.kb.z1, H.partial, out, s,
                        timer_hook(2));
  if (e != hipSuccess) return hip_fail(e, "kde_hybrid");
  return DEANN_OK;
}

size_t kde_exact_with_grad_workspace(int64_t n, int64_t q, int64_t d, deann_precision precision) {
  return kde_exact_backward_workspace(n, q, d, precision);
}

}  // extern "C"

static deann_status kde_exact_with_grad_impl(const void* prepared, size_t prepared_bytes,
                                             const float* X, int64_t n, const float* Y, int64_t q,
                                             int64_t d, double h, int kernel, int precision,
                                             double* out, float* grad_Y, double* grad_h, void* ws,
                                             size_t ws_bytes, void* stream) {
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (bad_exact_grad_prec(precision))
    return fail(DEANN_EINVAL, "precision must be DEANN_FP32 or DEANN_FP32_SPLIT");
  if (d > 128) return fail(DEANN_EUNSUPPORTED, "kde_exact_with_grad supports d <= 128");
  if (prepared && (st = check_prepared(prepared, prepared_bytes, n, d, DEANN_FP32)) != DEANN_OK)
    return st;
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_kde_bwd(nullptr, n, q, d, precision).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  KdeBwdPlan P = plan_kde_bwd(align_ws(ws), n, q, d, precision);
  record_last(P.cert.count, nullptr, q);
  SplitRows sp;
  const Prep pre = prepared ? prepared_of(prepared, n, d, DEANN_FP32) : Prep{};
  hipError_t e = prep_exact_grad(P, X, n, Y, q, d, precision, sp, s, prepared ? &pre : nullptr);
  if (e != hipSuccess) return hip_fail(e, "prep");
  TileProblem tp = make_problem(P.prep, n, q, DEANN_FP32, bwd_split_target(P.prep.dp));
  tp.map = make_tile_map(tp.qtiles, tp.splits, 1);
  e = launch_kde_backward(tp, X, Y, d, h, kernel, nullptr, P.gy_part, P.gh_part, grad_Y, nullptr,
                          s, timer_hook(1), out, grad_h, sp,
                          cert_args(P.cert, P.prep, sp.X ? P.dps + 4 : P.prep.dp, sp.X != nullptr));
  if (e != hipSuccess) return hip_fail(e, "kde value and gradient");
  return DEANN_OK;
}

extern "C" {

deann_status kde_exact_with_grad(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                        deann_kernel kernel, deann_precision precision, double* out, float* grad_Y, double* grad_h,
                        void* ws, size_t ws_bytes, void* stream) {
  return kde_exact_with_grad_impl(nullptr, 0, X, n, Y, q, d, h, kernel, precision, out, grad_Y,
                                  grad_h, ws, ws_bytes, stream);
}

deann_status kde_exact_with_grad_prepared(const void* prepared, size_t prepared_bytes,
                                          const float* X, int64_t n, const float* Y, int64_t q,
                                          int64_t d, double h, deann_kernel kernel,
                                          deann_precision precision, double* out, float* grad_Y,
                                          double* grad_h, void* ws, size_t ws_bytes,
                                          void* stream) {
  if (!prepared) return fail(DEANN_EINVAL, "prepared is NULL");
  return kde_exact_with_grad_impl(prepared, prepared_bytes, X, n, Y, q, d, h, kernel, precision,
                                  out, grad_Y, grad_h, ws, ws_bytes, stream);
}

}  // extern "C"

// ---- inverted-file index (Sec. 5) -------------------------------------------------
namespace {

constexpr int64_t kMaxClusters = 8192;       // cluster counters of one workgroup in LDS
constexpr int64_t kAssignBatch = 65536;      // rows per nearest-centroid k-NN call

int64_t ivf_cap(int64_t n, int64_t L) { return round_up(n + (BN - 1) * L, BN); }

// Most clusters one query inspects (n_probe, extended while they hold < k rows).
int64_t ivf_probe_cap(int64_t L, int64_t n_probe) {
  int64_t c = 2 * n_probe > n_probe + 64 ? 2 * n_probe : n_probe + 64;
  if (c > L) c = L;
  if (c > kMaxK) c = kMaxK;
  return c;
}

// Layout of the caller's index buffer.
struct IvfIndex {
  int32_t *off, *poff, *ids, *pids, *skipped;
  float* c;
  char* Xs;
  double* xnorm;
  float *xknorm, *xerr;
  uint32_t* err_max;
  int64_t cap, dp, bytes;
};

IvfIndex carve_index(void* base, int64_t n, int64_t d, int64_t L) {
  Carve cv(base);
  IvfIndex x{};
  x.cap = ivf_cap(n, L);
  x.dp = padded_d(d, DEANN_FP32);
  x.off = cv.take<int32_t>(L + 1);
  x.poff = cv.take<int32_t>(L + 1);
  x.ids = cv.take<int32_t>(n);
  x.pids = cv.take<int32_t>(x.cap);
  x.skipped = cv.take<int32_t>(1);
  x.c = cv.take<float>(d);
  x.Xs = cv.take<char>(x.cap * x.dp * 4);
  x.xnorm = cv.take<double>(x.cap);
  x.xknorm = cv.take<float>(x.cap);
  x.xerr = cv.take<float>(x.cap);
  x.err_max = cv.take<uint32_t>(2);
  x.bytes = cv.off + kAlign;
  return x;
}

struct IvfLayoutWs {
  int32_t *hist, *count;
  int64_t bytes;
};

IvfLayoutWs carve_layout_ws(Carve& cv, int64_t n, int64_t L) {
  IvfLayoutWs w{};
  w.hist = cv.take<int32_t>(ivf_hist_blocks(n) * L);
  w.count = cv.take<int32_t>(L);
  return w;
}

struct IvfBuildPlan {
  void* knn_ws;
  int64_t knn_bytes;
  float* C_tmp;
  IvfLayoutWs lw;
  int32_t *off, *ids, *skipped;
  int64_t bytes;
};

IvfBuildPlan plan_ivf_build(void* ws, int64_t n, int64_t d, int64_t L) {
  Carve cv(ws);
  IvfBuildPlan P{};
  const int64_t qb = n < kAssignBatch ? n : kAssignBatch;
  P.knn_bytes = plan_deann(nullptr, L, qb, d, 1, DEANN_FP32).bytes;
  P.knn_ws = cv.take<char>(P.knn_bytes);
  P.C_tmp = cv.take<float>(L * d);
  P.lw = carve_layout_ws(cv, n, L);
  P.off = cv.take<int32_t>(L + 1);
  P.ids = cv.take<int32_t>(n);
  P.skipped = cv.take<int32_t>(1);
  P.bytes = cv.off + kAlign;
  return P;
}

// assign[i] = the closest centroid of row i (exact k-NN with k = 1, in batches).
hipError_t assign_rows(void* knn_ws, const float* X, int64_t n, int64_t d, const float* C,
                       int64_t L, int32_t* assign, hipStream_t s) {
  for (int64_t r0 = 0; r0 < n; r0 += kAssignBatch) {
    const int64_t qb = n - r0 < kAssignBatch ? n - r0 : kAssignBatch;
    hipError_t e;
    if (L == 1) {   // the only centroid
      if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(assign + r0), qb, 0u, s)) != hipSuccess)
        return e;
      continue;
    }
    DeannPlan P = plan_deann(knn_ws, L, qb, d, 1, DEANN_FP32);
    P.kb.nn_work = assign + r0;
    const float* Xb = X + r0 * d;
    e = run_prep(P.prep, C, L, Xb, qb, d, DEANN_FP32, s);
    if (e != hipSuccess) return e;
    TileProblem tp = make_problem(P.prep, L, qb, DEANN_FP32, kKnnSplitTarget);
    TileProblem tc = make_problem(P.prep, L, qb, DEANN_FP32, kCollectSplitTarget);
    e = launch_knn(DEANN_FP32, tp, tc, P.kb, C, Xb, d, 1, 1.0, DEANN_GAUSSIAN, nullptr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct IvfCreatePlan {
  IvfLayoutWs lw;
  float* Xperm;
  double* cpart;
  int64_t bytes;
};

IvfCreatePlan plan_ivf_create(void* ws, int64_t n, int64_t d, int64_t L) {
  Carve cv(ws);
  IvfCreatePlan P{};
  P.lw = carve_layout_ws(cv, n, L);
  P.Xperm = cv.take<float>(ivf_cap(n, L) * d);
  P.cpart = cv.take<double>(kCenterRows * d);
  P.bytes = cv.off + kAlign;
  return P;
}

struct IvfQueryPlan {
  DeannPlan probe;        // k-NN of the queries among the centroids
  int32_t *order, *np_q;  // inspected clusters [q][kp] and their count [q]
  int64_t kp;
  char* Ys;
  double* ynorm;
  float *yknorm, *yerr;
  uint32_t* err_max;
  int32_t *pcount, *pfill, *pp, *pair_q, *pair_of, *lbase, *nparts;
  uint32_t* qthr;
  float *Yg, *ygk;
  KnnBuffers kb;
  int32_t* nn_internal;
  int64_t pcap, bytes;
};

IvfQueryPlan plan_ivf_query(void* ws, int64_t n, int64_t q, int64_t d, int64_t L, int64_t np,
                            int64_t k) {
  IvfQueryPlan P{};
  P.kp = ivf_probe_cap(L, np);
  P.probe = plan_deann(ws, L, q, d, P.kp, DEANN_FP32);
  Carve cv(ws);
  cv.off = P.probe.bytes;
  const int64_t dp = padded_d(d, DEANN_FP32), qp = round_up(q, BQ);
  P.order = cv.take<int32_t>(q * P.kp);
  P.np_q = cv.take<int32_t>(q > 0 ? q : 1);
  P.Ys = cv.take<char>(qp * dp * 4);
  P.ynorm = cv.take<double>(qp);
  P.yknorm = cv.take<float>(qp);
  P.yerr = cv.take<float>(qp);
  P.err_max = cv.take<uint32_t>(2);
  P.pcap = round_up(q * P.kp + (BN - 1) * L, BN);
  P.pcount = cv.take<int32_t>(L);
  P.pfill = cv.take<int32_t>(L + 1);
  P.pp = cv.take<int32_t>(L + 1);
  P.pair_q = cv.take<int32_t>(P.pcap);
  P.pair_of = cv.take<int32_t>(q * P.kp);
  P.lbase = cv.take<int32_t>(P.pcap / BN + 1);
  P.nparts = cv.take<int32_t>(2);
  P.qthr = cv.take<uint32_t>(q > 0 ? q : 1);
  P.Yg = cv.take<float>(P.pcap * dp);
  P.ygk = cv.take<float>(P.pcap);
  KnnBuffers& b = P.kb;
  b.K1 = knn_K1(k);
  b.cap1 = 256;
  while (b.cap1 < 2 * b.K1 + BN) b.cap1 <<= 1;
  b.cand = cv.take<uint64_t>(P.pcap * b.cap1);
  b.cand_cnt = cv.take<int32_t>(P.pcap);
  P.nn_internal = cv.take<int32_t>(q * (k > 0 ? k : 1));
  b.z1 = cv.take<double>(q > 0 ? q : 1);
  b.status = cv.take<int32_t>(q > 0 ? q : 1);
  b.thr2 = cv.take<float>(q > 0 ? q : 1);
  b.cand2 = cv.take<uint64_t>(q * kSortCapMax);
  b.cap2 = g_opt.knn_cap2;   // row stride of cand2 as well: within the carved rows
  b.cand2_cnt = cv.take<int32_t>(q > 0 ? q : 1);
  b.yerr = P.yerr;
  P.bytes = cv.off + kAlign;
  (void)n;
  return P;
}

}  // namespace

extern "C" {

size_t ivf_build_workspace(int64_t n, int64_t d, int64_t n_clusters) {
  if (n < 1 || d < 1 || n_clusters < 1 || n_clusters > n || n_clusters > kMaxClusters) return 0;
  return (size_t)plan_ivf_build(nullptr, n, d, n_clusters).bytes;
}

deann_status ivf_build(const float* X, int64_t n, int64_t d, int64_t n_clusters, int iters,
              float* centroids, int32_t* assign, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || d < 1) return fail(DEANN_EINVAL, "need n >= 1 and d >= 1");
  if (n >= (int64_t)1 << 31) return fail(DEANN_EINVAL, "n must be < 2^31");
  if (n_clusters < 1 || n_clusters > n)
    return fail(DEANN_EINVAL, "n_clusters must be in [1, n] (got %lld)", (long long)n_clusters);
  if (n_clusters > kMaxClusters)
    return fail(DEANN_EUNSUPPORTED, "n_clusters > %lld is not supported", (long long)kMaxClusters);
  if (iters < 0 || iters > 1000) return fail(DEANN_EINVAL, "iters must be in [0, 1000]");
  if (d > 4096) return fail(DEANN_EUNSUPPORTED, "d > 4096 is not supported");
  if (!X || !centroids || !assign) return fail(DEANN_EINVAL, "NULL array");
  const int64_t need = plan_ivf_build(nullptr, n, d, n_clusters).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IvfBuildPlan P = plan_ivf_build(align_ws(ws), n, d, n_clusters);
  hipError_t e = launch_kmeans_init(X, n, d, n_clusters, centroids, s);
  for (int it = 0; e == hipSuccess; ++it) {
    e = assign_rows(P.knn_ws, X, n, d, centroids, n_clusters, assign, s);
    if (e != hipSuccess || it == iters) break;
    e = launch_list_layout(assign, n, n_clusters, P.lw.hist, P.lw.count, P.off, nullptr, P.ids,
                           P.skipped, s);
    if (e != hipSuccess) break;
    e = launch_kmeans_mean(X, d, P.ids, P.off, n_clusters, centroids, P.C_tmp, s);
    if (e != hipSuccess) break;
    e = hipMemcpyAsync(centroids, P.C_tmp, (size_t)(n_clusters * d) * 4, hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return hip_fail(e, "ivf build");
  return DEANN_OK;
}

size_t ivf_index_bytes(int64_t n, int64_t d, int64_t n_clusters) {
  if (n < 1 || d < 1 || n_clusters < 1 || n_clusters > kMaxClusters) return 0;
  return (size_t)carve_index(nullptr, n, d, n_clusters).bytes;
}

size_t ivf_index_create_workspace(int64_t n, int64_t d, int64_t n_clusters) {
  if (n < 1 || d < 1 || n_clusters < 1 || n_clusters > kMaxClusters) return 0;
  return (size_t)plan_ivf_create(nullptr, n, d, n_clusters).bytes;
}

deann_status ivf_index_create(const float* X, int64_t n, int64_t d, const int32_t* assign,
                     int64_t n_clusters, void* index, size_t index_bytes, void* ws,
                     size_t ws_bytes, void* stream) {
  if (n < 1 || d < 1) return fail(DEANN_EINVAL, "need n >= 1 and d >= 1");
  if (n >= (int64_t)1 << 31) return fail(DEANN_EINVAL, "n must be < 2^31");
  if (n_clusters < 1) return fail(DEANN_EINVAL, "n_clusters must be >= 1");
  if (n_clusters > kMaxClusters)
    return fail(DEANN_EUNSUPPORTED, "n_clusters > %lld is not supported", (long long)kMaxClusters);
  if (d > 4096) return fail(DEANN_EUNSUPPORTED, "d > 4096 is not supported");
  if (!X || !assign || !index) return fail(DEANN_EINVAL, "NULL array");
  const int64_t need_i = carve_index(nullptr, n, d, n_clusters).bytes;
  if ((int64_t)index_bytes < need_i)
    return fail(DEANN_EWORKSPACE, "index buffer of %lld bytes needed", (long long)need_i);
  const int64_t need = plan_ivf_create(nullptr, n, d, n_clusters).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IvfIndex x = carve_index(align_ws(index), n, d, n_clusters);
  IvfCreatePlan P = plan_ivf_create(align_ws(ws), n, d, n_clusters);
  hipError_t e = launch_list_layout(assign, n, n_clusters, P.lw.hist, P.lw.count, x.off, x.poff,
                                    x.ids, x.skipped, s);
  if (e == hipSuccess)
    e = launch_list_tiles(X, d, x.ids, x.off, x.poff, n_clusters, x.cap, x.pids, P.Xperm, s);
  // the centring of the scan is the mean of the data rows
  const int64_t R = n < kCenterRows ? n : kCenterRows;
  if (e == hipSuccess) e = launch_center(X, n, d, P.cpart, R, x.c, s);
  if (e == hipSuccess) e = launch_fill_u32(x.err_max, 2, 0u, s);
  if (e == hipSuccess)
    e = launch_prep_rows_prec(DEANN_FP32, P.Xperm, x.cap, x.cap, d, x.dp, x.c, key_scale(x.dp),
                              x.Xs, x.xnorm, x.xknorm, x.xerr, x.err_max, s);
  if (e == hipSuccess) e = launch_empty_row_keys(x.pids, x.poff + n_clusters, x.cap, x.xknorm, s);
  if (e != hipSuccess) return hip_fail(e, "ivf index");
  return DEANN_OK;
}

size_t deann_ivf_query_workspace(int64_t n, int64_t q, int64_t d, int64_t n_clusters,
                                 int64_t n_probe, int64_t k, int64_t m) {
  (void)m;
  if (n < 1 || d < 1 || q < 0 || k < 0 || k > n || n_clusters < 1 || n_probe < 1 ||
      n_probe > n_clusters)
    return 0;
  return (size_t)plan_ivf_query(nullptr, n, q, d, n_clusters, n_probe, k).bytes;
}

deann_status deann_ivf_query(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                    const void* index, const float* centroids, int64_t n_clusters,
                    int64_t n_probe, double h, deann_kernel kernel, int64_t k, int64_t m, uint64_t seed,
                    uint64_t query_offset, double* out, int32_t* nn_idx, int32_t* sample_idx,
                    void* ws, size_t ws_bytes, void* stream) {
  deann_status st = check_common(X, n, Y, q, d, h, kernel);
  if (st != DEANN_OK) return st;
  if (k < 0 || k > n) return fail(DEANN_EINVAL, "k must be in [0, n] (got %lld)", (long long)k);
  if (m < 0) return fail(DEANN_EINVAL, "m must be >= 0 (got %lld)", (long long)m);
  if (k > kMaxK && k != n)
    return fail(DEANN_EUNSUPPORTED, "k = %lld: supported are k <= %lld and k = n", (long long)k,
                (long long)kMaxK);
  if (k > 0 && k < n && knn_K1(k) > 512)
    return fail(DEANN_EUNSUPPORTED, "k + knn_slack = %lld exceeds the 512 candidates of a list",
                (long long)(k + g_opt.knn_slack));
  if (d > 4096) return fail(DEANN_EUNSUPPORTED, "d > 4096 is not supported");
  if (n_clusters < 1 || n_clusters > kMaxClusters)
    return fail(DEANN_EINVAL, "n_clusters must be in [1, %lld]", (long long)kMaxClusters);
  if (n_probe < 1 || n_probe > n_clusters || n_probe > kMaxK)
    return fail(DEANN_EINVAL, "n_probe must be in [1, min(n_clusters, %lld)]", (long long)kMaxK);
  if (!index || !centroids) return fail(DEANN_EINVAL, "NULL index or centroids");
  if (q == 0) return DEANN_OK;
  if (!out) return fail(DEANN_EINVAL, "out is NULL");
  const int64_t need = plan_ivf_query(nullptr, n, q, d, n_clusters, n_probe, k).bytes;
  if (!ws || (int64_t)ws_bytes < need)
    return fail(DEANN_EWORKSPACE, "workspace of %lld bytes needed", (long long)need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IvfQueryPlan P = plan_ivf_query(align_ws(ws), n, q, d, n_clusters, n_probe, k);
  record_last(nullptr, nullptr, q);
  // the index buffer is read only
  IvfIndex x = carve_index(align_ws(const_cast<void*>(index)), n, d, n_clusters);
  P.kb.nn_work = nn_idx ? nn_idx : P.nn_internal;
  P.kb.xerr_max = x.err_max;
  hipError_t e = hipSuccess;
  if (k == n) {
    e = launch_knn_all(X, Y, n, q, d, h, kernel, P.kb.nn_work, P.kb.z1, s);
  } else if (k > 0) {
    // clusters to inspect: the kp closest centroids (exact k-NN), ordered by
    // distance; the query takes the shortest prefix of at least n_probe of
    // them that holds k rows
    int32_t* cand = P.probe.nn_internal;
    P.probe.kb.nn_work = cand;
    e = run_prep(P.probe.prep, centroids, n_clusters, Y, q, d, DEANN_FP32, s);
    if (e == hipSuccess) {
      TileProblem tp = make_problem(P.probe.prep, n_clusters, q, DEANN_FP32, kKnnSplitTarget);
      TileProblem tc = make_problem(P.probe.prep, n_clusters, q, DEANN_FP32, kCollectSplitTarget);
      if (P.kp == n_clusters)
        e = launch_knn_all(centroids, Y, n_clusters, q, d, h, kernel, cand, P.kb.z1, s);
      else
        e = launch_knn(DEANN_FP32, tp, tc, P.probe.kb, centroids, Y, d, P.kp, h, kernel,
                       nullptr, s);
    }
    if (e == hipSuccess)
      e = launch_probe_order(centroids, Y, q, d, cand, P.kp, x.off, n_probe, k, P.order, P.np_q,
                             s);
    const int32_t* probe = P.order;
    // the queries in the index's centring, then in (cluster, query) pair order
    const int64_t dp = x.dp, qp = round_up(q, BQ);
    if (e == hipSuccess) e = launch_fill_u32(P.err_max, 2, 0u, s);
    if (e == hipSuccess)
      e = launch_prep_rows_prec(DEANN_FP32, Y, q, qp, d, dp, x.c, key_scale(dp), P.Ys, P.ynorm,
                                P.yknorm, P.yerr, P.err_max + 1, s);
    if (e == hipSuccess)
      e = launch_pairs(probe, q, P.kp, P.np_q, n_clusters, P.pcount, P.pfill, P.pp, P.pair_q,
                       P.pair_of, P.pcap, reinterpret_cast<const float*>(P.Ys), P.yknorm, dp,
                       P.Yg, P.ygk, s);
    // long sweeps in parts: each list slot of the workspace holds one part
    if (e == hipSuccess)
      e = launch_pair_parts(P.pp, x.poff, n_clusters, P.pcap / BN, kIvfPartTarget, P.lbase,
                            P.nparts, s);
    if (e == hipSuccess) {
      IvfTiles t{reinterpret_cast<const char*>(P.Yg), x.Xs, dp * 4, (int)(dp * 4 / CHUNK_BYTES),
                 P.ygk, x.xknorm, P.pp, x.poff, n_clusters, P.pair_q, x.pids, P.lbase,
                 P.nparts, P.qthr};
      IvfRefine v{probe, P.kp, P.np_q, P.pair_of, x.off, x.ids, x.pids, P.lbase, P.qthr};
      e = launch_ivf_knn(t, P.pcap, P.kb, v, X, Y, n, q, d, k, h, kernel, nullptr, s);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "ivf neighbours");
  e = launch_sample(X, Y, n, q, d, h, kernel, k, m, seed, query_offset, 0, 0, 0, P.kb.nn_work,
                    P.kb.z1, out, sample_idx, s);
  if (e != hipSuccess) return hip_fail(e, "sample");
  return DEANN_OK;
}

}  // extern "C"
