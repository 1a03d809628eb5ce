/*
 * deann.h - C ABI of the DEANN query path on one AMD Instinct MI355X (gfx950).
 *
 * Paper: M. Karppa, M. Aumueller, R. Pagh, "DEANN: Speeding up Kernel-Density
 * Estimation using Approximate Nearest Neighbor Search", arXiv 2107.02736.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer, row-major and contiguous, owned
 *    by the caller.  The library never frees, keeps or modifies X and Y.
 *  - X[n, d] is the dataset, Y[q, d] the queries, both float32.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL for the
 *    default stream) and is asynchronous: outputs are valid once the stream has
 *    been synchronised.  No call synchronises the stream.
 *  - Scratch memory is supplied by the caller through (ws, ws_bytes); query the
 *    required size with the matching *_workspace function.  Its contents on
 *    entry are irrelevant.
 *  - Arguments are validated on the host before anything is launched; a
 *    violation returns DEANN_EINVAL (or DEANN_EWORKSPACE, DEANN_EUNSUPPORTED)
 *    and writes nothing.  A HIP launch failure returns DEANN_EHIP.
 *    deann_last_error() gives a message for the last non-OK status of the
 *    calling thread.
 *  - Calls that share a workspace must not overlap in time; calls with
 *    separate workspaces on different streams are independent.
 *  - Results are bitwise reproducible for identical inputs (no floating-point
 *    atomics; every reduction has a fixed order).
 */
#ifndef DEANN_H
#define DEANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Kernels: Gaussian exp(-||x-y||^2 / (2 h^2)) (Eq. (2)) and exponential
 * exp(-||x-y|| / h) (Sec. 1).  Both unnormalised, so the KDE lies in [0, 1]. */
typedef enum { DEANN_GAUSSIAN = 0, DEANN_EXPONENTIAL = 1 } deann_kernel;

/* Precision of the distance tiles on MFMA (FP32 accumulation in every case).
 * Values that reach an estimate in deann_query are always recomputed exactly
 * in FP64 from the float32 inputs, whatever the precision here. */
typedef enum { DEANN_FP32 = 0, DEANN_BF16 = 1, DEANN_FP16 = 2, DEANN_FP32_SPLIT = 3 } deann_precision;

typedef enum {
  DEANN_OK = 0,
  DEANN_EINVAL = 1,       /* invalid argument (size, pointer, h, k, m, enum) */
  DEANN_EWORKSPACE = 2,   /* ws_bytes smaller than the queried size, or ws NULL */
  DEANN_EHIP = 3,         /* a HIP launch failed */
  DEANN_EUNSUPPORTED = 4  /* valid but outside what this build implements */
} deann_status;

/* ---------------------------------------------------------------------------
 * Options of the calls a host thread makes (thread-local; the defaults hold
 * until deann_set_options is called on that thread).  Workspace sizes depend
 * on knn_slack: query them after setting the options.
 * ------------------------------------------------------------------------- */
typedef struct {
  /* float32-operand exact KDE (kde_exact with DEANN_FP32 or DEANN_FP32_SPLIT,
   * kde_exact_backward, kde_exact_with_grad): every query carries a bound of
   * the relative error of its kernel sum, from the sums of K and K^2 of the
   * tile sweep (probabilistic: roundings taken as independent, failure
   * probability below 3e-8 per query); a query whose bound exceeds rel_tol is
   * re-evaluated exactly (FP64 differences of the float32 rows), unless its
   * value is certainly below value_floor.  rel_tol in [1e-7, 1], default
   * 1e-5; value_floor >= 0, default 1e-16 (the paper reports no relative
   * error below 1e-16); value_floor = 0 re-evaluates every such query. */
  double rel_tol;
  double value_floor;
  /* exact k-NN: each candidate list keeps K1 = the power of two >= max(k +
   * knn_slack, 64) smallest keys (k + knn_slack <= 512; default 16); a query
   * whose second pass collects more than knn_cap2 rows (in [1, 4096], default
   * 4096) is scanned exhaustively in FP64.  Neither changes any result. */
  int64_t knn_slack;
  int64_t knn_cap2;
  /* 1 (default): rows are centred on the column mean of X before the
   * distance tiles (the KDE is translation invariant; centring shrinks the
   * norms the GEMM identity cancels); 0: raw coordinates. */
  int32_t center;
  /* 16-bit k-NN scans (DEANN_BF16, DEANN_FP16): the candidate pass that seeds
   * the distance bound of the second pass reads every knn_seed_stride-th data
   * tile of 128 rows (in [1, 64], default 4; lowered so that it reads at least
   * 16 tiles, if there are as many).  A larger
   * stride makes that pass cheaper and the bound looser (more rows for the
   * second pass to collect and sort); it changes no result. */
  int32_t knn_seed_stride;
} deann_options;

void deann_default_options(deann_options* opt);
deann_status deann_get_options(deann_options* opt);
/* DEANN_EINVAL (options unchanged) if a field is out of range. */
deann_status deann_set_options(const deann_options* opt);

/* Counts of the last call made on this thread (measurement and tests): the
 * queries the exact KDE re-evaluated in FP64, the queries of the k-NN that
 * needed its second pass and those scanned exhaustively; -1 where the call
 * had no such step.  Synchronises `stream` and copies counters from that
 * call's workspace, which must still be allocated. */
typedef struct {
  int64_t exact_refined;
  int64_t knn_second_pass;
  int64_t knn_exhaustive;
} deann_stats;
deann_status deann_last_stats(deann_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * Exact KDE, Eq. (1):  out[j] = (1/n) sum_i K_h(x_i, y_j).
 *
 * Distances use the identity ||x-y||^2 = ||x||^2 + ||y||^2 - 2<x,y> of App. F
 * (with both sides centred on the column mean of X) and the kernel sum is
 * fused into the MFMA tile; per-split sums are combined in FP64.
 *   precision  DEANN_FP32, DEANN_BF16 or DEANN_FP16 operands of the GEMM, or
 *              DEANN_FP32_SPLIT: float32-accurate dot products from three
 *              bfloat16 parts of every float32 value on BF16 MFMAs (six
 *              products per element); the float32 forms are certified per
 *              query (deann_options.rel_tol) like DEANN_FP32.
 *   out        [q] float64.
 * Requirements: n >= 1, d >= 1, q >= 0 (q = 0 is a no-op), h finite and > 0,
 * n and q < 2^31.
 * ------------------------------------------------------------------------- */
size_t kde_exact_workspace(int64_t n, int64_t q, int64_t d, deann_precision precision);
deann_status kde_exact(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
              deann_kernel kernel, deann_precision precision, double* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * DEANN estimate, Algorithm 1, with an exact k-NN in place of the ANN:
 *   X1  = the k nearest rows of X to y (exact; ties to the lower index),
 *   Z1  = sum over X1 of K_h,  S = m draws with repetition from X2 = X \ X1,
 *   Z2  = sum over S of K_h,   out = (Z1 + ((n-k)/m) Z2) / n,
 * which is the (k/n) Z1/k + ((n-k)/n) Z2/m of Algorithm 1, valid also for
 * k = 0 (random sampling) and m = 0 (far points dropped, biased).  With k = n
 * the result is the exact KDE and no draw is made.
 *
 * Draw j of query i is word (j mod 4) of Philox4x64-10 (Salmon et al., SC'11)
 * with key (seed, 0) and counter (j div 4, query_offset + i, word2, 0); the rank
 * r = floor(u (n-k) / 2^64) selects the r-th smallest index of X2.  Splitting a
 * query batch and passing query_offset reproduces the same draws.
 *
 *   precision   operand precision of the k-NN distance scan.  The neighbour set
 *               is exact in every precision: candidates are ranked by a rigorous
 *               lower bound and re-evaluated in FP64; a query whose candidate
 *               set cannot be certified is rescanned.
 *   out         [q] float64 estimates.
 *   nn_idx      [q, k] int32, neighbour indices sorted ascending, or NULL.
 *   sample_idx  [q, m] int32, drawn indices in draw order (-1 when X2 is
 *               empty), or NULL.  Both are needed by deann_query_backward.
 * Requirements: as kde_exact, plus 0 <= k <= n with k <= 496 or k == n,
 * m >= 0, n < 2^31.
 * ------------------------------------------------------------------------- */
size_t deann_query_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                             deann_precision precision);
deann_status deann_query(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                deann_kernel kernel, int64_t k, int64_t m, uint64_t seed, uint64_t query_offset,
                uint64_t word2, deann_precision precision, double* out, int32_t* nn_idx, int32_t* sample_idx,
                void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * DEANN estimates with their derivatives (Algorithm 1 and its adjoint with the
 * index sets held fixed, as deann_query_backward): the same neighbours, draws
 * and sample_idx as deann_query with the same arguments, and
 *   out[j]      the estimate, as deann_query up to the order of its FP64 sum
 *               (about 1e-16 relative)                        [q] float64
 *   grad_Y[j]   d out[j] / d y_j                               [q, d] float32, or NULL
 *   grad_h[j]   d out[j] / d h                                 [q] float64, or NULL
 * i.e. deann_query followed by deann_query_backward with grad_out = 1, except
 * that the h derivative is returned per query; the k + m rows of a query are
 * gathered once for all three (d % 4 == 0, 16-byte aligned X and Y, d <= 2048;
 * other shapes gather twice, with the same results).  nn_idx, sample_idx may
 * be NULL.  Requirements: as deann_query, plus d <= 2048.
 * ------------------------------------------------------------------------- */
size_t deann_query_with_grad_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                                       deann_precision precision);
deann_status deann_query_with_grad(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                                   double h, deann_kernel kernel, int64_t k, int64_t m,
                                   uint64_t seed, uint64_t query_offset, uint64_t word2,
                                   deann_precision precision, double* out, float* grad_Y,
                                   double* grad_h, int32_t* nn_idx, int32_t* sample_idx, void* ws,
                                   size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Prepared data set: the preprocessing of X that every call above performs
 * (Algorithm 1 fits its estimator to X once and then answers queries; App. F
 * keeps the row norms) -- X centred by its column mean (deann_options.center),
 * stored in the scan precision with its norms and rounding bounds -- done once
 * into caller-owned device memory and reused by the *_prepared calls, which
 * then prepare only the queries.
 *   deann_prepared_bytes  size for (n, d, precision); 0 for invalid arguments.
 *   deann_prepare         fills `prepared` (prepared_bytes at least that size)
 *                         from X[n, d]; asynchronous like every call.
 *   *_prepared            as kde_exact, kde_exact_backward, kde_exact_with_grad,
 *                         deann_query, deann_query_with_grad with
 *                         the same arguments (X is still read: the exact
 *                         re-evaluations and the gathers use its float32 rows),
 *                         plus the prepared set and its size.  Results are
 *                         bitwise those of the unprepared call.
 * The prepared set must come from deann_prepare with the same X, n, d and
 * precision (DEANN_FP32 for kde_exact_backward_prepared and
 * kde_exact_with_grad_prepared, and for kde_exact_prepared with
 * DEANN_FP32_SPLIT) and the
 * same centring option; only its size is checked (DEANN_EWORKSPACE when it is
 * too small for n, d and the precision).  It is read, never written, by the
 * query calls, so several streams may share it; the workspaces stay per call.
 * ------------------------------------------------------------------------- */
size_t deann_prepared_bytes(int64_t n, int64_t d, deann_precision precision);
deann_status deann_prepare(const float* X, int64_t n, int64_t d, deann_precision precision,
                           void* prepared, size_t prepared_bytes, void* stream);
deann_status kde_exact_prepared(const void* prepared, size_t prepared_bytes, const float* X,
                                int64_t n, const float* Y, int64_t q, int64_t d, double h,
                                deann_kernel kernel, deann_precision precision, double* out,
                                void* ws, size_t ws_bytes, void* stream);
deann_status deann_query_prepared(const void* prepared, size_t prepared_bytes, const float* X,
                                  int64_t n, const float* Y, int64_t q, int64_t d, double h,
                                  deann_kernel kernel, int64_t k, int64_t m, uint64_t seed,
                                  uint64_t query_offset, uint64_t word2,
                                  deann_precision precision, double* out, int32_t* nn_idx,
                                  int32_t* sample_idx, void* ws, size_t ws_bytes, void* stream);
deann_status kde_exact_backward_prepared(const void* prepared, size_t prepared_bytes,
                                         const float* X, int64_t n, const float* Y, int64_t q,
                                         int64_t d, double h, deann_kernel kernel,
                                         deann_precision precision, const double* grad_out,
                                         float* grad_Y, double* grad_h, void* ws,
                                         size_t ws_bytes, void* stream);
deann_status kde_exact_with_grad_prepared(const void* prepared, size_t prepared_bytes,
                                          const float* X, int64_t n, const float* Y, int64_t q,
                                          int64_t d, double h, deann_kernel kernel,
                                          deann_precision precision, double* out, float* grad_Y,
                                          double* grad_h, void* ws, size_t ws_bytes,
                                          void* stream);
deann_status deann_query_with_grad_prepared(const void* prepared, size_t prepared_bytes,
                                            const float* X, int64_t n, const float* Y, int64_t q,
                                            int64_t d, double h, deann_kernel kernel, int64_t k,
                                            int64_t m, uint64_t seed, uint64_t query_offset,
                                            uint64_t word2, deann_precision precision,
                                            double* out, float* grad_Y, double* grad_h,
                                            int32_t* nn_idx, int32_t* sample_idx, void* ws,
                                            size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * DEANN with permuted random sampling (DEANNP; App. G, Algorithm 2): as
 * deann_query, but the sample of query i is the block of the data's permuted
 * order that starts at the running index l_i = (start + i m) mod n, with the
 * query's neighbours skipped: m distinct rows of X2, without replacement.
 * The permutation is keyed by `seed`: a balanced 4-round Feistel network on
 * b-bit words (b the smallest even number >= 2 with 2^b >= n) whose round
 * function is word 0 of Philox4x64-10 with key (seed, 1) and counter
 * (half, round, 0, 0), restricted to [n] by cycle walking.  Passing start +
 * i0 m for a batch that begins at query i0 reproduces the same samples.
 *   sample_idx  [q, m] int32 rows in block order (or NULL); deann_query_backward
 *               accepts them unchanged.
 * Requirements: as deann_query, plus m <= n - k when k < n.
 * ------------------------------------------------------------------------- */
size_t deann_query_permuted_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m,
                                      deann_precision precision);
deann_status deann_query_permuted(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                         double h, deann_kernel kernel, int64_t k, int64_t m, uint64_t seed,
                         uint64_t start, deann_precision precision, double* out, int32_t* nn_idx,
                         int32_t* sample_idx, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Permuted random sampling with the preprocessing of Algorithm 2 (App. G) as
 * written: a permuted copy X' of the data, x'_i = x_pi(i), built once, from
 * which each query reads its block of positions contiguously.
 *   deann_perm_index_bytes   size of the index for n rows of width d (0 on bad
 *                            sizes): pi[n] and its inverse (int32) and X'
 *                            [n][d] float32, n d 4 + 8 n bytes and alignment.
 *   deann_perm_index_create  fills a caller-owned device buffer of at least
 *                            that size with the permutation keyed by `seed`
 *                            (the one deann_query_permuted evaluates on the
 *                            fly) and X'.  X must stay unchanged while the
 *                            index is used; the library keeps no pointer.
 *   deann_query_permuted_index  deann_query_permuted with that index: the same
 *                            neighbours, sample indices (rows of X) and
 *                            estimates bit for bit, for the seed the index was
 *                            made with and the given running index `start`;
 *                            the neighbours' positions come from pi's inverse
 *                            and the block's rows from X' (coalesced).  The
 *                            workspace is that of deann_query.
 * Requirements: as deann_query_permuted; index_bytes at least
 * deann_perm_index_bytes(n, d), else DEANN_EINVAL (query) or DEANN_EWORKSPACE
 * (create).
 * ------------------------------------------------------------------------- */
size_t deann_perm_index_bytes(int64_t n, int64_t d);
deann_status deann_perm_index_create(const float* X, int64_t n, int64_t d, uint64_t seed,
                                     void* index, size_t index_bytes, void* stream);
deann_status deann_query_permuted_index(const float* X, int64_t n, const float* Y, int64_t q,
                                        int64_t d, double h, deann_kernel kernel, int64_t k,
                                        int64_t m, const void* index, size_t index_bytes,
                                        uint64_t start, deann_precision precision, double* out,
                                        int32_t* nn_idx, int32_t* sample_idx, void* ws,
                                        size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Adjoint of deann_query with the index sets held fixed (the selection is
 * piecewise constant in y and h, so this is the derivative almost everywhere):
 *   grad_Y[j] = grad_out[j] * d out[j] / d y_j          [q, d] float32, or NULL
 *   grad_h    = sum_j grad_out[j] * d out[j] / d h      [1] float64, or NULL
 * Gaussian: dK/dy = K (x-y)/h^2, dK/dh = K r^2/h^3; exponential:
 * dK/dy = K (x-y)/(h r) (0 at r = 0), dK/dh = K r/h^2, with r = ||x-y||.
 * nn_idx and sample_idx are the outputs of the forward call with the same
 * (n, k, m).  Rows are gathered again and distances recomputed in FP64.
 * ------------------------------------------------------------------------- */
size_t deann_query_backward_workspace(int64_t n, int64_t q, int64_t d, int64_t k, int64_t m);
deann_status deann_query_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                         double h, deann_kernel kernel, int64_t k, int64_t m, const int32_t* nn_idx,
                         const int32_t* sample_idx, const double* grad_out, float* grad_Y,
                         double* grad_h, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same adjoint
 * as deann_query_backward, with the same arguments, kernels and results bit
 * for bit, but with no workspace.  Its per-query scratch (the dK/dh terms,
 * DEANN_NOALLOC_MAX_Q doubles = 8 MiB) is a device array of the library; each
 * GPU the library runs on holds its own copy from the first call on that
 * device until the process ends.  The entry point allocates nothing and frees
 * nothing.  `stream` must belong to the current device.
 *   q > DEANN_NOALLOC_MAX_Q  -> DEANN_EUNSUPPORTED (nothing launched).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams or host threads) race and must be ordered by the
 * caller.  Each call writes every entry it reads, so a call never sees the
 * contents a previous call left.
 * ------------------------------------------------------------------------- */
#define DEANN_NOALLOC_MAX_Q (1 << 20)
deann_status deann_query_backward_noalloc(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                                 double h, deann_kernel kernel, int64_t k, int64_t m,
                                 const int32_t* nn_idx, const int32_t* sample_idx,
                                 const double* grad_out, float* grad_Y, double* grad_h,
                                 void* stream);

/* ---------------------------------------------------------------------------
 * Adjoint of kde_exact (d <= 128):
 *   grad_Y[j] = grad_out[j] * (1/n) sum_i dK/dy (x_i, y_j),   [q, d] or NULL
 *   grad_h    = sum_j grad_out[j] * (1/n) sum_i dK/dh,        [1] or NULL.
 * The distance tiles are recomputed on MFMA, never stored.  precision:
 * DEANN_FP32 (float32 MFMAs) or DEANN_FP32_SPLIT (the distance product from
 * three-part bfloat16 operands as in kde_exact; the weighted sum W X on float32
 * MFMAs either way).
 * ------------------------------------------------------------------------- */
size_t kde_exact_backward_workspace(int64_t n, int64_t q, int64_t d, deann_precision precision);
deann_status kde_exact_backward(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                       deann_kernel kernel, deann_precision precision, const double* grad_out, float* grad_Y,
                       double* grad_h, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Exact KDE with its derivatives in one pass over the distance tiles (d <= 128;
 * precision DEANN_FP32 or DEANN_FP32_SPLIT as for kde_exact_backward), for
 * callers that need both (mean shift, fitting h):
 *   out[j]      = (1/n) sum_i K_h(x_i, y_j)                [q] float64
 *   grad_Y[j]   = d out[j] / d y_j                          [q, d] float32, or NULL
 *   grad_h[j]   = d out[j] / d h                            [q] float64, or NULL
 * i.e. kde_exact, and kde_exact_backward with grad_out = 1 except that the h
 * derivative is returned per query.  Costs one kde_exact_backward.
 * ------------------------------------------------------------------------- */
size_t kde_exact_with_grad_workspace(int64_t n, int64_t q, int64_t d, deann_precision precision);
deann_status kde_exact_with_grad(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
                        deann_kernel kernel, deann_precision precision, double* out, float* grad_Y, double* grad_h,
                        void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Near/far form of the exact KDE (derived from Algorithm 1: the near part is
 * Z1 over the k nearest rows X1, the far part is summed over all of X2 = X \ X1
 * instead of being sampled):
 *   out[j] = (1/n) (Z1_j + sum over X2 of K16_h(x_i, y_j)),
 * where Z1_j is computed in FP64 from the float32 rows and K16 is the kernel
 * value of kde_exact with 16-bit operands (precision DEANN_BF16 or DEANN_FP16),
 * so only the far rows carry the 16-bit operand error.  k = 0 gives
 * kde_exact with that precision, k = n the exact FP64 sum.
 *   nn_in   [q, k] int32 neighbour lists to use as X1 (distinct rows of [0, n)
 *           per query, any order; entries outside [0, n) are left out of both
 *           parts, repeated rows make Z1 count them again), e.g. the nn_idx
 *           of deann_query; NULL to compute the exact k nearest rows as
 *           deann_query does (then k <= 496 or k = n).
 *   out     [q] float64.
 *   nn_idx  [q, k] int32, the neighbour lists used (sorted ascending when
 *           computed here, a copy of nn_in otherwise), or NULL.
 * Requirements: as kde_exact, plus 0 <= k <= n, d <= 4096 when k > 0 and
 * q k < 2^31 when 0 < k < n.
 * ------------------------------------------------------------------------- */
size_t kde_hybrid_workspace(int64_t n, int64_t q, int64_t d, int64_t k, deann_precision precision);
deann_status kde_hybrid(const float* X, int64_t n, const float* Y, int64_t q, int64_t d, double h,
               deann_kernel kernel, int64_t k, deann_precision precision, const int32_t* nn_in, double* out,
               int32_t* nn_idx, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Inverted-file index: the approximate nearest neighbours of the experiments
 * (Sec. 5).  k-means over the data gives n_clusters centroids (the paper's
 * n_l); each row belongs to its closest centroid; a query inspects every row
 * of its n_probe closest centroids (the paper's n_q).  The DEANN estimate of
 * Algorithm 1 stays unbiased for any neighbour set, so these neighbours
 * replace the exact ones unchanged.
 *
 * ivf_build: Lloyd's k-means.  centroids[n_clusters, d] (float32, output) start
 *   as the rows floor(l n / n_clusters); each of `iters` steps assigns every row
 *   to its closest centroid (exact order (||c - x||^2, l), ties to the lower l)
 *   and replaces each centroid by the mean of its rows (FP64 sums in a fixed
 *   order, rounded once to float32; a centroid without rows stays).  assign[n] (int32,
 *   output) is the closest final centroid of every row.
 *   Requirements: 1 <= n_clusters <= min(n, 8192), 0 <= iters <= 1000, d <= 4096.
 *
 * ivf_index_create: lays the rows out by cluster in the caller's index buffer
 *   (ivf_index_bytes bytes, opaque, device memory): members in row order, each
 *   cluster padded to whole 128-row tiles, the rows centred and prepared for
 *   the FP32 tile scan.  assign[n] may come from ivf_build or from anywhere
 *   else; rows whose id is outside [0, n_clusters) are left out of the index.
 *   The index stays valid as long as X is unchanged; deann_ivf_query only
 *   reads it.
 *
 * deann_ivf_query: DEANN with the index's neighbours.  For query j: its
 *   clusters in the exact order (||c - y||^2, l); it inspects the n_probe
 *   closest, and while these hold fewer than k rows the next closest as well,
 *   up to min(n_clusters, max(2 n_probe, n_probe + 64), 496) clusters in all;
 *   the neighbours are the k nearest rows among their members (exact order
 *   (||x - y||^2, i), found by an FP32 MFMA scan of those clusters with
 *   certified lower-bound keys and an FP64 refinement).  If even the most
 *   clusters allowed hold fewer than k rows, the exact k nearest rows of all
 *   of X are used.  Sampling, the estimate and the
 *   outputs (out, nn_idx sorted by index, sample_idx) are those of deann_query
 *   with the same seed and query_offset; deann_query_backward accepts the
 *   indices unchanged.  centroids and n_clusters must be those the index was
 *   made with; 1 <= n_probe <= min(n_clusters, 496); k <= 496 or k = n.
 * ------------------------------------------------------------------------- */
size_t ivf_build_workspace(int64_t n, int64_t d, int64_t n_clusters);
deann_status ivf_build(const float* X, int64_t n, int64_t d, int64_t n_clusters, int iters,
              float* centroids, int32_t* assign, void* ws, size_t ws_bytes, void* stream);
size_t ivf_index_bytes(int64_t n, int64_t d, int64_t n_clusters);
size_t ivf_index_create_workspace(int64_t n, int64_t d, int64_t n_clusters);
deann_status ivf_index_create(const float* X, int64_t n, int64_t d, const int32_t* assign,
                     int64_t n_clusters, void* index, size_t index_bytes, void* ws,
                     size_t ws_bytes, void* stream);
size_t deann_ivf_query_workspace(int64_t n, int64_t q, int64_t d, int64_t n_clusters,
                                 int64_t n_probe, int64_t k, int64_t m);
deann_status deann_ivf_query(const float* X, int64_t n, const float* Y, int64_t q, int64_t d,
                    const void* index, const float* centroids, int64_t n_clusters,
                    int64_t n_probe, double h, deann_kernel kernel, int64_t k, int64_t m, uint64_t seed,
                    uint64_t query_offset, double* out, int32_t* nn_idx, int32_t* sample_idx,
                    void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Gaussian mean-shift step (the application the paper cites for density
 * gradients): Y_out[j] = Y[j] + h^2 grad_Y[j] / density[j], i.e. the
 * kernel-weighted mean of the rows when grad_Y and density come from
 * kde_exact_with_grad (or the DEANN estimate and its adjoint with
 * grad_out = 1).  Y, grad_Y, Y_out [q, d] float32 (Y_out may alias Y),
 * density [q] float64; a query with density 0 keeps its point.
 * ------------------------------------------------------------------------- */
deann_status mean_shift_update(const float* Y, const float* grad_Y, const double* density, int64_t q,
                      int64_t d, double h, float* Y_out, void* stream);

/* Message for the last non-OK status returned on the calling thread. */
const char* deann_last_error(void);

/* ---------------------------------------------------------------------------
 * Kernel timing, for measurement tools only (no effect on any result).
 * deann_kernel_timing(capacity): capacity in [1, 4096] makes the calling thread
 * record a pair of HIP events on the call's stream around the dense tile
 * kernel of each following call, for up to `capacity` calls per site:
 *   site 0 = kde_exact, site 1 = kde_exact_backward and kde_exact_with_grad,
 *   site 2 = the 16-bit tile sweep of kde_hybrid.
 * Recording happens only while a site has unread slots left.  capacity = 0
 * stops and releases the events (also done before a new capacity is set).
 * deann_kernel_times(site, ms, max_count): waits for the recorded events,
 * writes up to max_count durations in milliseconds to the host array ms (in
 * call order), frees the site's slots and returns the count, or -1 on error.
 * ------------------------------------------------------------------------- */
deann_status deann_kernel_timing(int capacity);
int deann_kernel_times(int site, float* ms, int max_count);

#ifdef __cplusplus
}
#endif
#endif /* DEANN_H */
