// Host-side launch interface of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace deann {

// Geometry of one (queries x data) tile sweep over the prepared operands.
struct TileProblem {
  const char* Ys;        // prepared queries  [qp][dp] in the scan type
  const char* Xs;        // prepared data     [np][dp]
  int64_t ld_bytes;      // row stride of Ys and Xs in bytes (multiple of 128)
  int nchunks;           // ld_bytes / 128
  const double* ynorm;   // ||y~||^2          [qp]
  const double* xnorm;   // ||x~||^2          [np]
  const float* yknorm;   // scaled norms for lower-bound keys [qp]
  const float* xknorm;   //                                   [np]
  int64_t n, q;          // true sizes
  int64_t np, qp;        // padded to multiples of 128
  int64_t qtiles, ntiles, splits;
  TileMap map;           // workgroup -> (query tile, split), see common.h
  int64_t tstride;       // sweep tile t is data tile t * tstride (1 but for the seed pass)
};

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, int64_t count, hipStream_t s);
// Largest of count non-negative floats, as float bits, into *out (atomic max:
// *out must hold a lower value first).
hipError_t launch_max_u32(const float* v, int64_t count, uint32_t* out, hipStream_t s);
hipError_t launch_center(const float* X, int64_t n, int64_t d, double* part, int64_t R, float* c,
                         hipStream_t s);
hipError_t launch_prep_rows_prec(int prec, const float* src, int64_t rows, int64_t rows_padded,
                                 int64_t d, int64_t dp, const float* c, double a_scale, void* dst,
                                 double* norm, float* knorm, float* err, uint32_t* err_max,
                                 hipStream_t s);

// Three bfloat16 planes per prepared float32 row (see prep.hip), dps >= dp32.
hipError_t launch_split_rows(const float* src, int64_t rows, int64_t dp32, int64_t dps,
                             void* dst, hipStream_t s);

// Optional pair of events recorded around a dense tile kernel (both null: none).
struct TimingHook {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Per-query accuracy certificate of the float32-operand sweeps (cert.hip): the
// sweeps write part; the reduction lists the queries whose error bound exceeds
// tau (and whose value is not certainly below floor) for an exact FP64
// re-evaluation.  fb_count must be zero before the reduction.
struct CertArgs {
  float2* part;            // [splits][qp] per split: sum of K^2, and (Gaussian) the sum of
                           // K times its exponent -log2 K or (exponential) the largest K
  const uint32_t* xnmax;   // float bits of the largest scaled data norm ||x~||^2 (1 - a)
  double a_scale;          // that scaling a
  int cd;                  // roundings of one dot product (its accumulation length)
  double tau;              // relative error bound of a certified query
  double floor;            // values certainly below it are not re-evaluated
  int32_t* fb_ids;         // [q] queries to re-evaluate
  int32_t* fb_count;       // [1]
  double sys;              // systematic dot-product error in units of u N per pair (the
                           // bfloat16 MFMA sums a group of eight products in a
                           // truncated register before rounding it into C: 2 for the
                           // three-part bfloat16 form, 0 for float32 MFMAs)
  float* pk;               // [splits][qp] per split: sum of K N (same units as pn), written
                           // by the split engine of the generic tile kernel only; it
                           // replaces the bias term sys u N by the pairs' own N
  float* pn;               // [splits][qp] per split: sum of (K N)^2 with N = ||x~||^2 +
                           // ||y~||^2 of the pair (Gaussian: times (L log2 e)^2), written by
                           // the generic float32 tile kernel only; null for the other sweeps
};

// Fixed-order sum of the float32 sweep's partials into out (Gaussian query
// factor and 1/n applied), the certificate of every query and the list of
// those to re-evaluate (clears *ca.fb_count first).
hipError_t launch_kde_reduce_cert(const double* partial, int64_t splits, int64_t qp, int64_t q,
                                  int64_t n, const double* ynorm, float Lf, int kern,
                                  const CertArgs& ca, double* out, hipStream_t s);
// Row splits of the exact re-evaluation for n data rows.
int64_t direct_splits(int64_t n);
// Exact FP64 value of the listed queries (ids[0 .. *count)): part [splits][q]
// scratch; overwrites out[ids[i]].
hipError_t launch_kde_direct(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                             double h, int kern, const int32_t* ids, const int32_t* count,
                             int64_t splits, double* part, double* out, hipStream_t s);
// Exact FP64 value, gradient and per-query d/dh of the listed queries (d <= 128):
// pval, pgh [splits][q] and pG [splits][q][ldg] scratch; overwrites the
// entries of grad_Y, ghq and mu (each may be NULL) of the listed queries.
// cap: entries of each scratch array (pval, pgh; pG holds cap * ldg), at least q
hipError_t launch_kde_direct_grad(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                  double h, int kern, const int32_t* ids, const int32_t* count,
                                  int64_t cap, double* pval, double* pgh, double* pG,
                                  int64_t ldg, const double* grad_out, float* grad_Y, double* ghq,
                                  double* mu, hipStream_t s);

// Float32 operands: the sweep, the reduction with the certificate (ca), and
// the exact re-evaluation of the listed queries from X and Y (fb_part:
// [direct_splits(n)][q] scratch).  16-bit operands: ca is not used.
hipError_t launch_kde_exact(int prec, const TileProblem& p, int kern, double h, double* partial,
                            double* out, hipStream_t s, TimingHook th, const CertArgs& ca,
                            const float* X, const float* Y, int64_t d, double* fb_part);
// Exact KDE from the three-part bfloat16 rows (Xsp, Ysp: [rows][3][dps]); p holds
// the float32 problem (norms, sizes, placement).
hipError_t launch_kde_exact_split(const TileProblem& p, const void* Xsp, const void* Ysp,
                                  int64_t dps, int kern, double h, double* partial, double* out,
                                  hipStream_t s, TimingHook th, const CertArgs& ca,
                                  const float* X, const float* Y, int64_t d, double* fb_part);

// ---- exact k nearest neighbours -------------------------------------------
struct KnnBuffers {
  uint64_t* cand;        // [splits][qp][cap1] packed (key, index), scan lists
  int32_t* cand_cnt;     // [splits][qp]
  int64_t cap1;          // list capacity per (split, query): 256, 512, 1024 or 2048
  int64_t K1;            // kept per list
  int32_t* nn_work;      // [q][k] neighbours sorted by index (internal copy)
  double* z1;            // [q] sum of kernel values over the neighbours
  float* thr2;           // [q] second-pass key threshold (>= 0 flagged)
  int32_t* flags;        // [qtiles] query tile needs a second pass
  uint64_t* cand2;       // [q][cap2] second-pass candidates: lower-bound key code << 32 | index
  int32_t* cand2_cnt;    // [q]
  int64_t cap2;
  int32_t* status;       // [q] 0 certified by the first pass, 1 second pass pending,
                         // 2 (3: too few inspected rows) exhaustive scan pending,
                         // 4 done by the second pass, 5 done by the exhaustive scan
  const float* yerr;     // [qp]
  const uint32_t* xerr_max;
  int64_t seed_stride;   // 16-bit candidate pass: every seed_stride-th data tile
};

// p: geometry of the selection scan, pc: of the second-pass collect (more splits)
hipError_t launch_knn(int prec, const TileProblem& p, const TileProblem& pc, const KnnBuffers& b,
                      const float* X, const float* Y, int64_t d, int64_t k, double h, int kern,
                      int32_t* nn_out, hipStream_t s);

hipError_t launch_knn_all(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                          double h, int kern, int32_t* nn, double* z1, hipStream_t s);
// Z1 over given neighbour lists nn[q][k] (entries outside [0, n) skipped).
hipError_t launch_knn_list_sum(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                               double h, int kern, const int32_t* nn, int64_t k, double* z1,
                               hipStream_t s);

// ---- near/far form of the exact KDE ----------------------------------------
// CSR of the neighbour pairs per (query tile, data tile): cnt [qtiles * ntiles]
// scratch, off [qtiles * ntiles + 1], tot [scan_blocks(qtiles * ntiles)],
// hits [q * k] entries (query mod 128) << 7 | (row mod 128).
int64_t scan_blocks(int64_t count);
hipError_t launch_hybrid_hits(const int32_t* nn, int64_t q, int64_t k, int64_t n, int64_t qtiles,
                              int64_t ntiles, int32_t* cnt, int32_t* off, int32_t* tot,
                              uint16_t* hits, hipStream_t s);
// 16-bit tile sweep without the listed pairs, then out = (sum + z1) / n.
hipError_t launch_kde_hybrid(int prec, const TileProblem& p, int kern, double h,
                             const int32_t* hoff, const uint16_t* hits, const double* z1,
                             double* partial, double* out, hipStream_t s, TimingHook th = {});

// ---- inverted-file neighbours --------------------------------------------------
int64_t ivf_hist_blocks(int64_t n);
hipError_t launch_kmeans_init(const float* X, int64_t n, int64_t d, int64_t L, float* C,
                              hipStream_t s);
// Cluster ranges off[L+1] (and poff[L+1] padded to the tile), member rows in
// index order ids[off[L]]; hist [ivf_hist_blocks(n)][L] is scratch.
hipError_t launch_list_layout(const int32_t* a, int64_t n, int64_t L, int32_t* hist,
                              int32_t* count, int32_t* off, int32_t* poff, int32_t* ids,
                              int32_t* skipped, hipStream_t s);
hipError_t launch_kmeans_mean(const float* X, int64_t d, const int32_t* ids, const int32_t* off,
                              int64_t L, const float* C_prev, float* C_new, hipStream_t s);
// Tile layout: pids[cap] (-1 for empty rows) and the float32 rows Xperm[cap][d].
hipError_t launch_list_tiles(const float* X, int64_t d, const int32_t* ids, const int32_t* off,
                             const int32_t* poff, int64_t L, int64_t cap, int32_t* pids,
                             float* Xperm, hipStream_t s);
hipError_t launch_empty_row_keys(const int32_t* pids, const int32_t* nrows, int64_t cap,
                                 float* xknorm, hipStream_t s);
// (cluster, query) pair rows of a batch: pp[L+1] (pfill needs L+1 entries);
// probe[q][kp] holds the inspected clusters, the first np_q[q] of them valid.
hipError_t launch_pairs(const int32_t* probe, int64_t q, int64_t kp, const int32_t* np_q,
                        int64_t L, int32_t* pcount, int32_t* pfill, int32_t* pp, int32_t* pair_q,
                        int32_t* pair_of, int64_t cap, const float* Ys, const float* yknorm,
                        int64_t dp, float* Yg, float* ygk, hipStream_t s);

// Parts of the pair tiles' sweeps (see pair_parts_kernel): lbase[nb+1] with
// nb = pp[L] / 128 <= budget; at most budget parts; nparts[2].
hipError_t launch_pair_parts(const int32_t* pp, const int32_t* poff, int64_t L, int64_t budget,
                             int64_t target, int32_t* lbase, int32_t* nparts, hipStream_t s);

struct IvfTiles {
  const char* Ys;          // prepared query rows in pair order [prow_cap][dp]
  const char* Xs;          // prepared index rows in tile layout [xrows][dp]
  int64_t ld_bytes;
  int nchunks;
  const float* yknorm;     // [prow_cap]
  const float* xknorm;     // [xrows], infinite for empty rows
  const int32_t* pp;       // [L+1] pair rows of each cluster (multiples of 128)
  const int32_t* poff;     // [L+1] index rows of each cluster (multiples of 128)
  int64_t L;
  const int32_t* pair_q;   // [prow_cap] query of each pair row (-1: padding)
  const int32_t* pids;     // [xrows] row of each tile-layout row (-1: empty)
  const int32_t* lbase;    // [nb+1] first part of each pair tile; part j lists at rows 128j..
  const int32_t* nparts;   // [0]: parts in all
  uint32_t* qthr;          // [q] smallest K1-th key published for each query (float_key order)
};

struct IvfRefine {
  const int32_t* probe;    // [q][kp] inspected clusters
  int64_t kp;
  const int32_t* np_q;     // [q] inspected clusters of each query (0: exact scan of all rows)
  const int32_t* pair_of;  // [q][kp] pair row of each inspected cluster
  const int32_t* off;      // [L+1] cluster ranges of ids
  const int32_t* ids;      // member rows in cluster order
  const int32_t* pids;     // [xrows] row of each tile-layout row (-1: empty)
  const int32_t* lbase;    // [nb+1] first part of each pair tile
  const uint32_t* qthr;    // [q] final shared bound of each query's scan
};

// Inspected clusters of each query (see probe_order_kernel); order[q][kp].
hipError_t launch_probe_order(const float* C, const float* Y, int64_t q, int64_t d,
                              const int32_t* cand, int64_t kp, const int32_t* off, int64_t n_probe,
                              int64_t k, int32_t* order, int32_t* np_q, hipStream_t s);

hipError_t launch_ivf_knn(const IvfTiles& t, int64_t prow_cap, const KnnBuffers& b,
                          const IvfRefine& v, const float* X, const float* Y, int64_t n,
                          int64_t q, int64_t d, int64_t k, double h, int kern, int32_t* nn_out,
                          hipStream_t s);

// ---- sampler, gather and combine --------------------------------------------
// Prepared permuted index of Algorithm 2: pi[n] (row at each position), inv[n]
// (position of each row), Xp[n][d] the rows in permuted order.
struct PermIndex {
  const int32_t* pi;
  const int32_t* inv;
  const float* Xp;
};
hipError_t launch_perm_index(const float* X, int64_t n, int64_t d, uint64_t seed,
                             const PermIndex& pidx, hipStream_t s);
// pidx (permuted sampling only; may be null): read the permutation and the
// rows from the prepared index instead of evaluating the permutation.
hipError_t launch_sample(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                         double h, int kern, int64_t k, int64_t m, uint64_t seed,
                         uint64_t query_offset, uint64_t word2, int permuted, uint64_t start,
                         const int32_t* nn_sorted, const double* z1, double* out,
                         int32_t* sample_idx, hipStream_t s, const PermIndex* pidx = nullptr);

// ---- adjoints ----------------------------------------------------------------
hipError_t launch_deann_backward(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                 double h, int kern, int64_t k, int64_t m, const int32_t* nn,
                                 const int32_t* samp, const double* grad_out /* NULL: ones */, float* grad_Y,
                                 double* gh_part, double* grad_h, hipStream_t s);
// DEANN's estimates (as launch_sample, plain sampling) and d out_j / d y_j,
// sum_j d out_j / d h from one gather of the k + m rows of each query; the
// draws go to sample_idx (required here: scratch for shapes that take the
// sampler and then the adjoint).
hipError_t launch_deann_value_grad(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                   double h, int kern, int64_t k, int64_t m, uint64_t seed,
                                   uint64_t query_offset, uint64_t word2, const int32_t* nn_sorted,
                                   const double* z1, double* out, int32_t* sample_idx,
                                   float* grad_Y, double* gh_part, double* grad_h, hipStream_t s);

// Three-part bfloat16 rows of the prepared operands ([rows][3][dps], see
// launch_split_rows); X null: the float32 distance product.
struct SplitRows {
  const void* X = nullptr;
  const void* Y = nullptr;
  int64_t dps = 0;
};

// The exact adjoint (and with mu the fused value + gradient): the sweep, the
// reduction with the certificate (ca, cd as for kde_exact), and the exact
// re-evaluation of the listed queries from the caller's X and Y (their
// scratch reuses gy_part and gh_part, so splits must be at least 1).
hipError_t launch_kde_backward(const TileProblem& p, const float* X, const float* Y, int64_t d,
                               double h, int kern, const double* grad_out, double* gy_part,
                               double* gh_part, float* grad_Y, double* grad_h, hipStream_t s,
                               TimingHook th, double* mu, double* gh_per_query, SplitRows split,
                               const CertArgs& ca);

hipError_t launch_mean_shift_update(const float* Y, const float* g, const double* mu, int64_t q,
                                    int64_t d, double h, float* Y_out, hipStream_t s);

}  // namespace deann
