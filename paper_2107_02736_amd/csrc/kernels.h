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
};

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);
hipError_t launch_center(const float* X, int64_t n, int64_t d, double* part, int64_t R, float* c,
                         hipStream_t s);
hipError_t launch_prep_rows_prec(int prec, const float* src, int64_t rows, int64_t rows_padded,
                                 int64_t d, int64_t dp, const float* c, double a_scale, void* dst,
                                 double* norm, float* knorm, float* err, uint32_t* err_max,
                                 hipStream_t s);

// Optional pair of events recorded around a dense tile kernel (both null: none).
struct TimingHook {
  hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_kde_exact(int prec, const TileProblem& p, int kern, double h, double* partial,
                            double* out, hipStream_t s, TimingHook th = {});

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
  uint64_t* cand2;       // [q][cap2] second-pass candidates (index only)
  int32_t* cand2_cnt;    // [q]
  int64_t cap2;
  int32_t* status;       // [q] 0 certified, 1 second pass, 2 exhaustive scan
  const float* yerr;     // [qp]
  const uint32_t* xerr_max;
};

// p: geometry of the selection scan, pc: of the second-pass collect (more splits)
hipError_t launch_knn(int prec, const TileProblem& p, const TileProblem& pc, const KnnBuffers& b,
                      const float* X, const float* Y, int64_t d, int64_t k, double h, int kern,
                      int32_t* nn_out, hipStream_t s);

hipError_t launch_knn_all(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                          double h, int kern, int32_t* nn, double* z1, hipStream_t s);

// ---- sampler, gather and combine --------------------------------------------
hipError_t launch_sample(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                         double h, int kern, int64_t k, int64_t m, uint64_t seed,
                         uint64_t query_offset, uint64_t word2, int permuted, uint64_t start,
                         const int32_t* nn_sorted, const double* z1, double* out,
                         int32_t* sample_idx, hipStream_t s);

// ---- adjoints ----------------------------------------------------------------
hipError_t launch_deann_backward(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                 double h, int kern, int64_t k, int64_t m, const int32_t* nn,
                                 const int32_t* samp, const double* grad_out, float* grad_Y,
                                 double* gh_part, double* grad_h, hipStream_t s);

hipError_t launch_kde_backward(const TileProblem& p, const float* Y, int64_t d, double h, int kern,
                               const double* grad_out, double* gy_part, double* gh_part,
                               float* grad_Y, double* grad_h, hipStream_t s, TimingHook th = {},
                               double* mu = nullptr, double* gh_per_query = nullptr);

hipError_t launch_mean_shift_update(const float* Y, const float* g, const double* mu, int64_t q,
                                    int64_t d, double h, float* Y_out, hipStream_t s);

}  // namespace deann
