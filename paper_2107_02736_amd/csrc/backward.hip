// Adjoints of the KDE (derived from Eq. (1)-(2); the paper has no gradients).
//
// For one query y and one data row x at distance r = ||x - y||:
//   Gaussian:    dK/dy = K (x - y) / h^2,        dK/dh = K r^2 / h^3
//   exponential: dK/dy = K (x - y) / (h r),      dK/dh = K r / h^2   (dK/dy = 0 at r = 0)
//
// DEANN estimate (Algorithm 1): the index sets are held fixed (the
// selection is piecewise constant in y and h), each neighbour weighs 1 and each
// draw (n-k)/m, all over n.  The rows are gathered again and the distances
// recomputed in FP64; nothing from the forward pass is stored but the indices.
//
// Exact KDE: the distance tile is recomputed on MFMA as S^T = X~ Y~^T so that
// the weights W = dK/dy-scale land in registers exactly in the A-operand layout
// of a second MFMA product G = W X~ (k dimension = data rows).  Then
// dKDE/dy = (G - y~ rowsum(W)) / n in the centred coordinates.
#include "cert.h"
#include "philox.h"

namespace deann {

// ---------------------------------------------------------------------------
// DEANN backward: one workgroup per query
// ---------------------------------------------------------------------------
constexpr int BWD_CHUNK = 512;
constexpr int BWD_MAX_COORD_PER_THREAD = 8;   // d <= 2048

__global__ void __launch_bounds__(WG)
deann_backward_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n,
                      int64_t d, double h, int kern, int64_t k, int64_t m,
                      const int32_t* __restrict__ nn, const int32_t* __restrict__ samp,
                      const double* __restrict__ grad_out, float* __restrict__ grad_Y,
                      double* __restrict__ gh_part) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  double* wc = reinterpret_cast<double*>(smem);          // BWD_CHUNK
  double* hh = wc + BWD_CHUNK;                            // BWD_CHUNK
  int32_t* rid = reinterpret_cast<int32_t*>(hh + BWD_CHUNK);   // BWD_CHUNK
  float* ys = reinterpret_cast<float*>(rid + BWD_CHUNK);        // d
  const int64_t qi = blockIdx.x;
  const int64_t size2 = n - k;
  const int64_t ms = (size2 > 0) ? m : 0;
  const int64_t R = k + ms;
  const double csamp = ms > 0 ? (double)size2 / (double)m : 0.0;
  for (int64_t t = threadIdx.x; t < d; t += WG) ys[t] = Y[qi * d + t];
  double acc[BWD_MAX_COORD_PER_THREAD];
#pragma unroll
  for (int u = 0; u < BWD_MAX_COORD_PER_THREAD; ++u) acc[u] = 0.0;
  double hsum = 0.0;   // thread 0
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  const double inv_h2 = 1.0 / (h * h);
  __syncthreads();
  for (int64_t r0 = 0; r0 < R; r0 += BWD_CHUNK) {
    const int cnt = (int)(R - r0 < BWD_CHUNK ? R - r0 : BWD_CHUNK);
    for (int jj = g; jj < cnt; jj += WG / 16) {
      const int64_t j = r0 + jj;
      const int32_t row = j < k ? nn[qi * k + j] : samp[qi * m + (j - k)];
      const double c = j < k ? 1.0 : csamp;
      const float* xr = X + (int64_t)row * d;
      double s = 0.0;
      for (int64_t t = l16; t < d; t += 16) {
        const double df = (double)xr[t] - (double)ys[t];
        s = __builtin_fma(df, df, s);
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 8, 64);
      if (l16 == 0) {
        double w, dh;
        if (kern == KERNEL_GAUSSIAN) {
          const double K = exp(-0.5 * s * inv_h2);
          w = K * inv_h2;
          dh = K * s * inv_h2 / h;
        } else {
          const double r = sqrt(s);
          const double K = exp(-r / h);
          w = r > 0.0 ? K / (h * r) : 0.0;
          dh = K * r * inv_h2;
        }
        wc[jj] = c * w;
        hh[jj] = c * dh;
        rid[jj] = row;
      }
    }
    __syncthreads();
    // coordinates owned by this thread, rows in fixed order
    for (int jj = 0; jj < cnt; ++jj) {
      const float* xr = X + (int64_t)rid[jj] * d;
      const double w = wc[jj];
#pragma unroll
      for (int u = 0; u < BWD_MAX_COORD_PER_THREAD; ++u) {
        const int64_t t = threadIdx.x + (int64_t)u * WG;
        if (t < d) acc[u] = __builtin_fma(w, (double)xr[t] - (double)ys[t], acc[u]);
      }
    }
    if (threadIdx.x == 0)
      for (int jj = 0; jj < cnt; ++jj) hsum += hh[jj];
    __syncthreads();
  }
  const double go = grad_out ? grad_out[qi] : 1.0;
  const double scale = go / (double)n;
  if (grad_Y) {
#pragma unroll
    for (int u = 0; u < BWD_MAX_COORD_PER_THREAD; ++u) {
      const int64_t t = threadIdx.x + (int64_t)u * WG;
      if (t < d) grad_Y[qi * d + t] = (float)(scale * acc[u]);
    }
  }
  if (threadIdx.x == 0 && gh_part) gh_part[qi] = scale * hsum;
}

// Register-resident variant for d % 4 == 0 and d <= 4 * GW * U: a group of GW
// lanes (16, or a whole wave for long rows) gathers a row once (float4 loads,
// 16 * GW contiguous bytes per group and step), reduces ||x - y||^2 with
// shuffles, and accumulates w (x - y) into its own FP64 coordinates; the group
// partials are summed in a fixed order.  The rows of each group are taken in
// the same order as before (row g, g + NG, ... of the query's neighbours then
// draws), so the sums do not change.
//
// DRAW: the fused value-and-gradient pass of DEANN.  The draws are made here
// (the sampler's rows, bit for bit: see philox.h) instead of read from samp,
// and the estimate itself, (1/n) sum of c K over the same rows, is written
// to dr.out beside d out / d y (grad_out NULL: a unit upstream gradient).
constexpr int BWD_IDX = 2048;   // row indices staged in LDS per chunk
struct DrawArgs {
  uint64_t seed, query_offset, word2;
  int32_t* sample_idx;   // [q][m] or NULL
  double* out;           // [q]
};
template <int U, int GW, bool DRAW>
__global__ void __launch_bounds__(WG)
deann_backward_vec_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n,
                          int64_t d, double h, int kern, int64_t k, int64_t m,
                          const int32_t* __restrict__ nn, const int32_t* __restrict__ samp,
                          const double* __restrict__ grad_out, float* __restrict__ grad_Y,
                          double* __restrict__ gh_part, DrawArgs dr) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int NG = WG / GW;   // groups (rows in flight) per workgroup
  double* part = reinterpret_cast<double*>(smem);   // [NG][d]
  double* hpart = part + NG * d;                    // [NG]
  double* vpart = hpart + NG;                       // [NG] (DRAW)
  int32_t* rid = reinterpret_cast<int32_t*>(vpart + NG);   // [BWD_IDX] row indices
  int32_t* gaps = rid + BWD_IDX;                    // [k] (DRAW)
  const int64_t qi = blockIdx.x;
  const int g = threadIdx.x / GW, lg = threadIdx.x % GW;
  const int64_t size2 = n - k;
  const int64_t ms = (size2 > 0) ? m : 0;
  const int64_t R = k + ms;
  const double csamp = ms > 0 ? (double)size2 / (double)m : 0.0;
  const double inv_h2 = 1.0 / (h * h);
  // this lane's coordinates: 4 * lg + 4 * GW * u + {0..3}
  float yv[U][4];
  double acc[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t t = 4 * lg + 4 * GW * u + c;
      yv[u][c] = t < d ? Y[qi * d + t] : 0.f;
      acc[u][c] = 0.0;
    }
  double hs = 0.0, vs = 0.0;
  if constexpr (DRAW) {
    if (ms > 0)
      for (int64_t t = threadIdx.x; t < k; t += WG) gaps[t] = nn[qi * k + t] - (int32_t)t;
    if (dr.sample_idx && ms == 0)
      for (int64_t j = threadIdx.x; j < m; j += WG) dr.sample_idx[qi * m + j] = -1;
  }
  auto load_row = [&](int32_t row, float (&dst)[U][4]) {
    const float* xr = X + (int64_t)row * d;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t t = 4 * lg + 4 * GW * u;
      if (t < d) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(xr + t);
        dst[u][0] = v[0]; dst[u][1] = v[1]; dst[u][2] = v[2]; dst[u][3] = v[3];
      } else {
        dst[u][0] = dst[u][1] = dst[u][2] = dst[u][3] = 0.f;
      }
    }
  };
  // Rows in chunks of BWD_IDX: the chunk's row indices are staged in LDS first
  // (one coalesced read instead of an index load in front of every row load),
  // and group g takes rows g, g + NG, ... of the chunk with the next rows in
  // flight behind the one it evaluates.
  // wide rows (a wave per row) and rows of up to 128 coordinates keep two rows
  // in flight per group, other 16-lane groups one (their extra registers would
  // cost occupancy)
  constexpr bool TWO = GW == 64 || U <= 2;
  float xv[U][4], xa[U][4], xb[U][4];
  for (int64_t c0 = 0; c0 < R; c0 += BWD_IDX) {
    const int cnt = (int)(R - c0 < BWD_IDX ? R - c0 : BWD_IDX);
    __syncthreads();   // the previous chunk's indices have been read (and gaps written)
    if constexpr (DRAW) {
      for (int i = threadIdx.x; i < cnt && c0 + i < k; i += WG) rid[i] = nn[qi * k + c0 + i];
      // draws [j_lo, j_hi) of this chunk, one Philox block (4 draws) per thread
      const int64_t j_lo = (c0 > k ? c0 : k) - k, j_hi = c0 + cnt - k;
      const uint64_t stream = dr.query_offset + (uint64_t)qi;
      for (int64_t jb = j_lo / 4 + threadIdx.x; jb * 4 < j_hi; jb += WG) {
        const Philox4x64 blk = philox4x64_10(dr.seed, 0, (uint64_t)jb, stream, dr.word2, 0);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int64_t jd = jb * 4 + w;
          if (jd >= j_lo && jd < j_hi) {
            const int32_t row = (int32_t)draw_row(blk.v[w], (uint64_t)size2, gaps, k);
            rid[jd + k - c0] = row;
            if (dr.sample_idx) dr.sample_idx[qi * m + jd] = row;
          }
        }
      }
    } else {
      for (int i = threadIdx.x; i < cnt; i += WG) {
        const int64_t j = c0 + i;
        rid[i] = j < k ? nn[qi * k + j] : samp[qi * m + (j - k)];
      }
    }
    __syncthreads();
    if (g < cnt) load_row(rid[g], xv);
    if (TWO && g + NG < cnt) load_row(rid[g + NG], xa);
    for (int i = g; i < cnt; i += NG) {
      if (TWO) {
        if (i + 2 * NG < cnt) load_row(rid[i + 2 * NG], xb);
      } else {
        if (i + NG < cnt) load_row(rid[i + NG], xa);
      }
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double df = (double)xv[u][c] - (double)yv[u][c];
          s = __builtin_fma(df, df, s);
        }
#pragma unroll
      for (int off = 1; off < GW; off <<= 1) s += __shfl_xor(s, off, 64);
      const double c = c0 + i < k ? 1.0 : csamp;
      double w, dh, K;
      if (kern == KERNEL_GAUSSIAN) {
        K = exp(-0.5 * s * inv_h2);
        w = K * inv_h2;
        dh = K * s * inv_h2 / h;
      } else {
        const double r = sqrt(s);
        K = exp(-r / h);
        w = r > 0.0 ? K / (h * r) : 0.0;
        dh = K * r * inv_h2;
      }
      w *= c;
      hs += c * dh;
      if constexpr (DRAW) vs += c * K;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc)
          acc[u][cc] = __builtin_fma(w, (double)xv[u][cc] - (double)yv[u][cc], acc[u][cc]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          xv[u][cc] = xa[u][cc];
          if (TWO) xa[u][cc] = xb[u][cc];
        }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t t = 4 * lg + 4 * GW * u + c;
      if (t < d) part[g * d + t] = acc[u][c];
    }
  if (lg == 0) {
    hpart[g] = hs;
    if constexpr (DRAW) vpart[g] = vs;
  }
  __syncthreads();
  const double scale = (grad_out ? grad_out[qi] : 1.0) / (double)n;
  if (grad_Y)
    for (int64_t t = threadIdx.x; t < d; t += WG) {
      double v = 0.0;
      for (int gg = 0; gg < NG; ++gg) v += part[gg * d + t];
      grad_Y[qi * d + t] = (float)(scale * v);
    }
  if (threadIdx.x == 0 && gh_part) {
    double v = 0.0;
    for (int gg = 0; gg < NG; ++gg) v += hpart[gg];
    gh_part[qi] = scale * v;
  }
  if constexpr (DRAW)
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int gg = 0; gg < NG; ++gg) v += vpart[gg];
      dr.out[qi] = v / (double)n;
    }
}

// Fixed-order sum of q per-query terms into one scalar (single workgroup).
__global__ void __launch_bounds__(WG) sum_scalar_kernel(const double* __restrict__ v, int64_t q,
                                                        double* __restrict__ out) {
  __shared__ double red[WG];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < q; i += WG) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = WG / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// The adjoint (DRAW = false: rows from samp) or the fused value-and-gradient
// pass (DRAW = true); false if the shape needs the generic kernel.
template <bool DRAW>
static bool launch_vec(const float* X, const float* Y, int64_t n, int64_t q, int64_t d, double h,
                       int kern, int64_t k, int64_t m, const int32_t* nn, const int32_t* samp,
                       const double* grad_out, float* grad_Y, double* gh_part, const DrawArgs& dr,
                       hipStream_t s) {
  const bool aligned = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0) &&
                       (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
  const dim3 g((unsigned)q), b(WG);
  const size_t extra = BWD_IDX * 4 + (DRAW && k < n && m > 0 ? (size_t)k * 4 : 0);   // gaps
#define DEANN_VEC(U_, GW_)                                                                    \
  deann_backward_vec_kernel<U_, GW_, DRAW><<<g, b, sm, s>>>(X, Y, n, d, h, kern, k, m, nn, samp, \
                                                             grad_out, grad_Y, gh_part, dr)
  if (aligned && d <= 256) {   // 16 lanes per row
    const size_t sm = (16 * d + 32) * 8 + extra;
    switch ((d + 63) / 64) {
      case 1: DEANN_VEC(1, 16); break;
      case 2: DEANN_VEC(2, 16); break;
      case 3: DEANN_VEC(3, 16); break;
      default: DEANN_VEC(4, 16); break;
    }
    return true;
  }
  if (aligned && d <= 2048) {   // a wave per row
    const size_t sm = (4 * d + 8) * 8 + extra;
    switch ((d + 255) / 256) {
      case 1:
      case 2: DEANN_VEC(2, 64); break;
      case 3:
      case 4: DEANN_VEC(4, 64); break;
      case 5:
      case 6: DEANN_VEC(6, 64); break;
      default: DEANN_VEC(8, 64); break;
    }
    return true;
  }
#undef DEANN_VEC
  return false;
}

hipError_t launch_deann_backward(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                 double h, int kern, int64_t k, int64_t m, const int32_t* nn,
                                 const int32_t* samp, const double* grad_out, float* grad_Y,
                                 double* gh_part, double* grad_h, hipStream_t s) {
  if (q == 0) return hipSuccess;
  if (!launch_vec<false>(X, Y, n, q, d, h, kern, k, m, nn, samp, grad_out, grad_Y, gh_part,
                         DrawArgs{}, s)) {
    const size_t sm = BWD_CHUNK * (8 + 8 + 4) + d * 4 + 16;
    deann_backward_kernel<<<dim3((unsigned)q), dim3(WG), sm, s>>>(
        X, Y, n, d, h, kern, k, m, nn, samp, grad_out, grad_Y, gh_part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad_h) return e;
  sum_scalar_kernel<<<dim3(1), dim3(WG), 0, s>>>(gh_part, q, grad_h);
  return hipGetLastError();
}

hipError_t launch_deann_value_grad(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                   double h, int kern, int64_t k, int64_t m, uint64_t seed,
                                   uint64_t query_offset, uint64_t word2, const int32_t* nn_sorted,
                                   const double* z1, double* out, int32_t* sample_idx,
                                   float* grad_Y, double* gh_part, double* grad_h, hipStream_t s) {
  if (q == 0) return hipSuccess;
  const DrawArgs dr{seed, query_offset, word2, sample_idx, out};
  if (!launch_vec<true>(X, Y, n, q, d, h, kern, k, m, nn_sorted, nullptr, nullptr, grad_Y,
                        gh_part, dr, s)) {
    // other shapes: the sampler, then the adjoint over its draws
    hipError_t e = launch_sample(X, Y, n, q, d, h, kern, k, m, seed, query_offset, word2, 0, 0,
                                 nn_sorted, z1, out, sample_idx, s);
    if (e != hipSuccess) return e;
    return launch_deann_backward(X, Y, n, q, d, h, kern, k, m, nn_sorted, sample_idx, nullptr,
                                 grad_Y, gh_part, grad_h, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad_h) return e;
  sum_scalar_kernel<<<dim3(1), dim3(WG), 0, s>>>(gh_part, q, grad_h);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact-KDE backward on MFMA (FP32 operands, padded d = DP <= 128)
// ---------------------------------------------------------------------------
// 512 threads (8 waves, two per SIMD).  Wave w owns queries w*16..+16 of the
// query tile; their FP32 rows stay in registers for the whole sweep (the
// B-operand fragments of every k-group).  Each 128-row data tile is staged
// whole in LDS (double-buffered, one barrier per tile) and serves both
// products of the wave:
//   S^T = X~ Y~^T   A = data-row fragments from LDS, B = the resident queries;
//                   lane (g, c) = (lane/16, lane%16) receives rows
//                   16*bi + 4*g + r (r = 0..3) of query column c;
//   weights         W = f(S^T) in place (FP32, same exponent arithmetic as the
//                   forward tiles);
//   G += W X~       16x16x4 MFMAs whose k index g stands for data row
//                   16*bi + 4*g + r: the A operand is the weight register
//                   itself, the B operand one 16-byte LDS read of that row
//                   (4 consecutive coordinates, used by 4 MFMAs whose output
//                   column c stands for coordinate 4*c + j of the block).
// Nothing goes through LDS but the data tile; G, the weight sums and the dK/dh
// sums stay in registers until the end of the split.
constexpr int BWG = 512;
// Rows staged per step of the exact adjoint: 64 for rows of 64 floats, where
// 64-row steps let two workgroups share a CU (measured 6% faster at d = 64);
// 128 otherwise (rows of 32 floats fit two workgroups per CU with 128-row
// steps already, rows of 96 and 128 floats do not fit two in the registers).
#ifndef BWD_TR_64
#define BWD_TR_64 64
#endif

template <int DP>
struct GradTile {
  static constexpr int KGS = DP / 16;            // 64-byte k-groups per row
  static constexpr int PITCH = DP * 4 + 16;      // LDS row pitch (bytes)
  static constexpr int NB = DP / 64;             // 64-coordinate blocks of G
  static constexpr int HB = (DP % 64) / 32;      // trailing 32-coordinate block
  static constexpr int GB = 4 * NB + 2 * HB;     // 16x16 G blocks per wave
  static constexpr int NPT = BN * DP / 4 / BWG;  // 16-byte tile pieces per thread
  static constexpr int PPR = DP / 4;             // 16-byte pieces per row
};

// The gradient tile G sums W x~ in FP32 MFMA accumulators. Its terms cancel
// (sum of w x against y times sum of w), so the FP32 sums are moved into the
// workgroup's FP64 partial every kGradFlushRows data rows and restarted: the
// rounding error then grows with that run, not with the split's whole range.
// G block (nb, j): lane (g, c), register rr holds query 4g + rr, coordinate
// nb*64 + 4c + j (trailing block: NB*64 + 2c + j).
constexpr int kGradFlushRows = 8192;

template <int DP>
__device__ inline void flush_grad(f32x4 (&gacc)[GradTile<DP>::GB], double* __restrict__ part,
                                  int g, int c, bool fresh) {
  using G = GradTile<DP>;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    double* dst = part + (4 * g + rr) * DP;
#pragma unroll
    for (int nb = 0; nb < G::NB; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double* o = dst + nb * 64 + 4 * c + j;
        *o = (fresh ? 0.0 : *o) + (double)gacc[4 * nb + j][rr];
      }
    if constexpr (G::HB)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        double* o = dst + G::NB * 64 + 2 * c + j;
        *o = (fresh ? 0.0 : *o) + (double)gacc[4 * G::NB + j][rr];
      }
  }
#pragma unroll
  for (int i = 0; i < G::GB; ++i) gacc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// VAL: also sum the kernel values themselves (the KDE); needed separately for
// the exponential kernel only, whose weights are K / r (Gaussian: K).
// TR: data rows staged per step, 128 (one workgroup per CU) or 64 (two
// workgroups per CU, whose steps need not line up, so one workgroup's MFMAs
// run while the other computes weights).
template <int KERN, int DP, bool VAL, int TR>
__global__ void __launch_bounds__(BWG, TR == 64 ? 4 : 1)
kde_backward_kernel(TileProblem p, float L, double* __restrict__ gy_part,
                    double* __restrict__ rw_part, double* __restrict__ gh_part,
                    double* __restrict__ ks_part, float2* __restrict__ cert) {
  using G = GradTile<DP>;
  // the certificate needs sum K for the exponential kernel (Gaussian: the weights)
  constexpr bool KS = KERN != KERNEL_GAUSSIAN;
  (void)VAL;
  constexpr int NBI = TR / 16, UPT = BN / TR;
  constexpr int NPT = TR * DP / 4 / BWG;   // 16-byte pieces per thread and step
  static_assert(NPT >= 1 && TR * DP / 4 == NPT * BWG, "row pieces must split evenly");
  __shared__ __attribute__((aligned(16))) char xs[2][TR * G::PITCH];
  __shared__ __attribute__((aligned(16))) float xvs[2][TR];   // per-row exponent terms
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t t0 = split * p.ntiles / p.splits * UPT, t1 = (split + 1) * p.ntiles / p.splits * UPT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;

  // resident query fragments and the query's exponent term
  const int64_t qrow = qt * BQ + wave * 16 + c;
  u32x4 yf[G::KGS];
#pragma unroll
  for (int kg = 0; kg < G::KGS; ++kg)
    yf[kg] = *reinterpret_cast<const u32x4*>(p.Ys + qrow * p.ld_bytes + kg * KG_BYTES + g * 16);
  const double ynq = p.ynorm[qrow];
  const float yv = KERN == KERNEL_GAUSSIAN ? (float)(-(double)L * ynq) : (float)ynq;

  // data rows: global -> registers -> LDS; row terms by the first TR threads
  u32x4 xr[NPT];
  float xvr = 0.f;
  auto gload = [&](int64_t t) {
    const char* base = p.Xs + t * TR * p.ld_bytes;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int v = threadIdx.x + i * BWG;
      xr[i] = *reinterpret_cast<const u32x4*>(base + (v / G::PPR) * p.ld_bytes + (v % G::PPR) * 16);
    }
    if (threadIdx.x < TR) {
      const int64_t row = t * TR + threadIdx.x;
      // padding rows: a huge finite term, so that K = 0 and K * d^2 = 0
      xvr = row < p.n ? (KERN == KERNEL_GAUSSIAN ? (float)(-(double)L * p.xnorm[row])
                                                 : (float)p.xnorm[row])
                      : (KERN == KERNEL_GAUSSIAN ? -1e30f : 1e30f);
    }
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int v = threadIdx.x + i * BWG;
      *reinterpret_cast<u32x4*>(&xs[b][(v / G::PPR) * G::PITCH + (v % G::PPR) * 16]) = xr[i];
    }
    if (threadIdx.x < TR) xvs[b][threadIdx.x] = xvr;
  };

  f32x4 gacc[G::GB];
#pragma unroll
  for (int i = 0; i < G::GB; ++i) gacc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  double rws = 0.0, dhs = 0.0, kss = 0.0;
  // certificate: sum of K^2; Gaussian: sum of K times its exponent, exponential: largest K
  float csq = 0.f, cmx = 0.f;

  const int64_t qbase = split * p.qp + qt * BQ + wave * 16;
  double* gpart = gy_part + qbase * DP;
  bool fresh = true;

  if (t0 < t1) {
    gload(t0);
    lstore(0);
  }
  __syncthreads();
  // runs of kGradFlushRows rows, each ending in a flush of G (a test inside
  // the tile loop instead costs registers, and occupancy)
  for (int64_t tc = t0; tc < t1; tc += kGradFlushRows / TR) {
  const int64_t te = tc + kGradFlushRows / TR < t1 ? tc + kGradFlushRows / TR : t1;
  for (int64_t t = tc; t < te; ++t) {
    const int b = (int)((t - t0) & 1);
    const bool more = t + 1 < t1;
    if (more) gload(t + 1);   // in flight behind the first product
    const char* xb = xs[b];

    // S^T for the TR staged rows against the wave's 16 queries
    f32x4 acc[NBI];
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) acc[bi] = f32x4{0.f, 0.f, 0.f, 0.f};
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kg = 0; kg < G::KGS; ++kg) {
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) {
        const u32x4 a = *reinterpret_cast<const u32x4*>(xb + (bi * 16 + c) * G::PITCH +
                                                         kg * KG_BYTES + g * 16);
        acc[bi] = mfma_kgroup<float>(a, yf[kg], acc[bi]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (more) lstore(b ^ 1);   // the other buffer was last read before the previous barrier

    // weights (constant factors 1/h^2, 1/h, -1/L and the Gaussian query
    // correction are applied per query by the reduction); FP32 partial sums of
    // eight rows folded into FP64
    const f32x4* xv4 = reinterpret_cast<const f32x4*>(xvs[b]);
#pragma unroll
    for (int bp = 0; bp < NBI / 2; ++bp) {
      float rw32 = 0.f, dh32 = 0.f, ks32 = 0.f;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int bi = 2 * bp + h2;
        const f32x4 xv = xv4[bi * 4 + g];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float s = acc[bi][r];
          float w, dh;
          if (KERN == KERNEL_GAUSSIAN) {
            const float a = fminf(__builtin_fmaf(2.f * L, s, yv + xv[r]), 0.f);   // -L d^2
            const float K = __builtin_amdgcn_exp2f(a);
            w = K;
            dh = K * a;
            csq = __builtin_fmaf(K, K, csq);
            cmx = __builtin_fmaf(-K, a, cmx);   // Gaussian: sum of K times its exponent
          } else {
            const float d2 = fmaxf(__builtin_fmaf(-2.f, s, yv + xv[r]), 0.f);
            const float rr = __builtin_sqrtf(d2);
            const float K = __builtin_amdgcn_exp2f(-L * rr);
            w = rr > 0.f ? K * __builtin_amdgcn_rcpf(rr) : 0.f;
            dh = K * rr;
            if constexpr (KS) ks32 += K;
            csq = __builtin_fmaf(K, K, csq);
            cmx = fmaxf(cmx, K);
          }
          acc[bi][r] = w;
          rw32 += w;
          dh32 += dh;
        }
      }
      rws += (double)rw32;
      dhs += (double)dh32;
      if constexpr (KS) kss += (double)ks32;
    }

    // G[q][t] += sum over the staged rows of W[q][i] x~[i][t]
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const char* row = xb + (bi * 16 + 4 * g + r) * G::PITCH;
        const float w = acc[bi][r];
#pragma unroll
        for (int nb = 0; nb < G::NB; ++nb) {
          const u32x4 xv = *reinterpret_cast<const u32x4*>(row + (nb * 64 + 4 * c) * 4);
          gacc[4 * nb + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.x), gacc[4 * nb + 0], 0, 0, 0);
          gacc[4 * nb + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.y), gacc[4 * nb + 1], 0, 0, 0);
          gacc[4 * nb + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.z), gacc[4 * nb + 2], 0, 0, 0);
          gacc[4 * nb + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.w), gacc[4 * nb + 3], 0, 0, 0);
        }
        if constexpr (G::HB) {
          const uint2 xv = *reinterpret_cast<const uint2*>(row + (G::NB * 64 + 2 * c) * 4);
          gacc[4 * G::NB + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.x), gacc[4 * G::NB + 0], 0, 0, 0);
          gacc[4 * G::NB + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.y), gacc[4 * G::NB + 1], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();   // tile t+1 staged; buffer b free for tile t+2
  }
  flush_grad<DP>(gacc, gpart, g, c, fresh);
  fresh = false;
  }

  // per-query sums: the four lane groups of a query column (fixed order)
  rws += __shfl_xor(rws, 16, 64);
  rws += __shfl_xor(rws, 32, 64);
  dhs += __shfl_xor(dhs, 16, 64);
  dhs += __shfl_xor(dhs, 32, 64);
  if constexpr (KS) {
    kss += __shfl_xor(kss, 16, 64);
    kss += __shfl_xor(kss, 32, 64);
  }
  csq += __shfl_xor(csq, 16, 64);
  csq += __shfl_xor(csq, 32, 64);
  if (KERN == KERNEL_GAUSSIAN) {
    cmx += __shfl_xor(cmx, 16, 64);
    cmx += __shfl_xor(cmx, 32, 64);
  } else {
    cmx = fmaxf(cmx, __shfl_xor(cmx, 16, 64));
    cmx = fmaxf(cmx, __shfl_xor(cmx, 32, 64));
  }
  if (g == 0) {
    rw_part[qbase + c] = rws;
    gh_part[qbase + c] = dhs;
    if constexpr (KS) ks_part[qbase + c] = kss;
    cert[qbase + c] = make_float2(csq, cmx);
  }
  if (fresh) flush_grad<DP>(gacc, gpart, g, c, true);   // empty range: zeros
}

// The same pass with the distance product from three-part bfloat16 rows (see
// kde_split_kernel): S^T on v_mfma_f32_16x16x32_bf16 (six products per element,
// float32-accurate), the second product G += W X~ on FP32 MFMAs as above.
// Data rows are staged 64 at a time: the split rows double-buffered for the
// first product, the float32 rows of the current 64 for the second (two
// barriers per staged tile).
template <int KERN, int DPS, int DP, bool VAL>
__global__ void __launch_bounds__(BWG, 1)
kde_backward_split_kernel(TileProblem p, const char* __restrict__ Xsp,
                          const char* __restrict__ Ysp, float L, double* __restrict__ gy_part,
                          double* __restrict__ rw_part, double* __restrict__ gh_part,
                          double* __restrict__ ks_part, float2* __restrict__ cert,
                          float* __restrict__ certk) {
  using G = GradTile<DP>;
  // the certificate needs sum K for the exponential kernel (Gaussian: the weights)
  constexpr bool KS = KERN != KERNEL_GAUSSIAN;
  (void)VAL;
  constexpr int TR = 64, NBI = TR / 16, UPT = BN / TR;
  constexpr int KC = DPS / 32;                 // 32-element k-chunks per plane
  constexpr int RB = 3 * DPS * 2;              // bytes per split row
  constexpr int SPITCH = RB + 16, SPPR = RB / 16, SNPT = TR * SPPR / BWG;
  constexpr int FNPT = TR * G::PPR / BWG;      // float32 pieces per thread
  static_assert(SNPT >= 1 && TR * SPPR == SNPT * BWG, "split pieces must split evenly");
  static_assert(FNPT >= 1 && TR * G::PPR == FNPT * BWG, "row pieces must split evenly");
  __shared__ __attribute__((aligned(16))) char xs[2][TR * SPITCH];   // split rows
  __shared__ __attribute__((aligned(16))) char xf[TR * G::PITCH];    // float32 rows
  __shared__ __attribute__((aligned(16))) float xvs[2][TR];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t u0 = split * p.ntiles / p.splits * UPT, u1 = (split + 1) * p.ntiles / p.splits * UPT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;

  const int64_t qrow = qt * BQ + wave * 16 + c;
  u32x4 yh[KC], ym[KC], yl[KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    const char* yr = Ysp + qrow * RB + kc * 64 + g * 16;
    yh[kc] = *reinterpret_cast<const u32x4*>(yr);
    ym[kc] = *reinterpret_cast<const u32x4*>(yr + DPS * 2);
    yl[kc] = *reinterpret_cast<const u32x4*>(yr + DPS * 4);
  }
  const double ynq = p.ynorm[qrow];
  const float yv = KERN == KERNEL_GAUSSIAN ? (float)(-(double)L * ynq) : (float)ynq;

  u32x4 xr[SNPT], xq[FNPT];
  float xvr = 0.f;
  auto gload = [&](int64_t u) {
    const char* sb = Xsp + u * TR * RB;
#pragma unroll
    for (int i = 0; i < SNPT; ++i) {
      const int v = threadIdx.x + i * BWG;
      xr[i] = *reinterpret_cast<const u32x4*>(sb + (v / SPPR) * RB + (v % SPPR) * 16);
    }
    const char* fb = p.Xs + u * TR * p.ld_bytes;
#pragma unroll
    for (int i = 0; i < FNPT; ++i) {
      const int v = threadIdx.x + i * BWG;
      xq[i] = *reinterpret_cast<const u32x4*>(fb + (v / G::PPR) * p.ld_bytes + (v % G::PPR) * 16);
    }
    if (threadIdx.x < TR) {
      const int64_t row = u * TR + threadIdx.x;
      xvr = row < p.n ? (KERN == KERNEL_GAUSSIAN ? (float)(-(double)L * p.xnorm[row])
                                                 : (float)p.xnorm[row])
                      : (KERN == KERNEL_GAUSSIAN ? -1e30f : 1e30f);
    }
  };
  auto store_split = [&](int b) {
#pragma unroll
    for (int i = 0; i < SNPT; ++i) {
      const int v = threadIdx.x + i * BWG;
      *reinterpret_cast<u32x4*>(&xs[b][(v / SPPR) * SPITCH + (v % SPPR) * 16]) = xr[i];
    }
    if (threadIdx.x < TR) xvs[b][threadIdx.x] = xvr;
  };
  auto store_rows = [&]() {
#pragma unroll
    for (int i = 0; i < FNPT; ++i) {
      const int v = threadIdx.x + i * BWG;
      *reinterpret_cast<u32x4*>(&xf[(v / G::PPR) * G::PITCH + (v % G::PPR) * 16]) = xq[i];
    }
  };

  f32x4 gacc[G::GB];
#pragma unroll
  for (int i = 0; i < G::GB; ++i) gacc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  double rws = 0.0, dhs = 0.0, kss = 0.0;
  // certificate: sum of K^2; Gaussian: sum of K times its exponent, exponential:
  // largest K; sum of K N (the bfloat16 MFMA's truncation bias, see cert.h)
  float csq = 0.f, cmx = 0.f, ckn = 0.f;

  const int64_t qbase = split * p.qp + qt * BQ + wave * 16;
  double* gpart = gy_part + qbase * DP;
  bool fresh = true;

  if (u0 < u1) {
    gload(u0);
    store_split(0);
    store_rows();
  }
  __syncthreads();
  for (int64_t uc = u0; uc < u1; uc += kGradFlushRows / TR) {
  const int64_t ue = uc + kGradFlushRows / TR < u1 ? uc + kGradFlushRows / TR : u1;
  for (int64_t u = uc; u < ue; ++u) {
    const int b = (int)((u - u0) & 1);
    const bool more = u + 1 < u1;
    if (more) gload(u + 1);
    const char* xb = xs[b];
    f32x4 acc[NBI], accx[NBI];
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) {
      acc[bi] = f32x4{0.f, 0.f, 0.f, 0.f};
      accx[bi] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) {
        const char* ar = xb + (bi * 16 + c) * SPITCH + kc * 64 + g * 16;
        const u32x4 ah = *reinterpret_cast<const u32x4*>(ar);
        const u32x4 am = *reinterpret_cast<const u32x4*>(ar + DPS * 2);
        const u32x4 al = *reinterpret_cast<const u32x4*>(ar + DPS * 4);
        f32x4 t = accx[bi];
        t = mfma_kgroup<__bf16>(al, yh[kc], t);
        t = mfma_kgroup<__bf16>(am, ym[kc], t);
        t = mfma_kgroup<__bf16>(ah, yl[kc], t);
        t = mfma_kgroup<__bf16>(am, yh[kc], t);
        accx[bi] = mfma_kgroup<__bf16>(ah, ym[kc], t);
        acc[bi] = mfma_kgroup<__bf16>(ah, yh[kc], acc[bi]);
      }
    }
    // the leading products and the five small ones accumulate apart: each MFMA
    // rounds into its accumulator, so the small terms do not round into the
    // large running sum
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) acc[bi] += accx[bi];
    __builtin_amdgcn_s_setprio(0);
    if (more) store_split(b ^ 1);   // that buffer was last read before the previous barriers

    const f32x4* xv4 = reinterpret_cast<const f32x4*>(xvs[b]);
#pragma unroll
    for (int bp = 0; bp < NBI / 2; ++bp) {
      float rw32 = 0.f, dh32 = 0.f, ks32 = 0.f;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int bi = 2 * bp + h2;
        const f32x4 xv = xv4[bi * 4 + g];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float sv = acc[bi][r];
          float w, dh;
          const float nl = yv + xv[r];   // -L N (Gaussian) or N; padding: huge
          if (KERN == KERNEL_GAUSSIAN) {
            const float a = fminf(__builtin_fmaf(2.f * L, sv, nl), 0.f);   // -L d^2
            const float K = __builtin_amdgcn_exp2f(a);
            w = K;
            dh = K * a;
            csq = __builtin_fmaf(K, K, csq);
            cmx = __builtin_fmaf(-K, a, cmx);   // Gaussian: sum of K times its exponent
            ckn = __builtin_fmaf(K, -nl, ckn);
          } else {
            const float d2 = fmaxf(__builtin_fmaf(-2.f, sv, nl), 0.f);
            const float rr = __builtin_sqrtf(d2);
            const float K = __builtin_amdgcn_exp2f(-L * rr);
            w = rr > 0.f ? K * __builtin_amdgcn_rcpf(rr) : 0.f;
            dh = K * rr;
            if constexpr (KS) ks32 += K;
            csq = __builtin_fmaf(K, K, csq);
            cmx = fmaxf(cmx, K);
            ckn = __builtin_fmaf(K, fminf(nl, 3.0e38f), ckn);
          }
          acc[bi][r] = w;
          rw32 += w;
          dh32 += dh;
        }
      }
      rws += (double)rw32;
      dhs += (double)dh32;
      if constexpr (KS) kss += (double)ks32;
    }

    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const char* row = xf + (bi * 16 + 4 * g + r) * G::PITCH;
        const float w = acc[bi][r];
#pragma unroll
        for (int nb = 0; nb < G::NB; ++nb) {
          const u32x4 xv = *reinterpret_cast<const u32x4*>(row + (nb * 64 + 4 * c) * 4);
          gacc[4 * nb + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.x), gacc[4 * nb + 0], 0, 0, 0);
          gacc[4 * nb + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.y), gacc[4 * nb + 1], 0, 0, 0);
          gacc[4 * nb + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.z), gacc[4 * nb + 2], 0, 0, 0);
          gacc[4 * nb + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.w), gacc[4 * nb + 3], 0, 0, 0);
        }
        if constexpr (G::HB) {
          const uint2 xv = *reinterpret_cast<const uint2*>(row + (G::NB * 64 + 2 * c) * 4);
          gacc[4 * G::NB + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.x), gacc[4 * G::NB + 0], 0, 0, 0);
          gacc[4 * G::NB + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, __uint_as_float(xv.y), gacc[4 * G::NB + 1], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();   // the float32 rows and split buffer b are no longer read
    if (more) store_rows();
    __syncthreads();   // staged tile u+1 published
  }
  flush_grad<DP>(gacc, gpart, g, c, fresh);
  fresh = false;
  }

  rws += __shfl_xor(rws, 16, 64);
  rws += __shfl_xor(rws, 32, 64);
  dhs += __shfl_xor(dhs, 16, 64);
  dhs += __shfl_xor(dhs, 32, 64);
  if constexpr (KS) {
    kss += __shfl_xor(kss, 16, 64);
    kss += __shfl_xor(kss, 32, 64);
  }
  csq += __shfl_xor(csq, 16, 64);
  csq += __shfl_xor(csq, 32, 64);
  ckn += __shfl_xor(ckn, 16, 64);
  ckn += __shfl_xor(ckn, 32, 64);
  if (KERN == KERNEL_GAUSSIAN) {
    cmx += __shfl_xor(cmx, 16, 64);
    cmx += __shfl_xor(cmx, 32, 64);
  } else {
    cmx = fmaxf(cmx, __shfl_xor(cmx, 16, 64));
    cmx = fmaxf(cmx, __shfl_xor(cmx, 32, 64));
  }
  if (g == 0) {
    rw_part[qbase + c] = rws;
    gh_part[qbase + c] = dhs;
    if constexpr (KS) ks_part[qbase + c] = kss;
    cert[qbase + c] = make_float2(csq, cmx);
    certk[qbase + c] = ckn;
  }
  if (fresh) flush_grad<DP>(gacc, gpart, g, c, true);   // empty range: zeros
}

// grad_Y[q] = g_q / n * c_y * f_q * (sum_s G_s[q] - y~_q sum_s rowsum_s[q]) and the
// per-query h term g_q / n * c_h * f_q * sum_s dh_s[q], where c_y, c_h are the
// constant factors left out of the tile weights and f_q is the Gaussian query
// factor 2^(rounding remainder of -L ||y||^2) (1 for the exponential kernel);
// g_q = grad_out[q], or 1 when grad_out is null.  With mu non-null also the
// KDE itself, f_q / n * sum_s K_s[q] (ks_part, or the Gaussian weight sums).
__global__ void kde_backward_reduce_kernel(const double* __restrict__ gy_part,
                                           const double* __restrict__ rw_part,
                                           const double* __restrict__ gh_part,
                                           const double* __restrict__ ks_part,
                                           const float* __restrict__ Ys, int64_t splits,
                                           int64_t qp, int64_t q, int64_t d, int64_t dp,
                                           int64_t n, double inv_n,
                                           const double* __restrict__ ynorm,
                                           float L, int kern, double c_y, double c_h,
                                           const double* __restrict__ grad_out,
                                           float* __restrict__ grad_Y, double* __restrict__ ghq,
                                           double* __restrict__ mu, CertArgs ca) {
  const int64_t qi = blockIdx.x;
  __shared__ double rw_s, f_s;
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0, A = 0.0, y2 = 0.0, AK = 0.0;
    for (int64_t s = 0; s < splits; ++s) {
      a += rw_part[s * qp + qi];
      b += gh_part[s * qp + qi];
      const float2 cc = ca.part[s * qp + qi];
      A += (double)cc.x;
      y2 = kern == KERNEL_GAUSSIAN ? y2 + (double)cc.y : fmax(y2, (double)cc.y);
      if (ca.pk) AK += (double)ca.pk[s * qp + qi];
    }
    if (ks_part)
      for (int64_t s = 0; s < splits; ++s) c += ks_part[s * qp + qi];
    double f = 1.0;
    if (kern == KERNEL_GAUSSIAN) {
      const double e = -(double)L * ynorm[qi];
      f = exp2(e - (double)(float)e);
    }
    const double g = grad_out ? grad_out[qi] : 1.0;
    rw_s = a;
    f_s = f;
    if (ghq) ghq[qi] = g * inv_n * c_h * f * b;
    const double T = ks_part ? c : a;   // sum of K (Gaussian: the weights themselves)
    if (mu) mu[qi] = f * T * inv_n;
    cert_check(qi, T, A * 1.01, kern == KERNEL_GAUSSIAN ? y2 * 1.01 : y2, f, ynorm[qi], n, L,
               kern, ca, -1.0, ca.pk ? AK * 1.02 : -1.0);
  }
  __syncthreads();
  if (!grad_Y) return;
  const double sc = (grad_out ? grad_out[qi] : 1.0) * inv_n * c_y * f_s;
  for (int64_t t = threadIdx.x; t < d; t += blockDim.x) {
    double g = 0.0;
    for (int64_t s = 0; s < splits; ++s) g += gy_part[(s * qp + qi) * dp + t];
    grad_Y[qi * d + t] = (float)(sc * (g - (double)Ys[qi * dp + t] * rw_s));
  }
}

// The weight loops no longer depend on VAL (the exponential kernel always sums
// K for the certificate), so one instantiation serves the adjoint and the fused
// value + gradient pass.
template <int KERN>
static hipError_t launch_kde_bwd_split(const TileProblem& p, const SplitRows& sp, int64_t dp,
                                       float L, double* gy, double* rw, double* gh, double* ks,
                                       float2* cert, float* ck, hipStream_t s) {
  const dim3 g((unsigned)p.map.grid), b(BWG);
  const char* Xs = reinterpret_cast<const char*>(sp.X);
  const char* Ys = reinterpret_cast<const char*>(sp.Y);
  if (sp.dps == 64 && dp == 32)
    kde_backward_split_kernel<KERN, 64, 32, false><<<g, b, 0, s>>>(p, Xs, Ys, L, gy, rw, gh, ks, cert, ck);
  else if (sp.dps == 64 && dp == 64)
    kde_backward_split_kernel<KERN, 64, 64, false><<<g, b, 0, s>>>(p, Xs, Ys, L, gy, rw, gh, ks, cert, ck);
  else if (sp.dps == 128 && dp == 96)
    kde_backward_split_kernel<KERN, 128, 96, false><<<g, b, 0, s>>>(p, Xs, Ys, L, gy, rw, gh, ks, cert, ck);
  else if (sp.dps == 128 && dp == 128)
    kde_backward_split_kernel<KERN, 128, 128, false><<<g, b, 0, s>>>(p, Xs, Ys, L, gy, rw, gh, ks, cert, ck);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int KERN>
static hipError_t launch_kde_bwd_k(const TileProblem& p, int64_t dp, float L, double* gy, double* rw,
                                   double* gh, double* ks, float2* cert, hipStream_t s) {
  const dim3 g((unsigned)p.map.grid), b(BWG);
  switch (dp) {
    case 32: kde_backward_kernel<KERN, 32, false, 128><<<g, b, 0, s>>>(p, L, gy, rw, gh, ks, cert); break;
    case 64: kde_backward_kernel<KERN, 64, false, BWD_TR_64><<<g, b, 0, s>>>(p, L, gy, rw, gh, ks, cert); break;
    case 96: kde_backward_kernel<KERN, 96, false, 128><<<g, b, 0, s>>>(p, L, gy, rw, gh, ks, cert); break;
    case 128: kde_backward_kernel<KERN, 128, false, 128><<<g, b, 0, s>>>(p, L, gy, rw, gh, ks, cert); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Gaussian mean-shift step from the density and its gradient:
// y <- y + h^2 grad / mu, which is the kernel-weighted mean of the rows.
__global__ void mean_shift_update_kernel(const float* Y, const float* __restrict__ g,
                                         const double* __restrict__ mu, int64_t q, int64_t d,
                                         double h2, float* Y_out) {   // Y_out may alias Y
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q * d) return;
  const double m = mu[i / d];
  Y_out[i] = m > 0.0 ? (float)((double)Y[i] + h2 * (double)g[i] / m) : Y[i];
}

hipError_t launch_mean_shift_update(const float* Y, const float* g, const double* mu, int64_t q,
                                    int64_t d, double h, float* Y_out, hipStream_t s) {
  if (q == 0) return hipSuccess;
  const int64_t total = q * d;
  mean_shift_update_kernel<<<dim3((unsigned)ceil_div(total, WG)), dim3(WG), 0, s>>>(
      Y, g, mu, q, d, h * h, Y_out);
  return hipGetLastError();
}

hipError_t launch_kde_backward(const TileProblem& p, const float* X, const float* Y, int64_t d,
                               double h, int kern, const double* grad_out, double* gy_part,
                               double* gh_part, float* grad_Y, double* grad_h, hipStream_t s,
                               TimingHook th, double* mu, double* gh_per_query, SplitRows split,
                               const CertArgs& ca) {
  const int64_t dp = p.ld_bytes / 4;
  const double log2e = 1.4426950408889634;
  const float L = (float)(kern == KERNEL_GAUSSIAN ? log2e / (2.0 * h * h) : log2e / h);
  // layout: gh [splits][qp], rw [splits][qp], ks [splits][qp], ghq [q]
  double* rw_part = gh_part + p.splits * p.qp;
  double* ks_part = rw_part + p.splits * p.qp;
  double* ghq = gh_per_query ? gh_per_query : ks_part + p.splits * p.qp;
  hipError_t e;
  if (th.start && (e = hipEventRecord(th.start, s)) != hipSuccess) return e;
  if (split.X)   // distance product from three-part bfloat16 rows
    e = kern == KERNEL_GAUSSIAN
            ? launch_kde_bwd_split<KERNEL_GAUSSIAN>(p, split, dp, L, gy_part, rw_part, gh_part,
                                                    ks_part, ca.part, ca.pk, s)
            : launch_kde_bwd_split<KERNEL_EXPONENTIAL>(p, split, dp, L, gy_part, rw_part, gh_part,
                                                       ks_part, ca.part, ca.pk, s);
  else
    e = kern == KERNEL_GAUSSIAN
            ? launch_kde_bwd_k<KERNEL_GAUSSIAN>(p, dp, L, gy_part, rw_part, gh_part, ks_part,
                                                ca.part, s)
            : launch_kde_bwd_k<KERNEL_EXPONENTIAL>(p, dp, L, gy_part, rw_part, gh_part, ks_part,
                                                   ca.part, s);
  if (e != hipSuccess) return e;
  if (th.stop && (e = hipEventRecord(th.stop, s)) != hipSuccess) return e;
  // Gaussian: weights K, dh terms K * (-L d^2); exponential: weights K / r, dh terms K r
  const double c_y = kern == KERNEL_GAUSSIAN ? 1.0 / (h * h) : 1.0 / h;
  const double c_h = kern == KERNEL_GAUSSIAN ? -1.0 / (h * h * h * (double)L) : 1.0 / (h * h);
  const bool need_ghq = grad_h || gh_per_query;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(ca.fb_count), 1, 0u, s)) != hipSuccess)
    return e;
  CertArgs cb = ca;
  if (!split.X) cb.pk = nullptr;   // float32 MFMAs round to nearest: no bias term
  kde_backward_reduce_kernel<<<dim3((unsigned)p.q), dim3(128), 0, s>>>(
      gy_part, rw_part, gh_part, kern != KERNEL_GAUSSIAN ? ks_part : nullptr,
      reinterpret_cast<const float*>(p.Ys), p.splits, p.qp, p.q, d, dp, p.n, 1.0 / (double)p.n,
      p.ynorm, L, kern, c_y, c_h, grad_out, grad_Y, need_ghq ? ghq : nullptr, mu, cb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // exact re-evaluation of the listed queries; its scratch reuses the sweep's
  // partials, which the reduction has consumed: value and h sums in the gh and
  // rw parts, the weighted row sums in gy_part ([splits][qp][dp] >= [fs][q][dp])
  e = launch_kde_direct_grad(X, Y, p.n, p.q, d, h, kern, ca.fb_ids, ca.fb_count,
                             p.splits * p.qp, gh_part, rw_part, gy_part, dp, grad_out, grad_Y,
                             need_ghq ? ghq : nullptr, mu, s);
  if (e != hipSuccess) return e;
  if (!grad_h) return hipSuccess;
  sum_scalar_kernel<<<dim3(1), dim3(WG), 0, s>>>(ghq, p.q, grad_h);
  return hipGetLastError();
}

}  // namespace deann
