// Preparation of the scan operands (the paper's norm precomputation, App. F).
//
// Every distance tile works on a centred copy of the data: x~ = T(x - c) with
// c the column mean of X (the KDE is translation invariant), stored in the
// scan precision T with rows zero-padded to a multiple of 128 bytes.  Per row
// we keep
//   norm  = ||x~||^2 (FP64),
//   knorm = ||x~||^2 (1 - a): scaled so that knorm_x + knorm_y - 2 x~.y~, as
//           computed in FP32, never exceeds the exact ||x~ - y~||^2,
//   err   = an upper bound of ||x~ - (x - c)||, the rounding of the row.
// Hence for every pair ||x - y|| >= sqrt(max(key, 0)) - err_x - err_y.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace deann {

// Column sums of X over a slice of rows: grid (ceil(d/64), R), 256 threads.
__global__ void __launch_bounds__(WG) center_partial_kernel(const float* __restrict__ X, int64_t n,
                                                            int64_t d, int64_t rows_per,
                                                            double* __restrict__ part) {
  __shared__ double red[WG];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + tx;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
  // four independent accumulators (rows r, r+4, r+8, r+12 of each step of 16),
  // combined in a fixed order
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (col < d) {
    int64_t r = r0 + ty;
    for (; r + 12 < r1; r += 16) {
      s0 += (double)X[r * d + col];
      s1 += (double)X[(r + 4) * d + col];
      s2 += (double)X[(r + 8) * d + col];
      s3 += (double)X[(r + 12) * d + col];
    }
    for (; r < r1; r += 4) s0 += (double)X[r * d + col];
  }
  red[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (ty == 0 && col < d)
    part[(int64_t)blockIdx.y * d + col] = ((red[tx] + red[tx + 64]) + red[tx + 128]) + red[tx + 192];
}

// One workgroup per column: strided partial sums, then a fixed-order tree.
__global__ void __launch_bounds__(WG) center_finalize_kernel(const double* __restrict__ part,
                                                             int64_t R, int64_t n, int64_t d,
                                                             float* __restrict__ c) {
  __shared__ double red[WG];
  const int64_t col = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < R; r += WG) s += part[r * d + col];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = WG / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) c[col] = (float)(red[0] / (double)n);
}

template <typename T>
__device__ __forceinline__ T to_elem(float v);
template <> __device__ __forceinline__ float to_elem<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 to_elem<__bf16>(float v) { return (__bf16)v; }
template <> __device__ __forceinline__ _Float16 to_elem<_Float16>(float v) { return (_Float16)v; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per row: centre, round, norms and rounding-error bound.
// Rows in [rows, rows_padded) are written as zeros.
template <typename T>
__global__ void __launch_bounds__(WG) prep_rows_kernel(const float* __restrict__ src, int64_t rows,
                                                       int64_t rows_padded, int64_t d, int64_t dp,
                                                       const float* __restrict__ c, double a_scale,
                                                       T* __restrict__ dst, double* __restrict__ norm,
                                                       float* __restrict__ knorm,
                                                       float* __restrict__ err,
                                                       uint32_t* __restrict__ err_max) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
  if (row >= rows_padded) return;
  T* out = dst + row * dp;
  if (row >= rows) {
    for (int64_t t = lane; t < dp; t += 64) out[t] = to_elem<T>(0.f);
    if (lane == 0) { norm[row] = 0.0; knorm[row] = 0.f; err[row] = 0.f; }
    return;
  }
  const float* in = src + row * d;
  double nn = 0.0, ee = 0.0;
  if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    // four consecutive coordinates per lane and step (16-byte loads; dp and d
    // are multiples of 4, the centre and the output rows 16- and 8-byte aligned)
    for (int64_t t = 4 * lane; t < dp; t += 256) {
      T r[4];
      if (t < d) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(in + t);
        const f32x4 cc = *reinterpret_cast<const f32x4*>(c + t);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          r[k] = to_elem<T>(v[k] - cc[k]);
          const double rd = (double)(float)r[k];
          nn += rd * rd;
          const double dlt = rd - ((double)v[k] - (double)cc[k]);   // exact in FP64
          ee += dlt * dlt;
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = to_elem<T>(0.f);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) out[t + k] = r[k];
    }
  } else {
    for (int64_t t = lane; t < dp; t += 64) {
      if (t < d) {
        const float v = in[t];
        const T r = to_elem<T>(v - c[t]);
        out[t] = r;
        const double rd = (double)(float)r;
        nn += rd * rd;
        const double exact = (double)v - (double)c[t];   // exact in FP64
        const double dlt = rd - exact;
        ee += dlt * dlt;
      } else {
        out[t] = to_elem<T>(0.f);
      }
    }
  }
  nn = wave_sum(nn);
  ee = wave_sum(ee);
  if (lane == 0) {
    norm[row] = nn;
    // round the scaled norm down and the error bound up
    knorm[row] = (float)(nn * (1.0 - a_scale));
    // FP32 rounding is below 6e-8 relative, so the 1e-6 margin keeps e an upper bound
    err[row] = (float)(sqrt(ee) * (1.0 + 1e-6));
  }
}

// Largest error bound over the rows: block maxima, one atomic per block
// (non-negative floats order like their bit patterns).
__global__ void __launch_bounds__(WG) max_u32_kernel(const float* __restrict__ v, int64_t count,
                                                     uint32_t* __restrict__ out) {
  __shared__ uint32_t red[WG / 64];
  uint32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < count; i += (int64_t)gridDim.x * WG)
    m = max(m, __builtin_bit_cast(uint32_t, v[i]));
  for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = red[0];
    for (int w = 1; w < WG / 64; ++w) r = max(r, red[w]);
    atomicMax(out, r);
  }
}

template <typename T>
hipError_t launch_prep_rows(const float* src, int64_t rows, int64_t rows_padded, int64_t d,
                            int64_t dp, const float* c, double a_scale, void* dst, double* norm,
                            float* knorm, float* err, uint32_t* err_max, hipStream_t s) {
  const int64_t blocks = ceil_div(rows_padded, WG / 64);
  prep_rows_kernel<T><<<dim3((unsigned)blocks), dim3(WG), 0, s>>>(
      src, rows, rows_padded, d, dp, c, a_scale, reinterpret_cast<T*>(dst), norm, knorm, err,
      err_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !err_max) return e;
  const int64_t mb = std::min<int64_t>(1024, ceil_div(rows, WG));
  max_u32_kernel<<<dim3((unsigned)mb), dim3(WG), 0, s>>>(err, rows, err_max);
  return hipGetLastError();
}

// Three bfloat16 parts of every prepared float32 value, v = h + m + l exactly
// (h the nearest bfloat16 to v, m the nearest to v - h, l = v - h - m, which
// has at most 8 significant bits): row r holds the planes h, m, l of dps
// elements each (zeros beyond dp32).
__global__ void __launch_bounds__(WG) split_rows_kernel(const float* __restrict__ src,
                                                        int64_t rows, int64_t dp32, int64_t dps,
                                                        __bf16* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= rows * dps) return;
  const int64_t r = i / dps, t = i % dps;
  const float v = t < dp32 ? src[r * dp32 + t] : 0.f;
  const __bf16 h = (__bf16)v;
  const float rem = v - (float)h;          // exact
  const __bf16 m = (__bf16)rem;
  const __bf16 l = (__bf16)(rem - (float)m);   // exact
  __bf16* out = dst + r * 3 * dps;
  out[t] = h;
  out[dps + t] = m;
  out[2 * dps + t] = l;
}

hipError_t launch_split_rows(const float* src, int64_t rows, int64_t dp32, int64_t dps,
                             void* dst, hipStream_t s) {
  const int64_t total = rows * dps;
  if (total == 0) return hipSuccess;
  split_rows_kernel<<<dim3((unsigned)ceil_div(total, WG)), dim3(WG), 0, s>>>(
      src, rows, dp32, dps, reinterpret_cast<__bf16*>(dst));
  return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_u32_kernel<<<dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s>>>(p, count, v);
  return hipGetLastError();
}

__global__ void copy_u32_kernel(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  copy_u32_kernel<<<dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s>>>(dst, src, count);
  return hipGetLastError();
}

hipError_t launch_max_u32(const float* v, int64_t count, uint32_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t mb = std::min<int64_t>(1024, ceil_div(count, WG));
  max_u32_kernel<<<dim3((unsigned)mb), dim3(WG), 0, s>>>(v, count, out);
  return hipGetLastError();
}

hipError_t launch_center(const float* X, int64_t n, int64_t d, double* part, int64_t R, float* c,
                         hipStream_t s) {
  const int64_t rows_per = ceil_div(n, R);
  center_partial_kernel<<<dim3((unsigned)ceil_div(d, 64), (unsigned)R), dim3(WG), 0, s>>>(
      X, n, d, rows_per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  center_finalize_kernel<<<dim3((unsigned)d), dim3(WG), 0, s>>>(part, R, n, d, c);
  return hipGetLastError();
}

hipError_t launch_prep_rows_prec(int prec, const float* src, int64_t rows, int64_t rows_padded,
                                 int64_t d, int64_t dp, const float* c, double a_scale, void* dst,
                                 double* norm, float* knorm, float* err, uint32_t* err_max,
                                 hipStream_t s) {
  switch (prec) {
    case PREC_FP32:
      return launch_prep_rows<float>(src, rows, rows_padded, d, dp, c, a_scale, dst, norm, knorm,
                                     err, err_max, s);
    case PREC_BF16:
      return launch_prep_rows<__bf16>(src, rows, rows_padded, d, dp, c, a_scale, dst, norm, knorm,
                                      err, err_max, s);
    default:
      return launch_prep_rows<_Float16>(src, rows, rows_padded, d, dp, c, a_scale, dst, norm,
                                        knorm, err, err_max, s);
  }
}

}  // namespace deann
