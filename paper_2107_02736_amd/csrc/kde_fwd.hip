// Exact KDE, Eq. (1), for the Gaussian kernel of Eq. (2) and the exponential
// kernel.  Distances come from the GEMM identity of App. F,
// ||x - y||^2 = ||x||^2 + ||y||^2 - 2 <x, y>, with <x, y> on MFMA; the kernel
// value and the row sum are fused into the tile epilogue (App. F steps
// (i)-(iii) without materialising the distance matrix).
//
// Grid: (query tile, data split) pairs, XCD-aware.  Each workgroup walks the
// data tiles of its split and keeps, per lane, FP32 sums of one tile folded
// into FP64 accumulators; the per-split FP64 partials are summed in a fixed
// order by kde_reduce_kernel, so results are bitwise reproducible.
//
// The epilogue is FP32.  Gaussian: with L = log2(e) / (2 h^2) rounded to FP32,
// the exponent -L d^2 = 2L <x,y> + (-L ||y||^2) + (-L ||x||^2) is one FMA on
// the MFMA result after one add of the two norm terms, each rounded to FP32
// from FP64 norms.  The rounding remainder of the query term is the same for
// every pair of that query, so it factors out of the kernel sum exactly:
// kde_reduce_kernel multiplies the query's FP64 total by 2^remainder.  The
// remaining roundings (data term, the add, the FMA) differ from pair to pair.
// Exponential: d^2 = ||y||^2 + ||x||^2 - 2 <x,y> in FP32, clamped at 0.
#include "common.h"
#include "kernels.h"

namespace deann {

template <typename T, int KERN, int ENG>   // ENG: see tile_engine
__global__ void __launch_bounds__(WG, 2)
kde_tile_kernel(const char* __restrict__ Ys, const char* __restrict__ Xs, int64_t ld_bytes,
                int nchunks, const double* __restrict__ ynorm, const double* __restrict__ xnorm,
                int64_t n, int64_t qtiles, int64_t splits, int64_t ntiles, float Lf,
                double* __restrict__ partial, int64_t qp, TileMap map) {
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, map, qtiles, splits, qt, split)) return;
  const int64_t t0 = split * ntiles / splits, t1 = (split + 1) * ntiles / splits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  const float L2 = 2.f * Lf;

  // per-row query terms (see the file comment)
  float yt[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double yn = ynorm[qt * BQ + wq * 64 + i * 16 + 4 * (lane >> 4) + r];
      yt[i][r] = KERN == KERNEL_GAUSSIAN ? (float)(-(double)Lf * yn) : (float)yn;
    }
  double sum[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum[i][r] = 0.0;

  const char* yq = Ys + qt * BQ * ld_bytes;
  constexpr int NK = 2;   // k-groups of the register-resident engine
  StreamState st;
  XStream<NK> xs;
  u32x4 yf[4][NK];
  QlState ql;
  if (t0 < t1) {
    if constexpr (ENG == 0) {
      stream_start(st, yq, Xs, ld_bytes, t0);
    } else if constexpr (ENG == 1) {
      ql_start(ql, yq, Xs, t0, lds);
    } else {
      yreg_load<NK>(yf, yq, ld_bytes, wq, lane);
      xs_load(xs, Xs + t0 * BN * ld_bytes, ld_bytes);
      xs.buf = 0;
    }
  }
  // The data norms of a tile are fetched one tile ahead, one per thread, and
  // staged in LDS (double-buffered) when the tile starts; the barrier inside
  // the tile sweep publishes them before the epilogue.  xnorm covers the
  // padded rows.
  __shared__ double xns[2][BN];
  double xn_reg = (threadIdx.x < BN && t0 < t1) ? xnorm[t0 * BN + threadIdx.x] : 0.0;
  for (int64_t t = t0; t < t1; ++t) {
    const int nb = (int)((t - t0) & 1);
    if (threadIdx.x < BN) {
      xns[nb][threadIdx.x] = xn_reg;
      if (t + 1 < t1) xn_reg = xnorm[(t + 1) * BN + threadIdx.x];
    }
    f32x4 acc[4][4];
    if constexpr (ENG == 0)
      stream_tile<T>(acc, st, yq, Xs, ld_bytes, nchunks, t, t1, lds, wq, wn, lane);
    else if constexpr (ENG == 1)
      ql_tile<T>(acc, ql, Xs, t, t1, lds, wq, wn, lane);
    else
      yreg_tile<T, NK>(acc, xs, yf, Xs, ld_bytes, t, t1, lds, wn, lane);
    // per-column data terms; padding columns get a term that zeroes the kernel
    float xt[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
      const double xn = xns[nb][wn * 64 + j * 16 + (lane & 15)];
      if (KERN == KERNEL_GAUSSIAN)
        xt[j] = col < n ? (float)(-(double)Lf * xn) : -__builtin_inff();
      else
        xt[j] = col < n ? (float)xn : __builtin_inff();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float part = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float kv;
          if (KERN == KERNEL_GAUSSIAN) {   // exp(-d^2 / (2 h^2))
            const float a = fminf(__builtin_fmaf(L2, acc[i][j][r], yt[i][r] + xt[j]), 0.f);
            kv = __builtin_amdgcn_exp2f(a);
          } else {                          // exp(-d / h)
            const float d2 = fmaxf(__builtin_fmaf(-2.f, acc[i][j][r], yt[i][r] + xt[j]), 0.f);
            kv = __builtin_amdgcn_exp2f(-Lf * __builtin_sqrtf(d2));
          }
          part += kv;
        }
        sum[i][r] += (double)part;
      }
    }
  }
  __syncthreads();

  // reduce over the 16 lanes that share rows, then over the two column waves
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = sum[i][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      sum[i][r] = v;
    }
  double* red = reinterpret_cast<double*>(lds);   // [2][BQ]
  if ((lane & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wn * BQ + wq * 64 + i * 16 + 4 * (lane >> 4) + r] = sum[i][r];
  }
  __syncthreads();
  if (threadIdx.x < BQ)
    partial[split * qp + qt * BQ + threadIdx.x] = red[threadIdx.x] + red[BQ + threadIdx.x];
}

// Sum of the per-split partials in split order, times the Gaussian query
// factor 2^(rounding remainder of -L ||y||^2), times 1/n.
__global__ void kde_reduce_kernel(const double* __restrict__ partial, int64_t splits, int64_t qp,
                                  int64_t q, double inv_n, const double* __restrict__ ynorm,
                                  float Lf, int kern, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  double s = 0.0;
  for (int64_t sp = 0; sp < splits; ++sp) s += partial[sp * qp + i];
  if (kern == KERNEL_GAUSSIAN) {
    const double e = -(double)Lf * ynorm[i];
    s *= exp2(e - (double)(float)e);
  }
  out[i] = s * inv_n;
}

template <typename T, int KERN, int ENG>
static void launch_kde_k(const TileProblem& p, float L, double* partial, hipStream_t s) {
  kde_tile_kernel<T, KERN, ENG><<<dim3((unsigned)p.map.grid), dim3(WG), 0, s>>>(
      p.Ys, p.Xs, p.ld_bytes, p.nchunks, p.ynorm, p.xnorm, p.n, p.qtiles, p.splits, p.ntiles, L,
      partial, p.qp, p.map);
}

template <typename T, int KERN>
static void launch_kde_n(const TileProblem& p, float L, double* partial, hipStream_t s) {
  if constexpr (elem_of<T>::bytes == 2) {
    const int eng = tile_engine<T>(p.ld_bytes);
    if (eng == 2) return launch_kde_k<T, KERN, 2>(p, L, partial, s);
    if (eng == 1) return launch_kde_k<T, KERN, 1>(p, L, partial, s);
  }
  launch_kde_k<T, KERN, 0>(p, L, partial, s);
}

template <typename T>
static hipError_t launch_kde_t(const TileProblem& p, int kern, float L, double* partial,
                               hipStream_t s) {
  if (kern == KERNEL_GAUSSIAN)
    launch_kde_n<T, KERNEL_GAUSSIAN>(p, L, partial, s);
  else
    launch_kde_n<T, KERNEL_EXPONENTIAL>(p, L, partial, s);
  return hipGetLastError();
}

hipError_t launch_kde_exact(int prec, const TileProblem& p, int kern, double h, double* partial,
                            double* out, hipStream_t s, TimingHook th) {
  const double log2e = 1.4426950408889634;
  const float L = (float)(kern == KERNEL_GAUSSIAN ? log2e / (2.0 * h * h) : log2e / h);
  hipError_t e;
  if (th.start && (e = hipEventRecord(th.start, s)) != hipSuccess) return e;
  switch (prec) {
    case PREC_FP32: e = launch_kde_t<float>(p, kern, L, partial, s); break;
    case PREC_BF16: e = launch_kde_t<__bf16>(p, kern, L, partial, s); break;
    default: e = launch_kde_t<_Float16>(p, kern, L, partial, s); break;
  }
  if (e != hipSuccess) return e;
  if (th.stop && (e = hipEventRecord(th.stop, s)) != hipSuccess) return e;
  kde_reduce_kernel<<<dim3((unsigned)ceil_div(p.q, 256)), dim3(256), 0, s>>>(
      partial, p.splits, p.qp, p.q, 1.0 / (double)p.n, p.ynorm, L, kern, out);
  return hipGetLastError();
}

}  // namespace deann
