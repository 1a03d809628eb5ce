// Accuracy certificate of the float32-operand exact KDE, and the exact
// re-evaluation of the queries it does not certify.
//
// The GEMM identity of App. F computes ||x~||^2 + ||y~||^2 - 2 <x~, y~> in
// float32, so each pair's exponent carries an absolute rounding error of the
// order u (||x~||^2 + ||y~||^2) / (2 h^2) (u = 2^-24): independent of the
// distance, large when h is small against the norms of the centred rows.
// Summed over many pairs of similar weight these errors average out; when a
// few pairs carry a query's mass they do not.  From the tile sweep's sums per
// query (T = sum K, A = sum K^2, and the K-weighted sum of the exponents
// for the Gaussian kernel, the largest K for the exponential one) the
// reduction bounds the relative error of T:
//
//   random part  Bernstein's inequality over the roundings, taken as
//                independent, zero-mean and with the variance of a uniform
//                error: the float32 MFMA accumulates a dot product like a
//                chain of round-to-nearest-even additions in k order, so each
//                of its c_d = d roundings is at most u |partial sum| <=
//                u ||x~|| ||y~||; with the data-norm term, the add and the FMA
//                every pair carries c_d + 6 roundings of at most u L N of the
//                exponent (L = 1/(2h^2); exponential kernel: 1/(2 h r_lo) per
//                unit of d^2, r_lo a lower bound of the query's smallest
//                distance; N = max ||x~||^2 + ||y~||^2), and the float32
//                partial sums add at most 8 more per pair.  Variance
//                A (u L N)^2 (c_d + 6) / 3 + ..., largest term u L N sqrt(A);
//                the bound fails with probability below 3e-8 per query.
//   systematic   the float32 rounding of the exponent scale (u per unit of the
//                K-weighted mean exponent; the exponential kernel bounds that
//                mean by ln(n/T) + ln n and adds its square root and product),
//                exp2 (2u), for the exponential kernel the rounding of ||y~||^2
//                that every pair of the query shares, and float32 underflow
//                (at most 2^-126 per term: n 2^-126 / T).
//
// A query whose bound exceeds tau, unless its value is certainly below the
// floor below which relative errors are not reported (the paper excludes
// KDE values under 1e-16 from its error statistics), is listed for an exact
// re-evaluation: direct differences x - y of the float32 rows in FP64, exp in
// FP64, and a fixed-order FP64 sum (Eq. (1) as written), which overwrites the
// value (and the gradient) the tile sweep gave.
#include "cert.h"

namespace deann {

// Sum of the per-split partials in split order (as kde_reduce_kernel), the
// certificate, and the list of queries to re-evaluate.
__global__ void kde_reduce_cert_kernel(const double* __restrict__ partial, int64_t splits,
                                       int64_t qp, int64_t q, int64_t n,
                                       const double* __restrict__ ynorm, float Lf, int kern,
                                       CertArgs ca, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  double s = 0.0, A = 0.0, y2 = 0.0, AN = 0.0, AK = 0.0;
  for (int64_t sp = 0; sp < splits; ++sp) {
    s += partial[sp * qp + i];
    const float2 c = ca.part[sp * qp + i];
    A += (double)c.x;
    if (ca.pn) AN += (double)ca.pn[sp * qp + i];
    if (ca.pk) AK += (double)ca.pk[sp * qp + i];
    // Gaussian: sum of K times its exponent; exponential: the largest K
    y2 = kern == KERNEL_GAUSSIAN ? y2 + (double)c.y : fmax(y2, (double)c.y);
  }
  double f = 1.0;
  if (kern == KERNEL_GAUSSIAN) {
    const double e = -(double)Lf * ynorm[i];
    f = exp2(e - (double)(float)e);
  }
  out[i] = s * f / (double)n;
  // FP32 sums of A and of the exponents lose at most a few 1e-4 relative: 1% margins
  // the norm terms of AN are float32 roundings of FP64 norms (a few u): inside the margin
  cert_check(i, s, A * 1.01, kern == KERNEL_GAUSSIAN ? y2 * 1.01 : y2, f, ynorm[i], n, Lf, kern,
             ca, ca.pn ? AN * 1.02 : -1.0, ca.pk ? AK * 1.02 : -1.0);
}

// ---------------------------------------------------------------------------
// Exact re-evaluation.  Work item = (16 listed queries, one of `splits` row
// ranges); a grid-stride loop over the items, whose count follows from the
// list length on the device.
// ---------------------------------------------------------------------------
constexpr int DQT = 16;      // queries per item
constexpr int DROWS = 64;    // data rows per block (gradient kernel)
constexpr int DG_MAXD = 128; // width limit of the gradient kernel

// Row ranges of the gradient kernel for F listed queries: about one per 2048
// rows (at most 512), as many as a scratch of cap entries per array holds
// (entry sp * F + slot; the weighted row sums take ldg of them each), so that
// a few listed queries still spread over the whole GPU.
__host__ __device__ inline int64_t direct_grad_splits(int64_t F, int64_t cap, int64_t n) {
  int64_t s = (n + 2047) / 2048;
  if (s > 512) s = 512;
  const int64_t room = F > 0 ? cap / F : cap;
  if (s > room) s = room;
  return s < 1 ? 1 : s;
}

// Value-only kernel: blocks of 256 rows, coordinates staged 32 at a time in
// LDS transposed ([coordinate][row], float) so that thread (rb, g) =
// (tid % 64, tid / 64) reads rows 4 rb .. 4 rb + 3 of one coordinate with one
// 16-byte load and the coordinates of queries 4 g .. 4 g + 3 (FP64, the same
// for the whole wave) as broadcasts; it keeps the 4 x 4 squared distances in
// registers: 16 differences and 16 FMAs in FP64 per coordinate and four loads.
constexpr int DXR = 256;          // rows per block
constexpr int DXC = 32;           // coordinates per LDS stage
constexpr int DXP = DXR + 4;      // LDS pitch of a coordinate (floats, 16-byte multiple)

template <int KERN>
__device__ __forceinline__ double kval(double d2, double h) {
  if (KERN == KERNEL_GAUSSIAN) return exp(-d2 / (2.0 * h * h));
  return exp(-sqrt(d2) / h);
}

template <int KERN, bool VEC>
__global__ void __launch_bounds__(WG)
kde_direct_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n, int64_t d,
                  double h, const int32_t* __restrict__ ids, const int32_t* __restrict__ count,
                  int64_t splits, int64_t q, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) float xs[DXC * DXP];
  __shared__ __attribute__((aligned(16))) double ys[DXC][DQT];
  const int64_t F = *count;
  const int64_t items = ceil_div(F, DQT) * splits;
  const int rb = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t nc = ceil_div(d, DXC);   // coordinate stages per row block
  constexpr int XV = DXR * DXC / 4 / WG;   // float4 pieces per thread and stage (8)
  constexpr int YV = DQT * DXC / WG;       // query values per thread and stage (2)
  f32x4 xr[XV];
  double yr[YV];
  // stage s of an item: row block s / nc, coordinates (s % nc) * DXC + [0, DXC)
  auto load = [&](int64_t tile, int64_t r0, int64_t r1, int64_t s) {
    const int64_t b0 = r0 + (s / nc) * DXR, c0 = (s % nc) * DXC;
#pragma unroll
    for (int i = 0; i < XV; ++i) {
      const int e = threadIdx.x + i * WG;          // row e / 8, coordinates 4 (e % 8) + [0, 4)
      const int64_t row = b0 + e / 8, col = c0 + 4 * (e % 8);
      if (VEC) {
        xr[i] = (row < r1 && col < d) ? *reinterpret_cast<const f32x4*>(X + row * d + col)
                                      : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) xr[i][k] = (row < r1 && col + k < d) ? X[row * d + col + k] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < YV; ++i) {
      const int e = threadIdx.x + i * WG;
      const int qq = e / DXC, cc = e % DXC;
      const int64_t slot = tile * DQT + qq, col = c0 + cc;
      yr[i] = (slot < F && col < d) ? (double)Y[(int64_t)ids[slot] * d + col] : 0.0;
    }
  };
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    const int64_t tile = w / splits, sp = w % splits;
    const int64_t r0 = sp * n / splits, r1 = (sp + 1) * n / splits;
    const int64_t stages = ceil_div(r1 - r0, DXR) * nc;
    double ks[4] = {0.0, 0.0, 0.0, 0.0};
    double acc[4][4];   // [row][query]
    if (stages > 0) load(tile, r0, r1, 0);
    for (int64_t s = 0; s < stages; ++s) {
      const int64_t b0 = r0 + (s / nc) * DXR, c0 = (s % nc) * DXC;
      if (s % nc == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
      __syncthreads();   // the previous stage has been read
#pragma unroll
      for (int i = 0; i < XV; ++i) {
        const int e = threadIdx.x + i * WG;
        const int rr = e / 8, cc = 4 * (e % 8);
#pragma unroll
        for (int k = 0; k < 4; ++k) xs[(cc + k) * DXP + rr] = xr[i][k];
      }
#pragma unroll
      for (int i = 0; i < YV; ++i) {
        const int e = threadIdx.x + i * WG;
        ys[e % DXC][e / DXC] = yr[i];
      }
      __syncthreads();
      if (s + 1 < stages) load(tile, r0, r1, s + 1);   // in flight behind this stage
      const int cn = (int)(d - c0 < DXC ? d - c0 : DXC);
      for (int t = 0; t < cn; ++t) {
        const f32x4 xv = *reinterpret_cast<const f32x4*>(&xs[t * DXP + 4 * rb]);
        double yv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) yv[j] = ys[t][4 * g + j];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double x = (double)xv[i];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double df = x - yv[j];
            acc[i][j] = __builtin_fma(df, df, acc[i][j]);
          }
        }
      }
      if (s % nc == nc - 1)   // the block's distances are complete
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (b0 + 4 * rb + i < r1)
#pragma unroll
            for (int j = 0; j < 4; ++j) ks[j] += kval<KERN>(acc[i][j], h);
    }
    // the 64 row groups of each query, in a fixed order
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = ks[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      const int64_t slot = tile * DQT + 4 * g + j;
      if (rb == 0 && slot < F) part[sp * q + slot] = v;
    }
  }
}

__global__ void kde_direct_reduce_kernel(const double* __restrict__ part,
                                         const int32_t* __restrict__ ids,
                                         const int32_t* __restrict__ count, int64_t splits,
                                         int64_t q, int64_t n, double* __restrict__ out) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= *count) return;
  double s = 0.0;
  for (int64_t sp = 0; sp < splits; ++sp) s += part[sp * q + slot];
  out[ids[slot]] = s / (double)n;
}

// Value, d/dy and d/dh of the listed queries (d <= 128): the rows of a block
// stay in LDS for both phases; phase 1 gives the distances and the weights
// (Gaussian K, exponential K / r), phase 2 the weighted sums of x - y, thread
// (query tid/16, coordinates tid%16 + 16 j).
template <int KERN>
__global__ void __launch_bounds__(WG)
kde_direct_grad_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n,
                       int64_t d, double h, const int32_t* __restrict__ ids,
                       const int32_t* __restrict__ count, int64_t cap,
                       double* __restrict__ pval, double* __restrict__ pgh,
                       double* __restrict__ pG, int64_t ldg) {
  __shared__ float xs[DROWS][DG_MAXD + 1];
  __shared__ double ys[DQT][DG_MAXD];
  __shared__ double ws[DQT][DROWS];
  const int64_t F = *count;
  const int64_t splits = direct_grad_splits(F, cap, n);
  const int64_t items = ceil_div(F, DQT) * splits;
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int qq = threadIdx.x >> 4, cl = threadIdx.x & 15;
  constexpr int NCT = DG_MAXD / 16;   // coordinates per thread in phase 2
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    const int64_t tile = w / splits, sp = w % splits;
    const int64_t r0 = sp * n / splits, r1 = (sp + 1) * n / splits;
    __syncthreads();   // the previous item's ys has been read
    for (int e = threadIdx.x; e < DQT * DG_MAXD; e += WG) {
      const int qi = e / DG_MAXD, cc = e % DG_MAXD;
      const int64_t slot = tile * DQT + qi;
      ys[qi][cc] = (slot < F && cc < d) ? (double)Y[(int64_t)ids[slot] * d + cc] : 0.0;
    }
    double kv[4] = {0.0, 0.0, 0.0, 0.0}, kh[4] = {0.0, 0.0, 0.0, 0.0};
    double G[NCT];
#pragma unroll
    for (int j = 0; j < NCT; ++j) G[j] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += DROWS) {
      __syncthreads();   // phase 2 of the previous block has read xs and ws
      for (int e = threadIdx.x; e < DROWS * DG_MAXD; e += WG) {
        const int rr = e / DG_MAXD, cc = e % DG_MAXD;
        const int64_t row = rb + rr;
        xs[rr][cc] = (row < r1 && cc < d) ? X[row * d + cc] : 0.f;
      }
      __syncthreads();
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < (int)d; ++t) {
        const double xv = (double)xs[r][t];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double df = xv - ys[4 * g + j][t];
          acc[j] = __builtin_fma(df, df, acc[j]);
        }
      }
      const bool valid = rb + r < r1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double wv = 0.0;
        if (valid) {
          const double K = kval<KERN>(acc[j], h);
          kv[j] += K;
          if (KERN == KERNEL_GAUSSIAN) {
            wv = K;
            kh[j] += K * acc[j];
          } else {
            const double rr = sqrt(acc[j]);
            wv = rr > 0.0 ? K / rr : 0.0;
            kh[j] += K * rr;
          }
        }
        ws[4 * g + j][r] = wv;
      }
      __syncthreads();
      for (int rr = 0; rr < DROWS; ++rr) {
        const double wv = ws[qq][rr];
#pragma unroll
        for (int j = 0; j < NCT; ++j) {
          const int t = cl + 16 * j;
          G[j] = __builtin_fma(wv, (double)xs[rr][t] - ys[qq][t], G[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double a = kv[j], b = kh[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
      }
      const int64_t slot = tile * DQT + 4 * g + j;
      if (r == 0 && slot < F) {
        pval[sp * F + slot] = a;
        pgh[sp * F + slot] = b;
      }
    }
    const int64_t slot = tile * DQT + qq;
    if (slot < F)
#pragma unroll
      for (int j = 0; j < NCT; ++j) {
        const int t = cl + 16 * j;
        if (t < d) pG[(sp * F + slot) * ldg + t] = G[j];
      }
  }
}

// Outputs of the listed queries, with the scaling of kde_backward_reduce_kernel:
// grad_Y = g/n * c_y * sum w (x - y), d/dh = g/n * c_h * sum dh, mu = sum K / n.
__global__ void kde_direct_grad_reduce_kernel(const double* __restrict__ pval,
                                              const double* __restrict__ pgh,
                                              const double* __restrict__ pG, int64_t ldg,
                                              const int32_t* __restrict__ ids,
                                              const int32_t* __restrict__ count, int64_t cap,
                                              int64_t n, int64_t d, double c_y,
                                              double c_h, const double* __restrict__ grad_out,
                                              float* __restrict__ grad_Y,
                                              double* __restrict__ ghq, double* __restrict__ mu) {
  const int64_t slot = blockIdx.x;
  const int64_t F = *count;
  if (slot >= F) return;
  const int64_t splits = direct_grad_splits(F, cap, n);
  const int64_t qi = ids[slot];
  const double g = grad_out ? grad_out[qi] : 1.0;
  const double inv_n = 1.0 / (double)n;
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int64_t sp = 0; sp < splits; ++sp) {
      a += pval[sp * F + slot];
      b += pgh[sp * F + slot];
    }
    if (ghq) ghq[qi] = g * inv_n * c_h * b;
    if (mu) mu[qi] = a * inv_n;
  }
  if (!grad_Y) return;
  for (int64_t t = threadIdx.x; t < d; t += blockDim.x) {
    double s = 0.0;
    for (int64_t sp = 0; sp < splits; ++sp) s += pG[(sp * F + slot) * ldg + t];
    grad_Y[qi * d + t] = (float)(g * inv_n * c_y * s);
  }
}

namespace {
constexpr int64_t kDirectGrid = 2048;      // workgroups of the gradient kernel's loop
constexpr int64_t kDirectResident = 768;   // value kernel: 3 workgroups on each of 256 CUs
}

hipError_t launch_kde_reduce_cert(const double* partial, int64_t splits, int64_t qp, int64_t q,
                                  int64_t n, const double* ynorm, float Lf, int kern,
                                  const CertArgs& ca, double* out, hipStream_t s) {
  if (q == 0) return hipSuccess;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ca.fb_count), 1, 0u, s);
  if (e != hipSuccess) return e;
  kde_reduce_cert_kernel<<<dim3((unsigned)ceil_div(q, 256)), dim3(256), 0, s>>>(
      partial, splits, qp, q, n, ynorm, Lf, kern, ca, out);
  return hipGetLastError();
}

int64_t direct_splits(int64_t n) {
  int64_t s = ceil_div(n, 2048);
  if (s < 1) s = 1;
  if (s > 512) s = 512;
  return s;
}

hipError_t launch_kde_direct(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                             double h, int kern, const int32_t* ids, const int32_t* count,
                             int64_t splits, double* part, double* out, hipStream_t s) {
  if (q == 0) return hipSuccess;
  const int64_t items = ceil_div(q, DQT) * splits;
  // workgroups that are all resident at once (3 per CU), each looping over items
  const dim3 grid((unsigned)(items < kDirectResident ? items : kDirectResident)), block(WG);
  const bool vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
  if (kern == KERNEL_GAUSSIAN) {
    if (vec)
      kde_direct_kernel<KERNEL_GAUSSIAN, true><<<grid, block, 0, s>>>(X, Y, n, d, h, ids, count,
                                                                      splits, q, part);
    else
      kde_direct_kernel<KERNEL_GAUSSIAN, false><<<grid, block, 0, s>>>(X, Y, n, d, h, ids, count,
                                                                       splits, q, part);
  } else {
    if (vec)
      kde_direct_kernel<KERNEL_EXPONENTIAL, true><<<grid, block, 0, s>>>(X, Y, n, d, h, ids,
                                                                         count, splits, q, part);
    else
      kde_direct_kernel<KERNEL_EXPONENTIAL, false><<<grid, block, 0, s>>>(X, Y, n, d, h, ids,
                                                                          count, splits, q, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  kde_direct_reduce_kernel<<<dim3((unsigned)ceil_div(q, 256)), dim3(256), 0, s>>>(
      part, ids, count, splits, q, n, out);
  return hipGetLastError();
}

hipError_t launch_kde_direct_grad(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                                  double h, int kern, const int32_t* ids, const int32_t* count,
                                  int64_t cap, double* pval, double* pgh, double* pG,
                                  int64_t ldg, const double* grad_out, float* grad_Y, double* ghq,
                                  double* mu, hipStream_t s) {
  if (q == 0) return hipSuccess;
  if (d > DG_MAXD || ldg < d || cap < q) return hipErrorInvalidValue;
  // the listed count is known on the device only: a grid-stride loop over the
  // items it implies, as many as the scratch holds (see direct_grad_splits)
  const dim3 grid((unsigned)kDirectGrid), block(WG);
  if (kern == KERNEL_GAUSSIAN)
    kde_direct_grad_kernel<KERNEL_GAUSSIAN><<<grid, block, 0, s>>>(X, Y, n, d, h, ids, count,
                                                                   cap, pval, pgh, pG, ldg);
  else
    kde_direct_grad_kernel<KERNEL_EXPONENTIAL><<<grid, block, 0, s>>>(
        X, Y, n, d, h, ids, count, cap, pval, pgh, pG, ldg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Gaussian: w = K, dh terms K d^2; exponential: w = K / r, dh terms K r
  const double c_y = kern == KERNEL_GAUSSIAN ? 1.0 / (h * h) : 1.0 / h;
  const double c_h = kern == KERNEL_GAUSSIAN ? 1.0 / (h * h * h) : 1.0 / (h * h);
  kde_direct_grad_reduce_kernel<<<dim3((unsigned)q), dim3(128), 0, s>>>(
      pval, pgh, pG, ldg, ids, count, cap, n, d, c_y, c_h, grad_out, grad_Y, ghq, mu);
  return hipGetLastError();
}

}  // namespace deann
