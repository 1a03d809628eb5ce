// Random-sampling part of DEANN (Algorithm 1): m uniform draws with
// repetition from X2 = X minus the k neighbours, the exact kernel sum over the
// drawn rows, and the combined estimate (Z1 + ((n-k)/m) Z2) / n.  The same
// kernel also takes the permuted blocks of App. G (Algorithm 2) instead of
// the draws; see `permute` below.
//
// Draw j of query i uses word (j mod 4) of Philox4x64-10 (Salmon et al., SC'11)
// with key (seed, 0) and counter (j div 4, query_offset + i, word2, 0).  The
// rank r = floor(u (n - k) / 2^64) picks the r-th smallest element of X2, found
// as r + #{t : nn_t - t <= r} over the neighbours sorted by index.  All of it is
// integer arithmetic, so the drawn indices are bit-reproducible.
//
// The gather reads each drawn row once with 16 lanes per row (64-byte
// coalesced segments) and evaluates ||x - y||^2 directly in FP64.
#include "common.h"
#include "kernels.h"
#include "philox.h"

namespace deann {

__host__ __device__ inline int next_pow2_i(int64_t v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Keyed pseudo-random permutation of [n] for permuted random sampling
// (App. G, Algorithm 2): a balanced 4-round Feistel network on b-bit words
// (b even, 2^b >= n) with round function word 0 of Philox4x64-10, key
// (seed, 1), counter (half, round, 0, 0); values outside [n] are walked
// through the network again until they fall inside (cycle walking, Black and
// Rogaway, CT-RSA 2002).
constexpr int PERM_ROUNDS = 4;

__host__ __device__ inline int perm_bits(int64_t n) {
  int b = 2;
  while (b < 62 && (int64_t(1) << b) < n) ++b;
  return b + (b & 1);
}

__device__ __forceinline__ uint64_t feistel(uint64_t x, int b, uint64_t seed, bool inverse) {
  const int half = b >> 1;
  const uint64_t mask = (uint64_t(1) << half) - 1;
  uint64_t left = x >> half, right = x & mask;
  if (!inverse) {
#pragma unroll
    for (int r = 0; r < PERM_ROUNDS; ++r) {
      const uint64_t f = philox4x64_10(seed, 1, right, (uint64_t)r, 0, 0).v[0] & mask;
      const uint64_t nl = right;
      right = left ^ f;
      left = nl;
    }
  } else {
#pragma unroll
    for (int r = PERM_ROUNDS - 1; r >= 0; --r) {
      const uint64_t f = philox4x64_10(seed, 1, left, (uint64_t)r, 0, 0).v[0] & mask;
      const uint64_t nr = left;
      left = right ^ f;
      right = nr;
    }
  }
  return (left << half) | right;
}

__device__ __forceinline__ int64_t permute(int64_t x, int64_t n, int b, uint64_t seed, bool inverse) {
  uint64_t y = feistel((uint64_t)x, b, seed, inverse);
  while (y >= (uint64_t)n) y = feistel(y, b, seed, inverse);   // ends: x lies on y's cycle
  return (int64_t)y;
}

// Workgroup bitonic sort of N int32 values in LDS (N a power of two).
__device__ void block_sort_i32(int32_t* a, int N) {
  for (int kk = 2; kk <= N; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int32_t x = a[i], y = a[ixj];
          if ((x > y) == ((i & kk) == 0)) { a[i] = y; a[ixj] = x; }
        }
      }
      __syncthreads();
    }
  }
}

constexpr int DRAW_CHUNK = 1024;   // draws handled per pass through LDS

__device__ __forceinline__ double kval(double d2, double h, int kern) {
  if (kern == KERNEL_GAUSSIAN) return exp(-d2 / (2.0 * h * h));
  return exp(-sqrt(d2) / h);
}

// PERM: permuted blocks (App. G) instead of draws with repetition; a template
// argument so that the draw loop of the plain sampler carries none of it.
// IDX (with PERM): the permutation is read from a prepared index instead of
// being evaluated: pi[pos] the row at position pos of the permuted order,
// inv[row] its position, and the rows themselves from the permuted copy Xp,
// where a query's block is contiguous (Algorithm 2 as written).
template <bool PERM, bool IDX>
__global__ void __launch_bounds__(WG)
deann_sample_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n,
                    int64_t d, double h, int kern, int64_t k, int64_t m, uint64_t seed,
                    uint64_t query_offset, uint64_t word2, uint64_t start,
                    const int32_t* __restrict__ nn_sorted, const double* __restrict__ z1,
                    double* __restrict__ out, int32_t* __restrict__ sample_idx,
                    const int32_t* __restrict__ pi, const int32_t* __restrict__ inv,
                    const float* __restrict__ Xp) {
  constexpr bool permuted = PERM;
  static_assert(PERM || !IDX, "a prepared index is for permuted sampling");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int kp = permuted ? next_pow2_i(k) : (int)k;   // sorted in place when permuted
  double* kv = reinterpret_cast<double*>(smem);                    // DRAW_CHUNK
  int32_t* sidx = reinterpret_cast<int32_t*>(kv + DRAW_CHUNK);     // DRAW_CHUNK
  int32_t* gaps = sidx + DRAW_CHUNK;                               // kp
  float* ys = reinterpret_cast<float*>(gaps + kp);                 // d
  const int64_t qi = blockIdx.x;
  const uint64_t size2 = (uint64_t)(n - k);
  const double zz1 = k > 0 ? z1[qi] : 0.0;
  if (m == 0 || size2 == 0) {
    if (sample_idx)
      for (int64_t j = threadIdx.x; j < m; j += WG) sample_idx[qi * m + j] = -1;
    if (threadIdx.x == 0) out[qi] = zz1 / (double)n;
    return;
  }
  // gaps[t] = e_t - t over the sorted excluded positions e_t: the neighbours'
  // indices (draws with repetition over X2), or, for permuted sampling, the
  // neighbours' positions in the permuted order relative to this query's
  // running index l = (start + i m) mod n
  const int bits = perm_bits(n);
  const int64_t run = permuted ? (int64_t)((start % (uint64_t)n + ((uint64_t)qi * (uint64_t)m) % (uint64_t)n) % (uint64_t)n) : 0;
  if constexpr (permuted) {
    for (int t = threadIdx.x; t < kp; t += WG) {
      int32_t gp = INT32_MAX;
      if (t < k) {
        const int64_t pos = IDX ? (int64_t)inv[nn_sorted[qi * k + t]]
                                : permute(nn_sorted[qi * k + t], n, bits, seed, true);
        gp = (int32_t)((pos - run + n) % n);
      }
      gaps[t] = gp;
    }
    __syncthreads();
    block_sort_i32(gaps, kp);
    for (int t = threadIdx.x; t < k; t += WG) gaps[t] -= t;
  } else {
    for (int64_t t = threadIdx.x; t < k; t += WG) gaps[t] = nn_sorted[qi * k + t] - (int32_t)t;
  }
  for (int64_t t = threadIdx.x; t < d; t += WG) ys[t] = Y[qi * d + t];
  __syncthreads();
  const uint64_t stream = query_offset + (uint64_t)qi;
  double total = 0.0;   // meaningful in thread 0
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  for (int64_t j0 = 0; j0 < m; j0 += DRAW_CHUNK) {
    const int cnt = (int)(m - j0 < DRAW_CHUNK ? m - j0 : DRAW_CHUNK);
    // draws: each thread makes one Philox block = 4 consecutive draws (with
    // repetition), or 4 consecutive positions of the permuted block
    for (int b = threadIdx.x; b * 4 < cnt; b += WG) {
      const int64_t jb = (j0 >> 2) + b;     // j0 is a multiple of 4
      Philox4x64 blk;
      if constexpr (!permuted) blk = philox4x64_10(seed, 0, (uint64_t)jb, stream, word2, 0);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int jj = b * 4 + w;
        if (jj < cnt) {
          int64_t u;
          if constexpr (permuted) {   // position j of the block, neighbours skipped
            u = rank_to_row((uint64_t)(j0 + jj), gaps, k);
          } else {
            u = draw_row(blk.v[w], size2, gaps, k);
          }
          int32_t idx;
          if constexpr (IDX) {   // gather from the permuted copy, report the row
            const int64_t pos = (run + u) % n;
            sidx[jj] = (int32_t)pos;
            idx = pi[pos];
          } else {
            idx = permuted ? (int32_t)permute((run + u) % n, n, bits, seed, false) : (int32_t)u;
            sidx[jj] = idx;
          }
          if (sample_idx) sample_idx[qi * m + j0 + jj] = idx;
        }
      }
    }
    __syncthreads();
    // gather and evaluate: 16 lanes per drawn row, four rows in flight
    for (int j0 = g; j0 < cnt; j0 += 4 * (WG / 16)) {
      int64_t rr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int jj = j0 + i * (WG / 16);
        rr[i] = jj < cnt ? (int64_t)sidx[jj] : -1;
      }
      double s4[4];
      group16_d2_4(IDX ? Xp : X, rr, d, ys, l16, s4);
      if (l16 == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int jj = j0 + i * (WG / 16);
          if (jj < cnt) kv[jj] = kval(s4[i], h, kern);
        }
    }
    __syncthreads();
    // fixed-order reduction of the chunk
    double* red = kv;   // reuse in place: tree over DRAW_CHUNK slots
    for (int i = cnt + threadIdx.x; i < DRAW_CHUNK; i += WG) red[i] = 0.0;
    __syncthreads();
    for (int w = DRAW_CHUNK / 2; w > 0; w >>= 1) {
      for (int i = threadIdx.x; i < w; i += WG) red[i] += red[i + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) total += red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[qi] = (zz1 + (double)size2 / (double)m * total) / (double)n;
}

hipError_t launch_sample(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                         double h, int kern, int64_t k, int64_t m, uint64_t seed,
                         uint64_t query_offset, uint64_t word2, int permuted, uint64_t start,
                         const int32_t* nn_sorted, const double* z1, double* out,
                         int32_t* sample_idx, hipStream_t s, const PermIndex* pidx) {
  if (q == 0) return hipSuccess;
  // without draws (m = 0 or k = n) the kernel only writes Z1 / n and needs no
  // gap table, whose size would otherwise grow with k
  const bool draws = m > 0 && k < n;
  const int64_t kp = !draws ? 0 : permuted ? next_pow2_i(k) : k;
  const size_t sm = DRAW_CHUNK * (8 + 4) + kp * 4 + d * 4 + 16;
  const dim3 g((unsigned)q), b(WG);
  if (permuted && pidx)
    deann_sample_kernel<true, true><<<g, b, sm, s>>>(
        X, Y, n, d, h, kern, k, m, seed, query_offset, word2, start, nn_sorted, z1, out,
        sample_idx, pidx->pi, pidx->inv, pidx->Xp);
  else if (permuted)
    deann_sample_kernel<true, false><<<g, b, sm, s>>>(
        X, Y, n, d, h, kern, k, m, seed, query_offset, word2, start, nn_sorted, z1, out,
        sample_idx, nullptr, nullptr, nullptr);
  else
    deann_sample_kernel<false, false><<<g, b, sm, s>>>(
        X, Y, n, d, h, kern, k, m, seed, query_offset, word2, start, nn_sorted, z1, out,
        sample_idx, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

// Permuted index (Algorithm 2's preprocessing): pi[pos] = the keyed
// permutation of pos, inv[pi[pos]] = pos, then the rows Xp[pos] = X[pi[pos]].
__global__ void perm_index_kernel(int64_t n, uint64_t seed, int32_t* __restrict__ pi,
                                  int32_t* __restrict__ inv) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const int64_t r = permute(pos, n, perm_bits(n), seed, false);
  pi[pos] = (int32_t)r;
  inv[r] = (int32_t)pos;
}

// One wave per permuted row: float4 copies when rows are 16-byte aligned.
__global__ void __launch_bounds__(WG) perm_rows_kernel(const float* __restrict__ X, int64_t n,
                                                       int64_t d, const int32_t* __restrict__ pi,
                                                       float* __restrict__ Xp, int vec) {
  const int64_t pos = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (pos >= n) return;
  const float* src = X + (int64_t)pi[pos] * d;
  float* dst = Xp + pos * d;
  if (vec) {
    for (int64_t t = 4 * lane; t < d; t += 256)
      *reinterpret_cast<f32x4*>(dst + t) = *reinterpret_cast<const f32x4*>(src + t);
  } else {
    for (int64_t t = lane; t < d; t += 64) dst[t] = src[t];
  }
}

hipError_t launch_perm_index(const float* X, int64_t n, int64_t d, uint64_t seed,
                             const PermIndex& pidx, hipStream_t s) {
  perm_index_kernel<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s>>>(
      n, seed, const_cast<int32_t*>(pidx.pi), const_cast<int32_t*>(pidx.inv));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(pidx.Xp) % 16 == 0;
  perm_rows_kernel<<<dim3((unsigned)ceil_div(n, WG / 64)), dim3(WG), 0, s>>>(
      X, n, d, pidx.pi, const_cast<float*>(pidx.Xp), vec);
  return hipGetLastError();
}

}  // namespace deann
