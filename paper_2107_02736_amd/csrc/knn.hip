// Exact k nearest neighbours: the ANN black box of Algorithm 1 replaced by
// an exact brute-force search whose result equals the sequence of
// points sorted by distance (Sec. 2) with ties broken towards the lower index.
//
// 1. scan     : the MFMA distance tile of the prepared operands gives a key per
//               pair that provably never exceeds ||x~ - y~||^2.
//               FP32: each (split, query) keeps the K1 smallest keys in a
//               global list (threshold in LDS, append on accept, wave-level
//               register sorts compact the list when it runs full).
//               BF16/FP16: each (split, query, lane column) keeps only its
//               smallest key ("cell" candidates), with no list traffic.
// 2. refine   : per query, the K1 smallest keys over all splits are re-evaluated
//               exactly (FP64 direct differences, double-double for near ties),
//               sorted by (d^2, index); the first k are the candidates.  FP32: a
//               certificate checks that every excluded point is provably farther
//               than the k-th candidate: sqrt(T) - E - e_y > d_k, with T the K1-th
//               key and E, e_y bounds of the rounding of the rows.  16-bit: the
//               candidates only bound d_k and the second pass always runs.
// 3. collect  : queries without a certificate rescan and gather every point
//               whose key admits a distance <= d_k; refine2 then sorts that set.
// 4. exhaustive: a query whose second-pass set overflowed is scanned with exact
//               FP64 distances by one workgroup (rare fallback).
#include "common.h"
#include "kernels.h"

namespace deann {

constexpr int SORT_CAP = 4096;   // entries of the workgroup LDS sorts
constexpr int K_MAX = 1024;      // largest K1 (and hence k) the refine kernels take

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Workgroup bitonic sort of N (power of two) packed uint64 keys, ascending.
// k0 > 2 skips the levels below k0: it requires the aligned blocks of k0 / 2
// entries to be sorted already, ascending in even blocks and descending in
// odd ones (the state the sort itself reaches after those levels).
__device__ void block_sort_u64(uint64_t* a, int N, int k0 = 2) {
  for (int kk = k0; kk <= N; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = a[i], y = a[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) { a[i] = y; a[ixj] = x; }
        }
      }
      __syncthreads();
    }
  }
}

// Workgroup bitonic sort of N pairs (key, idx) ascending by (key, idx).
__device__ void block_sort_pairs(uint64_t* key, uint32_t* idx, int N) {
  for (int kk = 2; kk <= N; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = key[i], b = key[ixj];
          const uint32_t ia = idx[i], ib = idx[ixj];
          const bool gt = a > b || (a == b && ia > ib);
          const bool up = (i & kk) == 0;
          if (gt == up) { key[i] = b; key[ixj] = a; idx[i] = ib; idx[ixj] = ia; }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Bitonic sort of 64*EPL packed keys held in registers by one wave, ascending;
// element e = lane * EPL + r.  Partners within a lane are swapped in
// registers, across lanes exchanged with shuffles; no LDS, no barrier.
template <int EPL>
__device__ __forceinline__ void wave_sort_u64(uint64_t (&v)[EPL], int lane) {
  constexpr int N = 64 * EPL;
#pragma unroll
  for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j < EPL) {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          if ((r & j) == 0) {
            const int e = lane * EPL + r;
            const bool up = (e & kk) == 0;
            const uint64_t a = v[r], b = v[r ^ j];
            const bool sw = (a > b) == up;
            v[r] = sw ? b : a;
            v[r ^ j] = sw ? a : b;
          }
        }
      } else {
        const int lj = j / EPL;
        const bool lower = (lane & lj) == 0;
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          const int e = lane * EPL + r;
          const bool up = (e & kk) == 0;
          const uint64_t o = __shfl_xor(v[r], lj, 64);
          const uint64_t mn = v[r] < o ? v[r] : o, mx = v[r] < o ? o : v[r];
          v[r] = (lower == up) ? mn : mx;
        }
      }
    }
  }
}

// Exact FP64 squared distance of row `row` of X to the query held in LDS,
// computed by a group of 16 consecutive lanes (all 16 get the result).  Rows
// whose start is 16-byte aligned are read as float4 (256 contiguous bytes per
// group and step).
__device__ __forceinline__ double group16_d2(const float* __restrict__ X, int64_t row, int64_t d,
                                             const float* ys, int l16) {
  const float* xr = X + row * d;
  double s = 0.0;
  if (((d & 3) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0)) {
    for (int64_t t = 4 * l16; t < d; t += 64) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(xr + t);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double df = (double)v[c] - (double)ys[t + c];
        s = __builtin_fma(df, df, s);
      }
    }
  } else {
    for (int64_t t = l16; t < d; t += 16) {
      const double df = (double)xr[t] - (double)ys[t];
      s = __builtin_fma(df, df, s);
    }
  }
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 4, 64);
  s += __shfl_xor(s, 8, 64);
  return s;
}

// ||x - y||^2 as an unevaluated double-double sum (error-free squares and
// two-sum accumulation); used only to order near ties.
__device__ void dd_d2(const float* __restrict__ xr, const float* ys, int64_t d, double& hi,
                      double& lo) {
  double s = 0.0, c = 0.0;
  for (int64_t t = 0; t < d; ++t) {
    const double df = (double)xr[t] - (double)ys[t];
    const double p = df * df;
    const double pe = __builtin_fma(df, df, -p);
    // two-sum s + p
    const double t1 = s + p;
    const double bp = t1 - s;
    const double e1 = (s - (t1 - bp)) + (p - bp);
    s = t1;
    c += e1 + pe;
  }
  hi = s + c;
  lo = c - (hi - s);
}

__device__ __forceinline__ double kernel_value(double d2, double h, int kern) {
  if (kern == KERNEL_GAUSSIAN) return exp(-d2 / (2.0 * h * h));
  return exp(-sqrt(d2) / h);
}

// Reorders the entries of [a, b] (inclusive; near-tied in FP64) by their
// double-double distance, then index.  Single thread, tiny ranges.
__device__ void resolve_band(uint64_t* key, uint32_t* idx, int a, int b, const float* X,
                             int64_t d, const float* ys) {
  constexpr int MAXB = 32;
  double hi[MAXB], lo[MAXB];
  uint32_t id[MAXB];
  const int cnt = b - a + 1;
  for (int i = 0; i < cnt; ++i) {
    id[i] = idx[a + i];
    dd_d2(X + (int64_t)id[i] * d, ys, d, hi[i], lo[i]);
  }
  for (int i = 1; i < cnt; ++i) {   // insertion sort by (hi, lo, id)
    const double h0 = hi[i], l0 = lo[i];
    const uint32_t i0 = id[i];
    int j = i - 1;
    while (j >= 0 && (hi[j] > h0 || (hi[j] == h0 && (lo[j] > l0 || (lo[j] == l0 && id[j] > i0))))) {
      hi[j + 1] = hi[j]; lo[j + 1] = lo[j]; id[j + 1] = id[j];
      --j;
    }
    hi[j + 1] = h0; lo[j + 1] = l0; id[j + 1] = i0;
  }
  for (int i = 0; i < cnt; ++i) {
    idx[a + i] = id[i];
    key[a + i] = __builtin_bit_cast(uint64_t, hi[i]);
  }
}

// Relative error bound of the FP64 direct squared distance.
__device__ __forceinline__ double fp64_rel(int64_t d) { return 4.0 * (double)(d + 2) * 0x1p-53; }

// After a (d^2 bits, index) sort of `cnt` exact candidates: fix the order of
// entries whose FP64 distances are too close to the k-th to be trusted.
__device__ void fix_boundary(uint64_t* key, uint32_t* idx, int cnt, int k, const float* X,
                             int64_t d, const float* ys) {
  if (threadIdx.x == 0 && k < cnt && k > 0) {
    const double D = __builtin_bit_cast(double, key[k - 1]);
    const double rel = fp64_rel(d);
    const double lo = D * (1.0 - rel), hi = D * (1.0 + rel);
    int a = k - 1, b = k - 1;
    while (a > 0 && __builtin_bit_cast(double, key[a - 1]) >= lo) --a;
    while (b + 1 < cnt && __builtin_bit_cast(double, key[b + 1]) <= hi) ++b;
    if (b > k - 1) {
      if (b - a + 1 > 32) { a = (k - 16 > a) ? k - 16 : a; b = (a + 31 < b) ? a + 31 : b; }
      resolve_band(key, idx, a, b, X, d, ys);
    }
  }
  __syncthreads();
}

// Neighbour list sorted by index, Z1 = sum of kernel values over it.
__device__ void emit_neighbours(const uint64_t* key, uint32_t* idx, uint32_t* tmp, int k,
                                double h, int kern, int32_t* nn_row, int32_t* nn_out_row,
                                double* z1_out, double* red) {
  // Z1 in the fixed (distance, index) order: per-thread strided partials, then a tree.
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x)
    s += kernel_value(__builtin_bit_cast(double, key[i]), h, kern);
  red[threadIdx.x] = s;
  const int N = next_pow2(k);
  for (int i = threadIdx.x; i < N; i += blockDim.x) tmp[i] = i < k ? idx[i] : 0xffffffffu;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  // sort the k indices ascending (bitonic on 32-bit values)
  for (int kk = 2; kk <= N; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint32_t a = tmp[i], b = tmp[ixj];
          if ((a > b) == ((i & kk) == 0)) { tmp[i] = b; tmp[ixj] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    nn_row[i] = (int32_t)tmp[i];
    if (nn_out_row) nn_out_row[i] = (int32_t)tmp[i];
  }
  if (threadIdx.x == 0) *z1_out = red[0];
}

// ---------------------------------------------------------------------------
// 1. scan
// ---------------------------------------------------------------------------

// Lists holding more than `lim` entries are cut to their K1 smallest keys;
// each wave sorts its own queries' lists in registers.  Whole block calls.
template <int EPL>
__device__ __forceinline__ void compact_lists(uint64_t* __restrict__ lists, int* cnt, float* thr,
                                              int lim, int K1, int wave, int lane) {
  constexpr int cap1 = 64 * EPL;
  for (int ql = wave; ql < BQ; ql += WG / 64) {
    const int c = cnt[ql];
    if (c <= lim) continue;
    uint64_t* lst = lists + (int64_t)ql * cap1;
    uint64_t v[EPL];
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
      const int e = lane * EPL + r;
      v[r] = e < c ? lst[e] : ~0ull;
    }
    wave_sort_u64<EPL>(v, lane);
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
      const int e = lane * EPL + r;
      if (e < K1) lst[e] = v[r];
    }
    uint64_t mine = 0;   // static register indexing only
#pragma unroll
    for (int r = 0; r < EPL; ++r)
      if (r == (K1 - 1) % EPL) mine = v[r];
    const uint64_t kth = __shfl(mine, (K1 - 1) / EPL, 64);
    if (lane == 0) {
      cnt[ql] = K1;
      thr[ql] = key_float((uint32_t)(kth >> 32));
    }
  }
  __syncthreads();
}
template <typename T, int EPL>   // list capacity = 64 * EPL
__global__ void __launch_bounds__(WG, 2)
knn_scan_kernel(TileProblem p, uint64_t* __restrict__ cand, int32_t* __restrict__ cand_cnt,
                int K1) {
  constexpr int cap1 = 64 * EPL;
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  __shared__ float thr[BQ];
  __shared__ float yks[BQ];
  __shared__ int cnt[BQ];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t t0 = split * p.ntiles / p.splits, t1 = (split + 1) * p.ntiles / p.splits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  if (threadIdx.x < BQ) {
    thr[threadIdx.x] = __builtin_inff();
    cnt[threadIdx.x] = 0;
    yks[threadIdx.x] = p.yknorm[qt * BQ + threadIdx.x];
  }
  uint64_t* lists = cand + (split * p.qp + qt * BQ) * (int64_t)cap1;

  const char* yq = p.Ys + qt * BQ * p.ld_bytes;
  const int limit = cap1 - BN;   // a list above this could overflow in the next tile

  __syncthreads();   // thr / cnt initialised
  StreamState st;
  if (t0 < t1) stream_start(st, yq, p.Xs, p.ld_bytes, t0);
  __shared__ float xks[2][BN];   // data key norms, one tile ahead (see kde_tile_kernel)
  float xk_reg = (threadIdx.x < BN && t0 < t1) ? p.xknorm[t0 * BN + threadIdx.x] : 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    const int nb = (int)((t - t0) & 1);
    if (threadIdx.x < BN) {
      xks[nb][threadIdx.x] = xk_reg;
      if (t + 1 < t1) xk_reg = p.xknorm[(t + 1) * BN + threadIdx.x];
    }
    f32x4 acc[4][4];
    stream_tile<T>(acc, st, yq, p.Xs, p.ld_bytes, p.nchunks, t, t1, lds, wq, wn, lane);
    float xk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
      xk[j] = col < p.n ? xks[nb][wn * 64 + j * 16 + (lane & 15)] : __builtin_inff();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ql = wq * 64 + i * 16 + 4 * (lane >> 4) + r;
        const float yk = yks[ql], th = thr[ql];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float key = __builtin_fmaf(-2.f, acc[i][j][r], yk + xk[j]);
          if (key < th) {
            const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
            const int slot = atomicAdd(&cnt[ql], 1);
            lists[(int64_t)ql * cap1 + slot] =
                ((uint64_t)float_key(key) << 32) | (uint64_t)(uint32_t)col;
          }
        }
      }
    __syncthreads();
    compact_lists<EPL>(lists, cnt, thr, limit, K1, wave, lane);
  }
  compact_lists<EPL>(lists, cnt, thr, K1, K1, wave, lane);
  if (threadIdx.x < BQ) cand_cnt[split * p.qp + qt * BQ + threadIdx.x] = cnt[threadIdx.x];
}

// ---------------------------------------------------------------------------
// 1'. candidate pass for 16-bit scans: every lane keeps, for each of its 16
//     queries, the smallest key among the data columns it sees (one "cell" =
//     one lane column of one wave, per split).  No list traffic at all; the
//     candidates only seed the exact distance d_k of the second pass, which is
//     what certifies the result.
// ---------------------------------------------------------------------------
constexpr int CELLS = 32;   // cells per (split, query): 16 lane columns x 2 waves

template <typename T, int ENG>   // ENG: see tile_engine
__global__ void __launch_bounds__(WG, 2)
knn_cand_kernel(TileProblem p, uint64_t* __restrict__ cand, int32_t* __restrict__ cand_cnt) {
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t t0 = split * p.ntiles / p.splits, t1 = (split + 1) * p.ntiles / p.splits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  // Per (query, cell): the smallest key seen, with the column block j (0..3)
  // packed into its two low mantissa bits so that one min tracks both, and
  // the tile it came from.  The packing perturbs keys by at most 3 ulp; the
  // candidates only seed the second pass, which alone decides the result.
  // The sweep tracks xk - 2 x.y; the query's key norm, the same for the whole
  // row, is added once per cell at the end.
  float best[4][4];
  int32_t btile[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      best[i][r] = __builtin_inff();
      btile[i][r] = -1;
    }
  const char* yq = p.Ys + qt * BQ * p.ld_bytes;
  constexpr int NK = 2;   // k-groups of the register-resident engine
  // sweep tile t is data tile t * ts: the seeds come from every ts-th tile
  const int64_t ts = p.tstride;
  StreamState st;
  XStream<NK> xs;
  u32x4 yf[4][NK];
  QlState ql;
  if (t0 < t1) {
    if constexpr (ENG == 0) {
      stream_start(st, yq, p.Xs, p.ld_bytes, t0, ts);
    } else if constexpr (ENG == 1) {
      ql_start(ql, yq, p.Xs, t0, lds, ts);
    } else {
      yreg_load<NK>(yf, yq, p.ld_bytes, wq, lane);
      xs_load(xs, p.Xs + t0 * ts * BN * p.ld_bytes, p.ld_bytes);
      xs.buf = 0;
    }
  }
  __shared__ float xks[2][BN];   // data key norms, one tile ahead (see kde_tile_kernel)
  float xk_reg = (threadIdx.x < BN && t0 < t1) ? p.xknorm[t0 * ts * BN + threadIdx.x] : 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    const int nb = (int)((t - t0) & 1);
    if (threadIdx.x < BN) {
      xks[nb][threadIdx.x] = xk_reg;
      if (t + 1 < t1) xk_reg = p.xknorm[(t + 1) * ts * BN + threadIdx.x];
    }
    f32x4 acc[4][4];
    if constexpr (ENG == 0)
      stream_tile<T>(acc, st, yq, p.Xs, p.ld_bytes, p.nchunks, t, t1, lds, wq, wn, lane, ts);
    else if constexpr (ENG == 1)
      ql_tile<T>(acc, ql, p.Xs, t, t1, lds, wq, wn, lane, ts);
    else
      yreg_tile<T, NK>(acc, xs, yf, p.Xs, p.ld_bytes, t, t1, lds, wn, lane, ts);
    const int64_t dt = t * ts;   // the data tile
    float xk[4];   // padding columns: a huge finite key (never NaN after packing)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = dt * BN + wn * 64 + j * 16 + (lane & 15);
      xk[j] = col < p.n ? xks[nb][wn * 64 + j * 16 + (lane & 15)] : 3.0e38f;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float m = __builtin_inff();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float part = __builtin_fmaf(-2.f, acc[i][j][r], xk[j]);
          m = fminf(m, __uint_as_float((__float_as_uint(part) & ~3u) | (uint32_t)j));
        }
        const bool better = m < best[i][r];
        best[i][r] = better ? m : best[i][r];
        btile[i][r] = better ? (int32_t)dt : btile[i][r];
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = qt * BQ + wq * 64 + i * 16 + 4 * (lane >> 4) + r;
      const int64_t col = (int64_t)btile[i][r] * BN + wn * 64 +
                          (int64_t)(__float_as_uint(best[i][r]) & 3u) * 16 + (lane & 15);
      const uint64_t v = (btile[i][r] < 0 || col >= p.n)
                             ? ~0ull
                             : ((uint64_t)float_key(best[i][r] + p.yknorm[row]) << 32) | (uint64_t)col;
      cand[(split * p.qp + row) * CELLS + wn * 16 + (lane & 15)] = v;
    }
  if (threadIdx.x < BQ) cand_cnt[split * p.qp + qt * BQ + threadIdx.x] = CELLS;
}

// ---------------------------------------------------------------------------
// 2. merge + exact refine + certificate (one workgroup per query)
// ---------------------------------------------------------------------------
struct RefineArgs {
  const float* X;
  const float* Y;
  int64_t n, q, d, k, qp, splits;
  double h;
  int kern;
  int approx;   // candidates come from the cell pass: no certificate, always collect
  // second refinement only: entries of its LDS sort and of its exact list (the
  // dynamic LDS of the launch is sized from them), and whether this launch
  // takes only the queries whose list fits (`small`: the others are left to a
  // launch with the full capacity)
  int sort_cap = SORT_CAP;   // keys of the sort of the list
  int ex_cap = SORT_CAP;     // exact (distance, index) pairs after it
  int kd_cap = K_MAX;
  int small = 0;
};

// The K1 smallest of a query's `cells` cell candidates (packed key, index;
// empty cells are ~0), sorted ascending, in buf[0 .. min(K1, valid)), and
// *fill = min(K1, number of non-empty cells).  Wave w takes cells
// [w * 64 * EPL, (w + 1) * 64 * EPL) and sorts them in registers; K1 <= 64 * EPL
// of each wave go to buf, where the upper levels of one workgroup bitonic sort
// merge them.  Whole block.
template <int EPL>
__device__ void cells_wave_select(const uint64_t* __restrict__ cand, int64_t qp, int64_t qi,
                                  int64_t cells, int K1, uint64_t* buf, int* fill) {
  __shared__ int valid_w[WG / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t v[EPL];
  int valid = 0;
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int64_t e = (int64_t)wave * 64 * EPL + lane * EPL + r;
    v[r] = e < cells ? cand[((e / CELLS) * qp + qi) * CELLS + e % CELLS] : ~0ull;
    valid += v[r] != ~0ull;
  }
  for (int off = 32; off > 0; off >>= 1) valid += __shfl_xor(valid, off, 64);
  wave_sort_u64<EPL>(v, lane);
  // each wave's K1 smallest, padded with empty cells to a block of kc (a power
  // of two), ascending in even waves' blocks and descending in odd ones: the
  // merge then runs only the bitonic levels above kc
  const int kc = next_pow2(K1), N = (WG / 64) * kc;
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int el = lane * EPL + r;
    if (el < kc) buf[wave * kc + ((wave & 1) ? kc - 1 - el : el)] = el < K1 ? v[r] : ~0ull;
  }
  if (lane == 0) valid_w[wave] = valid;
  __syncthreads();
  block_sort_u64(buf, N, 2 * kc);
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < WG / 64; ++w) tot += valid_w[w];
    *fill = tot < K1 ? tot : K1;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(WG, 6)
knn_refine_kernel(RefineArgs a, KnnBuffers b, int32_t* __restrict__ nn_out) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // sort_cap: merge buffer entries, kd_cap >= K1: exact candidates (even counts)
  const int bcap = a.sort_cap, kcap = a.kd_cap;
  uint64_t* buf = reinterpret_cast<uint64_t*>(smem);                  // bcap
  uint64_t* dkey = buf + bcap;                                         // kcap
  uint32_t* didx = reinterpret_cast<uint32_t*>(dkey + kcap);          // kcap
  uint32_t* tmp = didx + kcap;                                         // kcap
  double* red = reinterpret_cast<double*>(tmp + kcap);                // WG
  float* ys = reinterpret_cast<float*>(red + WG);                      // d
  __shared__ int fill_s;
  const int64_t qi = blockIdx.x;
  const int K1 = (int)b.K1;
  for (int64_t t = threadIdx.x; t < a.d; t += WG) ys[t] = a.Y[qi * a.d + t];
  if (threadIdx.x == 0) fill_s = 0;
  __syncthreads();
  // gather the split lists, keeping the K1 smallest keys
  int64_t seen = 0;
  const int64_t cells = a.approx ? a.splits * (int64_t)CELLS : 0;
  if (a.approx && cells <= (WG / 64) * 64 * 16 && K1 <= 512) {
    // at most 1024 cells per wave: each wave sorts its share in registers, the
    // K1 smallest of every wave meet in LDS, and one sort of those gives the
    // K1 smallest of all (empty cells sort last)
    if (cells <= (WG / 64) * 64 * 8)
      cells_wave_select<8>(b.cand, a.qp, qi, cells, K1, buf, &fill_s);
    else
      cells_wave_select<16>(b.cand, a.qp, qi, cells, K1, buf, &fill_s);
  } else if (a.approx) {
    // cell candidates: CELLS per (split, query), contiguous; read in chunks of
    // at most bcap - K1 entries whose loads are all in flight together
    const int64_t total = a.splits * (int64_t)CELLS, chunk = bcap - K1;
    for (int64_t c0 = 0; c0 < total; c0 += chunk) {
      const int64_t c1 = c0 + chunk < total ? c0 + chunk : total;
      __syncthreads();   // every thread has read fill_s for the previous decision
      for (int64_t i = c0 + threadIdx.x; i < c1; i += WG) {
        const uint64_t v = b.cand[((i / CELLS) * a.qp + qi) * CELLS + i % CELLS];
        if (v != ~0ull) buf[atomicAdd(&fill_s, 1)] = v;
      }
      __syncthreads();
      const bool last = c1 == total;
      // before another chunk the buffer is cut back to K1; after the last one
      // it is sorted whenever the K1-th key is used
      if ((last && fill_s >= K1) || (!last && fill_s > K1)) {
        const int F = fill_s;
        const int N = next_pow2(F);   // <= bcap
        for (int i = F + threadIdx.x; i < N; i += WG) buf[i] = ~0ull;
        __syncthreads();
        block_sort_u64(buf, N);
        if (threadIdx.x == 0) fill_s = K1;
        __syncthreads();
      }
    }
  }
  for (int64_t s = 0; s < (a.approx ? 0 : a.splits); ++s) {
    const int c = b.cand_cnt[s * a.qp + qi];
    const uint64_t* lst = b.cand + (s * a.qp + qi) * b.cap1;
    seen += c;
    __syncthreads();
    // append the list, dropping empty cells (order inside buf is irrelevant)
    for (int i = threadIdx.x; i < c; i += WG) {
      const uint64_t v = lst[i];
      if (v != ~0ull) buf[atomicAdd(&fill_s, 1)] = v;
    }
    __syncthreads();
    const bool flush = (fill_s + K1 > bcap) || (s + 1 == a.splits);
    if (flush && fill_s >= K1) {   // sorted whenever the K1-th key is used
      const int F = fill_s;
      const int N = next_pow2(F);   // <= bcap
      for (int i = F + threadIdx.x; i < N; i += WG) buf[i] = ~0ull;
      __syncthreads();
      block_sort_u64(buf, N);
      if (threadIdx.x == 0) fill_s = K1;
      __syncthreads();
    }
  }
  const int C = fill_s;            // candidates (<= K1)
  // all points were candidates iff no list ever dropped anything
  const bool complete = !a.approx && (seen == a.n) && (C == a.n);
  const float Tkey = (C == K1) ? key_float((uint32_t)(buf[K1 - 1] >> 32)) : __builtin_inff();
  // exact FP64 distances, four rows per 16-lane group at a time
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  for (int c0 = g; c0 < C; c0 += 4 * (WG / 16)) {
    int64_t rr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = c0 + i * (WG / 16);
      rr[i] = c < C ? (int64_t)(buf[c] & 0xffffffffu) : -1;
    }
    double d2[4];
    group16_d2_4(a.X, rr, a.d, ys, l16, d2);
    if (l16 == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = c0 + i * (WG / 16);
        if (c < C) { dkey[c] = __builtin_bit_cast(uint64_t, d2[i]); didx[c] = (uint32_t)rr[i]; }
      }
  }
  const int N = next_pow2(C > 1 ? C : 2);
  for (int i = C + threadIdx.x; i < N; i += WG) { dkey[i] = ~0ull; didx[i] = 0xffffffffu; }
  __syncthreads();
  block_sort_pairs(dkey, didx, N);
  const int k = (int)a.k;
  fix_boundary(dkey, didx, C, k, a.X, a.d, ys);
  bool ok = complete;
  if (!ok && C < k) {
    // too few candidates to bound d_k: the second pass collects every point
    if (threadIdx.x == 0) {
      b.thr2[qi] = __builtin_inff();
      b.status[qi] = 1;
      b.cand2_cnt[qi] = 0;
      b.flags[qi / BQ] = 1;
    }
    return;
  }
  if (!ok && C >= k) {
    const double Dk = __builtin_bit_cast(double, dkey[k - 1]) * (1.0 + fp64_rel(a.d));
    const double E = (double)__builtin_bit_cast(float, *b.xerr_max);
    const double ey = (double)b.yerr[qi];
    const double lhs = sqrt((double)fmaxf(Tkey, 0.f)) - E - ey;
    ok = !a.approx && lhs > 0.0 && lhs * lhs > Dk * (1.0 + 1e-14);
    if (!ok) {
      if (threadIdx.x == 0) {
        const double r = (sqrt(Dk) + E + ey) * (1.0 + 1e-6);
        b.thr2[qi] = (float)(r * r * (1.0 + 1e-6));
        b.status[qi] = 1;
        b.cand2_cnt[qi] = 0;
        b.flags[qi / BQ] = 1;
      }
      return;
    }
  }
  if (!ok) {   // fewer candidates than k cannot happen for k <= n; treat as exhaustive
    if (threadIdx.x == 0) { b.status[qi] = 2; b.flags[qi / BQ] = 1; }
    return;
  }
  if (threadIdx.x == 0) b.status[qi] = 0;
  emit_neighbours(dkey, didx, tmp, k, a.h, a.kern, b.nn_work + qi * k,
                  nn_out ? nn_out + qi * k : nullptr, b.z1 + qi, red);
}

// ---------------------------------------------------------------------------
// 3. second pass: collect every point whose key admits distance <= d_k
// ---------------------------------------------------------------------------
constexpr int COLLECT_STAGE = 128;   // staged second-pass hits per wave

template <typename T, int ENG>   // ENG: see tile_engine
__global__ void __launch_bounds__(WG, 2)
knn_collect_kernel(TileProblem p, KnnBuffers b) {
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  if (b.flags[qt] == 0) return;
  const int64_t t0 = split * p.ntiles / p.splits, t1 = (split + 1) * p.ntiles / p.splits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  // A column hits query row r when key = xk + yk - 2 x.y <= th_r.  The sweep
  // tests xk - 2 x.y (one fma) against tq_r = th_r - yk_r (one subtraction
  // per row, once): round-to-nearest is monotone, so whenever the exact key
  // is <= th_r the rounded sides compare the same way, and the test admits
  // every column the key bound requires.  th_r is -inf for a query without a
  // second pass and +inf for one that collects every point.  tq and the key
  // norms (for the key codes of the hits) of the tile's rows sit in LDS,
  // published by the first barrier of the sweep.
  __shared__ float tqs[BQ], yks[BQ];
  if (threadIdx.x < BQ) {
    const int64_t row = qt * BQ + threadIdx.x;
    const float th = (row < p.q && b.status[row] == 1) ? b.thr2[row] : -__builtin_inff();
    const float yk = p.yknorm[row];
    tqs[threadIdx.x] = th == __builtin_inff() ? th : th - yk;
    yks[threadIdx.x] = yk;
  }
  // Hits are staged per wave in LDS, (query row in the tile) << 57 | (key code
  // >> 7) << 32 | column, and appended to the global lists in bulk, so a wave
  // waits for one round of global atomics per drain rather than one per tile
  // with a hit.  The stage is private to its wave: no barrier is needed to
  // fill, test or drain it.  A hit that finds the stage full goes straight to
  // its query's list.
  __shared__ uint64_t stage[WG / 64][COLLECT_STAGE];
  __shared__ int nst[WG / 64];
  if (lane == 0) nst[wave] = 0;
  auto drain = [&]() {
    __builtin_amdgcn_wave_barrier();
    const int c = nst[wave];
    const int m = c < COLLECT_STAGE ? c : COLLECT_STAGE;
    for (int e = lane; e < m; e += 64) {
      const uint64_t v = stage[wave][e];
      const int64_t row = qt * BQ + (int64_t)(v >> 57);
      const int slot = atomicAdd(&b.cand2_cnt[row], 1);
      if (slot < b.cap2)
        b.cand2[row * b.cap2 + slot] = (((v >> 32) & 0x1ffffffull) << 39) | (v & 0xffffffffull);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) nst[wave] = 0;
    __builtin_amdgcn_wave_barrier();
  };
  const char* yq = p.Ys + qt * BQ * p.ld_bytes;
  constexpr int NK = 2;   // k-groups of the register-resident engine
  StreamState st;
  XStream<NK> xs;
  u32x4 yf[4][NK];
  QlState ql;
  if (t0 < t1) {
    if constexpr (ENG == 0) {
      stream_start(st, yq, p.Xs, p.ld_bytes, t0);
    } else if constexpr (ENG == 1) {
      ql_start(ql, yq, p.Xs, t0, lds);
    } else {
      yreg_load<NK>(yf, yq, p.ld_bytes, wq, lane);
      xs_load(xs, p.Xs + t0 * BN * p.ld_bytes, p.ld_bytes);
      xs.buf = 0;
    }
  }
  __shared__ float xks[2][BN];   // data key norms, one tile ahead (see kde_tile_kernel)
  float xk_reg = (threadIdx.x < BN && t0 < t1) ? p.xknorm[t0 * BN + threadIdx.x] : 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    const int nb = (int)((t - t0) & 1);
    if (threadIdx.x < BN) {
      xks[nb][threadIdx.x] = xk_reg;
      if (t + 1 < t1) xk_reg = p.xknorm[(t + 1) * BN + threadIdx.x];
    }
    f32x4 acc[4][4];
    if constexpr (ENG == 0)
      stream_tile<T>(acc, st, yq, p.Xs, p.ld_bytes, p.nchunks, t, t1, lds, wq, wn, lane);
    else if constexpr (ENG == 1)
      ql_tile<T>(acc, ql, p.Xs, t, t1, lds, wq, wn, lane);
    else
      yreg_tile<T, NK>(acc, xs, yf, p.Xs, p.ld_bytes, t, t1, lds, wn, lane);
    // queries without a second pass (th = -inf) never hit; padding columns
    // (infinite key) can only hit a query with th = +inf and are dropped by
    // the column check of the append
    float xk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
      xk[j] = col < p.n ? xks[nb][wn * 64 + j * 16 + (lane & 15)] : __builtin_inff();
    }
    // per query row (i, r): the lanes of the wave whose row has a hit in this
    // tile (some key of the row is <= its threshold), as a wave-wide mask
    uint64_t hitm[4][4], any = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float m = __builtin_fmaf(-2.f, acc[i][0][r], xk[0]);
#pragma unroll
        for (int j = 1; j < 4; ++j) m = fminf(m, __builtin_fmaf(-2.f, acc[i][j][r], xk[j]));
        hitm[i][r] = __builtin_amdgcn_ballot_w64(m <= tqs[wq * 64 + i * 16 + 4 * (lane >> 4) + r]);
        any |= hitm[i][r];
      }
    if (any) {   // append the hits, visiting only the rows where some lane has one
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!hitm[i][r]) continue;
          const int64_t row = qt * BQ + wq * 64 + i * 16 + 4 * (lane >> 4) + r;
          const float yk = yks[wq * 64 + i * 16 + 4 * (lane >> 4) + r];
          const float tq = tqs[wq * 64 + i * 16 + 4 * (lane >> 4) + r];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
            const float part = __builtin_fmaf(-2.f, acc[i][j][r], xk[j]);
            if (col < p.n && part <= tq) {
              // part + yk: two roundings, as fl(xk + yk) - 2 x.y has, within
              // the slack of the pre-scaled norms, so still a lower bound
              const uint32_t code = float_key(part + yk);
              const int e = atomicAdd(&nst[wave], 1);
              if (e < COLLECT_STAGE)
                stage[wave][e] = ((uint64_t)(row - qt * BQ) << 57) | ((uint64_t)(code >> 7) << 32) |
                                 (uint64_t)(uint32_t)col;
              else {   // stage full: straight to the list
                const int slot = atomicAdd(&b.cand2_cnt[row], 1);
                if (slot < b.cap2) b.cand2[row * b.cap2 + slot] = ((uint64_t)code << 32) | (uint64_t)col;
              }
            }
          }
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (nst[wave] >= COLLECT_STAGE / 2) drain();
  }
  drain();
}

// Second-pass entries are (key code << 32 | row): the row's lower-bound key,
// as float_key, rounded down (a valid lower bound still), and its index.
// The refinement sorts them by key, evaluates the K1 smallest exactly, and
// then only the entries that the k-th of those distances cannot exclude:
// an entry whose key gives sqrt(key) - E - e_y above it is farther than d_k.
__global__ void __launch_bounds__(WG, 6)
knn_refine2_kernel(RefineArgs a, KnnBuffers b, int32_t* __restrict__ nn_out) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // even counts: 8-byte alignment holds; ecap <= cap
  const int cap = a.sort_cap, ecap = a.ex_cap, kcap = a.kd_cap;
  uint64_t* dkey = reinterpret_cast<uint64_t*>(smem);                // cap
  uint32_t* didx = reinterpret_cast<uint32_t*>(dkey + cap);           // ecap
  uint64_t* kd = reinterpret_cast<uint64_t*>(didx + ecap);            // kcap
  uint32_t* tmp = reinterpret_cast<uint32_t*>(kd + kcap);             // kcap
  double* red = reinterpret_cast<double*>(tmp + kcap);                // WG
  float* ys = reinterpret_cast<float*>(red + WG);                      // d
  __shared__ int kept_s;
  const int64_t qi = blockIdx.x;
  if (b.status[qi] != 1) return;
  const int C = b.cand2_cnt[qi];
  // the second pass collects at least the k rows its threshold came from, so
  // C < k cannot occur; should it, the exhaustive scan answers the query
  if (C > b.cap2 || C > cap || C < a.k) {
    if (threadIdx.x == 0 && !a.small) b.status[qi] = 2;
    return;
  }
  for (int64_t t = threadIdx.x; t < a.d; t += WG) ys[t] = a.Y[qi * a.d + t];
  if (threadIdx.x == 0) kept_s = 0;
  // 1. the entries in key order
  const int N = next_pow2(C > 1 ? C : 2);
  for (int i = threadIdx.x; i < N; i += WG) dkey[i] = i < C ? b.cand2[qi * b.cap2 + i] : ~0ull;
  __syncthreads();
  block_sort_u64(dkey, N);
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  const int k = (int)a.k;
  // 2. exact distances of the P smallest keys (kd, tmp), sorted: their k-th bounds d_k
  const int P = C < (int)b.K1 ? C : (int)b.K1;
  for (int c0 = g; c0 < P; c0 += 4 * (WG / 16)) {
    int64_t rr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = c0 + i * (WG / 16);
      rr[i] = c < P ? (int64_t)(uint32_t)dkey[c] : -1;
    }
    double d2[4];
    group16_d2_4(a.X, rr, a.d, ys, l16, d2);
    if (l16 == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = c0 + i * (WG / 16);
        if (c < P) { kd[c] = __builtin_bit_cast(uint64_t, d2[i]); tmp[c] = (uint32_t)rr[i]; }
      }
  }
  const int NP = next_pow2(P > 1 ? P : 2);
  for (int i = P + threadIdx.x; i < NP; i += WG) { kd[i] = ~0ull; tmp[i] = 0xffffffffu; }
  __syncthreads();
  block_sort_pairs(kd, tmp, NP);
  // 3. entries [P, C) kept while their bound does not exclude them (keys
  // ascend, so the kept ones are a prefix)
  int cstar = C;
  if (C > P && P >= k && k > 0) {
    const double Dk = __builtin_bit_cast(double, kd[k - 1]) * (1.0 + fp64_rel(a.d));
    const double E = (double)__builtin_bit_cast(float, *b.xerr_max);
    const double ey = (double)b.yerr[qi];
    int kept = 0;
    for (int c = P + threadIdx.x; c < C; c += WG) {
      const float key = key_float((uint32_t)(dkey[c] >> 32));
      const double lhs = sqrt((double)fmaxf(key, 0.f)) - E - ey;
      kept += !(lhs > 0.0 && lhs * lhs > Dk * (1.0 + 1e-14));
    }
    if (kept) atomicAdd(&kept_s, kept);
    __syncthreads();
    cstar = P + kept_s;
  }
  // (uniform) more exact pairs than this launch holds: the query stays listed
  // for the launch with the full capacity
  if (next_pow2(cstar > 1 ? cstar : 2) > ecap) return;
  // 4. the P evaluated entries in front, then the exact distances of [P, cstar)
  for (int c0 = P + g; c0 < cstar; c0 += 4 * (WG / 16)) {
    int64_t rr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = c0 + i * (WG / 16);
      rr[i] = c < cstar ? (int64_t)(uint32_t)dkey[c] : -1;
    }
    double d2[4];
    group16_d2_4(a.X, rr, a.d, ys, l16, d2);
    if (l16 == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = c0 + i * (WG / 16);
        if (c < cstar) { dkey[c] = __builtin_bit_cast(uint64_t, d2[i]); didx[c] = (uint32_t)rr[i]; }
      }
  }
  for (int i = threadIdx.x; i < P; i += WG) { dkey[i] = kd[i]; didx[i] = tmp[i]; }
  const int N2 = next_pow2(cstar > 1 ? cstar : 2);
  for (int i = cstar + threadIdx.x; i < N2; i += WG) { dkey[i] = ~0ull; didx[i] = 0xffffffffu; }
  __syncthreads();
  block_sort_pairs(dkey, didx, N2);
  fix_boundary(dkey, didx, cstar, k, a.X, a.d, ys);
  if (threadIdx.x == 0) b.status[qi] = 4;   // done by the second pass
  emit_neighbours(dkey, didx, tmp, k, a.h, a.kern, b.nn_work + qi * k,
                  nn_out ? nn_out + qi * k : nullptr, b.z1 + qi, red);
}

// ---------------------------------------------------------------------------
// 4. exhaustive exact scan for the rare overflow (one workgroup per query)
// ---------------------------------------------------------------------------
constexpr int EXH_CHUNK = 512;   // rows examined between checks of the candidate buffer

// The k + 32 smallest (FP64 d^2 bits, index) pairs seen so far, in LDS.  Rows
// below the current (k+32)-th pair are appended; the buffer is sorted and cut
// back only when another chunk could overflow it (and after the last chunk),
// so once the cut-off is tight almost every row is a compare and nothing else.
struct ExhaustiveTop {
  int kkeep, cap;   // cap: buffer entries, a power of two >= kkeep + EXH_CHUNK
  uint64_t kth_key = ~0ull;
  uint32_t kth_idx = 0xffffffffu;
  __device__ ExhaustiveTop(int k, int cap_)
      : kkeep(k + 32 < cap_ - EXH_CHUNK ? k + 32 : cap_ - EXH_CHUNK), cap(cap_) {}
  __device__ void offer(uint64_t kb, uint32_t id, uint64_t* dkey, uint32_t* didx, int* fill) {
    if (kb < kth_key || (kb == kth_key && id < kth_idx)) {
      const int slot = atomicAdd(fill, 1);
      dkey[slot] = kb;
      didx[slot] = id;
    }
  }
  // whole block; `last`: after the final chunk (leaves the buffer sorted)
  __device__ void settle(uint64_t* dkey, uint32_t* didx, int* fill, bool last) {
    __syncthreads();
    const int F = *fill;
    if (F <= cap - EXH_CHUNK && !last) return;   // uniform: F read after the barrier
    const int N = next_pow2(F > 1 ? F : 2);
    for (int i = F + threadIdx.x; i < N; i += WG) { dkey[i] = ~0ull; didx[i] = 0xffffffffu; }
    __syncthreads();
    block_sort_pairs(dkey, didx, N);
    if (F >= kkeep) { kth_key = dkey[kkeep - 1]; kth_idx = didx[kkeep - 1]; }
    __syncthreads();
    if (threadIdx.x == 0) *fill = F < kkeep ? F : kkeep;
    __syncthreads();
  }
};
__global__ void __launch_bounds__(WG)
knn_exhaustive_kernel(RefineArgs a, KnnBuffers b, int32_t* __restrict__ nn_out) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // sort_cap: candidate buffer entries, kd_cap: next power of two >= k (even counts)
  const int cap = a.sort_cap, kcap = a.kd_cap;
  uint64_t* dkey = reinterpret_cast<uint64_t*>(smem);                // cap
  uint32_t* didx = reinterpret_cast<uint32_t*>(dkey + cap);           // cap
  uint32_t* tmp = didx + cap;                                          // kcap
  double* red = reinterpret_cast<double*>(tmp + kcap);                // WG
  float* ys = reinterpret_cast<float*>(red + WG);
  __shared__ int fill_s;
  const int64_t qi = blockIdx.x;
  if (b.status[qi] != 2) return;
  const int k = (int)a.k;
  for (int64_t t = threadIdx.x; t < a.d; t += WG) ys[t] = a.Y[qi * a.d + t];
  if (threadIdx.x == 0) fill_s = 0;
  __syncthreads();
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  ExhaustiveTop top(k, cap);
  for (int64_t r0 = 0; r0 < a.n; r0 += EXH_CHUNK) {
    const int64_t r1 = r0 + EXH_CHUNK < a.n ? r0 + EXH_CHUNK : a.n;
    // four rows per 16-lane group at a time (their loads in flight together)
    for (int64_t rb = r0 + g; rb < r1; rb += 4 * (WG / 16)) {
      int64_t rr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) rr[i] = rb + i * (WG / 16) < r1 ? rb + i * (WG / 16) : -1;
      double d2[4];
      group16_d2_4(a.X, rr, a.d, ys, l16, d2);
      if (l16 == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rr[i] >= 0)
            top.offer(__builtin_bit_cast(uint64_t, d2[i]), (uint32_t)rr[i], dkey, didx, &fill_s);
    }
    top.settle(dkey, didx, &fill_s, r1 == a.n);
  }
  fix_boundary(dkey, didx, fill_s, k, a.X, a.d, ys);
  if (threadIdx.x == 0) b.status[qi] = 5;   // done by the exhaustive scan
  emit_neighbours(dkey, didx, tmp, k, a.h, a.kern, b.nn_work + qi * k,
                  nn_out ? nn_out + qi * k : nullptr, b.z1 + qi, red);
}

// ---------------------------------------------------------------------------
// k = n: every row is a neighbour; Z1 is the exact FP64 kernel sum
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG)
knn_all_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n, int64_t d,
               double h, int kern, int32_t* __restrict__ nn, double* __restrict__ z1) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  double* red = reinterpret_cast<double*>(smem);   // WG / 16
  float* ys = reinterpret_cast<float*>(red + WG / 16);
  const int64_t qi = blockIdx.x;
  for (int64_t t = threadIdx.x; t < d; t += WG) ys[t] = Y[qi * d + t];
  for (int64_t i = threadIdx.x; i < n; i += WG) nn[qi * n + i] = (int32_t)i;
  __syncthreads();
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  double s = 0.0;
  // rows g, g + 16, ... in order, four at a time
  for (int64_t r0 = g; r0 < n; r0 += 4 * (WG / 16)) {
    int64_t rr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) rr[i] = r0 + i * (WG / 16) < n ? r0 + i * (WG / 16) : -1;
    double d2[4];
    group16_d2_4(X, rr, d, ys, l16, d2);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (rr[i] >= 0) s += kernel_value(d2[i], h, kern);
  }
  if (l16 == 0) red[g] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < WG / 16; ++i) t += red[i];
    z1[qi] = t;
  }
}

hipError_t launch_knn_all(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                          double h, int kern, int32_t* nn, double* z1, hipStream_t s) {
  if (q == 0) return hipSuccess;
  const size_t sm = (WG / 16) * 8 + d * 4 + 16;
  knn_all_kernel<<<dim3((unsigned)q), dim3(WG), sm, s>>>(X, Y, n, d, h, kern, nn, z1);
  return hipGetLastError();
}

// Z1 over given neighbour lists nn[q][k]: FP64 kernel sum in a fixed order
// (16-lane groups take every 16th entry, then the groups in order); entries
// outside [0, n) are skipped.
__global__ void __launch_bounds__(WG)
knn_list_sum_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t n,
                    int64_t d, double h, int kern, const int32_t* __restrict__ nn, int64_t k,
                    double* __restrict__ z1) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  double* red = reinterpret_cast<double*>(smem);   // WG / 16
  float* ys = reinterpret_cast<float*>(red + WG / 16);
  const int64_t qi = blockIdx.x;
  for (int64_t t = threadIdx.x; t < d; t += WG) ys[t] = Y[qi * d + t];
  __syncthreads();
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  double s = 0.0;
  for (int64_t j0 = g; j0 < k; j0 += 4 * (WG / 16)) {   // entries j0, j0 + 16, ... in order
    int64_t rr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t j = j0 + i * (WG / 16);
      const int32_t r = j < k ? nn[qi * k + j] : -1;
      rr[i] = (r >= 0 && r < n) ? (int64_t)r : -1;
    }
    double d2[4];
    group16_d2_4(X, rr, d, ys, l16, d2);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (rr[i] >= 0) s += kernel_value(d2[i], h, kern);
  }
  if (l16 == 0) red[g] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < WG / 16; ++i) t += red[i];
    z1[qi] = t;
  }
}

hipError_t launch_knn_list_sum(const float* X, const float* Y, int64_t n, int64_t q, int64_t d,
                               double h, int kern, const int32_t* nn, int64_t k, double* z1,
                               hipStream_t s) {
  if (q == 0) return hipSuccess;
  const size_t sm = (WG / 16) * 8 + d * 4 + 16;
  knn_list_sum_kernel<<<dim3((unsigned)q), dim3(WG), sm, s>>>(X, Y, n, d, h, kern, nn, k, z1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host launch
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t launch_tiles(const TileProblem& p, const KnnBuffers& b, bool collect,
                               hipStream_t s) {
  const dim3 g((unsigned)p.map.grid), blk(WG);
  if (collect) {
    const int eng = tile_engine<T>(p.ld_bytes);
    if constexpr (elem_of<T>::bytes == 2) {
      if (eng == 2) knn_collect_kernel<T, 2><<<g, blk, 0, s>>>(p, b);
      else if (eng == 1) knn_collect_kernel<T, 1><<<g, blk, 0, s>>>(p, b);
      else knn_collect_kernel<T, 0><<<g, blk, 0, s>>>(p, b);
    } else {
      knn_collect_kernel<T, 0><<<g, blk, 0, s>>>(p, b);
    }
  } else if constexpr (elem_of<T>::bytes == 4) {   // 16-bit scans use the candidate pass
    switch (b.cap1) {
      case 256: knn_scan_kernel<T, 4><<<g, blk, 0, s>>>(p, b.cand, b.cand_cnt, (int)b.K1); break;
      case 512: knn_scan_kernel<T, 8><<<g, blk, 0, s>>>(p, b.cand, b.cand_cnt, (int)b.K1); break;
      case 1024: knn_scan_kernel<T, 16><<<g, blk, 0, s>>>(p, b.cand, b.cand_cnt, (int)b.K1); break;
      default: knn_scan_kernel<T, 32><<<g, blk, 0, s>>>(p, b.cand, b.cand_cnt, (int)b.K1); break;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_tiles_prec(int prec, const TileProblem& p, const KnnBuffers& b,
                                    bool collect, hipStream_t s) {
  switch (prec) {
    case PREC_FP32: return launch_tiles<float>(p, b, collect, s);
    case PREC_BF16: return launch_tiles<__bf16>(p, b, collect, s);
    default: return launch_tiles<_Float16>(p, b, collect, s);
  }
}

// Tile stride of the 16-bit candidate pass: the requested one, unless that
// leaves fewer than 16 seed tiles.
static int64_t seed_stride(int64_t ntiles, int64_t want) {
  if (want < 1) return 1;
  const int64_t most = ntiles / 16;
  return want < most ? want : (most > 1 ? most : 1);
}

// The second refinement in two launches: first with LDS for lists of at most
// REFINE2_SORT entries of which at most REFINE2_EXACT are evaluated exactly
// (five or six workgroups per CU), then with the full capacity for the queries
// left (longer lists, and the ones for the exhaustive scan).
constexpr int REFINE2_SORT = 2048, REFINE2_EXACT = 1024;

hipError_t launch_refine2(RefineArgs a, const KnnBuffers& b, int32_t* nn_out, int64_t d,
                          hipStream_t s) {
  int kcap = 2;
  while (kcap < (int)b.K1) kcap <<= 1;
  if (kcap > K_MAX) kcap = K_MAX;
  const dim3 g((unsigned)a.q), blk(WG);
  RefineArgs sa = a;
  sa.sort_cap = REFINE2_SORT;
  sa.ex_cap = REFINE2_EXACT;
  sa.kd_cap = kcap;
  sa.small = 1;
  const size_t sm_small = (size_t)REFINE2_SORT * 8 + (size_t)REFINE2_EXACT * 4 +
                          (size_t)kcap * (8 + 4) + WG * 8 + d * 4;
  knn_refine2_kernel<<<g, blk, sm_small, s>>>(sa, b, nn_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  RefineArgs la = a;
  la.sort_cap = SORT_CAP;
  la.ex_cap = SORT_CAP;
  la.kd_cap = K_MAX;
  la.small = 0;
  const size_t sm = (size_t)SORT_CAP * (8 + 4) + (size_t)K_MAX * (8 + 4) + WG * 8 + d * 4;
  knn_refine2_kernel<<<g, blk, sm, s>>>(la, b, nn_out);
  return hipGetLastError();
}

hipError_t launch_knn(int prec, const TileProblem& p, const TileProblem& pc, const KnnBuffers& b,
                      const float* X, const float* Y, int64_t d, int64_t k, double h, int kern,
                      int32_t* nn_out, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(b.flags), p.qtiles, 0u, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(reinterpret_cast<uint32_t*>(b.status), p.q, 0u, s);
  if (e != hipSuccess) return e;
  const bool approx = prec != PREC_FP32;
  KnnBuffers bb = b;
  RefineArgs a{X, Y, p.n, p.q, d, k, p.qp, p.splits, h, kern, 0};
  if (approx) {
    // 16-bit scans: cheap cell candidates from every ts-th data tile (at least
    // 16 of them), then the certified second pass over all tiles
    TileProblem ps = pc;
    ps.tstride = seed_stride(pc.ntiles, b.seed_stride);
    ps.ntiles = (pc.ntiles + ps.tstride - 1) / ps.tstride;
    // at most as many splits as keep a query's cells (CELLS per split) within
    // the refinement's in-register selection (4096 cells): small query batches
    // would otherwise get thousands of splits and a slow merge of their cells
    constexpr int64_t kMaxSeedSplits = (WG / 64) * 64 * 16 / CELLS;
    ps.splits = pc.splits < ps.ntiles ? pc.splits : ps.ntiles;
    if (ps.splits > kMaxSeedSplits) ps.splits = kMaxSeedSplits;
    ps.map = make_tile_map(ps.qtiles, ps.splits, pc.map.group);
    const dim3 g((unsigned)ps.map.grid), blk(WG);
    const int eng = tile_engine<__bf16>(ps.ld_bytes);
    if (prec == PREC_BF16) {
      if (eng == 2) knn_cand_kernel<__bf16, 2><<<g, blk, 0, s>>>(ps, b.cand, b.cand_cnt);
      else if (eng == 1) knn_cand_kernel<__bf16, 1><<<g, blk, 0, s>>>(ps, b.cand, b.cand_cnt);
      else knn_cand_kernel<__bf16, 0><<<g, blk, 0, s>>>(ps, b.cand, b.cand_cnt);
    } else {
      if (eng == 2) knn_cand_kernel<_Float16, 2><<<g, blk, 0, s>>>(ps, b.cand, b.cand_cnt);
      else if (eng == 1) knn_cand_kernel<_Float16, 1><<<g, blk, 0, s>>>(ps, b.cand, b.cand_cnt);
      else knn_cand_kernel<_Float16, 0><<<g, blk, 0, s>>>(ps, b.cand, b.cand_cnt);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bb.cap1 = CELLS;
    a.splits = ps.splits;
    a.approx = 1;
  } else {
    e = launch_tiles_prec(prec, p, b, false, s);
    if (e != hipSuccess) return e;
  }
  // the cell selection in registers needs 4 K1 merge entries (rounded up to a
  // power of two) and K1 exact ones: several workgroups per CU; list merges
  // take the full buffers
  RefineArgs ra = a;
  if (a.approx && a.splits * (int64_t)CELLS <= (WG / 64) * 64 * 16 && bb.K1 <= 512) {
    int kcap = 2;
    while (kcap < (int)bb.K1) kcap <<= 1;
    ra.sort_cap = (WG / 64) * kcap;
    ra.kd_cap = kcap;
  } else {
    ra.sort_cap = SORT_CAP;
    ra.kd_cap = K_MAX;
  }
  const size_t sm1 = (size_t)ra.sort_cap * 8 + (size_t)ra.kd_cap * (8 + 4 + 4) + WG * 8 + d * 4;
  knn_refine_kernel<<<dim3((unsigned)p.q), dim3(WG), sm1, s>>>(ra, bb, nn_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = launch_tiles_prec(prec, pc, b, true, s);
  if (e != hipSuccess) return e;
  if ((e = launch_refine2(a, bb, nn_out, d, s)) != hipSuccess) return e;
  // the exhaustive scan keeps k + 32 pairs plus a chunk of appends
  RefineArgs ea = a;
  int kcap = 2;
  while (kcap < (int)k) kcap <<= 1;
  int cap = 2;
  while (cap < (int)k + 32 + EXH_CHUNK) cap <<= 1;
  ea.sort_cap = cap < SORT_CAP ? cap : SORT_CAP;
  ea.kd_cap = kcap;
  const size_t sm2 = (size_t)ea.sort_cap * (8 + 4) + (size_t)kcap * 4 + WG * 8 + d * 4;
  knn_exhaustive_kernel<<<dim3((unsigned)p.q), dim3(WG), sm2, s>>>(ea, bb, nn_out);
  return hipGetLastError();
}

}  // namespace deann

namespace deann {

// ---------------------------------------------------------------------------
// Inverted-file neighbours (Sec. 5): the k nearest rows among the clusters a
// query inspects.  Pair row r of a batch is one (cluster, query) pair; the pair
// rows of cluster l form the range [pp[l], pp[l+1]) (a multiple of the tile),
// so one query tile of one cluster sweeps that cluster's rows [poff[l],
// poff[l+1]) of the index, in one or more parts (one workgroup each), keeping
// per pair and part the K1 smallest lower-bound keys exactly as the FP32 scan
// keeps them per (split, query).  The refinement then merges the lists of the
// query's pairs and parts; keys are exact lower bounds and the merged K1
// smallest are those of the whole sweep, so the certificate of the FP32 scan
// carries over unchanged.
// ---------------------------------------------------------------------------
// Pair tile and data-tile range of part w of the sweeps (see
// pair_parts_kernel: part p of P sweeps tiles [t0 + p*tiles/P, t0 +
// (p+1)*tiles/P) of the cluster); false past the last part.
struct IvfPart {
  int64_t row0, t0, t1;
};
__device__ __forceinline__ bool ivf_part(const IvfTiles& v, int64_t w, IvfPart& o) {
  if (w >= v.nparts[0]) return false;
  int64_t lo = 0, hi = v.pp[v.L] / BQ;   // lbase[lo] <= w < lbase[lo + 1]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (v.lbase[mid] <= w) lo = mid; else hi = mid;
  }
  o.row0 = lo * BQ;
  int64_t a = 0, z = v.L;   // the cluster: pp[a] <= row0 < pp[a + 1]
  while (z - a > 1) {
    const int64_t mid = (a + z) >> 1;
    if (v.pp[mid] <= o.row0) a = mid; else z = mid;
  }
  const int64_t c0 = v.poff[a] / BN, tiles = v.poff[a + 1] / BN - c0;
  const int64_t P = v.lbase[lo + 1] - v.lbase[lo], p = w - v.lbase[lo];
  o.t0 = c0 + tiles * p / P;
  o.t1 = c0 + tiles * (p + 1) / P;
  return true;
}

template <int EPL>   // list capacity = 64 * EPL
__global__ void __launch_bounds__(WG, 2)
ivf_scan_kernel(IvfTiles v, uint64_t* __restrict__ cand, int32_t* __restrict__ cand_cnt, int K1) {
  constexpr int cap1 = 64 * EPL;
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  __shared__ float thr[BQ];
  __shared__ float yks[BQ];
  __shared__ int cnt[BQ];
  IvfPart pt;
  if (!ivf_part(v, blockIdx.x, pt)) return;
  const int64_t row0 = pt.row0, t0 = pt.t0, t1 = pt.t1;
  const int64_t lrow0 = (int64_t)blockIdx.x * BQ;   // list rows of this part
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  // The query's own bound: thr is the K1-th key of this list or a value of
  // qthr[query], the smallest K1-th key any list of the query has published.
  // Either has K1 keys at or below it among the query's lists, so a key at or
  // above it is not among the K1 smallest of the query's inspected rows.
  const int32_t qi = threadIdx.x < BQ ? v.pair_q[row0 + threadIdx.x] : -1;
  auto share_bound = [&]() {
    if (qi >= 0) {
      const float th = thr[threadIdx.x];
      const uint32_t was = atomicMin(&v.qthr[qi], float_key(th));
      thr[threadIdx.x] = fminf(th, key_float(was));
    }
  };
  if (threadIdx.x < BQ) {
    thr[threadIdx.x] = qi >= 0 ? key_float(v.qthr[qi]) : __builtin_inff();
    cnt[threadIdx.x] = 0;
    yks[threadIdx.x] = v.yknorm[row0 + threadIdx.x];
  }
  uint64_t* lists = cand + lrow0 * (int64_t)cap1;
  const char* yq = v.Ys + row0 * v.ld_bytes;
  const int limit = cap1 - BN;
  __syncthreads();
  StreamState st;
  if (t0 < t1) stream_start(st, yq, v.Xs, v.ld_bytes, t0);
  __shared__ float xks[2][BN];
  float xk_reg = (threadIdx.x < BN && t0 < t1) ? v.xknorm[t0 * BN + threadIdx.x] : 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    const int nb = (int)((t - t0) & 1);
    if (threadIdx.x < BN) {
      xks[nb][threadIdx.x] = xk_reg;
      if (t + 1 < t1) xk_reg = v.xknorm[(t + 1) * BN + threadIdx.x];
    }
    f32x4 acc[4][4];
    stream_tile<float>(acc, st, yq, v.Xs, v.ld_bytes, v.nchunks, t, t1, lds, wq, wn, lane);
    float xk[4];   // empty rows carry an infinite key norm
#pragma unroll
    for (int j = 0; j < 4; ++j) xk[j] = xks[nb][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ql = wq * 64 + i * 16 + 4 * (lane >> 4) + r;
        const float yk = yks[ql], th = thr[ql];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float key = __builtin_fmaf(-2.f, acc[i][j][r], yk + xk[j]);
          if (key < th) {
            const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
            const int slot = atomicAdd(&cnt[ql], 1);
            lists[(int64_t)ql * cap1 + slot] =
                ((uint64_t)float_key(key) << 32) | (uint64_t)(uint32_t)col;
          }
        }
      }
    __syncthreads();
    compact_lists<EPL>(lists, cnt, thr, limit, K1, wave, lane);
    share_bound();
    __syncthreads();
  }
  compact_lists<EPL>(lists, cnt, thr, K1, K1, wave, lane);
  share_bound();
  if (threadIdx.x < BQ) cand_cnt[lrow0 + threadIdx.x] = cnt[threadIdx.x];
}

// Rows the query's clusters hold (clusters probed by one query are distinct).
__device__ __forceinline__ int64_t ivf_rows(const IvfRefine& v, int64_t qi) {
  int64_t tot = 0;
  for (int64_t p = 0; p < v.np_q[qi]; ++p) {
    const int32_t l = v.probe[qi * v.kp + p];
    tot += v.off[l + 1] - v.off[l];
  }
  return tot;
}

// status: 0 certified, 1 second pass over the inspected clusters (collect
// every row whose key admits a distance <= d_k), 2 exact scan of the
// inspected clusters (second-pass overflow), 3 exact scan of all rows (the
// inspected clusters hold fewer than k rows).
__global__ void __launch_bounds__(WG)
ivf_refine_kernel(RefineArgs a, KnnBuffers b, IvfRefine v, int32_t* __restrict__ nn_out) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  uint64_t* buf = reinterpret_cast<uint64_t*>(smem);                  // SORT_CAP
  uint64_t* dkey = buf + SORT_CAP;                                     // K_MAX
  uint32_t* didx = reinterpret_cast<uint32_t*>(dkey + K_MAX);         // K_MAX
  uint32_t* tmp = didx + K_MAX;                                        // K_MAX
  double* red = reinterpret_cast<double*>(tmp + K_MAX);               // WG
  float* ys = reinterpret_cast<float*>(red + WG);                      // d
  __shared__ int fill_s;
  const int64_t qi = blockIdx.x;
  const int K1 = (int)b.K1;
  const int k = (int)a.k;
  const int64_t rows = ivf_rows(v, qi);
  if (rows < k) {
    if (threadIdx.x == 0) b.status[qi] = 3;
    return;
  }
  for (int64_t t = threadIdx.x; t < a.d; t += WG) ys[t] = a.Y[qi * a.d + t];
  if (threadIdx.x == 0) fill_s = 0;
  __syncthreads();
  int64_t seen = 0;
  const int64_t np = v.np_q[qi];
  // the query's lists hold at least K1 keys at or below its final shared
  // bound, so the K1 smallest are among the entries at or below it
  const uint64_t cut = ((uint64_t)v.qthr[qi] << 32) | 0xffffffffull;
  for (int64_t p = 0; p < np; ++p) {
    const int32_t row = v.pair_of[qi * v.kp + p];
    const int64_t tile = row / BQ, ql = row % BQ;
    const int32_t j1 = v.lbase[tile + 1];
    for (int32_t j = v.lbase[tile]; j < j1; ++j) {   // the parts of the pair's sweep
      const int64_t lrow = (int64_t)j * BQ + ql;
      const uint64_t* lst = b.cand + lrow * b.cap1;
      const uint64_t e0 = lst[threadIdx.x];   // issued with the count (WG <= cap1 slots)
      const int c = b.cand_cnt[lrow];
      seen += c;
      __syncthreads();
      for (int i = threadIdx.x; i < c; i += WG) {
        const uint64_t e = i < WG ? e0 : lst[i];
        if (e <= cut) buf[atomicAdd(&fill_s, 1)] = e;
      }
      __syncthreads();
      const bool flush = (fill_s + K1 > SORT_CAP) || (p + 1 == np && j + 1 == j1);
      if (flush && fill_s >= K1) {
        const int F = fill_s;
        const int N = next_pow2(F);
        for (int i = F + threadIdx.x; i < N; i += WG) buf[i] = ~0ull;
        __syncthreads();
        block_sort_u64(buf, N);
        if (threadIdx.x == 0) fill_s = K1;
        __syncthreads();
      }
    }
  }
  const int C = fill_s;
  const bool complete = (seen == rows) && (C == rows);
  const float Tkey = (C == K1) ? key_float((uint32_t)(buf[K1 - 1] >> 32)) : __builtin_inff();
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  for (int c0 = g; c0 < C; c0 += 4 * (WG / 16)) {   // four rows per group at a time
    int64_t rr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = c0 + i * (WG / 16);
      // a real row (empty rows have infinite keys and are never listed)
      const int32_t pid = c < C ? v.pids[(uint32_t)(buf[c] & 0xffffffffu)] : -1;
      rr[i] = c < C ? (int64_t)(pid >= 0 ? pid : 0) : -1;
    }
    double d2[4];
    group16_d2_4(a.X, rr, a.d, ys, l16, d2);
    if (l16 == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = c0 + i * (WG / 16);
        if (c < C) { dkey[c] = __builtin_bit_cast(uint64_t, d2[i]); didx[c] = (uint32_t)rr[i]; }
      }
  }
  const int N = next_pow2(C > 1 ? C : 2);
  for (int i = C + threadIdx.x; i < N; i += WG) { dkey[i] = ~0ull; didx[i] = 0xffffffffu; }
  __syncthreads();
  block_sort_pairs(dkey, didx, N);
  fix_boundary(dkey, didx, C, k, a.X, a.d, ys);
  bool ok = complete;
  if (!ok && C >= k) {
    const double Dk = __builtin_bit_cast(double, dkey[k - 1]) * (1.0 + fp64_rel(a.d));
    const double E = (double)__builtin_bit_cast(float, *b.xerr_max);
    const double ey = (double)b.yerr[qi];
    const double lhs = sqrt((double)fmaxf(Tkey, 0.f)) - E - ey;
    ok = lhs > 0.0 && lhs * lhs > Dk * (1.0 + 1e-14);
  }
  if (!ok) {   // C = K1 >= k here: d_k is bounded, the second pass collects
    if (threadIdx.x == 0) {
      const double Dk = __builtin_bit_cast(double, dkey[k - 1]) * (1.0 + fp64_rel(a.d));
      const double E = (double)__builtin_bit_cast(float, *b.xerr_max);
      const double ey = (double)b.yerr[qi];
      const double r = (sqrt(Dk) + E + ey) * (1.0 + 1e-6);
      b.thr2[qi] = (float)(r * r * (1.0 + 1e-6));
      b.cand2_cnt[qi] = 0;
      b.status[qi] = 1;
    }
    return;
  }
  if (threadIdx.x == 0) b.status[qi] = 0;
  emit_neighbours(dkey, didx, tmp, k, a.h, a.kern, b.nn_work + qi * k,
                  nn_out ? nn_out + qi * k : nullptr, b.z1 + qi, red);
}

// Second pass over the pair tiles: every row of an inspected cluster whose key
// is <= the threshold of the pair's query (status 1) is appended to that
// query's candidates, as its row index.
__global__ void __launch_bounds__(WG, 2)
ivf_collect_kernel(IvfTiles v, KnnBuffers b) {
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  __shared__ float yks[BQ], ths[BQ];
  __shared__ int qry[BQ];
  IvfPart pt;
  if (!ivf_part(v, blockIdx.x, pt)) return;
  const int64_t row0 = pt.row0, t0 = pt.t0, t1 = pt.t1;
  int need = 0;
  if (threadIdx.x < BQ) {
    const int32_t qi = v.pair_q[row0 + threadIdx.x];
    const bool on = qi >= 0 && b.status[qi] == 1;
    qry[threadIdx.x] = qi;
    yks[threadIdx.x] = v.yknorm[row0 + threadIdx.x];
    ths[threadIdx.x] = on ? b.thr2[qi] : -__builtin_inff();
    need = on;
  }
  if (!__syncthreads_or(need)) return;   // no query of this tile needs the pass
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  const char* yq = v.Ys + row0 * v.ld_bytes;
  StreamState st;
  if (t0 < t1) stream_start(st, yq, v.Xs, v.ld_bytes, t0);
  __shared__ float xks[2][BN];
  float xk_reg = (threadIdx.x < BN && t0 < t1) ? v.xknorm[t0 * BN + threadIdx.x] : 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    const int nb = (int)((t - t0) & 1);
    if (threadIdx.x < BN) {
      xks[nb][threadIdx.x] = xk_reg;
      if (t + 1 < t1) xk_reg = v.xknorm[(t + 1) * BN + threadIdx.x];
    }
    f32x4 acc[4][4];
    stream_tile<float>(acc, st, yq, v.Xs, v.ld_bytes, v.nchunks, t, t1, lds, wq, wn, lane);
    float xk[4];   // empty rows carry an infinite key norm
#pragma unroll
    for (int j = 0; j < 4; ++j) xk[j] = xks[nb][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ql = wq * 64 + i * 16 + 4 * (lane >> 4) + r;
        const float yk = yks[ql], th = ths[ql];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float key = __builtin_fmaf(-2.f, acc[i][j][r], yk + xk[j]);
          if (key <= th) {   // th = -inf for rows without a second pass
            const int32_t id = v.pids[t * BN + wn * 64 + j * 16 + (lane & 15)];
            if (id >= 0) {
              const int32_t qi = qry[ql];
              const int slot = atomicAdd(&b.cand2_cnt[qi], 1);
              if (slot < b.cap2)
                b.cand2[(int64_t)qi * b.cap2 + slot] = ((uint64_t)float_key(key) << 32) | (uint64_t)(uint32_t)id;
            }
          }
        }
      }
  }
}

// Exact FP64 scan for status 2 (rows of the inspected clusters) and status 3
// (all rows), one workgroup per query, as knn_exhaustive_kernel.
__global__ void __launch_bounds__(WG)
ivf_exhaustive_kernel(RefineArgs a, KnnBuffers b, IvfRefine v, int32_t* __restrict__ nn_out) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  uint64_t* dkey = reinterpret_cast<uint64_t*>(smem);
  uint32_t* didx = reinterpret_cast<uint32_t*>(dkey + SORT_CAP);
  uint32_t* tmp = didx + SORT_CAP;
  double* red = reinterpret_cast<double*>(tmp + K_MAX);
  float* ys = reinterpret_cast<float*>(red + WG);
  int64_t* cum = reinterpret_cast<int64_t*>(ys + ((a.d + 3) & ~3ll));   // [kp + 1]
  __shared__ int fill_s;
  const int64_t qi = blockIdx.x;
  const int st = b.status[qi];
  if (st != 2 && st != 3) return;
  const int k = (int)a.k;
  for (int64_t t = threadIdx.x; t < a.d; t += WG) ys[t] = a.Y[qi * a.d + t];
  const int64_t np = v.np_q[qi];
  if (threadIdx.x == 0) {
    fill_s = 0;
    int64_t c = 0;
    for (int64_t p = 0; p < np; ++p) {
      cum[p] = c;
      const int32_t l = v.probe[qi * v.kp + p];
      c += v.off[l + 1] - v.off[l];
    }
    cum[np] = c;
  }
  __syncthreads();
  const int64_t R = st == 3 ? a.n : cum[np];
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  ExhaustiveTop top(k, SORT_CAP);
  for (int64_t r0 = 0; r0 < R; r0 += EXH_CHUNK) {
    const int64_t r1 = r0 + EXH_CHUNK < R ? r0 + EXH_CHUNK : R;
    // four rows per 16-lane group at a time (their loads in flight together)
    for (int64_t rb = r0 + g; rb < r1; rb += 4 * (WG / 16)) {
      int64_t rr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = rb + i * (WG / 16);
        int64_t id = r < r1 ? r : -1;
        if (st == 2 && r < r1) {   // r-th row of the inspected clusters
          int64_t lo = 0, hi = np;   // cum[lo] <= r < cum[hi]
          while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (cum[mid] <= r) lo = mid; else hi = mid;
          }
          const int32_t l = v.probe[qi * v.kp + lo];
          id = v.ids[v.off[l] + (r - cum[lo])];
        }
        rr[i] = id;
      }
      double d2[4];
      group16_d2_4(a.X, rr, a.d, ys, l16, d2);
      if (l16 == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rr[i] >= 0)
            top.offer(__builtin_bit_cast(uint64_t, d2[i]), (uint32_t)rr[i], dkey, didx, &fill_s);
    }
    top.settle(dkey, didx, &fill_s, r1 == R);
  }
  fix_boundary(dkey, didx, fill_s, k, a.X, a.d, ys);
  if (threadIdx.x == 0) b.status[qi] = 5;   // done by the exhaustive scan
  emit_neighbours(dkey, didx, tmp, k, a.h, a.kern, b.nn_work + qi * k,
                  nn_out ? nn_out + qi * k : nullptr, b.z1 + qi, red);
}

// Inspected clusters of each query: its kp closest clusters (an exact k-NN
// among the centroids, cand[q][kp] ascending by id) put in the exact order
// (||c - y||^2, l): FP64 distances, then every run of values too close for
// FP64 to decide re-ordered in double-double (runs of at most 32; longer runs
// keep the FP64 order, which is exact for identical centroids).  The query
// inspects the shortest prefix of at least n_probe clusters holding k rows,
// or none (np_q = 0: exact scan of all rows) if all kp hold fewer.
constexpr int PROBE_MAX = 512;
__global__ void __launch_bounds__(WG)
probe_order_kernel(const float* __restrict__ C, const float* __restrict__ Y, int64_t d,
                   const int32_t* __restrict__ cand, int kp, const int32_t* __restrict__ off,
                   int n_probe, int64_t k, int32_t* __restrict__ order, int32_t* __restrict__ np_q) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  uint64_t* dkey = reinterpret_cast<uint64_t*>(smem);                 // PROBE_MAX
  uint32_t* didx = reinterpret_cast<uint32_t*>(dkey + PROBE_MAX);     // PROBE_MAX
  float* ys = reinterpret_cast<float*>(didx + PROBE_MAX);             // d
  const int64_t qi = blockIdx.x;
  for (int64_t t = threadIdx.x; t < d; t += WG) ys[t] = Y[qi * d + t];
  __syncthreads();
  const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  for (int i = g; i < kp; i += WG / 16) {
    const int32_t l = cand[qi * kp + i];
    const double d2 = group16_d2(C, l, d, ys, l16);
    if (l16 == 0) { dkey[i] = __builtin_bit_cast(uint64_t, d2); didx[i] = (uint32_t)l; }
  }
  const int N = next_pow2(kp > 1 ? kp : 2);
  for (int i = kp + threadIdx.x; i < N; i += WG) { dkey[i] = ~0ull; didx[i] = 0xffffffffu; }
  __syncthreads();
  block_sort_pairs(dkey, didx, N);
  if (threadIdx.x == 0) {
    const double rel = fp64_rel(d);
    for (int i = 0; i < kp;) {
      int j = i;
      while (j + 1 < kp && __builtin_bit_cast(double, dkey[j + 1]) <=
                               __builtin_bit_cast(double, dkey[j]) * (1.0 + 2.0 * rel) + 1e-300)
        ++j;
      if (j > i && j - i < 32) resolve_band(dkey, didx, i, j, C, d, ys);
      i = j + 1;
    }
    int64_t rows = 0;
    int p = 0;
    while (p < kp && (p < n_probe || rows < k)) {
      rows += off[didx[p] + 1] - off[didx[p]];
      ++p;
    }
    np_q[qi] = rows >= k ? p : 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kp; i += WG) order[qi * kp + i] = (int32_t)didx[i];
}

hipError_t launch_probe_order(const float* C, const float* Y, int64_t q, int64_t d,
                              const int32_t* cand, int64_t kp, const int32_t* off, int64_t n_probe,
                              int64_t k, int32_t* order, int32_t* np_q, hipStream_t s) {
  if (kp > PROBE_MAX) return hipErrorInvalidValue;
  const size_t sm = PROBE_MAX * (8 + 4) + d * 4;
  probe_order_kernel<<<dim3((unsigned)q), dim3(WG), sm, s>>>(C, Y, d, cand, (int)kp, off,
                                                             (int)n_probe, k, order, np_q);
  return hipGetLastError();
}

hipError_t launch_ivf_knn(const IvfTiles& t, int64_t prow_cap, const KnnBuffers& b,
                          const IvfRefine& v, const float* X, const float* Y, int64_t n,
                          int64_t q, int64_t d, int64_t k, double h, int kern, int32_t* nn_out,
                          hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(b.status), q, 0u, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(t.qthr, q, 0xff800000u, s)) != hipSuccess) return e;   // +inf key
  const dim3 g((unsigned)(prow_cap / BQ)), blk(WG);
  switch (b.cap1) {
    case 256: ivf_scan_kernel<4><<<g, blk, 0, s>>>(t, b.cand, b.cand_cnt, (int)b.K1); break;
    case 512: ivf_scan_kernel<8><<<g, blk, 0, s>>>(t, b.cand, b.cand_cnt, (int)b.K1); break;
    case 1024: ivf_scan_kernel<16><<<g, blk, 0, s>>>(t, b.cand, b.cand_cnt, (int)b.K1); break;
    default: ivf_scan_kernel<32><<<g, blk, 0, s>>>(t, b.cand, b.cand_cnt, (int)b.K1); break;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  RefineArgs a{X, Y, n, q, d, k, 0, 0, h, kern, 0};
  const size_t sm1 = SORT_CAP * 8 + K_MAX * (8 + 4 + 4) + WG * 8 + d * 4;
  ivf_refine_kernel<<<dim3((unsigned)q), dim3(WG), sm1, s>>>(a, b, v, nn_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  ivf_collect_kernel<<<g, blk, 0, s>>>(t, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_refine2(a, b, nn_out, d, s)) != hipSuccess) return e;
  const size_t sm2 = SORT_CAP * (8 + 4) + K_MAX * 4 + WG * 8 + ((d + 3) & ~3ll) * 4 +
                     (v.kp + 1) * 8;
  ivf_exhaustive_kernel<<<dim3((unsigned)q), dim3(WG), sm2, s>>>(a, b, v, nn_out);
  return hipGetLastError();
}

}  // namespace deann
