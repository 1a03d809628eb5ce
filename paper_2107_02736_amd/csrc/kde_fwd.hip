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
//
// The float32-operand sweeps also keep, per query and split, the sum of the
// squared kernel values (and for the exponential kernel their maximum) for the
// per-query error certificate of cert.hip.
#include "common.h"
#include "kernels.h"

namespace deann {

template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};

// Neighbour pairs staged in LDS per workgroup (near/far form); a workgroup
// whose tiles hold more reads them from global memory.
constexpr int HYB_LDS = 1024;

// HYB: near/far form.  hoff[(qt * ntiles + t) .. + 1] delimit the entries
// (query mod 128) << 7 | (row mod 128) in hits of the neighbour pairs of query
// tile qt in data tile t; those elements are left out of the sums.
// Split-operand engine (ENG 3) for rows wider than 128 floats with float32-
// accurate dot products from bfloat16 MFMAs (DEANN_FP32_SPLIT): every prepared
// value is held as three bfloat16 parts v = h + m + l (row = planes h, m, l of
// dps elements, see split_rows_kernel).  A 32-element k-chunk of a row is its
// 64-byte slice of each plane; both tiles' chunks go global -> registers ->
// LDS (double-buffered, one barrier per chunk, the next chunk in flight behind
// the MFMAs).  Per chunk each wave forms, for its 64 x 64 quarter, the six
// products h h, h m, m h, h l, m m, l h on v_mfma_f32_16x16x32_bf16 (products
// exact in FP32); the three dropped products are below 2^-23 |x||y| together.
// The leading products h h and the five small ones accumulate apart for the
// whole tile and are added at its end: every MFMA rounds into its accumulator,
// and rounding the small terms into the large running sum (one accumulator)
// measured errors up to 1.5e-5 at d = 960 against a few 1e-7 for the float32
// MFMAs.  One workgroup of 4 waves per CU (the staging of both
// tiles' three planes takes two 53 KB buffers), so each wave may hold up to
// 512 registers.
constexpr int SPL_KB = 64;                                    // one plane's slice of a chunk
constexpr int SPL_ROWB = 3 * SPL_KB;                          // a row's chunk, three planes
constexpr int SPL_PITCH = SPL_ROWB + 16;                      // LDS row pitch (bytes)
constexpr int SPL_BUF = (BQ + BN) * SPL_PITCH;                // one staged chunk, both tiles
constexpr int SPL_NPT = (BQ + BN) * (SPL_ROWB / 16) / WG;     // 16-byte pieces per thread
static_assert(SPL_NPT * WG == (BQ + BN) * (SPL_ROWB / 16), "chunk pieces must split evenly");

struct SplitStream {
  u32x4 r[SPL_NPT];
  int buf;
};

// Chunk c of the query tile at yq and the data tile at xt: piece v is 16 bytes
// (v % 4) of plane (v % 12) / 4 of row v / 12 (query rows first).  rowb: bytes
// of a split row (3 planes), planeb: of one plane.
__device__ __forceinline__ void split_load(SplitStream& st, const char* __restrict__ yq,
                                           const char* __restrict__ xt, int64_t rowb,
                                           int64_t planeb, int c) {
#pragma unroll
  for (int i = 0; i < SPL_NPT; ++i) {
    const int v = threadIdx.x + i * WG;
    const int row = v / 12, w = v % 12;
    const char* base = row < BQ ? yq + (int64_t)row * rowb : xt + (int64_t)(row - BQ) * rowb;
    st.r[i] = *reinterpret_cast<const u32x4*>(base + (w >> 2) * planeb + c * SPL_KB + (w & 3) * 16);
  }
}

__device__ __forceinline__ void split_store(const SplitStream& st, char* buf) {
#pragma unroll
  for (int i = 0; i < SPL_NPT; ++i) {
    const int v = threadIdx.x + i * WG;
    *reinterpret_cast<u32x4*>(buf + (v / 12) * SPL_PITCH + (v % 12) * 16) = st.r[i];
  }
}

__device__ __forceinline__ void split_start(SplitStream& st, const char* __restrict__ yq,
                                            const char* __restrict__ Xs, int64_t rowb,
                                            int64_t t0) {
  split_load(st, yq, Xs + t0 * BN * rowb, rowb, rowb / 3, 0);
  st.buf = 0;
  __syncthreads();   // previous users of the staging area are done
}

__device__ __forceinline__ void split_tile(f32x4 (&acc)[4][4], SplitStream& st,
                                           const char* __restrict__ yq,
                                           const char* __restrict__ Xs, int64_t rowb,
                                           int nchunks, int64_t t, int64_t t1, char* lds, int wq,
                                           int wn, int lane) {
  const int64_t planeb = rowb / 3;
  f32x4 accx[4][4];   // the five small products
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      accx[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  for (int c = 0; c < nchunks; ++c) {
    char* b = lds + st.buf * SPL_BUF;
    split_store(st, b);
    __syncthreads();   // chunk c staged; the buffer written next was read two chunks ago
    int nc = c + 1;
    int64_t nt = t;
    if (nc == nchunks) { nc = 0; nt = t + 1; }
    if (nt < t1) split_load(st, yq, Xs + nt * BN * rowb, rowb, planeb, nc);
    __builtin_amdgcn_s_setprio(1);   // favour the wave issuing MFMAs
    u32x4 bh[4], bm[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const char* pr = b + (BQ + wn * 64 + j * 16 + (lane & 15)) * SPL_PITCH + (lane >> 4) * 16;
      bh[j] = *reinterpret_cast<const u32x4*>(pr);
      bm[j] = *reinterpret_cast<const u32x4*>(pr + SPL_KB);
      bl[j] = *reinterpret_cast<const u32x4*>(pr + 2 * SPL_KB);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const char* pr = b + (wq * 64 + i * 16 + (lane & 15)) * SPL_PITCH + (lane >> 4) * 16;
      const u32x4 ah = *reinterpret_cast<const u32x4*>(pr);
      const u32x4 am = *reinterpret_cast<const u32x4*>(pr + SPL_KB);
      const u32x4 al = *reinterpret_cast<const u32x4*>(pr + 2 * SPL_KB);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        f32x4 v = accx[i][j];
        v = mfma_kgroup<__bf16>(al, bh[j], v);
        v = mfma_kgroup<__bf16>(am, bm[j], v);
        v = mfma_kgroup<__bf16>(ah, bl[j], v);
        v = mfma_kgroup<__bf16>(am, bh[j], v);
        accx[i][j] = mfma_kgroup<__bf16>(ah, bm[j], v);
        acc[i][j] = mfma_kgroup<__bf16>(ah, bh[j], acc[i][j]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    st.buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] += accx[i][j];
}

template <typename T, int KERN, int ENG, bool HYB>   // ENG: see tile_engine; 3: split (above)
__global__ void __launch_bounds__(WG, ENG == 3 ? 1 : 2)
kde_tile_kernel(const char* __restrict__ Ys, const char* __restrict__ Xs, int64_t ld_bytes,
                int nchunks, const double* __restrict__ ynorm, const double* __restrict__ xnorm,
                int64_t n, int64_t qtiles, int64_t splits, int64_t ntiles, float Lf,
                double* __restrict__ partial, int64_t qp, TileMap map,
                const int32_t* __restrict__ hoff, const uint16_t* __restrict__ hits,
                float2* __restrict__ cert, float* __restrict__ certn,
                float* __restrict__ certk) {
  // float32 operands: certificate sums (see the file comment), and per pair
  // the squared product of K and the pair's norm term N = ||x~||^2 + ||y~||^2
  // (Gaussian: -L N, the exponent's norm part), so that the bound takes each
  // pair's rounding scale instead of the largest row norm's
  constexpr bool CERT = elem_of<T>::bytes == 4 && !HYB;
  static_assert(ENG != 3 || (CERT && elem_of<T>::bytes == 4), "split rows carry float32 values");
  __shared__ __attribute__((aligned(16))) char lds[ENG == 3 ? 2 * SPL_BUF : 4 * TILE_LDS];
  __shared__ uint16_t hl[HYB ? HYB_LDS : 1];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, map, qtiles, splits, qt, split)) return;
  const int64_t t0 = split * ntiles / splits, t1 = (split + 1) * ntiles / splits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  const float L2 = 2.f * Lf;

  // the neighbour pairs of this workgroup's tiles are contiguous in hits; the
  // barrier inside the first tile sweep publishes the LDS copy
  int32_t hbase = 0;
  bool hlds = true;
  if constexpr (HYB) {
    if (t0 < t1) {
      hbase = hoff[qt * ntiles + t0];
      const int32_t hcnt = hoff[qt * ntiles + t1] - hbase;
      hlds = hcnt <= HYB_LDS;
      if (hlds)
        for (int i = threadIdx.x; i < hcnt; i += WG) hl[i] = hits[hbase + i];
    }
  }

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
  // certificate (CERT only): sum of K^2; Gaussian: sum of K times its exponent,
  // exponential: largest K; sum of (K N)^2; split engine: sum of K N (the
  // bfloat16 MFMA's truncated group sums bias each dot product by up to u N / 2)
  constexpr bool KN = ENG == 3;
  float csq[4][4], cmx[4][4], cqn[4][4], ckn[KN ? 4 : 1][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sum[i][r] = 0.0;
      csq[i][r] = 0.f;
      cmx[i][r] = 0.f;
      cqn[i][r] = 0.f;
      if constexpr (KN) ckn[i][r] = 0.f;
    }

  const char* yq = Ys + qt * BQ * ld_bytes;
  constexpr int NK = 2;   // k-groups of the register-resident engine
  StreamState st;
  XStream<NK> xs;
  u32x4 yf[4][NK];
  QlState ql;
  SplitStream sst;
  if (t0 < t1) {
    if constexpr (ENG == 0) {
      stream_start(st, yq, Xs, ld_bytes, t0);
    } else if constexpr (ENG == 1) {
      ql_start(ql, yq, Xs, t0, lds);
    } else if constexpr (ENG == 2) {
      yreg_load<NK>(yf, yq, ld_bytes, wq, lane);
      xs_load(xs, Xs + t0 * BN * ld_bytes, ld_bytes);
      xs.buf = 0;
    } else {
      split_start(sst, yq, Xs, ld_bytes, t0);
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
    else if constexpr (ENG == 2)
      yreg_tile<T, NK>(acc, xs, yf, Xs, ld_bytes, t, t1, lds, wn, lane);
    else
      split_tile(acc, sst, yq, Xs, ld_bytes, nchunks, t, t1, lds, wq, wn, lane);
    // bit (4 i + j) * 4 + r of hm: element acc[i][j][r] of this lane is a
    // neighbour pair
    uint64_t hm = 0;
    if constexpr (HYB) {
      const int32_t ha = hoff[qt * ntiles + t] - hbase, hb = hoff[qt * ntiles + t + 1] - hbase;
      for (int32_t e = ha; e < hb; ++e) {
        const unsigned v = hlds ? hl[e] : hits[hbase + e];
        const int ql_ = (int)(v >> 7), cl = (int)(v & 127);
        const bool own = (ql_ >> 6) == wq && (cl >> 6) == wn &&
                         lane == ((((ql_ & 15) >> 2) << 4) | (cl & 15));
        if (own)
          hm |= 1ull << (((((ql_ & 63) >> 4) << 2) + ((cl & 63) >> 4)) * 4 + (ql_ & 3));
      }
    }
    // per-column data terms; padding columns get a term that zeroes the kernel
    float xt[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = t * BN + wn * 64 + j * 16 + (lane & 15);
      const double xn = xns[nb][wn * 64 + j * 16 + (lane & 15)];
      if (KERN == KERNEL_GAUSSIAN)
        xt[j] = col < n ? (float)(-(double)Lf * xn) : -1e30f;
      else
        xt[j] = col < n ? (float)xn : __builtin_inff();
    }
    if constexpr (HYB) {
      // one 16-row block i of the lane's rows (bits i*16 .. i*16+15 of hm);
      // the masked copy runs only for the blocks in which some lane of the
      // wave holds a neighbour pair
      auto block = [&](auto tag, const int i) {
        constexpr bool MASK = decltype(tag)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float part = 0.f;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float kv;
            if (KERN == KERNEL_GAUSSIAN) {
              const float a = fminf(__builtin_fmaf(L2, acc[i][j][r], yt[i][r] + xt[j]), 0.f);
              kv = __builtin_amdgcn_exp2f(a);
            } else {
              const float d2 = fmaxf(__builtin_fmaf(-2.f, acc[i][j][r], yt[i][r] + xt[j]), 0.f);
              kv = __builtin_amdgcn_exp2f(-Lf * __builtin_sqrtf(d2));
            }
            if constexpr (MASK)
              if ((hm >> ((i * 4 + j) * 4 + r)) & 1ull) kv = 0.f;
            part += kv;
          }
          sum[i][r] += (double)part;
        }
      };
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (__any(((hm >> (16 * i)) & 0xffffull) != 0ull))
          block(BoolTag<true>{}, i);
        else
          block(BoolTag<false>{}, i);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float part = 0.f;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float kv;
            float a = 0.f;
            const float nl = yt[i][r] + xt[j];
            if (KERN == KERNEL_GAUSSIAN) {   // exp(-d^2 / (2 h^2))
              a = fminf(__builtin_fmaf(L2, acc[i][j][r], nl), 0.f);
              kv = __builtin_amdgcn_exp2f(a);
            } else {                          // exp(-d / h)
              const float d2 = fmaxf(__builtin_fmaf(-2.f, acc[i][j][r], nl), 0.f);
              kv = __builtin_amdgcn_exp2f(-Lf * __builtin_sqrtf(d2));
            }
            part += kv;
            if constexpr (CERT) {
              csq[i][r] = __builtin_fmaf(kv, kv, csq[i][r]);
              if (KERN == KERNEL_GAUSSIAN) cmx[i][r] = __builtin_fmaf(-kv, a, cmx[i][r]);
              else cmx[i][r] = fmaxf(cmx[i][r], kv);
              // padding columns: K = 0 times a finite norm term
              const float w = kv * (KERN == KERNEL_GAUSSIAN ? nl : fminf(nl, 3.0e38f));
              cqn[i][r] = __builtin_fmaf(w, w, cqn[i][r]);
              if constexpr (KN) ckn[i][r] += fabsf(w);
            }
          }
          sum[i][r] += (double)part;
        }
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
  if constexpr (CERT) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float a = csq[i][r], m = cmx[i][r], w = cqn[i][r], kk = KN ? ckn[i][r] : 0.f;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          a += __shfl_xor(a, o, 64);
          w += __shfl_xor(w, o, 64);
          if constexpr (KN) kk += __shfl_xor(kk, o, 64);
          const float mo = __shfl_xor(m, o, 64);
          m = KERN == KERNEL_GAUSSIAN ? m + mo : fmaxf(m, mo);
        }
        csq[i][r] = a;
        cmx[i][r] = m;
        cqn[i][r] = w;
        if constexpr (KN) ckn[i][r] = kk;
      }
    __syncthreads();   // red is reused
    float2* cr = reinterpret_cast<float2*>(lds);   // [2][BQ]
    float* cw = reinterpret_cast<float*>(cr + 2 * BQ);   // [2][BQ]
    float* ck = cw + 2 * BQ;                              // [2][BQ]
    if ((lane & 15) == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = wn * BQ + wq * 64 + i * 16 + 4 * (lane >> 4) + r;
          cr[e] = make_float2(csq[i][r], cmx[i][r]);
          cw[e] = cqn[i][r];
          if constexpr (KN) ck[e] = ckn[i][r];
        }
    }
    __syncthreads();
    if (threadIdx.x < BQ) {
      const float2 a = cr[threadIdx.x], b = cr[BQ + threadIdx.x];
      cert[split * qp + qt * BQ + threadIdx.x] =
          make_float2(a.x + b.x, KERN == KERNEL_GAUSSIAN ? a.y + b.y : fmaxf(a.y, b.y));
      certn[split * qp + qt * BQ + threadIdx.x] = cw[threadIdx.x] + cw[BQ + threadIdx.x];
      if constexpr (KN) certk[split * qp + qt * BQ + threadIdx.x] = ck[threadIdx.x] + ck[BQ + threadIdx.x];
    }
  }
}

// FP32 operands, padded width DP <= 128: the queries stay in registers.  512
// threads (8 waves); wave w owns queries w*16..+16 of the query tile, and its
// FP32 rows are the B-operand fragments of every k-group for the whole sweep.
// Data rows are staged TR = 16 * NBI at a time in LDS (double-buffered, rows
// padded to 16 bytes past the width, one barrier per staged tile); each wave
// multiplies all of them against its 16 queries (1 LDS read per 4 MFMAs), so
// lane (g, c) = (lane/16, lane%16) receives rows 16*bi + 4*g + r of query c.
// Epilogue as above; FP32 sums of eight values folded into FP64.
constexpr int YWG = 512;
// 64 data rows per staged tile: 2 x 66 KB of LDS at d <= 128, so two
// workgroups (16 waves) share a CU (measured 7% faster than 128-row tiles
// with one workgroup per CU)
#ifndef YRES_NBI
#define YRES_NBI 4
#endif

template <int KERN, int DP, int NBI>
__global__ void __launch_bounds__(YWG, NBI == 8 ? 1 : 2)
kde_yres_kernel(TileProblem p, float Lf, double* __restrict__ partial, float2* __restrict__ cert) {
  constexpr int TR = 16 * NBI;                // data rows per staged tile
  constexpr int KGS = DP / 16;                // 64-byte k-groups per row
  constexpr int PITCH = DP * 4 + 16;          // LDS row pitch (bytes)
  constexpr int PPR = DP / 4;                 // 16-byte pieces per row
  constexpr int NPT = TR * PPR / YWG;         // pieces per thread per staged tile
  constexpr int UPT = BN / TR;                // staged tiles per 128-row tile
  static_assert(NPT >= 1 && TR * PPR == NPT * YWG, "tile pieces must split evenly");
  __shared__ __attribute__((aligned(16))) char xs[2][TR * PITCH];
  __shared__ __attribute__((aligned(16))) float xvs[2][TR];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t u0 = split * p.ntiles / p.splits * UPT, u1 = (split + 1) * p.ntiles / p.splits * UPT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const float L2 = 2.f * Lf;

  const int64_t qrow = qt * BQ + wave * 16 + c;
  u32x4 yf[KGS];
#pragma unroll
  for (int kg = 0; kg < KGS; ++kg)
    yf[kg] = *reinterpret_cast<const u32x4*>(p.Ys + qrow * p.ld_bytes + kg * KG_BYTES + g * 16);
  const double ynq = p.ynorm[qrow];
  const float yt = KERN == KERNEL_GAUSSIAN ? (float)(-(double)Lf * ynq) : (float)ynq;

  u32x4 xr[NPT];
  float xvr = 0.f;
  auto gload = [&](int64_t u) {
    const char* base = p.Xs + u * TR * p.ld_bytes;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int v = threadIdx.x + i * YWG;
      xr[i] = *reinterpret_cast<const u32x4*>(base + (v / PPR) * p.ld_bytes + (v % PPR) * 16);
    }
    if (threadIdx.x < TR) {   // padding rows: a term that zeroes the kernel
      const int64_t row = u * TR + threadIdx.x;
      if (KERN == KERNEL_GAUSSIAN)   // finite: K = 0 and K times the exponent = 0
        xvr = row < p.n ? (float)(-(double)Lf * p.xnorm[row]) : -1e30f;
      else
        xvr = row < p.n ? (float)p.xnorm[row] : __builtin_inff();
    }
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int v = threadIdx.x + i * YWG;
      *reinterpret_cast<u32x4*>(&xs[b][(v / PPR) * PITCH + (v % PPR) * 16]) = xr[i];
    }
    if (threadIdx.x < TR) xvs[b][threadIdx.x] = xvr;
  };

  double sum = 0.0;
  // certificate: sum of K^2; Gaussian: sum of K times its exponent, exponential: largest K
  float csq = 0.f, cmx = 0.f;
  if (u0 < u1) {
    gload(u0);
    lstore(0);
  }
  __syncthreads();
  for (int64_t u = u0; u < u1; ++u) {
    const int b = (int)((u - u0) & 1);
    const bool more = u + 1 < u1;
    if (more) gload(u + 1);
    const char* xb = xs[b];
    f32x4 acc[NBI];
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) acc[bi] = f32x4{0.f, 0.f, 0.f, 0.f};
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kg = 0; kg < KGS; ++kg) {
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) {
        const u32x4 a = *reinterpret_cast<const u32x4*>(xb + (bi * 16 + c) * PITCH + kg * KG_BYTES +
                                                         g * 16);
        acc[bi] = mfma_kgroup<float>(a, yf[kg], acc[bi]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (more) lstore(b ^ 1);
    const f32x4* xv4 = reinterpret_cast<const f32x4*>(xvs[b]);
#pragma unroll
    for (int bp = 0; bp < NBI / 2; ++bp) {
      float part = 0.f;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int bi = 2 * bp + h2;
        const f32x4 xt = xv4[bi * 4 + g];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float kv;
          if (KERN == KERNEL_GAUSSIAN) {   // exp(-d^2 / (2 h^2))
            const float a = fminf(__builtin_fmaf(L2, acc[bi][r], yt + xt[r]), 0.f);
            kv = __builtin_amdgcn_exp2f(a);
            cmx = __builtin_fmaf(-kv, a, cmx);
          } else {                          // exp(-d / h)
            const float d2 = fmaxf(__builtin_fmaf(-2.f, acc[bi][r], yt + xt[r]), 0.f);
            kv = __builtin_amdgcn_exp2f(-Lf * __builtin_sqrtf(d2));
            cmx = fmaxf(cmx, kv);
          }
          part += kv;
          csq = __builtin_fmaf(kv, kv, csq);
        }
      }
      sum += (double)part;
    }
    __syncthreads();   // next staged tile published; buffer b free
  }
  // the four lane groups of a query column, in a fixed order
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
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
    partial[split * p.qp + qt * BQ + wave * 16 + c] = sum;
    cert[split * p.qp + qt * BQ + wave * 16 + c] = make_float2(csq, cmx);
  }
}

// The same sweep with float32-accurate dot products from bfloat16 MFMAs: every
// prepared value is split into three bfloat16 parts (v = h + m + l exactly) and
// <x, y> is accumulated from the six products h h, h m, m h, h l, m m, l h of
// each 32-element k-chunk (v_mfma_f32_16x16x32_bf16, products exact in FP32);
// the three dropped products are below 2^-23 |x||y| together.  Rows hold the
// planes h, m, l of DPS elements each; the queries' planes stay in registers.
template <int KERN, int DPS, int NBI>
__global__ void __launch_bounds__(YWG, NBI <= 2 ? 2 : 1)
kde_split_kernel(TileProblem p, const char* __restrict__ Xsp, const char* __restrict__ Ysp,
                 float Lf, double* __restrict__ partial, float2* __restrict__ cert,
                 float* __restrict__ certk) {
  constexpr int TR = 16 * NBI;
  constexpr int KC = DPS / 32;                // 32-element k-chunks per plane
  constexpr int RB = 3 * DPS * 2;             // bytes per split row
  constexpr int PITCH = RB + 16;
  constexpr int PPR = RB / 16;
  constexpr int NPT = TR * PPR / YWG;
  constexpr int UPT = BN / TR;
  static_assert(NPT >= 1 && TR * PPR == NPT * YWG, "tile pieces must split evenly");
  __shared__ __attribute__((aligned(16))) char xs[2][TR * PITCH];
  __shared__ __attribute__((aligned(16))) float xvs[2][TR];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t u0 = split * p.ntiles / p.splits * UPT, u1 = (split + 1) * p.ntiles / p.splits * UPT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const float L2 = 2.f * Lf;
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
  const float yt = KERN == KERNEL_GAUSSIAN ? (float)(-(double)Lf * ynq) : (float)ynq;

  u32x4 xr[NPT];
  float xvr = 0.f;
  auto gload = [&](int64_t u) {
    const char* base = Xsp + u * TR * RB;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int v = threadIdx.x + i * YWG;
      xr[i] = *reinterpret_cast<const u32x4*>(base + (v / PPR) * RB + (v % PPR) * 16);
    }
    if (threadIdx.x < TR) {
      const int64_t row = u * TR + threadIdx.x;
      if (KERN == KERNEL_GAUSSIAN)   // finite: K = 0 and K times the exponent = 0
        xvr = row < p.n ? (float)(-(double)Lf * p.xnorm[row]) : -1e30f;
      else
        xvr = row < p.n ? (float)p.xnorm[row] : __builtin_inff();
    }
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int v = threadIdx.x + i * YWG;
      *reinterpret_cast<u32x4*>(&xs[b][(v / PPR) * PITCH + (v % PPR) * 16]) = xr[i];
    }
    if (threadIdx.x < TR) xvs[b][threadIdx.x] = xvr;
  };

  double sum = 0.0;
  // certificate: sum of K^2; Gaussian: sum of K times its exponent, exponential:
  // largest K; sum of K N (the bfloat16 MFMA's truncation bias, see cert.h)
  float csq = 0.f, cmx = 0.f, ckn = 0.f;
  if (u0 < u1) {
    gload(u0);
    lstore(0);
  }
  __syncthreads();
  for (int64_t u = u0; u < u1; ++u) {
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
        const char* ar = xb + (bi * 16 + c) * PITCH + kc * 64 + g * 16;
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
    if (more) lstore(b ^ 1);
    const f32x4* xv4 = reinterpret_cast<const f32x4*>(xvs[b]);
#pragma unroll
    for (int bp = 0; bp < (NBI + 1) / 2; ++bp) {
      float part = 0.f;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int bi = 2 * bp + h2;
        if (bi >= NBI) break;
        const f32x4 xt = xv4[bi * 4 + g];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float kv;
          const float nl = yt + xt[r];   // -L N (Gaussian) or N; padding: huge
          if (KERN == KERNEL_GAUSSIAN) {
            const float a = fminf(__builtin_fmaf(L2, acc[bi][r], nl), 0.f);
            kv = __builtin_amdgcn_exp2f(a);
            cmx = __builtin_fmaf(-kv, a, cmx);
            ckn = __builtin_fmaf(kv, -nl, ckn);
          } else {
            const float d2 = fmaxf(__builtin_fmaf(-2.f, acc[bi][r], nl), 0.f);
            kv = __builtin_amdgcn_exp2f(-Lf * __builtin_sqrtf(d2));
            cmx = fmaxf(cmx, kv);
            ckn = __builtin_fmaf(kv, fminf(nl, 3.0e38f), ckn);
          }
          part += kv;
          csq = __builtin_fmaf(kv, kv, csq);
        }
      }
      sum += (double)part;
    }
    __syncthreads();
  }
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
  csq += __shfl_xor(csq, 16, 64);
  csq += __shfl_xor(csq, 32, 64);
  if (KERN == KERNEL_GAUSSIAN) {
    cmx += __shfl_xor(cmx, 16, 64);
    cmx += __shfl_xor(cmx, 32, 64);
  } else {
    cmx = fmaxf(cmx, __shfl_xor(cmx, 16, 64));
    cmx = fmaxf(cmx, __shfl_xor(cmx, 32, 64));
  }
  ckn += __shfl_xor(ckn, 16, 64);
  ckn += __shfl_xor(ckn, 32, 64);
  if (g == 0) {
    partial[split * p.qp + qt * BQ + wave * 16 + c] = sum;
    cert[split * p.qp + qt * BQ + wave * 16 + c] = make_float2(csq, cmx);
    certk[split * p.qp + qt * BQ + wave * 16 + c] = ckn;
  }
}

#ifndef SPLIT_NBI
#define SPLIT_NBI 2
#endif

__global__ void kde_reduce_kernel(const double* __restrict__ partial, int64_t splits, int64_t qp,
                                  int64_t q, double inv_n, const double* __restrict__ ynorm,
                                  float Lf, int kern, const double* __restrict__ add,
                                  double* __restrict__ out);

static hipError_t finish_fp32(const TileProblem& p, int kern, double h, float L, double* partial,
                              double* out, hipStream_t s, const CertArgs& ca, const float* X,
                              const float* Y, int64_t d, double* fb_part);

template <int KERN, int DPS>
static void launch_split(const TileProblem& p, const void* Xsp, const void* Ysp, float L,
                         double* partial, float2* cert, float* certk, hipStream_t s) {
  TileProblem q = p;
  q.map = make_tile_map(p.qtiles, p.splits, 1);
  constexpr int NBI = DPS == 64 ? 4 : SPLIT_NBI;   // whole 16-byte pieces per thread
  kde_split_kernel<KERN, DPS, NBI><<<dim3((unsigned)q.map.grid), dim3(YWG), 0, s>>>(
      q, reinterpret_cast<const char*>(Xsp), reinterpret_cast<const char*>(Ysp), L, partial,
      cert, certk);
}

template <typename T, int KERN, int ENG, bool HYB = false>
static void launch_kde_k(const TileProblem& p, float L, double* partial, hipStream_t s,
                         const int32_t* hoff = nullptr, const uint16_t* hits = nullptr,
                         float2* cert = nullptr, float* certn = nullptr, float* certk = nullptr);

hipError_t launch_kde_exact_split(const TileProblem& p, const void* Xsp, const void* Ysp,
                                  int64_t dps, int kern, double h, double* partial, double* out,
                                  hipStream_t s, TimingHook th, const CertArgs& ca,
                                  const float* X, const float* Y, int64_t d, double* fb_part) {
  const double log2e = 1.4426950408889634;
  const float L = (float)(kern == KERNEL_GAUSSIAN ? log2e / (2.0 * h * h) : log2e / h);
  hipError_t e;
  if (th.start && (e = hipEventRecord(th.start, s)) != hipSuccess) return e;
  if (dps == 64) {
    if (kern == KERNEL_GAUSSIAN)
      launch_split<KERNEL_GAUSSIAN, 64>(p, Xsp, Ysp, L, partial, ca.part, ca.pk, s);
    else
      launch_split<KERNEL_EXPONENTIAL, 64>(p, Xsp, Ysp, L, partial, ca.part, ca.pk, s);
  } else if (dps == 128) {
    if (kern == KERNEL_GAUSSIAN)
      launch_split<KERNEL_GAUSSIAN, 128>(p, Xsp, Ysp, L, partial, ca.part, ca.pk, s);
    else
      launch_split<KERNEL_EXPONENTIAL, 128>(p, Xsp, Ysp, L, partial, ca.part, ca.pk, s);
  } else if (dps > 128 && dps % 32 == 0) {
    // wider rows: the generic tile kernel's split engine (query tiles streamed)
    TileProblem q = p;
    q.Ys = reinterpret_cast<const char*>(Ysp);
    q.Xs = reinterpret_cast<const char*>(Xsp);
    q.ld_bytes = 6 * dps;
    q.nchunks = (int)(dps / 32);
    if (kern == KERNEL_GAUSSIAN)
      launch_kde_k<float, KERNEL_GAUSSIAN, 3>(q, L, partial, s, nullptr, nullptr, ca.part, ca.pn,
                                              ca.pk);
    else
      launch_kde_k<float, KERNEL_EXPONENTIAL, 3>(q, L, partial, s, nullptr, nullptr, ca.part,
                                                 ca.pn, ca.pk);
  } else {
    return hipErrorInvalidValue;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (th.stop && (e = hipEventRecord(th.stop, s)) != hipSuccess) return e;
  CertArgs cb = ca;
  if (dps <= 128) cb.pn = nullptr;   // the resident-query split kernel keeps no sums of (K N)^2
  return finish_fp32(p, kern, h, L, partial, out, s, cb, X, Y, d, fb_part);
}

// Sum of the per-split partials in split order, times the Gaussian query
// factor 2^(rounding remainder of -L ||y||^2), plus add[i] (the exact sum over
// the neighbours in the near/far form; NULL otherwise), times 1/n.
__global__ void kde_reduce_kernel(const double* __restrict__ partial, int64_t splits, int64_t qp,
                                  int64_t q, double inv_n, const double* __restrict__ ynorm,
                                  float Lf, int kern, const double* __restrict__ add,
                                  double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  double s = 0.0;
  for (int64_t sp = 0; sp < splits; ++sp) s += partial[sp * qp + i];
  if (kern == KERNEL_GAUSSIAN) {
    const double e = -(double)Lf * ynorm[i];
    s *= exp2(e - (double)(float)e);
  }
  if (add) s += add[i];
  out[i] = s * inv_n;
}

template <typename T, int KERN, int ENG, bool HYB>
static void launch_kde_k(const TileProblem& p, float L, double* partial, hipStream_t s,
                         const int32_t* hoff, const uint16_t* hits, float2* cert, float* certn,
                         float* certk) {
  kde_tile_kernel<T, KERN, ENG, HYB><<<dim3((unsigned)p.map.grid), dim3(WG), 0, s>>>(
      p.Ys, p.Xs, p.ld_bytes, p.nchunks, p.ynorm, p.xnorm, p.n, p.qtiles, p.splits, p.ntiles, L,
      partial, p.qp, p.map, hoff, hits, cert, certn, certk);
}

template <typename T, int KERN>
static void launch_kde_n(const TileProblem& p, float L, double* partial, float2* cert,
                         float* certn, hipStream_t s) {
  if constexpr (elem_of<T>::bytes == 2) {
    const int eng = tile_engine<T>(p.ld_bytes);
    if (eng == 2) return launch_kde_k<T, KERN, 2>(p, L, partial, s);
    if (eng == 1) return launch_kde_k<T, KERN, 1>(p, L, partial, s);
  }
  launch_kde_k<T, KERN, 0>(p, L, partial, s, nullptr, nullptr, cert, certn);
}

template <typename T, int KERN>
static void launch_hyb_n(const TileProblem& p, float L, double* partial, const int32_t* hoff,
                         const uint16_t* hits, hipStream_t s) {
  const int eng = tile_engine<T>(p.ld_bytes);
  if (eng == 2) return launch_kde_k<T, KERN, 2, true>(p, L, partial, s, hoff, hits);
  if (eng == 1) return launch_kde_k<T, KERN, 1, true>(p, L, partial, s, hoff, hits);
  launch_kde_k<T, KERN, 0, true>(p, L, partial, s, hoff, hits);
}

template <typename T>
static void launch_hyb_t(const TileProblem& p, int kern, float L, double* partial,
                         const int32_t* hoff, const uint16_t* hits, hipStream_t s) {
  if (kern == KERNEL_GAUSSIAN)
    launch_hyb_n<T, KERNEL_GAUSSIAN>(p, L, partial, hoff, hits, s);
  else
    launch_hyb_n<T, KERNEL_EXPONENTIAL>(p, L, partial, hoff, hits, s);
}

template <int KERN, int DP>
static void launch_yres(const TileProblem& p, float L, double* partial, float2* cert,
                        hipStream_t s) {
  // one workgroup sweeps a query tile over a data split; split-major placement
  TileProblem q = p;
  q.map = make_tile_map(p.qtiles, p.splits, 1);
  kde_yres_kernel<KERN, DP, YRES_NBI><<<dim3((unsigned)q.map.grid), dim3(YWG), 0, s>>>(
      q, L, partial, cert);
}

template <int KERN>
static bool launch_yres_d(const TileProblem& p, float L, double* partial, float2* cert,
                          hipStream_t s) {
  switch (p.ld_bytes / 4) {
    case 32: launch_yres<KERN, 32>(p, L, partial, cert, s); return true;
    case 64: launch_yres<KERN, 64>(p, L, partial, cert, s); return true;
    case 96: launch_yres<KERN, 96>(p, L, partial, cert, s); return true;
    case 128: launch_yres<KERN, 128>(p, L, partial, cert, s); return true;
    default: return false;
  }
}

// certn (float32 operands): set to null when the sweep does not write the
// per-pair norm sums (rows of at most 512 bytes take kde_yres_kernel)
template <typename T>
static hipError_t launch_kde_t(const TileProblem& p, int kern, float L, double* partial,
                               float2* cert, float** certn, hipStream_t s) {
  if constexpr (elem_of<T>::bytes == 4) {   // FP32 rows of at most 512 bytes
    const bool done = kern == KERNEL_GAUSSIAN
                          ? launch_yres_d<KERNEL_GAUSSIAN>(p, L, partial, cert, s)
                          : launch_yres_d<KERNEL_EXPONENTIAL>(p, L, partial, cert, s);
    if (done) {
      *certn = nullptr;
      return hipGetLastError();
    }
  }
  float* cn = certn ? *certn : nullptr;
  if (kern == KERNEL_GAUSSIAN)
    launch_kde_n<T, KERNEL_GAUSSIAN>(p, L, partial, cert, cn, s);
  else
    launch_kde_n<T, KERNEL_EXPONENTIAL>(p, L, partial, cert, cn, s);
  return hipGetLastError();
}

// Reduction of a float32-operand sweep with the certificate, then the exact
// re-evaluation of the queries it lists.
static hipError_t finish_fp32(const TileProblem& p, int kern, double h, float L, double* partial,
                              double* out, hipStream_t s, const CertArgs& ca, const float* X,
                              const float* Y, int64_t d, double* fb_part) {
  hipError_t e = launch_kde_reduce_cert(partial, p.splits, p.qp, p.q, p.n, p.ynorm, L, kern, ca,
                                        out, s);
  if (e != hipSuccess) return e;
  return launch_kde_direct(X, Y, p.n, p.q, d, h, kern, ca.fb_ids, ca.fb_count,
                           direct_splits(p.n), fb_part, out, s);
}

hipError_t launch_kde_exact(int prec, const TileProblem& p, int kern, double h, double* partial,
                            double* out, hipStream_t s, TimingHook th, const CertArgs& ca,
                            const float* X, const float* Y, int64_t d, double* fb_part) {
  const double log2e = 1.4426950408889634;
  const float L = (float)(kern == KERNEL_GAUSSIAN ? log2e / (2.0 * h * h) : log2e / h);
  hipError_t e;
  if (th.start && (e = hipEventRecord(th.start, s)) != hipSuccess) return e;
  CertArgs cb = ca;
  cb.pk = nullptr;   // float32 MFMAs round to nearest: no bias term
  switch (prec) {
    case PREC_FP32: e = launch_kde_t<float>(p, kern, L, partial, ca.part, &cb.pn, s); break;
    case PREC_BF16: e = launch_kde_t<__bf16>(p, kern, L, partial, nullptr, nullptr, s); break;
    default: e = launch_kde_t<_Float16>(p, kern, L, partial, nullptr, nullptr, s); break;
  }
  if (e != hipSuccess) return e;
  if (th.stop && (e = hipEventRecord(th.stop, s)) != hipSuccess) return e;
  if (prec == PREC_FP32) return finish_fp32(p, kern, h, L, partial, out, s, cb, X, Y, d, fb_part);
  kde_reduce_kernel<<<dim3((unsigned)ceil_div(p.q, 256)), dim3(256), 0, s>>>(
      partial, p.splits, p.qp, p.q, 1.0 / (double)p.n, p.ynorm, L, kern, nullptr, out);
  return hipGetLastError();
}

hipError_t launch_kde_hybrid(int prec, const TileProblem& p, int kern, double h,
                             const int32_t* hoff, const uint16_t* hits, const double* z1,
                             double* partial, double* out, hipStream_t s, TimingHook th) {
  const double log2e = 1.4426950408889634;
  const float L = (float)(kern == KERNEL_GAUSSIAN ? log2e / (2.0 * h * h) : log2e / h);
  hipError_t e;
  if (th.start && (e = hipEventRecord(th.start, s)) != hipSuccess) return e;
  if (prec == PREC_BF16)
    launch_hyb_t<__bf16>(p, kern, L, partial, hoff, hits, s);
  else if (prec == PREC_FP16)
    launch_hyb_t<_Float16>(p, kern, L, partial, hoff, hits, s);
  else
    return hipErrorInvalidValue;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (th.stop && (e = hipEventRecord(th.stop, s)) != hipSuccess) return e;
  kde_reduce_kernel<<<dim3((unsigned)ceil_div(p.q, 256)), dim3(256), 0, s>>>(
      partial, p.splits, p.qp, p.q, 1.0 / (double)p.n, p.ynorm, L, kern, z1, out);
  return hipGetLastError();
}

}  // namespace deann
