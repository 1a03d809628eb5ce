// Shared device helpers for the DEANN HIP library (gfx950 / CDNA4).
//
// Tiles: a workgroup of 256 threads (4 wave64) owns a BQ x BN block of
// (query, data-row) pairs.  Both operands are staged through LDS in k-chunks
// of DK elements; each wave owns a 64 x 64 quarter and issues 16 x 16 MFMA
// blocks (v_mfma_f32_16x16x4_f32 for FP32 operands, v_mfma_f32_16x16x32_{bf16,f16}
// for 16-bit operands), accumulating in FP32.
//
// Operand layout convention (identical for A = query rows and B = data rows):
// a k-group is 64 bytes of a row.  Lane l of a wave reads the 16 bytes at
// offset 16*(l/16) of the k-group of row (l%16).  For FP32 those 4 floats feed
// 4 successive 16x16x4 MFMAs; for 16-bit types the 8 values feed one 16x16x32
// MFMA.  The k order inside a group is thereby permuted, identically for both
// operands, which leaves every dot product unchanged.
//
// Accumulator layout of a 16x16 block: lane l, register r holds
// row 4*(l/16) + r, column l%16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace deann {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int WG = 256;          // threads per workgroup
constexpr int BQ = 128;          // queries per tile
constexpr int BN = 128;          // data rows per tile
constexpr int KG_BYTES = 64;     // bytes of a row per k-group
constexpr int CHUNK_BYTES = 128; // bytes of a row per LDS k-chunk (2 k-groups)
constexpr int ROW_PAD = 16;      // LDS row padding in bytes
constexpr int LDS_ROW = CHUNK_BYTES + ROW_PAD;
constexpr int TILE_LDS = BQ * LDS_ROW;   // one operand chunk in LDS (bytes)

enum : int { KERNEL_GAUSSIAN = 0, KERNEL_EXPONENTIAL = 1 };
enum : int { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP16 = 2 };

template <typename T> struct elem_of;
template <> struct elem_of<float> { static constexpr int bytes = 4; };
template <> struct elem_of<__bf16> { static constexpr int bytes = 2; };
template <> struct elem_of<_Float16> { static constexpr int bytes = 2; };

// Elements per padded row unit: every scan operand row is padded with zeros
// to a multiple of CHUNK_BYTES so that tile loads need no k masking.
template <typename T>
__host__ __device__ constexpr int64_t padded_dim(int64_t d) {
  const int64_t per = CHUNK_BYTES / elem_of<T>::bytes;
  return (d + per - 1) / per * per;
}

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// MFMA on one 64-byte k-group: acc += A(16 x kgroup) * B(kgroup x 16)^T
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ f32x4 mfma_kgroup(u32x4 a, u32x4 b, f32x4 acc);

template <>
__device__ __forceinline__ f32x4 mfma_kgroup<float>(u32x4 a, u32x4 b, f32x4 acc) {
  // element-wise reinterpretation (a bit_cast of a vector element would
  // reinterpret the whole vector's first bytes)
  const uint32_t a0 = a.x, a1 = a.y, a2 = a.z, a3 = a.w;
  const uint32_t b0 = b.x, b1 = b.y, b2 = b.z, b3 = b.w;
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a0), __uint_as_float(b0), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a1), __uint_as_float(b1), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a2), __uint_as_float(b2), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a3), __uint_as_float(b3), acc, 0, 0, 0);
  return acc;
}

template <>
__device__ __forceinline__ f32x4 mfma_kgroup<__bf16>(u32x4 a, u32x4 b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}

template <>
__device__ __forceinline__ f32x4 mfma_kgroup<_Float16>(u32x4 a, u32x4 b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Global -> register -> LDS staging of one k-chunk (CHUNK_BYTES per row) of a
// 128-row tile.  Rows are padded in global memory (row stride `ld_bytes`, a
// multiple of CHUNK_BYTES) and the row count is padded to a multiple of 128,
// so every load is in bounds and 16-byte aligned.
// ---------------------------------------------------------------------------
constexpr int CHUNK_VECS = BQ * CHUNK_BYTES / 16 / WG;   // 16-byte loads per thread (= 4)

struct ChunkRegs { u32x4 v[CHUNK_VECS]; };

__device__ __forceinline__ void load_chunk(ChunkRegs& r, const char* __restrict__ base,
                                           int64_t ld_bytes, int64_t kbyte) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < CHUNK_VECS; ++i) {
    const int v = t + i * WG;                 // vector id within the tile chunk
    const int row = v / (CHUNK_BYTES / 16);
    const int col = v % (CHUNK_BYTES / 16);
    r.v[i] = *reinterpret_cast<const u32x4*>(base + row * ld_bytes + kbyte + col * 16);
  }
}

__device__ __forceinline__ void store_chunk(const ChunkRegs& r, char* lds) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < CHUNK_VECS; ++i) {
    const int v = t + i * WG;
    const int row = v / (CHUNK_BYTES / 16);
    const int col = v % (CHUNK_BYTES / 16);
    *reinterpret_cast<u32x4*>(lds + row * LDS_ROW + col * 16) = r.v[i];
  }
}

// Fragment of 16 rows starting at `row0` for k-group `kg` of the LDS chunk.
__device__ __forceinline__ u32x4 lds_frag(const char* lds, int row0, int kg, int lane) {
  return *reinterpret_cast<const u32x4*>(lds + (row0 + (lane & 15)) * LDS_ROW + kg * KG_BYTES +
                                         (lane >> 4) * 16);
}

// Accumulate the wave's 64 x 64 quarter over one LDS chunk.
// qa: LDS chunk of the query tile, xa: LDS chunk of the data tile.
template <typename T>
__device__ __forceinline__ void mfma_chunk(f32x4 (&acc)[4][4], const char* qa, const char* xa,
                                           int wq, int wn, int lane) {
#pragma unroll
  for (int kg = 0; kg < CHUNK_BYTES / KG_BYTES; ++kg) {
    u32x4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = lds_frag(qa, wq * 64 + i * 16, kg, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = lds_frag(xa, wn * 64 + j * 16, kg, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma_kgroup<T>(a[i], b[j], acc[i][j]);
  }
}

// Streamed sweep over data tiles [t0, t1) against one query tile.  The chunk
// sequence is continuous across tiles: the registers always hold the next
// chunk (of this tile or of the next one) while the current one is multiplied,
// so global latency is hidden behind the MFMAs and the epilogue.  One barrier
// per chunk: a buffer is refilled two chunks after it was last read, and every
// wave has passed the barrier in between.  Usage:
//   StreamState st;  stream_start(st, ...);
//   for (t = t0; t < t1; ++t) { stream_tile<T>(acc, st, ..., t, ...); epilogue; }
//   __syncthreads();   // before reusing the staging area
// The epilogue may use LDS outside the 4 * TILE_LDS staging area.  ts: sweep
// tile t reads data tile t * ts (every ts-th tile; the engines below alike).
struct StreamState {
  ChunkRegs rq, rx;
  int buf;
};

__device__ __forceinline__ void stream_start(StreamState& st, const char* __restrict__ yq,
                                             const char* __restrict__ Xs, int64_t ld_bytes,
                                             int64_t t0, int64_t ts = 1) {
  load_chunk(st.rq, yq, ld_bytes, 0);
  load_chunk(st.rx, Xs + t0 * ts * BN * ld_bytes, ld_bytes, 0);
  st.buf = 0;
  __syncthreads();   // previous users of the staging area are done
}

// SWAP = false: acc rows are queries (wq), columns data rows (wn).
// SWAP = true : acc rows are data rows (wq), columns queries (wn), i.e. S^T.
template <typename T, bool SWAP = false>
__device__ __forceinline__ void stream_tile(f32x4 (&acc)[4][4], StreamState& st,
                                            const char* __restrict__ yq,
                                            const char* __restrict__ Xs, int64_t ld_bytes,
                                            int nchunks, int64_t t, int64_t t1, char* lds,
                                            int wq, int wn, int lane, int64_t ts = 1) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < nchunks; ++c) {
    char* qa = lds + st.buf * 2 * TILE_LDS;
    char* xa = qa + TILE_LDS;
    store_chunk(st.rq, qa);
    store_chunk(st.rx, xa);
    __syncthreads();
    int nc = c + 1;
    int64_t nt = t;
    if (nc == nchunks) { nc = 0; nt = t + 1; }
    if (nt < t1) {
      load_chunk(st.rq, yq, ld_bytes, (int64_t)nc * CHUNK_BYTES);
      load_chunk(st.rx, Xs + nt * ts * BN * ld_bytes, ld_bytes, (int64_t)nc * CHUNK_BYTES);
    }
    __builtin_amdgcn_s_setprio(1);   // favour the wave issuing MFMAs
    if (SWAP)
      mfma_chunk<T>(acc, xa, qa, wq, wn, lane);
    else
      mfma_chunk<T>(acc, qa, xa, wq, wn, lane);
    __builtin_amdgcn_s_setprio(0);
    st.buf ^= 1;
  }
}

// Query tile resident in LDS, data chunks two steps ahead, for rows of exactly
// 256 bytes (16-bit operands with 64 < d <= 128: two chunks per tile).  The
// query tile is copied to LDS once per workgroup; per chunk only the data
// chunk is stored, and the registers of chunk c are refilled with chunk c of
// the next tile right after the barrier, so a load has a whole tile (both
// chunks and the epilogue) to arrive.  LDS: QL_Y_BYTES + 2 * TILE_LDS bytes.
// Usage as stream_tile: ql_start once, ql_tile per data tile, __syncthreads()
// before reusing the staging area.
constexpr int QL_ROWB = 2 * CHUNK_BYTES;
constexpr int QL_YROW = QL_ROWB + ROW_PAD;
constexpr int QL_Y_BYTES = BQ * QL_YROW;

struct QlState {
  ChunkRegs rx[2];
};

__device__ __forceinline__ void ql_start(QlState& st, const char* __restrict__ yq,
                                         const char* __restrict__ Xs, int64_t t0, char* lds,
                                         int64_t ts = 1) {
  __syncthreads();   // previous users of the staging area are done
  constexpr int VECS = BQ * QL_ROWB / 16;
#pragma unroll
  for (int i = 0; i < VECS / WG; ++i) {
    const int v = threadIdx.x + i * WG;
    const int row = v / (QL_ROWB / 16), col = v % (QL_ROWB / 16);
    *reinterpret_cast<u32x4*>(lds + row * QL_YROW + col * 16) =
        *reinterpret_cast<const u32x4*>(yq + row * QL_ROWB + col * 16);
  }
  load_chunk(st.rx[0], Xs + t0 * ts * BN * QL_ROWB, QL_ROWB, 0);
  load_chunk(st.rx[1], Xs + t0 * ts * BN * QL_ROWB, QL_ROWB, CHUNK_BYTES);
}

template <typename T>
__device__ __forceinline__ void ql_tile(f32x4 (&acc)[4][4], QlState& st,
                                        const char* __restrict__ Xs, int64_t t, int64_t t1,
                                        char* lds, int wq, int wn, int lane, int64_t ts = 1) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    char* xa = lds + QL_Y_BYTES + c * TILE_LDS;
    store_chunk(st.rx[c], xa);
    __syncthreads();
    if (t + 1 < t1) load_chunk(st.rx[c], Xs + (t + 1) * ts * BN * QL_ROWB, QL_ROWB, c * CHUNK_BYTES);
    __builtin_amdgcn_s_setprio(1);   // favour the wave issuing MFMAs
#pragma unroll
    for (int kg = 0; kg < CHUNK_BYTES / KG_BYTES; ++kg) {
      u32x4 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *reinterpret_cast<const u32x4*>(lds + (wq * 64 + i * 16 + (lane & 15)) * QL_YROW +
                                               c * CHUNK_BYTES + kg * KG_BYTES + (lane >> 4) * 16);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = lds_frag(xa, wn * 64 + j * 16, kg, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_kgroup<T>(a[i], b[j], acc[i][j]);
    }
    __builtin_amdgcn_s_setprio(0);
  }
}

// Query fragments resident in registers, for 16-bit rows of 128 bytes
// (d <= 64): each wave keeps its 64 query rows' A fragments for the whole
// kernel and only the data tiles stream through LDS, a whole tile (NKG 64-byte
// k-groups of 128 rows) per barrier, prefetched a tile ahead in registers.
template <int NKG>
struct XStream {
  static constexpr int ROWB = NKG * KG_BYTES;          // bytes of a row
  static constexpr int LROW = ROWB + ROW_PAD;          // LDS row stride
  static constexpr int VEC = BN * ROWB / 16 / WG;      // 16-byte loads per thread
  static constexpr int BUF = BN * LROW;                // one buffer (bytes)
  u32x4 r[VEC];
  int buf;
};

template <int NKG>
__device__ __forceinline__ void xs_load(XStream<NKG>& st, const char* __restrict__ xt,
                                        int64_t ld_bytes) {
#pragma unroll
  for (int i = 0; i < XStream<NKG>::VEC; ++i) {
    const int v = threadIdx.x + i * WG;
    const int row = v / (XStream<NKG>::ROWB / 16), col = v % (XStream<NKG>::ROWB / 16);
    st.r[i] = *reinterpret_cast<const u32x4*>(xt + row * ld_bytes + col * 16);
  }
}

template <int NKG>
__device__ __forceinline__ void xs_store(const XStream<NKG>& st, char* lds) {
#pragma unroll
  for (int i = 0; i < XStream<NKG>::VEC; ++i) {
    const int v = threadIdx.x + i * WG;
    const int row = v / (XStream<NKG>::ROWB / 16), col = v % (XStream<NKG>::ROWB / 16);
    *reinterpret_cast<u32x4*>(lds + row * XStream<NKG>::LROW + col * 16) = st.r[i];
  }
}

// A fragments of the wave's 64 query rows, all k-groups, straight from global.
template <int NKG>
__device__ __forceinline__ void yreg_load(u32x4 (&yf)[4][NKG], const char* __restrict__ yq,
                                          int64_t ld_bytes, int wq, int lane) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int g = 0; g < NKG; ++g)
      yf[i][g] = *reinterpret_cast<const u32x4*>(yq + (wq * 64 + i * 16 + (lane & 15)) * ld_bytes +
                                                  g * KG_BYTES + (lane >> 4) * 16);
}

// One data tile t (data already prefetched in st): store, barrier, prefetch
// tile t + 1 if any, multiply.  lds holds 2 * XStream<NKG>::BUF bytes.
template <typename T, int NKG>
__device__ __forceinline__ void yreg_tile(f32x4 (&acc)[4][4], XStream<NKG>& st,
                                          const u32x4 (&yf)[4][NKG], const char* __restrict__ Xs,
                                          int64_t ld_bytes, int64_t t, int64_t t1, char* lds,
                                          int wn, int lane, int64_t ts = 1) {
  char* xa = lds + st.buf * XStream<NKG>::BUF;
  xs_store(st, xa);
  __syncthreads();
  if (t + 1 < t1) xs_load(st, Xs + (t + 1) * ts * BN * ld_bytes, ld_bytes);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int g = 0; g < NKG; ++g) {
    u32x4 b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const u32x4*>(xa + (wn * 64 + j * 16 + (lane & 15)) * XStream<NKG>::LROW +
                                             g * KG_BYTES + (lane >> 4) * 16);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma_kgroup<T>(yf[i][g], b[j], acc[i][j]);
  }
  st.buf ^= 1;
}

// Engine for a tile kernel: 2 = query fragments in registers (16-bit rows of
// 128 bytes, d <= 64); 1 = query tile in LDS (16-bit rows of 256 bytes,
// 64 < d <= 128); 0 = generic stream.  Query fragments in registers for 256-byte
// rows would not leave room for two workgroups per CU.
template <typename T>
inline int tile_engine(int64_t ld_bytes) {
  if (elem_of<T>::bytes != 2) return 0;
  if (ld_bytes == 2 * KG_BYTES) return 2;
  if (ld_bytes == QL_ROWB) return 1;
  return 0;
}

// XCD-aware placement.  Workgroups are dispatched round-robin over the 8 XCDs,
// so hardware id hw runs on XCD hw % 8 as its (hw / 8)-th workgroup.  Each XCD
// receives a contiguous eighth of the (split-major) work items, so the
// workgroups an XCD holds at a time share one data split -- the same data
// tiles, read once into that XCD's L2 -- and differ in their query tile.
// Returns false for the padding items beyond qtiles * splits.
struct TileMap {
  int64_t grid;     // launched workgroups: qtiles * splits rounded up to 8
  int64_t group;    // data splits per group (see map_tile)
};

// Workgroup placement.  Hardware workgroup ids are dealt round-robin to the 8
// XCDs, so v below enumerates, for each XCD in turn, the workgroups it runs in
// dispatch order.  Consecutive v cover `group` data splits for every query
// tile in turn (query tile major within the group): the workgroups resident
// on one XCD at a time then share the data tiles of a few splits in its L2
// while their query tiles (re-read every data tile by the generic stream)
// stay few enough to remain cached too.  With group = 1 it is split-major.
__device__ __forceinline__ bool map_tile(int64_t hw, const TileMap& m, int64_t qtiles,
                                         int64_t splits, int64_t& qt, int64_t& split) {
  const int64_t v = (hw % 8) * (m.grid / 8) + hw / 8;
  const int64_t span = qtiles * m.group;
  const int64_t sg = v / span, rem = v % span;
  const int64_t g = splits - sg * m.group < m.group ? splits - sg * m.group : m.group;
  if (g <= 0) return false;
  qt = rem / g;
  split = sg * m.group + rem % g;
  return qt < qtiles;
}

inline TileMap make_tile_map(int64_t qtiles, int64_t splits, int64_t group) {
  TileMap m;
  m.grid = (qtiles * splits + 7) / 8 * 8;
  m.group = group < 1 ? 1 : (group > splits ? splits : group);
  return m;
}

// Order-preserving map float -> uint32 (total order matching <, -0 < +0).
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t b = __builtin_bit_cast(uint32_t, f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, b);
}

// Exact FP64 squared distances of four rows of X to the query ys (LDS), by a
// group of 16 consecutive lanes (all 16 get the results); the four rows'
// loads are in flight together.  Rows whose start is 16-byte aligned are read
// as float4.  Each sum is formed in a fixed order (coordinates of a lane in
// ascending order, then a butterfly over the 16 lanes), the same for one row
// at a time.  Rows r[i] < 0 give 0.
__device__ __forceinline__ void group16_d2_4(const float* __restrict__ X, const int64_t (&r)[4],
                                             int64_t d, const float* ys, int l16, double (&out)[4]) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (((d & 3) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0)) {
    for (int64_t t = 4 * l16; t < d; t += 64) {
      f32x4 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v[i] = r[i] >= 0 ? *reinterpret_cast<const f32x4*>(X + r[i] * d + t)
                         : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double df = (double)v[i][c] - (double)ys[t + c];
          s[i] = __builtin_fma(df, df, s[i]);
        }
    }
  } else {
    for (int64_t t = l16; t < d; t += 16) {
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = r[i] >= 0 ? X[r[i] * d + t] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double df = (double)v[i] - (double)ys[t];
        s[i] = __builtin_fma(df, df, s[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = s[i];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    out[i] = r[i] >= 0 ? v : 0.0;
  }
}

}  // namespace deann
