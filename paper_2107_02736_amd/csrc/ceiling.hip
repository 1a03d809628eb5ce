// Measurement support, not part of the DEANN library: the two data-movement
// patterns of the hot path with all of their arithmetic removed, so that each
// product kernel can be set against what its own access pattern reaches on
// the device.
//
//  * ceiling_gather: random whole-row reads, GW lanes per row and two rows in
//    flight per lane group, as the DEANN gather (deann_backward_vec_kernel)
//    reads the k + m rows of a query; the row data only feeds a sum.
//  * ceiling_tile_sweep: the 16-bit distance tile sweep of the k-NN passes
//    (the same tile engines, placement and split count as knn_collect_kernel)
//    with the epilogue reduced to a running sum of the accumulators.
//
// Built into its own libdeann_ceiling.so; the benchmark's --ceilings mode
// calls it.  Both entry points return a hipError_t value (0 = success).
#include "common.h"
#include "kernels.h"

namespace deann {
namespace {

template <int GW, int U>
__global__ void __launch_bounds__(WG) ceiling_gather_kernel(const float* __restrict__ X, int64_t d,
                                                            const int32_t* __restrict__ idx,
                                                            int64_t rows, float* __restrict__ out) {
  constexpr int NG = WG / GW;
  const int g = threadIdx.x / GW, lg = threadIdx.x % GW;
  const int32_t* id = idx + (int64_t)blockIdx.x * rows;
  auto load_row = [&](int32_t row, f32x4 (&dst)[U]) {
    const float* xr = X + (int64_t)row * d;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t t = 4 * lg + 4 * GW * u;
      dst[u] = t < d ? *reinterpret_cast<const f32x4*>(xr + t) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  f32x4 xv[U], xa[U];
  float s = 0.f;
  if (g < rows) load_row(id[g], xv);
  for (int64_t i = g; i < rows; i += NG) {
    if (i + NG < rows) load_row(id[i + NG], xa);
#pragma unroll
    for (int u = 0; u < U; ++u) s += (xv[u][0] + xv[u][1]) + (xv[u][2] + xv[u][3]);
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = xa[u];
  }
  // never true for finite data; keeps the loads live
  if (s == -1.0e30f) out[(int64_t)blockIdx.x * WG + threadIdx.x] = s;
}

template <typename T, int ENG>
__global__ void __launch_bounds__(WG, 2) ceiling_sweep_kernel(TileProblem p, float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char lds[4 * TILE_LDS];
  int64_t qt, split;
  if (!map_tile(blockIdx.x, p.map, p.qtiles, p.splits, qt, split)) return;
  const int64_t t0 = split * p.ntiles / p.splits, t1 = (split + 1) * p.ntiles / p.splits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = wave >> 1, wn = wave & 1;
  const char* yq = p.Ys + qt * BQ * p.ld_bytes;
  constexpr int NK = 2;
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
  float s = 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    f32x4 acc[4][4];
    if constexpr (ENG == 0)
      stream_tile<T>(acc, st, yq, p.Xs, p.ld_bytes, p.nchunks, t, t1, lds, wq, wn, lane);
    else if constexpr (ENG == 1)
      ql_tile<T>(acc, ql, p.Xs, t, t1, lds, wq, wn, lane);
    else
      yreg_tile<T, NK>(acc, xs, yf, p.Xs, p.ld_bytes, t, t1, lds, wn, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) s += acc[i][j][0];
  }
  if (s == -1.0e30f) out[threadIdx.x] = s;
}

}  // namespace
}  // namespace deann

using namespace deann;

// X: [n, d] float32 device rows (d a multiple of 4, 16-byte aligned), idx:
// [q, rows] int32 device row indices in [0, n), out: q * 256 floats of device
// scratch (never written for finite X).  One workgroup per index row.
extern "C" int ceiling_gather(const float* X, int64_t n, int64_t d, const int32_t* idx, int64_t q,
                              int64_t rows, float* out, void* stream) {
  if (!X || !idx || !out || n <= 0 || q <= 0 || rows <= 0 || d <= 0 || d % 4 != 0 || d > 2048)
    return (int)hipErrorInvalidValue;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 g((unsigned)q), blk(WG);
  if (d <= 64) ceiling_gather_kernel<16, 1><<<g, blk, 0, s>>>(X, d, idx, rows, out);
  else if (d <= 128) ceiling_gather_kernel<16, 2><<<g, blk, 0, s>>>(X, d, idx, rows, out);
  else if (d <= 256) ceiling_gather_kernel<64, 1><<<g, blk, 0, s>>>(X, d, idx, rows, out);
  else if (d <= 512) ceiling_gather_kernel<64, 2><<<g, blk, 0, s>>>(X, d, idx, rows, out);
  else if (d <= 1024) ceiling_gather_kernel<64, 4><<<g, blk, 0, s>>>(X, d, idx, rows, out);
  else ceiling_gather_kernel<64, 8><<<g, blk, 0, s>>>(X, d, idx, rows, out);
  return (int)hipGetLastError();
}

// Ys: [qp, dp] and Xs: [np, dp] bfloat16 device operands, qp and np multiples
// of 128, dp a multiple of 64 (rows of dp * 2 bytes); split_target: workgroups
// wanted (the k-NN passes use 4096); group: data splits per placement group
// (0: the k-NN passes' choice); out: 256 floats of device scratch.
extern "C" int ceiling_tile_sweep(const void* Ys, int64_t qp, const void* Xs, int64_t np,
                                  int64_t dp, int64_t split_target, int64_t group, float* out,
                                  void* stream) {
  if (!Ys || !Xs || !out || qp <= 0 || np <= 0 || qp % BQ || np % BN || dp <= 0 || dp % 64 ||
      split_target <= 0 || group < 0)
    return (int)hipErrorInvalidValue;
  TileProblem p{};
  p.Ys = static_cast<const char*>(Ys);
  p.Xs = static_cast<const char*>(Xs);
  p.ld_bytes = dp * 2;
  p.nchunks = (int)(p.ld_bytes / CHUNK_BYTES);
  p.qtiles = qp / BQ;
  p.ntiles = np / BN;
  p.splits = split_target / p.qtiles;
  if (p.splits < 1) p.splits = 1;
  if (p.splits > p.ntiles) p.splits = p.ntiles;
  const bool resident_query = p.ld_bytes <= 2 * CHUNK_BYTES;
  p.map = make_tile_map(p.qtiles, p.splits, group > 0 ? group : (resident_query ? 1 : 4));
  p.tstride = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 g((unsigned)p.map.grid), blk(WG);
  const int eng = tile_engine<__bf16>(p.ld_bytes);
  if (eng == 2) ceiling_sweep_kernel<__bf16, 2><<<g, blk, 0, s>>>(p, out);
  else if (eng == 1) ceiling_sweep_kernel<__bf16, 1><<<g, blk, 0, s>>>(p, out);
  else ceiling_sweep_kernel<__bf16, 0><<<g, blk, 0, s>>>(p, out);
  return (int)hipGetLastError();
}
