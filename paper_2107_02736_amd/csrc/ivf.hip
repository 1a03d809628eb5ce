// Inverted-file index (the approximate nearest neighbours of the experiments,
// Sec. 5): k-means training, the list layout of the data rows, and the
// (cluster, query) pairs of a query batch.  The tile sweep over the inspected
// clusters and the refinement live with the other k-NN kernels.
//
// Clusters are stored as contiguous row ranges.  The stable order inside a
// cluster is the row index, obtained by a block histogram, a per-cluster scan
// over blocks and a block-local stable rank, so every layout is deterministic.
// In the tile layout each cluster is padded with empty rows to a multiple of
// the 128-row tile; an empty row has index -1.
#include "common.h"
#include "kernels.h"

namespace deann {

constexpr int IVF_HIST_ROWS = 1024;   // rows per histogram block
constexpr int IVF_SCAN_THREADS = 1024;

// Centroid l <- row floor(l n / n_l).
__global__ void kmeans_init_kernel(const float* __restrict__ X, int64_t n, int64_t d,
                                   int64_t L, float* __restrict__ C) {
  const int64_t l = blockIdx.x;
  const int64_t row = l * n / L;
  for (int64_t t = threadIdx.x; t < d; t += blockDim.x) C[l * d + t] = X[row * d + t];
}

// hist[b][l] = rows of block b in cluster l; out-of-range ids are counted in
// *skipped and left out.
__global__ void __launch_bounds__(WG)
list_hist_kernel(const int32_t* __restrict__ a, int64_t n, int64_t L, int32_t* __restrict__ hist,
                 int32_t* __restrict__ skipped) {
  extern __shared__ int32_t cnt[];   // [L]
  for (int64_t l = threadIdx.x; l < L; l += WG) cnt[l] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * IVF_HIST_ROWS;
  int bad = 0;
  for (int64_t i = r0 + threadIdx.x; i < n && i < r0 + IVF_HIST_ROWS; i += WG) {
    const int32_t l = a[i];
    if (l >= 0 && l < L) atomicAdd(&cnt[l], 1);
    else ++bad;
  }
  if (bad) atomicAdd(skipped, bad);
  __syncthreads();
  for (int64_t l = threadIdx.x; l < L; l += WG) hist[(int64_t)blockIdx.x * L + l] = cnt[l];
}

// Exclusive prefix of hist over blocks, per cluster; count[l] = cluster size.
__global__ void list_colscan_kernel(int32_t* __restrict__ hist, int64_t B, int64_t L,
                                    int32_t* __restrict__ count) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  int32_t run = 0;
  for (int64_t b = 0; b < B; ++b) {
    const int32_t v = hist[b * L + l];
    hist[b * L + l] = run;
    run += v;
  }
  count[l] = run;
}

// off = exclusive prefix of count (off[L] = total); poff the same over the
// sizes rounded up to `pad` (one workgroup).
__global__ void __launch_bounds__(IVF_SCAN_THREADS)
list_offsets_kernel(const int32_t* __restrict__ count, int64_t L, int pad,
                    int32_t* __restrict__ off, int32_t* __restrict__ poff) {
  __shared__ int64_t s_a[IVF_SCAN_THREADS], s_b[IVF_SCAN_THREADS];
  const int64_t per = (L + IVF_SCAN_THREADS - 1) / IVF_SCAN_THREADS;
  const int64_t l0 = threadIdx.x * per, l1 = l0 + per < L ? l0 + per : L;
  int64_t a = 0, b = 0;
  for (int64_t l = l0; l < l1; ++l) {
    a += count[l];
    b += (count[l] + pad - 1) / pad * pad;
  }
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {   // serial scan of the 1024 partial sums
    int64_t ra = 0, rb = 0;
    for (int i = 0; i < IVF_SCAN_THREADS; ++i) {
      const int64_t va = s_a[i], vb = s_b[i];
      s_a[i] = ra;
      s_b[i] = rb;
      ra += va;
      rb += vb;
    }
    off[L] = (int32_t)ra;
    if (poff) poff[L] = (int32_t)rb;
  }
  __syncthreads();
  a = s_a[threadIdx.x];
  b = s_b[threadIdx.x];
  for (int64_t l = l0; l < l1; ++l) {
    off[l] = (int32_t)a;
    if (poff) poff[l] = (int32_t)b;
    a += count[l];
    b += (count[l] + pad - 1) / pad * pad;
  }
}

// ids[off[l] + rank] = i, where rank orders the rows of cluster l by index:
// rows of earlier blocks come first (hist prefix), inside a block the rows are
// taken in rounds of WG in index order.
__global__ void __launch_bounds__(WG)
list_scatter_kernel(const int32_t* __restrict__ a, int64_t n, int64_t L,
                    const int32_t* __restrict__ hist, const int32_t* __restrict__ off,
                    int32_t* __restrict__ ids) {
  extern __shared__ int32_t base[];   // [L] next slot of each cluster in this block
  __shared__ int32_t lab[WG];
  for (int64_t l = threadIdx.x; l < L; l += WG)
    base[l] = off[l] + hist[(int64_t)blockIdx.x * L + l];
  const int64_t r0 = (int64_t)blockIdx.x * IVF_HIST_ROWS;
  for (int64_t s = r0; s < n && s < r0 + IVF_HIST_ROWS; s += WG) {
    const int64_t i = s + threadIdx.x;
    const bool in = i < n && i < r0 + IVF_HIST_ROWS;
    int32_t l = in ? a[i] : -1;
    if (l >= L) l = -1;
    lab[threadIdx.x] = l;
    __syncthreads();   // also publishes base[] on the first round
    int rank = 0;
    if (l >= 0)
      for (int j = 0; j < (int)threadIdx.x; ++j) rank += lab[j] == l;
    const int32_t slot = l >= 0 ? base[l] + rank : 0;
    __syncthreads();
    if (l >= 0) {
      ids[slot] = (int32_t)i;
      atomicAdd(&base[l], 1);
    }
    __syncthreads();
  }
}

// Lloyd update: centroid l <- mean of its rows (FP64 sums, one rounding to
// float32); a cluster without rows keeps its centroid.  Workgroup (l, 64
// coordinates); its four waves sum the members j = j0 + w, j0 + w + 4, ... in
// order and the four partial sums are added in a fixed order, so the result
// does not depend on scheduling.
constexpr int MEAN_COLS = 64;
__global__ void __launch_bounds__(WG)
kmeans_mean_kernel(const float* __restrict__ X, int64_t d, const int32_t* __restrict__ ids,
                   const int32_t* __restrict__ off, const float* __restrict__ C_prev,
                   float* __restrict__ C_new) {
  __shared__ double part[WG / MEAN_COLS][MEAN_COLS];
  const int64_t l = blockIdx.x;
  const int64_t t = (int64_t)blockIdx.y * MEAN_COLS + (threadIdx.x % MEAN_COLS);
  const int ph = threadIdx.x / MEAN_COLS;
  const int32_t j0 = off[l], j1 = off[l + 1];
  double s = 0.0;
  if (t < d)
    for (int32_t j = j0 + ph; j < j1; j += WG / MEAN_COLS) s += (double)X[(int64_t)ids[j] * d + t];
  part[ph][threadIdx.x % MEAN_COLS] = s;
  __syncthreads();
  if (ph == 0 && t < d) {
    const int c = threadIdx.x;
    const double tot = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
    C_new[l * d + t] = j1 > j0 ? (float)(tot / (double)(j1 - j0)) : C_prev[l * d + t];
  }
}

// Padded row ids of the tile layout: cluster l occupies rows
// [poff[l], poff[l+1]), the first off[l+1]-off[l] of them real.
__global__ void list_pad_ids_kernel(const int32_t* __restrict__ ids, const int32_t* __restrict__ off,
                                    const int32_t* __restrict__ poff, int32_t* __restrict__ pids) {
  const int64_t l = blockIdx.x;
  const int32_t c = off[l + 1] - off[l];
  for (int32_t j = threadIdx.x; j < poff[l + 1] - poff[l]; j += blockDim.x)
    pids[poff[l] + j] = j < c ? ids[off[l] + j] : -1;
}

// out[r] = X[pids[r]] (zeros for empty rows); rows in [0, rows).
__global__ void gather_rows_kernel(const float* __restrict__ X, int64_t d,
                                   const int32_t* __restrict__ pids, const int32_t* __restrict__ nrows,
                                   int64_t cap, float* __restrict__ out) {
  const int64_t r = blockIdx.x;
  if (r >= cap) return;
  const int32_t src = r < *nrows ? pids[r] : -1;
  for (int64_t t = threadIdx.x; t < d; t += blockDim.x)
    out[r * d + t] = src >= 0 ? X[(int64_t)src * d + t] : 0.f;
}

// Empty rows get an infinite key norm so that no tile key selects them.
__global__ void empty_row_keys_kernel(const int32_t* __restrict__ pids,
                                      const int32_t* __restrict__ nrows, int64_t cap,
                                      float* __restrict__ xknorm) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= cap) return;
  if (r >= *nrows || pids[r] < 0) xknorm[r] = __builtin_inff();
}

// ---- query batch: (cluster, query) pairs ------------------------------------
// probe[q][kp]: inspected clusters of each query, the first np_q[q] valid.
// A workgroup takes PAIR_CHUNK consecutive (query, slot) entries and counts
// its pairs per cluster in LDS, so the global counters of the few clusters
// see one atomic per workgroup instead of one per pair.
constexpr int64_t PAIR_CHUNK = 16384;
__global__ void __launch_bounds__(WG)
pair_count_kernel(const int32_t* __restrict__ probe, int64_t total, int64_t kp,
                  const int32_t* __restrict__ np_q, int64_t L, int32_t* __restrict__ pcount) {
  extern __shared__ int32_t hist[];   // [L]
  for (int64_t l = threadIdx.x; l < L; l += WG) hist[l] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * PAIR_CHUNK;
  const int64_t i1 = i0 + PAIR_CHUNK < total ? i0 + PAIR_CHUNK : total;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += WG)
    if (i % kp < np_q[i / kp]) atomicAdd(&hist[probe[i]], 1);
  __syncthreads();
  for (int64_t l = threadIdx.x; l < L; l += WG)
    if (hist[l] != 0) atomicAdd(&pcount[l], hist[l]);
}

// Pair rows of cluster l: [pp[l], pp[l] + pcount[l]), padded to the tile.  A
// workgroup reserves one range of slots per cluster (one global atomic) and
// hands them out to its pairs from LDS; the order of pairs inside a cluster
// is unspecified.
__global__ void __launch_bounds__(WG)
pair_scatter_kernel(const int32_t* __restrict__ probe, int64_t total, int64_t kp,
                    const int32_t* __restrict__ np_q, int64_t L, const int32_t* __restrict__ pp,
                    int32_t* __restrict__ pfill, int32_t* __restrict__ pair_q,
                    int32_t* __restrict__ pair_of) {
  extern __shared__ int32_t hist[];   // [2L]: counts, then slot bases
  int32_t* base = hist + L;
  for (int64_t l = threadIdx.x; l < L; l += WG) hist[l] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * PAIR_CHUNK;
  const int64_t i1 = i0 + PAIR_CHUNK < total ? i0 + PAIR_CHUNK : total;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += WG)
    if (i % kp < np_q[i / kp]) atomicAdd(&hist[probe[i]], 1);
  __syncthreads();
  for (int64_t l = threadIdx.x; l < L; l += WG) {
    base[l] = hist[l] != 0 ? pp[l] + atomicAdd(&pfill[l], hist[l]) : 0;
    hist[l] = 0;
  }
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += WG) {
    if (i % kp >= np_q[i / kp]) continue;
    const int32_t l = probe[i];
    const int32_t row = base[l] + atomicAdd(&hist[l], 1);
    pair_q[row] = (int32_t)(i / kp);
    pair_of[i] = row;
  }
}

// Prepared query rows and key norms in pair order (zeros for padding rows),
// one row per workgroup in turn; rows from pp[L] on belong to no pair tile
// and are left unwritten.
constexpr int64_t PAIR_GATHER_WGS = 8192;
__global__ void pair_gather_kernel(const float* __restrict__ Ys, const float* __restrict__ yknorm,
                                   int64_t dp, const int32_t* __restrict__ pair_q,
                                   const int32_t* __restrict__ pp, int64_t L, int64_t cap,
                                   float* __restrict__ Yg, float* __restrict__ ygk) {
  const int64_t rows = (int64_t)pp[L] < cap ? (int64_t)pp[L] : cap;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int32_t qi = pair_q[r];
    for (int64_t t = threadIdx.x; t < dp; t += blockDim.x)
      Yg[r * dp + t] = qi >= 0 ? Ys[(int64_t)qi * dp + t] : 0.f;
    if (threadIdx.x == 0) ygk[r] = qi >= 0 ? yknorm[qi] : 0.f;
  }
}

// Parts of the pair tiles' sweeps.  Pair tile b (pair rows [128b, 128b+128))
// sweeps the tiles_b data tiles of its cluster; it is split into
// P_b = max(1, ceil(tiles_b / T)) parts of near-equal length, each with lists
// of its own, so that the longest workgroup of the scan is at most T tiles
// rather than the largest cluster.  T = max(PART_MIN, ceil(S / target),
// ceil(S / (budget - nb))) over the S tiles of all nb pair tiles keeps the parts
// at most budget: sum P_b <= nb + S / T (no tile is split when budget <= nb).
// lbase[b] is the first part of pair tile b, lbase[nb] = nparts[0] the number
// of parts; nparts[1] = T.
constexpr int64_t PART_MIN = 8;
__global__ void __launch_bounds__(IVF_SCAN_THREADS)
pair_parts_kernel(const int32_t* __restrict__ pp, const int32_t* __restrict__ poff, int64_t L,
                  int64_t budget, int64_t target, int32_t* __restrict__ lbase,
                  int32_t* __restrict__ nparts) {
  __shared__ int64_t red[IVF_SCAN_THREADS];
  __shared__ int32_t s[IVF_SCAN_THREADS];
  const int64_t nb = pp[L] / BN;
  auto tiles_of = [&](int64_t b) -> int64_t {   // the cluster l with pp[l] <= 128b < pp[l+1]
    int64_t lo = 0, hi = L;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)pp[mid] <= b * BN) lo = mid; else hi = mid;
    }
    return (int64_t)(poff[lo + 1] - poff[lo]) / BN;
  };
  int64_t acc = 0;
  for (int64_t b = threadIdx.x; b < nb; b += IVF_SCAN_THREADS) acc += tiles_of(b);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = IVF_SCAN_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const int64_t S = red[0];
  int64_t T = PART_MIN;
  if (target > 0 && (S + target - 1) / target > T) T = (S + target - 1) / target;
  const int64_t room = budget - nb;
  if (room <= 0) T = S + 1;   // no room for a second part anywhere
  else if ((S + room - 1) / room > T) T = (S + room - 1) / room;
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += IVF_SCAN_THREADS) {
    const int64_t b = c0 + threadIdx.x;
    const int64_t tb = b < nb ? tiles_of(b) : 0;
    const int32_t v = b < nb ? (int32_t)(tb > T ? (tb + T - 1) / T : 1) : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < IVF_SCAN_THREADS; off <<= 1) {
      const int32_t a = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    const int32_t incl = s[threadIdx.x], total = s[IVF_SCAN_THREADS - 1];
    __syncthreads();
    if (b < nb) lbase[b] = carry + incl - v;
    carry += total;
  }
  if (threadIdx.x == 0) {
    lbase[nb] = carry;
    nparts[0] = carry;
    nparts[1] = (int32_t)(T < 0x7fffffff ? T : 0x7fffffff);
  }
}

// ---- host launches -------------------------------------------------------------
int64_t ivf_hist_blocks(int64_t n) { return ceil_div(n, IVF_HIST_ROWS); }

hipError_t launch_kmeans_init(const float* X, int64_t n, int64_t d, int64_t L, float* C,
                              hipStream_t s) {
  kmeans_init_kernel<<<dim3((unsigned)L), dim3(128), 0, s>>>(X, n, d, L, C);
  return hipGetLastError();
}

hipError_t launch_list_layout(const int32_t* a, int64_t n, int64_t L, int32_t* hist,
                              int32_t* count, int32_t* off, int32_t* poff, int32_t* ids,
                              int32_t* skipped, hipStream_t s) {
  const int64_t B = ivf_hist_blocks(n);
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(skipped), 1, 0u, s);
  if (e != hipSuccess) return e;
  const size_t sm = (size_t)L * 4;
  list_hist_kernel<<<dim3((unsigned)B), dim3(WG), sm, s>>>(a, n, L, hist, skipped);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  list_colscan_kernel<<<dim3((unsigned)ceil_div(L, WG)), dim3(WG), 0, s>>>(hist, B, L, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  list_offsets_kernel<<<dim3(1), dim3(IVF_SCAN_THREADS), 0, s>>>(count, L, BN, off, poff);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  list_scatter_kernel<<<dim3((unsigned)B), dim3(WG), sm, s>>>(a, n, L, hist, off, ids);
  return hipGetLastError();
}

hipError_t launch_kmeans_mean(const float* X, int64_t d, const int32_t* ids, const int32_t* off,
                              int64_t L, const float* C_prev, float* C_new, hipStream_t s) {
  static_assert(WG / MEAN_COLS == 4, "four partial sums per coordinate");
  kmeans_mean_kernel<<<dim3((unsigned)L, (unsigned)ceil_div(d, MEAN_COLS)), dim3(WG), 0, s>>>(
      X, d, ids, off, C_prev, C_new);
  return hipGetLastError();
}

hipError_t launch_list_tiles(const float* X, int64_t d, const int32_t* ids, const int32_t* off,
                             const int32_t* poff, int64_t L, int64_t cap, int32_t* pids,
                             float* Xperm, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(pids), cap, 0xffffffffu, s);
  if (e != hipSuccess) return e;
  list_pad_ids_kernel<<<dim3((unsigned)L), dim3(WG), 0, s>>>(ids, off, poff, pids);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  gather_rows_kernel<<<dim3((unsigned)cap), dim3(128), 0, s>>>(X, d, pids, poff + L, cap, Xperm);
  return hipGetLastError();
}

hipError_t launch_empty_row_keys(const int32_t* pids, const int32_t* nrows, int64_t cap,
                                 float* xknorm, hipStream_t s) {
  empty_row_keys_kernel<<<dim3((unsigned)ceil_div(cap, WG)), dim3(WG), 0, s>>>(pids, nrows, cap,
                                                                            xknorm);
  return hipGetLastError();
}

hipError_t launch_pairs(const int32_t* probe, int64_t q, int64_t kp, const int32_t* np_q,
                        int64_t L, int32_t* pcount, int32_t* pfill, int32_t* pp, int32_t* pair_q,
                        int32_t* pair_of, int64_t cap, const float* Ys, const float* yknorm,
                        int64_t dp, float* Yg, float* ygk, hipStream_t s) {
  const int64_t total = q * kp;
  hipError_t e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(pcount), L, 0u, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(pfill), L, 0u, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(pair_q), cap, 0xffffffffu, s)) != hipSuccess)
    return e;
  const unsigned g = (unsigned)ceil_div(total, PAIR_CHUNK);
  const size_t sm = (size_t)L * 4;
  if (g > 0) pair_count_kernel<<<dim3(g), dim3(WG), sm, s>>>(probe, total, kp, np_q, L, pcount);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  list_offsets_kernel<<<dim3(1), dim3(IVF_SCAN_THREADS), 0, s>>>(pcount, L, BN, pfill, pp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // pfill held the unpadded prefix; reset it to count the slots
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(pfill), L, 0u, s)) != hipSuccess) return e;
  if (g > 0)
    pair_scatter_kernel<<<dim3(g), dim3(WG), 2 * sm, s>>>(probe, total, kp, np_q, L, pp, pfill,
                                                          pair_q, pair_of);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t gw = cap < PAIR_GATHER_WGS ? cap : PAIR_GATHER_WGS;
  if (gw == 0) return hipSuccess;
  pair_gather_kernel<<<dim3((unsigned)gw), dim3(128), 0, s>>>(Ys, yknorm, dp, pair_q, pp, L, cap,
                                                              Yg, ygk);
  return hipGetLastError();
}

hipError_t launch_pair_parts(const int32_t* pp, const int32_t* poff, int64_t L, int64_t budget,
                             int64_t target, int32_t* lbase, int32_t* nparts, hipStream_t s) {
  pair_parts_kernel<<<dim3(1), dim3(IVF_SCAN_THREADS), 0, s>>>(pp, poff, L, budget, target, lbase,
                                                                nparts);
  return hipGetLastError();
}

}  // namespace deann
