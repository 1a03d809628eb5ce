// Near/far form of the exact KDE.  Algorithm 1 splits a query's kernel sum
// into the k nearest rows, summed exactly, and the remaining rows; here the
// remaining rows are not sampled but summed in full by the 16-bit tile sweep
// of Eq. (1), which leaves out the (query, row) pairs of the neighbours.  So
// the largest kernel values are exact (FP64 from the float32 rows) and only
// the far rows carry the 16-bit operand error.
//
// This file lists, per (query tile, data tile), the neighbour pairs that fall
// into that tile: a CSR over the keys (query / 128) * ntiles + row / 128 with
// one 16-bit entry (query mod 128) << 7 | (row mod 128) per pair.  Entries of
// one key are in no particular order; the tile sweep turns them into a set of
// masked elements, so its result does not depend on that order.
#include "common.h"
#include "kernels.h"

namespace deann {

constexpr int SCAN_WG = 256;
constexpr int SCAN_ITEMS = 16;                        // consecutive elements per thread
constexpr int64_t SCAN_BLOCK = SCAN_WG * SCAN_ITEMS;  // elements per block

// cnt[key] += 1 per (query, neighbour) pair; rows outside [0, n) are skipped.
__global__ void hyb_count_kernel(const int32_t* __restrict__ nn, int64_t q, int64_t k, int64_t n,
                                 int64_t ntiles, int32_t* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= q * k) return;
  const int32_t r = nn[t];
  if (r < 0 || r >= n) return;
  atomicAdd(&cnt[(t / k / BQ) * ntiles + r / BN], 1);
}

// Inclusive prefix within one block of SCAN_BLOCK elements, written to
// out[i + 1]; the block total goes to tot[block].
__global__ void __launch_bounds__(SCAN_WG)
scan_block_kernel(const int32_t* __restrict__ in, int64_t count, int32_t* __restrict__ out,
                  int32_t* __restrict__ tot) {
  __shared__ int32_t s[SCAN_WG];
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    run += base + i < count ? in[base + i] : 0;
    v[i] = run;
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < SCAN_WG; off <<= 1) {   // inclusive scan of the thread totals
    const int32_t a = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += a;
    __syncthreads();
  }
  const int32_t before = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < count) out[base + i + 1] = v[i] + before;
  if (threadIdx.x == SCAN_WG - 1) tot[blockIdx.x] = s[SCAN_WG - 1];
}

// Exclusive prefix of the block totals, in place (one workgroup).
__global__ void __launch_bounds__(1024) scan_totals_kernel(int32_t* __restrict__ tot, int64_t nb) {
  __shared__ int32_t s[1024];
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t j = c0 + threadIdx.x;
    const int32_t v = j < nb ? tot[j] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t a = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    const int32_t incl = s[threadIdx.x], total = s[1023];
    __syncthreads();
    if (j < nb) tot[j] = carry + incl - v;
    carry += total;
  }
}

__global__ void scan_add_kernel(int32_t* __restrict__ out, int64_t count,
                                const int32_t* __restrict__ tot) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) out[0] = 0;
  if (j < count) out[j + 1] += tot[j / SCAN_BLOCK];
}

// hits[off[key] + slot] = entry; cnt counts down to zero as the slots fill.
__global__ void hyb_scatter_kernel(const int32_t* __restrict__ nn, int64_t q, int64_t k, int64_t n,
                                   int64_t ntiles, const int32_t* __restrict__ off,
                                   int32_t* __restrict__ cnt, uint16_t* __restrict__ hits) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= q * k) return;
  const int32_t r = nn[t];
  if (r < 0 || r >= n) return;
  const int64_t qi = t / k;
  const int64_t key = (qi / BQ) * ntiles + r / BN;
  const int32_t slot = atomicSub(&cnt[key], 1) - 1;
  hits[off[key] + slot] = (uint16_t)(((qi % BQ) << 7) | (r % BN));
}

int64_t scan_blocks(int64_t count) { return ceil_div(count, SCAN_BLOCK); }

hipError_t launch_hybrid_hits(const int32_t* nn, int64_t q, int64_t k, int64_t n, int64_t qtiles,
                              int64_t ntiles, int32_t* cnt, int32_t* off, int32_t* tot,
                              uint16_t* hits, hipStream_t s) {
  const int64_t keys = qtiles * ntiles, pairs = q * k;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), keys, 0u, s);
  if (e != hipSuccess || keys == 0) return e;
  const unsigned gp = (unsigned)ceil_div(pairs, 256);
  if (pairs > 0) {
    hyb_count_kernel<<<dim3(gp), dim3(256), 0, s>>>(nn, q, k, n, ntiles, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int64_t nb = scan_blocks(keys);
  scan_block_kernel<<<dim3((unsigned)nb), dim3(SCAN_WG), 0, s>>>(cnt, keys, off, tot);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  scan_totals_kernel<<<dim3(1), dim3(1024), 0, s>>>(tot, nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  scan_add_kernel<<<dim3((unsigned)ceil_div(keys, 256)), dim3(256), 0, s>>>(off, keys, tot);
  if ((e = hipGetLastError()) != hipSuccess || pairs == 0) return e;
  hyb_scatter_kernel<<<dim3(gp), dim3(256), 0, s>>>(nn, q, k, n, ntiles, off, cnt, hits);
  return hipGetLastError();
}

}  // namespace deann
