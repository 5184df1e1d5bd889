// Device exclusive prefix sum (u32).  Up to kSingleTile elements: one
// workgroup, one launch, the total written by the same kernel.  Up to
// kDirectTiles tiles: tile totals, then each tile adds the totals before it
// (read from L2) to its own scan (two launches).  Beyond: per-tile scans
// with tile totals, the scan of the totals (which also gives the grand
// total), add-back.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, size_t n,
             uint32_t *__restrict__ tile_sums) {
  __shared__ uint32_t smem[kScanThreads / kWave + 1];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_excl_scan<kScanThreads>(s, smem, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_add(uint32_t *__restrict__ out, size_t n, const uint32_t *__restrict__ tile_off) {
  const size_t base = (size_t)blockIdx.x * kScanTile;
  const uint32_t add = tile_off[blockIdx.x];
  for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
    if (base + k < n) out[base + k] += add;
}

// tile totals only
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const uint32_t *__restrict__ in, size_t n, uint32_t *__restrict__ tile_sums) {
  __shared__ uint32_t red[kScanThreads / kWave];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += (base + k < n) ? in[base + k] : 0u;
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    tile_sums[blockIdx.x] = t;
  }
}

constexpr size_t kDirectTiles = 4096;

// the tile's scan plus the totals of the tiles before it; the last tile
// writes the grand total
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, size_t n,
             const uint32_t *__restrict__ tile_sums, unsigned long long *__restrict__ total_dev) {
  __shared__ uint32_t smem[kScanThreads / kWave + 1];
  __shared__ uint32_t red[kScanThreads / kWave];
  __shared__ uint32_t s_off;
  uint32_t before = 0;
  for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kScanThreads) before += tile_sums[t];
  before = wave_sum(before);
  if (lane_id() == 0) red[threadIdx.x / kWave] = before;
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    s_off = t;
  }
  uint32_t total;
  uint32_t run = block_excl_scan<kScanThreads>(s, smem, &total) + s_off;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    *total_dev = (unsigned long long)s_off + total;
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

constexpr int kSingleThreads = 1024;
constexpr int kSingleItems = 16;
constexpr int kSingleTile = kSingleThreads * kSingleItems;

// in and out may be the same array: every element is read before it is
// written, within the tile that holds it
__global__ void __launch_bounds__(kSingleThreads)
k_scan_single(const uint32_t *in, uint32_t *out, uint32_t n, unsigned long long *total) {
  __shared__ uint32_t smem[kSingleThreads / kWave + 1];
  uint32_t carry = 0;
  for (uint32_t t0 = 0; t0 < n; t0 += kSingleTile) {
    const uint32_t base = t0 + threadIdx.x * kSingleItems;
    uint32_t v[kSingleItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kSingleItems; ++k) {
      v[k] = (base + k < n) ? in[base + k] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_excl_scan<kSingleThreads>(sum, smem, &tot);
#pragma unroll
    for (int k = 0; k < kSingleItems; ++k) {
      if (base + k < n) out[base + k] = run;
      run += v[k];
    }
    carry += tot;
    __syncthreads();   // smem is reused by the next tile's scan
  }
  if (total && threadIdx.x == 0) *total = carry;
}

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n, hipStream_t s, Arena &ar,
                        unsigned long long *total_dev) {
  if (n == 0) {
    if (total_dev) {
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, total_dev);
      GPA_LAUNCH_CHECK();
    }
    return;
  }
  if (n <= (size_t)kSingleTile) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kSingleThreads), 0, s, in, out, (uint32_t)n,
                       total_dev);
    GPA_LAUNCH_CHECK();
    return;
  }
  const size_t tiles = (n + kScanTile - 1) / kScanTile;
  uint32_t *sums = ar.get<uint32_t>(tiles);
  if (tiles <= kDirectTiles) {
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n, sums);
    GPA_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       sums, total_dev);
    GPA_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                     sums);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(sums, sums, tiles, s, ar, total_dev);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, n, sums);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
