// Device exclusive prefix sum (u32), three phases: per-tile scan with tile
// totals, recursive scan of the totals, add-back.
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

__global__ void k_copy_last(const uint32_t *in, size_t n, uint32_t *last) { *last = in[n - 1]; }

__global__ void k_scan_total(const uint32_t *last, const uint32_t *out, size_t n,
                             unsigned long long *total) {
  *total = (unsigned long long)out[n - 1] + *last;
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n, hipStream_t s, Arena &ar,
                        unsigned long long *total_dev) {
  if (n == 0) {
    if (total_dev) {
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, total_dev);
      GPA_LAUNCH_CHECK();
    }
    return;
  }
  // the last input element is needed for the total after `out` overwrote it
  uint32_t *last = nullptr;
  if (total_dev) {
    last = ar.get<uint32_t>(1);
    hipLaunchKernelGGL(k_copy_last, dim3(1), dim3(1), 0, s, in, n, last);
    GPA_LAUNCH_CHECK();
  }
  size_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, in, out, n, nullptr);
    GPA_LAUNCH_CHECK();
  } else {
    uint32_t *sums = ar.get<uint32_t>(tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       sums);
    GPA_LAUNCH_CHECK();
    exclusive_scan_u32(sums, sums, tiles, s, ar, nullptr);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, n, sums);
    GPA_LAUNCH_CHECK();
  }
  if (total_dev) {
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, s, last, out, n, total_dev);
    GPA_LAUNCH_CHECK();
  }
}

}  // namespace gpa
