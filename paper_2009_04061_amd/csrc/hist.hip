// Sample aggregation (Sec. 2.1): C[pc][stall][latency] over valid records.
//
// Device-wide atomics on MI355X retire far slower than HBM streams records,
// and Zipf-distributed PCs serialize them on hot bins, so the histogram is
// built without them:
//   k_partition   one workgroup per tile of kTile records: validity check,
//                 LDS counting sort by PC bucket (kBucketPCs consecutive PCs),
//                 the tile's valid records written back as 2-byte payloads
//                 (pc offset in bucket, stall, latency bit) grouped by bucket,
//                 plus the tile's bucket offsets and its totals;
//   k_bucket_plan per bucket: records over all tiles, number of work items;
//   k_count       one workgroup per work item (a bucket and a range of tiles):
//                 LDS histogram of the bucket's 512 x 24 bins, written once to
//                 the output (single item) or to a partial slot;
//   k_merge       per split bucket: sum of its partial slots.
// Every output bin is written exactly once; integer sums are exact in any order.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kHistThreads = 256;
constexpr int kTile = 16384;                    // records per partition tile (u16 offsets)
constexpr int kPerThread = kTile / kHistThreads;
constexpr int kBucketShift = 9;
constexpr int kBucketPCs = 1 << kBucketShift;   // 512 PCs -> 12288 bins = 48 KiB of LDS
constexpr int kBucketBins = kBucketPCs * 24;
constexpr int kMaxBuckets = 8192;
constexpr uint32_t kItemRecords = 1u << 16;     // target records per counting work item

struct TileTotals {
  uint32_t valid, latency, dropped, pad;
};

__global__ void __launch_bounds__(kHistThreads)
k_partition(const uint64_t *__restrict__ rec, uint64_t n, uint32_t n_instr, uint32_t n_buckets,
            uint16_t *__restrict__ payload, uint16_t *__restrict__ tile_off,
            TileTotals *__restrict__ tile_tot) {
  extern __shared__ uint32_t smem[];
  uint32_t *cnt = smem;                                   // [n_buckets + 1]
  uint16_t *arrival = (uint16_t *)(smem + ((n_buckets + 4) & ~3u));
  uint16_t *sorted = arrival + kTile;
  __shared__ uint32_t scan_tmp[kHistThreads / kWave + 1];
  __shared__ uint32_t red[3];
  const unsigned tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  for (uint32_t b = tid; b <= n_buckets; b += kHistThreads) cnt[b] = 0;
  if (tid < 3) red[tid] = 0;
  __syncthreads();
  uint32_t rank[kPerThread];
  uint32_t my_valid = 0, my_lat = 0, my_drop = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const uint64_t idx = base + (uint64_t)k * kHistThreads + tid;
    rank[k] = 0xFFFFFFFFu;
    if (idx < n) {
      const uint64_t r = __builtin_nontemporal_load(&rec[idx]);
      const uint32_t lo = (uint32_t)r, hi = (uint32_t)(r >> 32);
      const uint32_t pc = lo, stall = hi & 0xFFu, flags = (hi >> 8) & 0xFFu, resv = hi >> 16;
      if (pc < n_instr && stall < 12u && (flags & ~1u) == 0u && resv == 0u) {
        const uint32_t b = pc >> kBucketShift;
        const uint32_t pl = ((pc & (kBucketPCs - 1)) << 5) | (stall * 2u + flags);
        const uint32_t rk = atomicAdd(&cnt[b], 1u);
        arrival[k * kHistThreads + tid] = (uint16_t)pl;
        rank[k] = (b << 16) | rk;
        my_valid += 1;
        my_lat += flags;
      } else {
        my_drop += 1;
      }
    }
  }
  // exclusive scan of the bucket counts (n_buckets <= kMaxBuckets)
  __syncthreads();
  {
    const uint32_t per = (n_buckets + kHistThreads - 1) / kHistThreads;
    const uint32_t b0 = tid * per, b1 = min(b0 + per, n_buckets);
    uint32_t s = 0;
    for (uint32_t b = b0; b < b1; ++b) s += cnt[b];
    uint32_t total;
    uint32_t run = block_excl_scan<kHistThreads>(s, scan_tmp, &total);
    for (uint32_t b = b0; b < b1; ++b) {
      uint32_t c = cnt[b];
      cnt[b] = run;
      run += c;
    }
    if (tid == 0) cnt[n_buckets] = total;
  }
  __syncthreads();
  uint16_t *toff = tile_off + (size_t)blockIdx.x * (n_buckets + 1);
  for (uint32_t b = tid; b <= n_buckets; b += kHistThreads) toff[b] = (uint16_t)cnt[b];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    if (rank[k] != 0xFFFFFFFFu) {
      const uint32_t b = rank[k] >> 16, rk = rank[k] & 0xFFFFu;
      sorted[cnt[b] + rk] = arrival[k * kHistThreads + tid];
    }
  }
  atomicAdd(&red[0], my_valid);
  atomicAdd(&red[1], my_lat);
  atomicAdd(&red[2], my_drop);
  __syncthreads();
  const uint32_t nvalid = cnt[n_buckets];
  uint16_t *out = payload + base;
  // coalesced write-back of the grouped payloads, two per 32-bit word
  const uint32_t *s32 = (const uint32_t *)sorted;
  uint32_t *o32 = (uint32_t *)out;
  for (uint32_t w = tid; w < (nvalid + 1) / 2; w += kHistThreads) o32[w] = s32[w];
  if (tid == 0) {
    TileTotals t;
    t.valid = red[0];
    t.latency = red[1];
    t.dropped = red[2];
    t.pad = 0;
    tile_tot[blockIdx.x] = t;
  }
}

// per bucket: records over all tiles and the number of counting items
__global__ void __launch_bounds__(kHistThreads)
k_bucket_plan(const uint16_t *__restrict__ tile_off, uint32_t n_tiles, uint32_t n_buckets,
              uint32_t *__restrict__ items) {
  __shared__ uint32_t red[kHistThreads / kWave];
  const uint32_t b = blockIdx.x;
  uint32_t s = 0;
  for (uint32_t t = threadIdx.x; t < n_tiles; t += kHistThreads) {
    const uint16_t *o = tile_off + (size_t)t * (n_buckets + 1);
    s += (uint32_t)o[b + 1] - (uint32_t)o[b];
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kHistThreads / kWave; ++w) tot += red[w];
    uint32_t r = (tot + kItemRecords - 1) / kItemRecords;
    if (r < 1) r = 1;
    if (r > n_tiles) r = n_tiles > 0 ? n_tiles : 1;
    items[b] = r;
  }
}

__global__ void k_hist_totals(const TileTotals *__restrict__ tt, uint32_t n_tiles,
                              unsigned long long *__restrict__ totals) {
  __shared__ unsigned long long red[3][kHistThreads / kWave];
  unsigned long long v = 0, l = 0, d = 0;
  for (uint32_t t = threadIdx.x; t < n_tiles; t += kHistThreads) {
    v += tt[t].valid;
    l += tt[t].latency;
    d += tt[t].dropped;
  }
  v = wave_sum(v);
  l = wave_sum(l);
  d = wave_sum(d);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = v;
    red[1][threadIdx.x / kWave] = l;
    red[2][threadIdx.x / kWave] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0, c = 0;
    for (int w = 0; w < kHistThreads / kWave; ++w) {
      a += red[0][w];
      b += red[1][w];
      c += red[2][w];
    }
    totals[0] = a;
    totals[1] = b;
    totals[2] = c;
    totals[3] = 0;
  }
}

// work item -> (bucket, part) via the prefix of items per bucket
__global__ void __launch_bounds__(kHistThreads)
k_count(const uint16_t *__restrict__ payload, const uint16_t *__restrict__ tile_off,
        uint32_t n_tiles, uint32_t n_buckets, uint32_t n_instr,
        const uint32_t *__restrict__ items, const uint32_t *__restrict__ item_start,
        uint32_t *__restrict__ counts, uint32_t *__restrict__ partial) {
  __shared__ uint32_t bins[kBucketBins];
  const uint32_t it = blockIdx.x;
  const uint32_t total_items = item_start[n_buckets - 1] + items[n_buckets - 1];
  if (it >= total_items) return;
  const uint32_t b = upper_index_u32(item_start, 0, n_buckets, it);
  const uint32_t parts = items[b], part = it - item_start[b];
  const uint32_t t0 = (uint32_t)((uint64_t)n_tiles * part / parts);
  const uint32_t t1 = (uint32_t)((uint64_t)n_tiles * (part + 1) / parts);
  for (uint32_t k = threadIdx.x; k < kBucketBins; k += kHistThreads) bins[k] = 0;
  __syncthreads();
  const unsigned w = threadIdx.x / kWave, lane = lane_id();
  constexpr unsigned kWaves = kHistThreads / kWave;
  for (uint32_t t = t0 + w; t < t1; t += kWaves) {
    const uint16_t *o = tile_off + (size_t)t * (n_buckets + 1);
    const uint32_t lo = o[b], hi = o[b + 1];
    const uint16_t *src = payload + (size_t)t * kTile;
    for (uint32_t q = lo + lane; q < hi; q += kWave) {
      const uint32_t pl = src[q];
      atomicAdd(&bins[(pl >> 5) * 24u + (pl & 31u)], 1u);
    }
  }
  __syncthreads();
  if (parts == 1) {
    const uint32_t pc0 = b * kBucketPCs;
    const uint32_t npc = min((uint32_t)kBucketPCs, n_instr - pc0);
    uint32_t *dst = counts + (size_t)pc0 * 24u;
    for (uint32_t k = threadIdx.x; k < npc * 24u; k += kHistThreads) dst[k] = bins[k];
  } else {
    uint32_t *dst = partial + (size_t)it * kBucketBins;
    for (uint32_t k = threadIdx.x; k < kBucketBins; k += kHistThreads) dst[k] = bins[k];
  }
}

__global__ void __launch_bounds__(kHistThreads)
k_merge(const uint32_t *__restrict__ partial, const uint32_t *__restrict__ items,
        const uint32_t *__restrict__ item_start, uint32_t n_instr, uint32_t *__restrict__ counts) {
  const uint32_t b = blockIdx.x;
  const uint32_t parts = items[b];
  if (parts == 1) return;
  const uint32_t pc0 = b * kBucketPCs;
  const uint32_t npc = min((uint32_t)kBucketPCs, n_instr - pc0);
  const uint32_t *src = partial + (size_t)item_start[b] * kBucketBins;
  for (uint32_t k = threadIdx.x; k < npc * 24u; k += kHistThreads) {
    uint32_t s = 0;
    for (uint32_t p = 0; p < parts; ++p) s += src[(size_t)p * kBucketBins + k];
    counts[(size_t)pc0 * 24u + k] = s;
  }
}

__global__ void k_hist_empty(uint32_t *counts, size_t nbins, unsigned long long *totals) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nbins;
       k += (size_t)gridDim.x * blockDim.x)
    counts[k] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 4) totals[threadIdx.x] = 0;
}

void run_hist(const gpa_program &p, const gpa_sample *samples, uint64_t n, uint32_t *counts,
              unsigned long long *totals, hipStream_t s, Arena &ar) {
  const uint32_t n_instr = p.n_instr;
  const uint32_t n_buckets = (n_instr + kBucketPCs - 1) / kBucketPCs;
  if (n_buckets > kMaxBuckets)
    fail(GPA_E_UNSUPPORTED, "histogram supports up to %d instructions", kMaxBuckets * kBucketPCs);
  if (n == 0) {
    hipLaunchKernelGGL(k_hist_empty, dim3(grid_for((size_t)n_instr * 24, 256, 4096)), dim3(256), 0,
                       s, counts, (size_t)n_instr * 24, totals);
    GPA_LAUNCH_CHECK();
    return;
  }
  const uint64_t n_tiles64 = (n + kTile - 1) / kTile;
  if (n_tiles64 > 0x7FFFFFFFull) fail(GPA_E_UNSUPPORTED, "too many samples in one call");
  const uint32_t n_tiles = (uint32_t)n_tiles64;
  uint16_t *payload = ar.get<uint16_t>(n_tiles64 * kTile);
  uint16_t *tile_off = ar.get<uint16_t>((size_t)n_tiles * (n_buckets + 1));
  TileTotals *tt = ar.get<TileTotals>(n_tiles);
  const size_t lds = (size_t)((n_buckets + 4) & ~3u) * 4 + 2 * (size_t)kTile * 2;
  GPA_HIP(hipFuncSetAttribute((const void *)k_partition, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  hipLaunchKernelGGL(k_partition, dim3(n_tiles), dim3(kHistThreads), lds, s,
                     (const uint64_t *)samples, n, n_instr, n_buckets, payload, tile_off, tt);
  GPA_LAUNCH_CHECK();
  uint32_t *items = ar.get<uint32_t>(n_buckets);
  uint32_t *item_start = ar.get<uint32_t>(n_buckets);
  hipLaunchKernelGGL(k_bucket_plan, dim3(n_buckets), dim3(kHistThreads), 0, s, tile_off, n_tiles,
                     n_buckets, items);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hist_totals, dim3(1), dim3(kHistThreads), 0, s, tt, n_tiles, totals);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(items, item_start, n_buckets, s, ar);
  // upper bound on the number of items: one per bucket plus one per kItemRecords records
  const uint64_t max_items = n_buckets + n / kItemRecords + 1;
  uint32_t *partial = ar.get<uint32_t>((size_t)max_items * kBucketBins);
  hipLaunchKernelGGL(k_count, dim3((unsigned)max_items), dim3(kHistThreads), 0, s, payload,
                     tile_off, n_tiles, n_buckets, n_instr, items, item_start, counts, partial);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_merge, dim3(n_buckets), dim3(kHistThreads), 0, s, partial, items,
                     item_start, n_instr, counts);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
