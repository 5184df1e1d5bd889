// Sample aggregation (Sec. 2.1): C[pc][stall][latency] over valid records.
//
// Device-wide atomics on MI355X retire far slower than HBM streams records,
// and Zipf-distributed PCs serialize them on hot bins, so the histogram is
// built by partitioning the records into buckets of kBucketPCs consecutive
// PCs whose 512 x 24 bins fit in LDS, reading the records once:
//   k_hsample     every kSampleStride-th tile: bucket sizes, scaled up, give
//                 each bucket a region of the payload array (capacity with
//                 head-room and slack; k_hregions lays them out);
//   k_partition   per tile of kTile records: an LDS counting sort by bucket,
//                 one device atomic per (tile, bucket) reserving room in the
//                 bucket's region, and the runs written as 2-byte payloads
//                 (pc offset in bucket, stall, latency bit); a run that does
//                 not fit goes to an overflow area as 4-byte keys;
//   k_count       per work item (a contiguous range of one bucket's region):
//                 LDS histogram of the bucket's bins, written once to the
//                 output (whole bucket) or to a partial slot;
//   k_merge       per split bucket: sum of its partial slots;
//   k_hoverflow   overflow keys added with integer atomics (only when a
//                 bucket outgrew its estimate).
// Integer sums are exact in any order, so the result does not depend on
// where runs land.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kHistThreads = 256;
constexpr int kTile = 16384;                    // records per tile
constexpr int kBatch = 16;                      // records per thread per batch (8 x 16 B loads)
constexpr int kBatches = kTile / (kHistThreads * kBatch);
constexpr int kBucketShift = 9;
constexpr int kBucketPCs = 1 << kBucketShift;   // 512 PCs -> 12288 bins = 48 KiB of LDS
constexpr int kBucketBins = kBucketPCs * 24;
constexpr int kMaxBuckets = 8192;
constexpr uint32_t kItemRecords = 1u << 17;     // records per counting work item
constexpr uint32_t kSampleStride = 32;          // one sampled tile in this many
constexpr uint32_t kBucketSlack = 4 * kTile;    // region slack per bucket, records

typedef unsigned long u64x2 __attribute__((ext_vector_type(2)));

struct TileTotals {
  uint32_t valid, latency, dropped, pad;
};

__device__ __forceinline__ bool rec_valid(uint64_t r, uint32_t n_instr) {
  const uint32_t pc = (uint32_t)r, hi = (uint32_t)(r >> 32);
  return pc < n_instr && (hi & 0xFFu) < 12u && ((hi >> 8) & 0xFEu) == 0u && (hi >> 16) == 0u;
}

// The tile's records in batches of kBatch per thread: record q of a batch
// sits at local index bt*4096 + (q/2)*512 + 2*tid + (q&1); two records per
// 16-byte load, 1 KiB contiguous per wave instruction.
template <bool VEC>
__device__ __forceinline__ void load_batch(const uint64_t *__restrict__ rec, uint64_t n,
                                           uint64_t base, int bt, uint64_t (&v)[kBatch]) {
  const unsigned tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kBatch / 2; ++j) {
    const uint64_t idx = base + (uint64_t)bt * 4096 + (uint64_t)j * 512 + 2 * tid;
    if (VEC && idx + 1 < n) {
      const u64x2 x = __builtin_nontemporal_load((const u64x2 *)(rec + idx));
      v[2 * j] = x.x;
      v[2 * j + 1] = x.y;
    } else {
      v[2 * j] = idx < n ? rec[idx] : 0ull;
      v[2 * j + 1] = idx + 1 < n ? rec[idx + 1] : 0ull;
    }
  }
}

__device__ __forceinline__ uint32_t local_index(int bt, int q) {
  return (uint32_t)bt * 4096u + (uint32_t)(q / 2) * 512u + 2u * threadIdx.x + (uint32_t)(q & 1);
}

// bucket sizes of every kSampleStride-th tile, added into est[]
template <bool VEC>
__global__ void __launch_bounds__(kHistThreads)
k_hsample(const uint64_t *__restrict__ rec, uint64_t n, uint32_t n_instr, uint32_t n_buckets,
          uint32_t *__restrict__ est) {
  extern __shared__ uint32_t cnt[];   // [n_buckets]
  const unsigned tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * kSampleStride * kTile;
  for (uint32_t b = tid; b < n_buckets; b += kHistThreads) cnt[b] = 0;
  __syncthreads();
#pragma unroll
  for (int bt = 0; bt < kBatches; ++bt) {
    uint64_t v[kBatch];
    load_batch<VEC>(rec, n, base, bt, v);
#pragma unroll
    for (int q = 0; q < kBatch; ++q)
      if (base + local_index(bt, q) < n && rec_valid(v[q], n_instr))
        atomicAdd(&cnt[(uint32_t)v[q] >> kBucketShift], 1u);
  }
  __syncthreads();
  for (uint32_t b = tid; b < n_buckets; b += kHistThreads)
    if (cnt[b]) atomicAdd(&est[b], cnt[b]);
}

// regions: capacity = estimate * 5/4 + slack per bucket, laid out in bucket
// order by one workgroup; cursors start at zero
__global__ void __launch_bounds__(kHistThreads)
k_hregions(uint32_t n_buckets, const uint32_t *__restrict__ est, uint32_t *__restrict__ cap,
           uint32_t *__restrict__ region, uint32_t *__restrict__ cursor) {
  __shared__ uint32_t tmp[kHistThreads / kWave + 1];
  const uint32_t per = (n_buckets + kHistThreads - 1) / kHistThreads;
  const uint32_t b0 = min(threadIdx.x * per, n_buckets), b1 = min(b0 + per, n_buckets);
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    const uint64_t e = (uint64_t)est[b] * kSampleStride;
    const uint32_t c = (uint32_t)min<uint64_t>(e + e / 4 + kBucketSlack, 0x40000000ull);
    cap[b] = c;
    sum += c;
  }
  uint32_t total;
  uint32_t run = block_excl_scan<kHistThreads>(sum, tmp, &total);
  for (uint32_t b = b0; b < b1; ++b) {
    region[b] = run;
    run += cap[b];
    cursor[b] = 0;
  }
}

template <bool VEC>
__global__ void __launch_bounds__(kHistThreads)
k_partition(const uint64_t *__restrict__ rec, uint64_t n, uint32_t n_instr, uint32_t n_buckets,
            const uint32_t *__restrict__ cap, const uint32_t *__restrict__ region,
            uint32_t *__restrict__ cursor, uint16_t *__restrict__ payload,
            uint32_t *__restrict__ ov_keys, uint32_t *__restrict__ ov_count,
            TileTotals *__restrict__ tile_tot) {
  extern __shared__ uint32_t smem[];
  uint32_t *cnt = smem;                                   // [n_buckets + 1]
  uint32_t *dst = cnt + n_buckets + 1;                    // [n_buckets] where each run goes
  uint32_t *staged = dst + n_buckets;                     // [kTile]: bucket << 16 | payload
  __shared__ uint32_t scan_tmp[kHistThreads / kWave + 1];
  __shared__ uint32_t red[3];
  const unsigned tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  for (uint32_t b = tid; b <= n_buckets; b += kHistThreads) cnt[b] = 0;
  if (tid < 3) red[tid] = 0;
  __syncthreads();
  uint32_t rank[kTile / kHistThreads];
  uint32_t my_lat = 0, my_drop = 0;
#pragma unroll
  for (int bt = 0; bt < kBatches; ++bt) {
    uint64_t v[kBatch];
    load_batch<VEC>(rec, n, base, bt, v);
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      uint32_t rk = 0xFFFFFFFFu;
      if (base + local_index(bt, q) < n) {
        if (rec_valid(v[q], n_instr)) {
          const uint32_t pc = (uint32_t)v[q], hi = (uint32_t)(v[q] >> 32);
          const uint32_t b = pc >> kBucketShift;
          const uint32_t pl = ((pc & (kBucketPCs - 1)) << 5) | ((hi & 0xFFu) * 2u + ((hi >> 8) & 1u));
          rk = (b << 16) | atomicAdd(&cnt[b], 1u);
          staged[local_index(bt, q)] = pl;   // parked; moved to its sorted slot below
          my_lat += (hi >> 8) & 1u;
        } else {
          ++my_drop;
        }
      }
      rank[bt * kBatch + q] = rk;
    }
  }
  my_lat = wave_sum(my_lat);
  my_drop = wave_sum(my_drop);
  if (lane_id() == 0) {
    atomicAdd(&red[1], my_lat);
    atomicAdd(&red[2], my_drop);
  }
  __syncthreads();
  // room for each run: a device atomic per non-empty bucket of the tile
  for (uint32_t b = tid; b < n_buckets; b += kHistThreads) {
    const uint32_t c = cnt[b];
    uint32_t d = 0;
    if (c) {
      const uint32_t pos = atomicAdd(&cursor[b], c);
      if (pos + c <= cap[b]) d = region[b] + pos;
      else d = 0x80000000u | atomicAdd(ov_count, c);   // overflow area, 4-byte keys
    }
    dst[b] = d;
  }
  __syncthreads();
  // exclusive scan of the bucket counts
  {
    const uint32_t per = (n_buckets + kHistThreads - 1) / kHistThreads;
    const uint32_t b0 = min(tid * per, n_buckets), b1 = min(b0 + per, n_buckets);
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; ++b) sum += cnt[b];
    uint32_t total;
    uint32_t run = block_excl_scan<kHistThreads>(sum, scan_tmp, &total);
    for (uint32_t b = b0; b < b1; ++b) {
      const uint32_t c = cnt[b];
      cnt[b] = run;
      run += c;
    }
    if (tid == 0) cnt[n_buckets] = total;
  }
  __syncthreads();
  // move every parked payload to its sorted slot; parked and sorted slots
  // share [0, kTile), so every parked value is read before any is moved
  uint32_t val[kTile / kHistThreads];
#pragma unroll
  for (int bt = 0; bt < kBatches; ++bt)
#pragma unroll
    for (int q = 0; q < kBatch; ++q)
      val[bt * kBatch + q] = (rank[bt * kBatch + q] != 0xFFFFFFFFu) ? staged[local_index(bt, q)] : 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTile / kHistThreads; ++k) {
    if (rank[k] != 0xFFFFFFFFu) {
      const uint32_t b = rank[k] >> 16;
      staged[cnt[b] + (rank[k] & 0xFFFFu)] = (b << 16) | val[k];
    }
  }
  __syncthreads();
  const uint32_t nvalid = cnt[n_buckets];
  for (uint32_t k = tid; k < nvalid; k += kHistThreads) {
    const uint32_t x = staged[k];
    const uint32_t b = x >> 16;
    const uint32_t d = dst[b];
    if (!(d & 0x80000000u)) payload[d + (k - cnt[b])] = (uint16_t)x;
    else ov_keys[(d & 0x7FFFFFFFu) + (k - cnt[b])] = x;
  }
  if (tid == 0) {
    TileTotals t;
    t.valid = nvalid;
    t.latency = red[1];
    t.dropped = red[2];
    t.pad = 0;
    tile_tot[blockIdx.x] = t;
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

// per bucket: its start and fill in the payload array, and its work items
__global__ void k_bucket_plan(uint32_t n_buckets, const uint32_t *region, const uint32_t *cursor,
                              const uint32_t *cap, uint32_t *bstart, uint32_t *bfill,
                              uint32_t *items) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_buckets;
       b += gridDim.x * blockDim.x) {
    const uint32_t fill = min(cursor[b], cap[b]);
    bstart[b] = region[b];
    bfill[b] = fill;
    const uint32_t r = (fill + kItemRecords - 1) / kItemRecords;
    items[b] = r < 1 ? 1 : r;
  }
}

// work item -> (bucket, part) via the prefix of items per bucket
__global__ void __launch_bounds__(kHistThreads)
k_count(const uint16_t *__restrict__ payload, const uint32_t *__restrict__ bstart,
        const uint32_t *__restrict__ bfill, uint32_t n_buckets, uint32_t n_instr,
        const uint32_t *__restrict__ items, const uint32_t *__restrict__ item_start,
        uint32_t *__restrict__ counts, uint32_t *__restrict__ partial) {
  __shared__ uint32_t bins[kBucketBins];
  const uint32_t it = blockIdx.x;
  const uint32_t total_items = item_start[n_buckets - 1] + items[n_buckets - 1];
  if (it >= total_items) return;
  const uint32_t b = upper_index_u32(item_start, 0, n_buckets, it);
  const uint32_t parts = items[b], part = it - item_start[b];
  const uint32_t s0 = bstart[b];
  const uint32_t fill = bfill[b];
  const uint32_t q0 = s0 + (uint32_t)((uint64_t)fill * part / parts);
  const uint32_t q1 = s0 + (uint32_t)((uint64_t)fill * (part + 1) / parts);
  for (uint32_t k = threadIdx.x; k < kBucketBins; k += kHistThreads) bins[k] = 0;
  __syncthreads();
  uint32_t q = q0 + threadIdx.x;
  for (; q + 3 * kHistThreads < q1; q += 4 * kHistThreads) {
    const uint32_t p0 = payload[q], p1 = payload[q + kHistThreads];
    const uint32_t p2 = payload[q + 2 * kHistThreads], p3 = payload[q + 3 * kHistThreads];
    atomicAdd(&bins[(p0 >> 5) * 24u + (p0 & 31u)], 1u);
    atomicAdd(&bins[(p1 >> 5) * 24u + (p1 & 31u)], 1u);
    atomicAdd(&bins[(p2 >> 5) * 24u + (p2 & 31u)], 1u);
    atomicAdd(&bins[(p3 >> 5) * 24u + (p3 & 31u)], 1u);
  }
  for (; q < q1; q += kHistThreads) {
    const uint32_t pl = payload[q];
    atomicAdd(&bins[(pl >> 5) * 24u + (pl & 31u)], 1u);
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

// grid (bucket, slice of kHistThreads bins): each thread sums one bin over
// the bucket's parts, four loads in flight
__global__ void __launch_bounds__(kHistThreads)
k_merge(const uint32_t *__restrict__ partial, const uint32_t *__restrict__ items,
        const uint32_t *__restrict__ item_start, uint32_t n_instr, uint32_t *__restrict__ counts) {
  const uint32_t b = blockIdx.x;
  const uint32_t parts = items[b];
  if (parts == 1) return;
  const uint32_t pc0 = b * kBucketPCs;
  const uint32_t npc = min((uint32_t)kBucketPCs, n_instr - pc0);
  const uint32_t k = blockIdx.y * kHistThreads + threadIdx.x;
  if (k >= npc * 24u) return;
  const uint32_t *src = partial + (size_t)item_start[b] * kBucketBins + k;
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  uint32_t p = 0;
  for (; p + 3 < parts; p += 4) {
    s0 += src[(size_t)p * kBucketBins];
    s1 += src[(size_t)(p + 1) * kBucketBins];
    s2 += src[(size_t)(p + 2) * kBucketBins];
    s3 += src[(size_t)(p + 3) * kBucketBins];
  }
  for (; p < parts; ++p) s0 += src[(size_t)p * kBucketBins];
  counts[(size_t)pc0 * 24u + k] = (s0 + s1) + (s2 + s3);
}

// keys of runs that did not fit their bucket's region (bucket << 16 | payload)
__global__ void k_hoverflow(const uint32_t *__restrict__ ov_keys, const uint32_t *__restrict__ ov_count,
                            uint32_t *__restrict__ counts) {
  const uint32_t n = *ov_count;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const uint32_t x = ov_keys[k];
    const uint32_t pc = (x >> 16) * kBucketPCs + ((x & 0xFFFFu) >> 5);
    atomicAdd(&counts[(size_t)pc * 24u + (x & 31u)], 1u);
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
  if (n >= 0x40000000ull) fail(GPA_E_UNSUPPORTED, "at most 2^30 samples in one call");
  const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
  const uint64_t *rec = (const uint64_t *)samples;
  const bool vec = ((uintptr_t)samples % 16) == 0;
  // bucket regions from a sample of the tiles
  const uint32_t n_samp = (n_tiles + kSampleStride - 1) / kSampleStride;
  uint32_t *est = ar.get<uint32_t>(n_buckets), *cap = ar.get<uint32_t>(n_buckets);
  uint32_t *region = ar.get<uint32_t>(n_buckets), *cursor = ar.get<uint32_t>(n_buckets);
  uint32_t *ov_count = ar.get<uint32_t>(1);
  GPA_HIP(hipMemsetAsync(est, 0, 4 * (size_t)n_buckets, s));
  GPA_HIP(hipMemsetAsync(ov_count, 0, 4, s));
  const size_t lds_count = (size_t)n_buckets * 4;
  if (vec)
    hipLaunchKernelGGL(k_hsample<true>, dim3(n_samp), dim3(kHistThreads), lds_count, s, rec, n,
                       n_instr, n_buckets, est);
  else
    hipLaunchKernelGGL(k_hsample<false>, dim3(n_samp), dim3(kHistThreads), lds_count, s, rec, n,
                       n_instr, n_buckets, est);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hregions, dim3(1), dim3(kHistThreads), 0, s, n_buckets, est, cap, region,
                     cursor);
  GPA_LAUNCH_CHECK();
  // the regions hold at most 5/4 of the scaled sample plus the slack
  const uint64_t max_region = (uint64_t)n_samp * kTile * kSampleStride * 5 / 4 +
                              (uint64_t)n_buckets * (kBucketSlack + 1);
  uint16_t *payload = ar.get<uint16_t>(max_region);
  uint32_t *ov_keys = ar.get<uint32_t>(n);
  TileTotals *tt = ar.get<TileTotals>(n_tiles);
  const size_t lds_part = (2 * (size_t)n_buckets + 1) * 4 + (size_t)kTile * 4;
  if (vec) {
    GPA_HIP(hipFuncSetAttribute((const void *)k_partition<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_part));
    hipLaunchKernelGGL(k_partition<true>, dim3(n_tiles), dim3(kHistThreads), lds_part, s, rec, n,
                       n_instr, n_buckets, cap, region, cursor, payload, ov_keys, ov_count, tt);
  } else {
    GPA_HIP(hipFuncSetAttribute((const void *)k_partition<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_part));
    hipLaunchKernelGGL(k_partition<false>, dim3(n_tiles), dim3(kHistThreads), lds_part, s, rec, n,
                       n_instr, n_buckets, cap, region, cursor, payload, ov_keys, ov_count, tt);
  }
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hist_totals, dim3(1), dim3(kHistThreads), 0, s, tt, n_tiles, totals);
  uint32_t *bstart = ar.get<uint32_t>(n_buckets), *bfill = ar.get<uint32_t>(n_buckets);
  uint32_t *items = ar.get<uint32_t>(n_buckets);
  uint32_t *item_start = ar.get<uint32_t>(n_buckets);
  hipLaunchKernelGGL(k_bucket_plan, dim3(grid_for(n_buckets, 256, 64)), dim3(256), 0, s,
                     n_buckets, region, cursor, cap, bstart, bfill, items);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(items, item_start, n_buckets, s, ar);
  // items <= one per bucket plus one per kItemRecords records
  const uint64_t max_items = n_buckets + n / kItemRecords + 1;
  uint32_t *partial = ar.get<uint32_t>((size_t)max_items * kBucketBins);
  hipLaunchKernelGGL(k_count, dim3((unsigned)max_items), dim3(kHistThreads), 0, s, payload, bstart,
                     bfill, n_buckets, n_instr, items, item_start, counts, partial);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_merge, dim3(n_buckets, kBucketBins / kHistThreads), dim3(kHistThreads), 0,
                     s, partial, items, item_start, n_instr, counts);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hoverflow, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, ov_keys, ov_count,
                     counts);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
