// Sample aggregation (Sec. 2.1): C[pc][stall][latency] over valid records.
//
// Device-wide atomics on MI355X retire far slower than HBM streams records,
// and Zipf-distributed PCs serialize them on hot bins, so the histogram is
// built by partitioning the records into buckets of kBucketPCs consecutive
// PCs whose 512 x 24 bins fit in LDS, reading the records once:
//   k_hsample     every kSampleStride-th slice of records: bucket sizes;
//   k_hregions    one workgroup lays out kSubs sub-regions per bucket in the
//                 payload array (scaled estimate with head-room and slack)
//                 and clears their cursors;
//   k_partition   per tile of kTile records: an LDS counting sort by bucket,
//                 one device atomic per (tile, bucket) reserving room in one
//                 of the bucket's sub-regions, and the runs written as 2-byte
//                 payloads (pc offset in bucket, stall, latency bit); a run
//                 that does not fit goes to an overflow area as 4-byte keys;
//   k_hplan       one workgroup sums the tile totals and plans the counting
//                 work items (a range of one bucket's filled sub-regions,
//                 taken end to end);
//   k_count       per work item: LDS histogram of the bucket's bins, written
//                 once to the output (whole bucket) or to a partial slot;
//   k_merge       per split bucket: sum of its partial slots;
//   k_hoverflow   overflow keys added with integer atomics (only when a
//                 bucket outgrew its estimate).
// Integer sums are exact in any order, so the result does not depend on
// where runs land.  (A last-workgroup-does-the-rest scheme would save the
// small launches, but the device-scope fence it needs in every workgroup
// costs far more on this part.)
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kHistThreads = 256;
constexpr int kTile = 8192;                     // records per tile
constexpr int kBatch = 16;                      // records per thread per batch (8 x 16 B loads)
constexpr int kBatches = kTile / (kHistThreads * kBatch);
constexpr int kBucketShift = 9;
constexpr int kBucketPCs = 1 << kBucketShift;   // 512 PCs -> 12288 bins = 48 KiB of LDS
constexpr int kBucketBins = kBucketPCs * 24;
constexpr int kMaxBuckets = 8192;
constexpr uint32_t kItemRecords = 1u << 17;     // records per counting work item
constexpr uint32_t kSampleStride = 32;          // one sampled slice in this many
constexpr uint32_t kSampleSlice = 512;          // records per sampled slice
constexpr int kCountThreads = 1024;
// Each bucket's region is split into kSubs sub-regions, tile t reserving in
// sub-region t % kSubs, so that no cursor takes more than 1/kSubs of the
// tiles' device atomics; cursors sit kCursorStride words apart (one line
// each).  Word 1 of a cursor's line holds the start of the first run that
// did not fit: runs are reserved in position order, so the sub-region is
// written exactly up to there (or up to the cursor when nothing overflowed).
constexpr uint32_t kSubs = 8;
constexpr uint32_t kCursorStride = 32;
constexpr uint32_t kSubSlack = kTile;           // region slack per sub-region, records

typedef unsigned long u64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct TileTotals {
  uint32_t valid, latency, dropped, pad;
};

__device__ __forceinline__ bool rec_valid(uint64_t r, uint32_t n_instr) {
  const uint32_t pc = (uint32_t)r, hi = (uint32_t)(r >> 32);
  return pc < n_instr && (hi & 0xFFu) < 12u && ((hi >> 8) & 0xFEu) == 0u && (hi >> 16) == 0u;
}

// The tile's records in batches of kBatch per thread: record q of a batch
// sits at local index bt*4096 + (q/2)*512 + 2*tid + (q&1); two records per
// 16-byte load, 1 KiB contiguous per wave instruction.  FULL: the whole tile
// is in range and 16-byte aligned; otherwise every record is bounds-checked.
template <bool FULL>
__device__ __forceinline__ void load_batch(const uint64_t *__restrict__ rec, uint64_t n,
                                           uint64_t base, int bt, uint64_t (&v)[kBatch]) {
  const unsigned tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kBatch / 2; ++j) {
    const uint64_t idx = base + (uint64_t)bt * 4096 + (uint64_t)j * 512 + 2 * tid;
    if (FULL) {
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

// where record (bt, q) of a thread is parked in LDS before the sort: any
// one-to-one map onto [0, kTile) serves; consecutive lanes take consecutive
// words, so the parking stores and loads are free of bank conflicts
__device__ __forceinline__ uint32_t park_index(int bt, int q) {
  return (uint32_t)(bt * kBatch + q) * kHistThreads + threadIdx.x;
}

// sub-regions: capacity = estimate / kSubs * 5/4 + slack, laid out in
// (bucket, sub-region) order by one workgroup; cursors start at zero
__device__ void lay_out_regions(uint32_t n_buckets, const uint32_t *est, uint32_t *cap,
                                uint32_t *region, uint32_t *cursor) {
  __shared__ uint32_t tmp[kHistThreads / kWave + 1];
  const uint32_t per = (n_buckets + kHistThreads - 1) / kHistThreads;
  const uint32_t b0 = min(threadIdx.x * per, n_buckets), b1 = min(b0 + per, n_buckets);
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    uint64_t e = 0;
    for (uint32_t u = 0; u < kSubs; ++u) e += est[(b * kSubs + u) * kCursorStride];
    e = e * kSampleStride / kSubs;
    const uint32_t c = (uint32_t)min<uint64_t>(e + e / 4 + kSubSlack, 0x10000000ull);
    for (uint32_t u = 0; u < kSubs; ++u) cap[b * kSubs + u] = c;
    sum += c * kSubs;
  }
  uint32_t total;
  uint32_t run = block_excl_scan<kHistThreads>(sum, tmp, &total);
  for (uint32_t b = b0; b < b1; ++b)
    for (uint32_t u = 0; u < kSubs; ++u) {
      region[b * kSubs + u] = run;
      run += cap[b * kSubs + u];
      cursor[(b * kSubs + u) * kCursorStride] = 0;
      cursor[(b * kSubs + u) * kCursorStride + 1] = 0xFFFFFFFFu;
    }
}

// bucket sizes of every kSampleStride-th slice of kSampleSlice records
// (two records per thread), added into the workgroup's copy of est[] (one of
// kSubs copies, kCursorStride words apart, so that the atomics spread)
__global__ void __launch_bounds__(kHistThreads)
k_hsample(const uint64_t *__restrict__ rec, uint64_t n, uint32_t n_instr, uint32_t n_buckets,
          uint32_t *__restrict__ est) {
  extern __shared__ uint32_t cnt[];   // [n_buckets]
  const unsigned tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * kSampleStride * kSampleSlice;
  for (uint32_t b = tid; b < n_buckets; b += kHistThreads) cnt[b] = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint64_t i = base + 2 * tid + q;
    if (i < n) {
      const uint64_t v = rec[i];
      if (rec_valid(v, n_instr)) atomicAdd(&cnt[(uint32_t)v >> kBucketShift], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = tid; b < n_buckets; b += kHistThreads)
    if (cnt[b]) atomicAdd(&est[(b * kSubs + blockIdx.x % kSubs) * kCursorStride], cnt[b]);
}

__global__ void __launch_bounds__(kHistThreads)
k_hregions(uint32_t n_buckets, const uint32_t *__restrict__ est, uint32_t *__restrict__ cap,
           uint32_t *__restrict__ region, uint32_t *__restrict__ cursor) {
  lay_out_regions(n_buckets, est, cap, region, cursor);
}

// totals = {valid, latency, dropped, 0} over the tiles, by one workgroup
__device__ void sum_tile_totals(const TileTotals *tt, uint32_t n_tiles,
                                unsigned long long *totals) {
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

// per sub-region: how far it is filled; per bucket: the total fill, the
// number of work items and the first item's index, by one workgroup
__device__ void plan_items(uint32_t n_buckets, const uint32_t *cursor, const uint32_t *cap,
                           uint32_t *sfill, uint32_t *bfill, uint32_t *items,
                           uint32_t *item_start) {
  __shared__ uint32_t tmp[kHistThreads / kWave + 1];
  const uint32_t per = (n_buckets + kHistThreads - 1) / kHistThreads;
  const uint32_t b0 = min(threadIdx.x * per, n_buckets), b1 = min(b0 + per, n_buckets);
  uint32_t my_items = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    uint32_t fill = 0;
    for (uint32_t u = 0; u < kSubs; ++u) {
      const uint32_t slot = b * kSubs + u;
      const uint32_t f = min(min(cursor[slot * kCursorStride], cap[slot]),
                             cursor[slot * kCursorStride + 1]);
      sfill[slot] = f;
      fill += f;
    }
    bfill[b] = fill;
    const uint32_t r = (fill + kItemRecords - 1) / kItemRecords;
    items[b] = r < 1 ? 1 : r;
    my_items += r < 1 ? 1 : r;
  }
  uint32_t total;
  uint32_t run = block_excl_scan<kHistThreads>(my_items, tmp, &total);
  for (uint32_t b = b0; b < b1; ++b) {
    item_start[b] = run;
    run += items[b];
  }
}

// LDS words k_partition needs beyond its static arrays
__host__ __device__ constexpr size_t partition_lds_words(uint32_t n_buckets) {
  return 2 * (size_t)n_buckets + 2 + kTile + kWave;
}

template <bool VEC>
__global__ void __launch_bounds__(kHistThreads)
k_partition(const uint64_t *__restrict__ rec, uint64_t n, uint32_t n_instr, uint32_t n_buckets,
            const uint32_t *__restrict__ cap, const uint32_t *__restrict__ region,
            uint32_t *__restrict__ cursor, uint16_t *__restrict__ payload,
            uint32_t *__restrict__ ov_keys, uint32_t *__restrict__ ov_count,
            TileTotals *__restrict__ tile_tot) {
  extern __shared__ uint32_t smem[];
  // cnt: one counter per bucket, then two sink counters: records that fail
  // validation (bucket n_buckets) and records past the end (n_buckets + 1)
  uint32_t *cnt = smem;                                   // [n_buckets + 2]
  uint32_t *dst = cnt + n_buckets + 2;                    // [n_buckets] run destination - run start
  uint32_t *staged = dst + n_buckets;                     // [kTile + kWave], tail = sink slots
  __shared__ uint32_t scan_tmp[kHistThreads / kWave + 1];
  __shared__ uint32_t s_lat, s_ovf, s_total;
  const unsigned tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  const uint32_t lim = (uint32_t)min<uint64_t>(n - base, (uint64_t)kTile);
  for (uint32_t b = tid; b < n_buckets + 2; b += kHistThreads) cnt[b] = 0;
  if (tid == 0) {
    s_lat = 0;
    s_ovf = 0;
  }
  __syncthreads();
  // every load of the tile is issued before any record is ranked
  uint64_t vb[kBatches][kBatch];
  if (VEC && lim == (uint32_t)kTile) {
#pragma unroll
    for (int bt = 0; bt < kBatches; ++bt) load_batch<true>(rec, n, base, bt, vb[bt]);
  } else {
#pragma unroll
    for (int bt = 0; bt < kBatches; ++bt) load_batch<false>(rec, n, base, bt, vb[bt]);
  }
  // rank of each record within its bucket (or sink); branch-free per record
  uint32_t rank[kTile / kHistThreads];
  uint32_t my_lat = 0;
#pragma unroll
  for (int bt = 0; bt < kBatches; ++bt) {
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const uint64_t r = vb[bt][q];
      const uint32_t pc = (uint32_t)r, hi = (uint32_t)(r >> 32);
      const bool in = local_index(bt, q) < lim;
      const bool ok = in & rec_valid(r, n_instr);
      const uint32_t b = ok ? (pc >> kBucketShift) : (in ? n_buckets : n_buckets + 1);
      rank[bt * kBatch + q] = (b << 16) | atomicAdd(&cnt[b], 1u);
      // parked; moved to its sorted slot below
      staged[park_index(bt, q)] = ((pc & (kBucketPCs - 1)) << 5) | ((hi & 0xFFu) * 2u + ((hi >> 8) & 1u));
      my_lat += ok ? (hi >> 8) & 1u : 0u;
    }
  }
  my_lat = wave_sum(my_lat);
  if (lane_id() == 0) atomicAdd(&s_lat, my_lat);
  __syncthreads();
  // room for each run: a device atomic per non-empty bucket of the tile, in
  // the tile's sub-region of the bucket
  const uint32_t sub = blockIdx.x % kSubs;
  uint32_t any_ovf = 0;
  for (uint32_t b = tid; b < n_buckets; b += kHistThreads) {
    const uint32_t c = cnt[b];
    uint32_t d = 0;
    if (c) {
      const uint32_t slot = b * kSubs + sub;
      const uint32_t pos = atomicAdd(&cursor[slot * kCursorStride], c);
      if (pos + c <= cap[slot]) {
        d = region[slot] + pos;
      } else {
        d = 0x80000000u | atomicAdd(ov_count, c);   // overflow area, 4-byte keys
        any_ovf = 1;
        atomicMin(&cursor[slot * kCursorStride + 1], pos);
      }
    }
    dst[b] = d;
  }
  if (any_ovf) s_ovf = 1;
  __syncthreads();   // the scan below rewrites cnt[] and dst[] of other threads' buckets
  // exclusive scan of the bucket counts; dst[] becomes destination minus
  // run start, so that tile slot k of bucket b goes to dst[b] + k
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
      dst[b] -= run;
      run += c;
    }
    if (tid == 0) s_total = total;
  }
  __syncthreads();
  // move every parked payload to its sorted slot; parked and sorted slots
  // share [0, kTile), so every parked value is read before any is moved;
  // sink records go to the spare slots past kTile
  uint32_t val[kTile / kHistThreads];
#pragma unroll
  for (int bt = 0; bt < kBatches; ++bt)
#pragma unroll
    for (int q = 0; q < kBatch; ++q) val[bt * kBatch + q] = staged[park_index(bt, q)];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTile / kHistThreads; ++k) {
    const uint32_t b = rank[k] >> 16;
    const uint32_t slot = b < n_buckets ? cnt[b] + (rank[k] & 0xFFFFu) : (uint32_t)kTile + lane_id();
    staged[slot] = (b << 16) | val[k];
  }
  __syncthreads();
  const uint32_t nvalid = s_total;
  if (!s_ovf) {
    uint32_t k = tid;
    for (; k + 3 * kHistThreads < nvalid; k += 4 * kHistThreads) {
      const uint32_t x0 = staged[k], x1 = staged[k + kHistThreads];
      const uint32_t x2 = staged[k + 2 * kHistThreads], x3 = staged[k + 3 * kHistThreads];
      payload[dst[x0 >> 16] + k] = (uint16_t)x0;
      payload[dst[x1 >> 16] + k + kHistThreads] = (uint16_t)x1;
      payload[dst[x2 >> 16] + k + 2 * kHistThreads] = (uint16_t)x2;
      payload[dst[x3 >> 16] + k + 3 * kHistThreads] = (uint16_t)x3;
    }
    for (; k < nvalid; k += kHistThreads) {
      const uint32_t x = staged[k];
      payload[dst[x >> 16] + k] = (uint16_t)x;
    }
  } else {
    for (uint32_t k = tid; k < nvalid; k += kHistThreads) {
      const uint32_t x = staged[k];
      const uint32_t b = x >> 16;
      const uint32_t d = dst[b] + cnt[b];   // the run's destination
      if (!(d & 0x80000000u)) payload[d + (k - cnt[b])] = (uint16_t)x;
      else ov_keys[(d & 0x7FFFFFFFu) + (k - cnt[b])] = x;
    }
  }
  if (tid == 0) {
    TileTotals t;
    t.valid = nvalid;
    t.latency = s_lat;
    t.dropped = cnt[n_buckets];
    t.pad = 0;
    tile_tot[blockIdx.x] = t;
  }
}

// one workgroup: the totals over the tiles and the counting plan
__global__ void __launch_bounds__(kHistThreads)
k_hplan(const TileTotals *__restrict__ tt, uint32_t n_tiles, unsigned long long *__restrict__ totals,
        uint32_t n_buckets, const uint32_t *__restrict__ cursor, const uint32_t *__restrict__ cap,
        uint32_t *__restrict__ sfill, uint32_t *__restrict__ bfill, uint32_t *__restrict__ items,
        uint32_t *__restrict__ item_start) {
  sum_tile_totals(tt, n_tiles, totals);
  plan_items(n_buckets, cursor, cap, sfill, bfill, items, item_start);
}

// k_count's LDS bins: each 16-lane group of a wave adds into its own copy,
// so that a hot bin takes at most 16 same-address atomics per instruction;
// a copy holds the 12288 bins as 16-bit counters, bin k in the low half of
// word k when k < 6144, else in the high half of word k - 6144 (the two
// latency bins of a stall reason land in different words); copies start 16
// banks apart.  A copy receives a quarter of a work item's vector loads plus
// at most one partial round of them and the unaligned ends per sub-region,
// which stays below 2^16.
constexpr uint32_t kCountCopies = 4;
constexpr uint32_t kHalfWords = kBucketBins / 2;
constexpr uint32_t kCopyStride = kHalfWords + 16;
static_assert(kItemRecords / kCountCopies + kSubs * (2 * kCountThreads + 16) < 65536u,
              "16-bit counters of a copy must not carry");

__device__ __forceinline__ void count_one(uint32_t pl, uint32_t *bins) {
  const uint32_t k = (pl >> 5) * 24u + (pl & 31u);
  const bool hi = k >= kHalfWords;
  atomicAdd(&bins[hi ? k - kHalfWords : k], hi ? 0x10000u : 1u);
}

__device__ __forceinline__ void count_word(uint32_t w, uint32_t *bins) {
  count_one(w & 0xFFFFu, bins);
  count_one(w >> 16, bins);
}

// payload[q0, q1) into the thread's copy of the bins: the unaligned head and
// tail one by one, the rest as 16-byte loads (eight payloads), two per
// thread in flight
__device__ __forceinline__ void count_range(const uint16_t *__restrict__ payload, uint32_t q0,
                                            uint32_t q1, uint32_t *bins) {
  const uint32_t a = min(q1, (q0 + 7u) & ~7u);
  const uint32_t z = max(a, q1 & ~7u);
  for (uint32_t q = q0 + threadIdx.x; q < a; q += kCountThreads) count_one(payload[q], bins);
  for (uint32_t q = z + threadIdx.x; q < q1; q += kCountThreads) count_one(payload[q], bins);
  const u32x4 *vec = (const u32x4 *)(payload + a);
  const uint32_t nv = (z - a) / 8u;
  uint32_t k = threadIdx.x;
  for (; k + kCountThreads < nv; k += 2 * kCountThreads) {
    const u32x4 x = __builtin_nontemporal_load(vec + k);
    const u32x4 y = __builtin_nontemporal_load(vec + k + kCountThreads);
    count_word(x.x, bins);
    count_word(x.y, bins);
    count_word(x.z, bins);
    count_word(x.w, bins);
    count_word(y.x, bins);
    count_word(y.y, bins);
    count_word(y.z, bins);
    count_word(y.w, bins);
  }
  if (k < nv) {
    const u32x4 x = __builtin_nontemporal_load(vec + k);
    count_word(x.x, bins);
    count_word(x.y, bins);
    count_word(x.z, bins);
    count_word(x.w, bins);
  }
}

// work item -> (bucket, part) via the prefix of items per bucket
__global__ void __launch_bounds__(kCountThreads)
k_count(const uint16_t *__restrict__ payload, const uint32_t *__restrict__ region,
        const uint32_t *__restrict__ sfill, const uint32_t *__restrict__ bfill,
        uint32_t n_buckets, uint32_t n_instr,
        const uint32_t *__restrict__ items, const uint32_t *__restrict__ item_start,
        uint32_t *__restrict__ counts, uint32_t *__restrict__ partial) {
  __shared__ uint32_t bins[kCountCopies * kCopyStride];
  const uint32_t it = blockIdx.x;
  const uint32_t total_items = item_start[n_buckets - 1] + items[n_buckets - 1];
  if (it >= total_items) return;
  const uint32_t b = upper_index_u32(item_start, 0, n_buckets, it);
  const uint32_t parts = items[b], part = it - item_start[b];
  // the item's share [q0, q1) of the bucket's sub-regions taken end to end
  const uint32_t fill = bfill[b];
  const uint32_t q0 = (uint32_t)((uint64_t)fill * part / parts);
  const uint32_t q1 = (uint32_t)((uint64_t)fill * (part + 1) / parts);
  for (uint32_t k = threadIdx.x; k < kCountCopies * kCopyStride; k += kCountThreads) bins[k] = 0;
  __syncthreads();
  uint32_t *mine = bins + ((threadIdx.x >> 4) & (kCountCopies - 1)) * kCopyStride;
  uint32_t v = 0;
  for (uint32_t u = 0; u < kSubs; ++u) {
    const uint32_t slot = b * kSubs + u;
    const uint32_t f = sfill[slot];
    const uint32_t lo = max(q0, v), hi = min(q1, v + f);
    if (lo < hi) count_range(payload, region[slot] + (lo - v), region[slot] + (hi - v), mine);
    v += f;
  }
  __syncthreads();
  // bin k = sum over the copies of its 16-bit counter
  uint32_t *dst;
  uint32_t nbins;
  if (parts == 1) {
    const uint32_t pc0 = b * kBucketPCs;
    nbins = min((uint32_t)kBucketPCs, n_instr - pc0) * 24u;
    dst = counts + (size_t)pc0 * 24u;
  } else {
    nbins = kBucketBins;
    dst = partial + (size_t)it * kBucketBins;
  }
  for (uint32_t k = threadIdx.x; k < nbins; k += kCountThreads) {
    const bool hi = k >= kHalfWords;
    const uint32_t w = hi ? k - kHalfWords : k, sh = hi ? 16u : 0u;
    uint32_t t = 0;
#pragma unroll
    for (uint32_t c = 0; c < kCountCopies; ++c) t += (bins[c * kCopyStride + w] >> sh) & 0xFFFFu;
    dst[k] = t;
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

// ------------------------------------------------------------ hot-set path
// For programs of up to kHotMaxPCs instructions, a sample of the records
// picks a hot set of at most kHotH PCs.  One read of the records adds every
// hot record into a workgroup-private LDS copy of the hot bins (two 16-bit
// counters per word, as in the direct mode) and appends every other (cold)
// record as a 4-byte key to the workgroup's own slice of a key array.  A hot
// counter that wraps is caught from the atomic's returned value and its
// 65,536 (less the carry it pushed into its neighbour) added to a
// per-profile correction array: the only device atomics, at most a few per
// 2^16 records.  The workgroup then sorts its cold keys by bucket of
// kColdPCs PCs within tiles, and a last launch sums the packed hot copies
// with the corrections and counts each bucket's cold keys in LDS.  Hot and
// cold PCs are disjoint, so every bin is written exactly once.
//   k_hot_select  one workgroup: 16-bit LDS counters (one per PC, or per
//                 pair of PCs beyond 65,536) over kSelSample records in
//                 evenly spread runs; a counter that reaches kSelMin makes
//                 its PCs hot
//                 (first come, at most kHotH), each placed in one of two
//                 candidate slots of the lookup table;
//   k_hot_pass    one workgroup per contiguous range of records, which
//                 then sorts its cold keys by bucket in tiles of kColdTile;
//   k_hot_finish  cold buckets, hot-bin sums and the totals.
constexpr int kHotThreads = 1024;
constexpr uint32_t kHotH = 1024;                 // hot PCs at most
constexpr uint32_t kHotTBits = 12;
constexpr uint32_t kHotT = 1u << kHotTBits;      // lookup slots (load <= 1/4)
constexpr uint32_t kHotBins = kHotH * 24;        // hot bins (the merge's columns)
constexpr uint32_t kHotWords = kHotH * 12;       // packed: two 16-bit counters per word
constexpr uint32_t kHotMaxPCs = 1u << 17;        // cold keys pc << 5 | bin fit 22 bits
// table entries: pc | id << kPcBits; the pc field of an empty slot (all
// ones) is above every pc, and an id field of all ones marks a claim
constexpr uint32_t kPcBits = 18;
constexpr uint32_t kPcMask = (1u << kPcBits) - 1;
constexpr uint32_t kIdClaim = 0xFFFFFFFFu >> kPcBits;
static_assert(kHotMaxPCs < kPcMask && kHotH < kIdClaim, "table entry fields");
constexpr uint32_t kColdShift = 8;
constexpr uint32_t kColdPCs = 1u << kColdShift;  // PCs per cold bucket
constexpr uint32_t kColdBins = kColdPCs * 24;
constexpr uint32_t kColdMaxBuckets = kHotMaxPCs / kColdPCs;
constexpr uint32_t kColdTile = 16384;            // cold keys per sorted tile
constexpr uint32_t kSelSample = 32768;           // sampled records
constexpr uint32_t kSelRun = 128;                // records per sampled run
constexpr uint32_t kSelCounters = 1u << 16;      // 16-bit, two per word
constexpr uint32_t kSelMin = 2;                  // sampled count that makes a PC hot
constexpr int kHotUnroll = 4;                    // 16-byte loads per thread per step
constexpr uint32_t kHotStep = kHotThreads * kHotUnroll * 2;   // records per step
constexpr uint32_t kHotGrid = 256;               // workgroups of the pass at most
constexpr uint32_t kMaxRuns = 4096;              // cold runs listed at a time
constexpr uint32_t kMergeSlice = 16;             // partials one merging thread sums at most
constexpr uint32_t kMergeWords = 4;              // words one merging thread takes
static_assert(kHotGrid / kMergeSlice <= (uint32_t)kHotThreads && 2 * kHotThreads <= kColdPCs * 24,
              "merge slices and their LDS sums");
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
static_assert(kColdMaxBuckets <= (uint32_t)kHotThreads, "one cold bucket per thread in scans");
static_assert(kSelSample < 65536u, "16-bit sample counters");

// a hot PC sits in one of its two slots (entry pc | id << kPcBits), given by two
// multiplicative hashes of the pc (< 2^17 on this path) taken as 24-bit
// products, which issue at full rate where a 32-bit multiply takes four
// cycles (HIP's __umul24 returns int: the product is made unsigned before
// the shift)
static_assert(kHotMaxPCs <= (1u << 24), "24-bit hash operands");
__device__ __forceinline__ uint32_t hot_slot1(uint32_t pc) {
  return (uint32_t)__umul24(pc, 0x9E3779u) >> (32 - kHotTBits);
}
__device__ __forceinline__ uint32_t hot_slot2(uint32_t pc) {
  return ((uint32_t)__umul24(pc, 0x85EBCBu) + 0x6A09E667u) >> (32 - kHotTBits);
}
__device__ __forceinline__ uint32_t cold_bucket(uint32_t key) { return key >> (5 + kColdShift); }
__device__ __forceinline__ uint32_t cold_local_bin(uint32_t key) {
  return ((key >> 5) & (kColdPCs - 1)) * 24u + (key & 31u);
}

// LDS words of k_hot_select (dynamic): counters and the table
constexpr size_t kSelLdsWords = kSelCounters / 2 + kHotT;

// Direct mode: a program of at most kDirectPCs instructions keeps every bin
// of the pass workgroup in LDS, two 16-bit counters per word (bins 2w and
// 2w + 1 of word w = pc * 12 + stall), so there is no selection, no lookup
// and no cold key.  A counter that wraps is caught from the value the LDS
// atomic returns and logged (kind and word), and the workgroup's totals are
// rebuilt exactly at the end: with c_lo wraps of the low counter and c_hi of
// the high one (a carried low wrap adds 1 to the high counter, which can
// wrap it too), the word's final value W gives
//   low  = (W & 0xFFFF) + 65536 c_lo,
//   high = (W >> 16) + 65536 c_hi - c_lo.
// A wrap takes 65,536 additions to one counter since its last wrap, so a
// range of at most kDirectMaxPer records logs at most 2 * 64 + 1 events.
constexpr uint32_t kDirectPCs = 3072;
constexpr uint32_t kDirectWords = kDirectPCs * 12;
constexpr uint32_t kDirectMarks = kDirectWords / 32;
constexpr uint32_t kMaxEvents = 256;
constexpr uint64_t kDirectMaxPer = 1ull << 22;
static_assert(2 * (kDirectMaxPer >> 16) + 1 <= kMaxEvents, "event log bound");

// The pass's LDS: one pool laid out per mode.
//   hot/cold: hot bins, lookup table, the first cold tile, bucket counters,
//             scan scratch;
//   direct:   packed counters, wrap marks (one bit per word), the event log,
//             its count and reduction scratch.
constexpr uint32_t kHotPoolWords = kHotWords + kHotT + kColdTile + kColdMaxBuckets +
                                   kHotThreads / kWave + 1;
constexpr uint32_t kDirectPoolWords = kDirectWords + kDirectMarks + kMaxEvents + 1 +
                                      2 * (kHotThreads / kWave);
constexpr uint32_t kPassPoolWords =
    kHotPoolWords > kDirectPoolWords ? kHotPoolWords : kDirectPoolWords;
static_assert(kPassPoolWords * 4 + 64 <= 160u * 1024u, "the pass's LDS fits one CU");

// Everything one profile's hot-set histogram needs: its records and sizes,
// the pass's shape, its scratch and its outputs.  A launch for one profile
// takes it by value; a batched launch reads one per profile from a device
// table, each workgroup finding its profile and its block index within that
// profile's grid in a work list.
struct HotArgs {
  const uint64_t *rec;
  uint64_t n, per, run_stride;
  uint32_t n_instr, n_cb, G, T;
  uint32_t n_merge, merge_slices;   // hot-bin merge workgroups (0 when G = 1) and their slices
  uint32_t direct, pad;             // direct mode: every bin in LDS, no selection, no cold keys
  uint32_t *hot_tab, *hot_pc, *n_hot, *partial, *cold, *cold_sorted, *tile_off, *n_cold;
  uint32_t *corr;   // hot mode: kHotBins wrap corrections, cleared by the selection
  TileTotals *wtot;
  uint32_t *counts, *issued;
  unsigned long long *totals;
};

template <bool BATCH>
__device__ __forceinline__ void hot_item(const HotArgs &one, const HotArgs *many,
                                         const WorkItem *items, HotArgs &a, uint32_t &local) {
  if (BATCH) {
    const WorkItem it = items[blockIdx.x];
    a = many[it.entry];
    local = it.local;
  } else {
    a = one;
    local = blockIdx.x;
  }
}

// Sampled record k: k itself when n <= kSelSample, else offset k % kSelRun
// of run k / kSelRun, the runs run_stride apart
// ((kSelSample / kSelRun - 1) run_stride + kSelRun <= n).
template <bool BATCH>
__global__ void __launch_bounds__(kHotThreads)
k_hot_select(HotArgs one, const HotArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  HotArgs a;
  uint32_t local;
  hot_item<BATCH>(one, many, items, a, local);
  const uint64_t *__restrict__ rec = a.rec;
  const uint64_t n = a.n, run_stride = a.run_stride;
  const uint32_t n_instr = a.n_instr;
  uint32_t *__restrict__ hot_tab = a.hot_tab;
  uint32_t *__restrict__ hot_pc = a.hot_pc;
  uint32_t *__restrict__ n_hot = a.n_hot;
  extern __shared__ uint32_t sm[];
  uint32_t *cnt = sm, *tab = cnt + kSelCounters / 2;
  __shared__ uint32_t s_nsel;
  const unsigned tid = threadIdx.x;
  const uint32_t sh = n_instr > kSelCounters ? 1u : 0u;   // counter = pc >> sh
  // the sample in rounds of kPer records per thread (a round's loads issued
  // together, held in registers)
  constexpr uint32_t kPer = 16;
  constexpr uint32_t kRounds = kSelSample / (kPer * kHotThreads);
  static_assert(kRounds * kPer * kHotThreads == kSelSample, "whole rounds");
  uint64_t r[kPer];
  auto load = [&](uint32_t round) {
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint32_t k = (round * kPer + j) * kHotThreads + tid;
      const uint64_t i = n <= kSelSample ? k : (k / kSelRun) * run_stride + k % kSelRun;
      r[j] = i < n ? rec[i] : ~0ull;
    }
  };
  load(0);
  for (uint32_t k = tid; k < kSelCounters / 2; k += kHotThreads) cnt[k] = 0;
  for (uint32_t k = tid; k < kHotT; k += kHotThreads) tab[k] = kEmpty;
  if (tid == 0) s_nsel = 0;
  __syncthreads();
  for (uint32_t round = 0; round < kRounds; ++round) {
  if (round > 0) load(round);
  // a rolled loop: this kernel runs once per call, so its code is fetched
  // cold and a short body costs less than unrolled copies
#pragma unroll 1
  for (uint32_t j = 0; j < kPer; ++j) {
    if (!rec_valid(r[j], n_instr)) continue;
    const uint32_t c = (uint32_t)r[j] >> sh, half = 16 * (c & 1);
    const uint32_t old = (atomicAdd(&cnt[c >> 1], 1u << half) >> half) & 0xFFFFu;
    if (old + 1 != kSelMin) continue;
    // this sample made counter c reach kSelMin: its PCs become hot
    for (uint32_t pc = c << sh; pc < ((c + 1) << sh) && pc < n_instr; ++pc) {
      const uint32_t prov = pc | (kIdClaim << kPcBits);   // claimed, not yet numbered
      uint32_t slot = hot_slot1(pc);
      if (atomicCAS(&tab[slot], kEmpty, prov) != kEmpty) {
        slot = hot_slot2(pc);
        if (atomicCAS(&tab[slot], kEmpty, prov) != kEmpty) continue;   // stays cold
      }
      const uint32_t id = atomicAdd(&s_nsel, 1u);
      if (id < kHotH) {
        hot_pc[id] = pc;
        tab[slot] = pc | (id << kPcBits);
      } else {
        tab[slot] = kEmpty;   // the hot set is full: stays cold
      }
    }
  }
  }
  __syncthreads();
  for (uint32_t k = tid; k < kHotT; k += kHotThreads) hot_tab[k] = tab[k];
  if (tid == 0) *n_hot = min(s_nsel, kHotH);
  for (uint32_t k = tid; k < kHotBins; k += kHotThreads) a.corr[k] = 0;
}

// one step's records of a thread: FULL steps lie wholly below n (16-byte
// loads when VEC); otherwise the indices are clamped and the records past n
// zeroed (no branches, so that the loads are issued back to back)
template <bool VEC, bool FULL>
__device__ __forceinline__ void hot_load(const uint64_t *__restrict__ rec, uint64_t n, uint64_t i0,
                                         uint64_t (&v)[2 * kHotUnroll]) {
#pragma unroll
  for (int u = 0; u < kHotUnroll; ++u) {
    const uint64_t i = i0 + 2 * ((uint64_t)u * kHotThreads + threadIdx.x);
    if (FULL && VEC) {
      const u64x2 x = __builtin_nontemporal_load((const u64x2 *)(rec + i));
      v[2 * u] = x.x;
      v[2 * u + 1] = x.y;
    } else if (FULL) {
      v[2 * u] = rec[i];
      v[2 * u + 1] = rec[i + 1];
    } else {
      const uint64_t a = rec[min(i, n - 1)], b = rec[min(i + 1, n - 1)];
      v[2 * u] = i < n ? a : 0ull;
      v[2 * u + 1] = i + 1 < n ? b : 0ull;
    }
  }
}

// m <= kColdTile cold keys src[0, m) (in global memory, or in sorted[]
// itself: every key is in registers before sorted[] is written) sorted by
// bucket into cold_sorted[base, base + m); the bucket starts (absolute
// indices) to off[0, n_cb), the end to off[n_cb].  Every thread of the
// workgroup calls it; it ends on a barrier.
__device__ void sort_cold_tile(uint32_t n_cb, uint64_t base, uint32_t m, const uint32_t *src,
                               uint32_t *__restrict__ cold_sorted, uint32_t *__restrict__ off,
                               uint32_t *sorted, uint32_t *bc, uint32_t *scan_tmp) {
  const unsigned tid = threadIdx.x;
  constexpr uint32_t kPer = kColdTile / kHotThreads;
  uint32_t key[kPer];
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t k = j * kHotThreads + tid;
    key[j] = k < m ? src[k] : kEmpty;
  }
  for (uint32_t b = tid; b < n_cb; b += kHotThreads) bc[b] = 0;
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j)
    if (key[j] != kEmpty) atomicAdd(&bc[cold_bucket(key[j])], 1u);
  __syncthreads();
  {
    const uint32_t c = tid < n_cb ? bc[tid] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<kHotThreads>(c, scan_tmp, &total);
    if (tid < n_cb) {
      bc[tid] = ex;
      off[tid] = (uint32_t)(base + ex);
    }
    if (tid == 0) off[n_cb] = (uint32_t)(base + total);
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j)
    if (key[j] != kEmpty) sorted[atomicAdd(&bc[cold_bucket(key[j])], 1u)] = key[j];
  __syncthreads();
  for (uint32_t k = tid; k < m; k += kHotThreads) cold_sorted[base + k] = sorted[k];
  __syncthreads();
}

// Workgroup w reads records [w per, min((w + 1) per, n)) in steps of
// kHotStep (per is even; a last step that is not whole reads its records
// one by one, clamped), the loads of the next two steps in flight while a
// step is counted; its cold keys are appended in arrival order (one LDS
// reservation per wave and step), their number to n_cold[w]: the first
// kColdTile to the LDS array that the tile sort uses (idle until then), so
// that the first tile is sorted without a round trip through memory, and
// the rest to cold[] at their positions from index w per on.  Then the
// workgroup sorts its cold keys by bucket in tiles of kColdTile: tile t's
// bucket starts go to tile_off[(w T + t) (n_cb + 1) + b] (entry n_cb: the
// end).
// a hot counter wrapped (rare): the word's low counter is bin 2w of the hot
// bins, its high counter bin 2w + 1.  A low wrap loses 65,536 from the low
// counter and pushed a carry into the high one (which also wrapped if it
// held 0xFFFF); a high wrap loses 65,536 from the high counter.
__device__ __attribute__((noinline)) void hot_wrap(uint32_t *corr, uint32_t w, uint32_t sh,
                                                   uint32_t old) {
  if (sh == 0) {
    atomicAdd(&corr[2 * w], 65536u);
    atomicAdd(&corr[2 * w + 1], ((old >> 16) == 0xFFFFu ? 65536u : 0u) - 1u);
  } else {
    atomicAdd(&corr[2 * w + 1], 65536u);
  }
}

// a direct-mode counter wrapped (rare): log it and mark its word.  A low
// counter's wrap carried 1 into the high counter, which wrapped as well when
// it held 0xFFFF; entries are word << 1 | (1 for a high-counter wrap).
__device__ __attribute__((noinline)) void direct_wrap(uint32_t w, uint32_t sh, uint32_t old,
                                                      uint32_t *mark, uint32_t *evlog,
                                                      uint32_t *n_ev) {
  const uint32_t kinds = sh ? 2u : (1u | ((old >> 16) == 0xFFFFu ? 2u : 0u));
  for (uint32_t k = 1; k <= 2; k <<= 1) {
    if (!(kinds & k)) continue;
    const uint32_t i = atomicAdd(n_ev, 1u);
    if (i < kMaxEvents) evlog[i] = (w << 1) | (k >> 1);
  }
  atomicOr(&mark[w >> 5], 1u << (w & 31));
}

// Direct mode of the pass: records [wg per, min((wg + 1) per, n)) counted in
// LDS (two 16-bit counters per word), then the workgroup's exact bins and
// totals written: to the counts when the profile has one workgroup, else to
// its partial table (n_instr * 24, merged by the finish).
template <bool VEC>
__device__ void direct_pass(const HotArgs &a, uint32_t wg, uint32_t *pool) {
  const uint64_t *__restrict__ rec = a.rec;
  const uint64_t n = a.n, per = a.per;
  const uint32_t n_instr = a.n_instr, nw = a.n_instr * 12u;
  uint32_t *words = pool;
  uint32_t *mark = pool + kDirectWords;
  uint32_t *evlog = mark + kDirectMarks;
  uint32_t *n_ev = evlog + kMaxEvents;
  uint32_t *red = n_ev + 1;   // [2][kHotThreads / kWave]
  const unsigned tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  const uint64_t r0 = (uint64_t)wg * per, r1 = min(r0 + per, n);
  const uint64_t rf = r0 + (r1 - r0) / kHotStep * kHotStep;
  uint64_t va[2 * kHotUnroll], vb[2 * kHotUnroll], vc[2 * kHotUnroll];
  auto issue = [&](uint64_t i0, uint64_t (&v)[2 * kHotUnroll]) {
    if (i0 < rf) hot_load<VEC, true>(rec, r1, i0, v);
  };
  issue(r0, va);
  issue(r0 + kHotStep, vb);
  for (uint32_t k = tid; k < nw; k += kHotThreads) words[k] = 0;
  for (uint32_t k = tid; k < (nw + 31) / 32; k += kHotThreads) mark[k] = 0;
  if (tid == 0) *n_ev = 0;
  lds_barrier();
  auto step = [&](auto full, uint64_t i0, const uint64_t (&cur)[2 * kHotUnroll]) {
    constexpr bool FULL = decltype(full)::value;
#pragma unroll
    for (int q = 0; q < 2 * kHotUnroll; ++q) {
      const uint64_t r = cur[q];
      const uint32_t pc = (uint32_t)r, hi = (uint32_t)(r >> 32);
      bool ok = pc < n_instr && hi < 0x200u && (hi & 0xFFu) < 12u;   // rec_valid
      if (!FULL) ok = ok && i0 + 2 * ((uint64_t)(q / 2) * kHotThreads + tid) + (q & 1) < r1;
      if (ok) {
        const uint32_t w = (uint32_t)__umul24(pc, 12u) + (hi & 0xFFu);
        const uint32_t sh = (hi >> 4) & 16u;   // the latency bit selects the high counter
        const uint32_t old = atomicAdd(&words[w], 1u << sh);
        if (((old >> sh) & 0xFFFFu) == 0xFFFFu) direct_wrap(w, sh, old, mark, evlog, n_ev);
      }
    }
  };
  constexpr std::true_type kFull{};
  constexpr std::false_type kPart{};
  for (uint64_t i0 = r0; i0 < rf;) {
    issue(i0 + 2 * kHotStep, vc);
    step(kFull, i0, va);
    if ((i0 += kHotStep) >= rf) break;
    issue(i0 + 2 * kHotStep, va);
    step(kFull, i0, vb);
    if ((i0 += kHotStep) >= rf) break;
    issue(i0 + 2 * kHotStep, vb);
    step(kFull, i0, vc);
    i0 += kHotStep;
  }
  if (rf < r1) {
    hot_load<VEC, false>(rec, r1, rf, va);
    step(kPart, rf, va);
  }
  __syncthreads();
  const uint32_t nev = min(*n_ev, kMaxEvents);
  uint32_t *dst = a.G == 1 ? a.counts : a.partial + (size_t)wg * n_instr * 24u;
  uint32_t valid = 0, lat = 0;
  for (uint32_t w = tid; w < nw; w += kHotThreads) {
    const uint32_t W = words[w];
    uint32_t lo = W & 0xFFFFu, hi = W >> 16;
    if (nev && ((mark[w >> 5] >> (w & 31)) & 1u)) {
      uint32_t c_lo = 0, c_hi = 0;
      for (uint32_t e = 0; e < nev; ++e) {
        const uint32_t v = evlog[e];
        if ((v >> 1) == w) {
          c_hi += v & 1u;
          c_lo += (v & 1u) ^ 1u;
        }
      }
      lo += c_lo << 16;
      hi = hi + (c_hi << 16) - c_lo;
    }
    valid += lo + hi;
    lat += hi;
    *(uint2 *)(dst + 2 * (size_t)w) = make_uint2(lo, hi);
    if (a.G == 1 && w % 12u == GPA_ST_SELECTED) a.issued[w / 12u] = lo + hi;
  }
  valid = wave_sum(valid);
  lat = wave_sum(lat);
  if (lane == 0) {
    red[wv] = valid;
    red[kHotThreads / kWave + wv] = lat;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t v = 0, l = 0;
    for (uint32_t k = 0; k < kHotThreads / kWave; ++k) {
      v += red[k];
      l += red[kHotThreads / kWave + k];
    }
    const uint32_t dropped = (uint32_t)(r1 - r0) - v;
    if (a.G == 1) {
      a.totals[0] = v;
      a.totals[1] = l;
      a.totals[2] = dropped;
      a.totals[3] = 0;
    } else {
      TileTotals t;
      t.valid = v;
      t.latency = l;
      t.dropped = dropped;
      t.pad = 0;
      a.wtot[wg] = t;
    }
  }
}

template <bool VEC, bool BATCH>
__global__ void __launch_bounds__(kHotThreads)
k_hot_pass(HotArgs one, const HotArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  HotArgs a;
  uint32_t wg;
  hot_item<BATCH>(one, many, items, a, wg);
  __shared__ __align__(16) uint32_t pool[kPassPoolWords];
  if (a.direct) {
    direct_pass<VEC>(a, wg, pool);
    return;
  }
  const uint64_t *__restrict__ rec = a.rec;
  const uint64_t n = a.n, per = a.per;
  const uint32_t n_instr = a.n_instr, n_cb = a.n_cb, T = a.T;
  const uint32_t *__restrict__ hot_tab = a.hot_tab;
  uint32_t *__restrict__ cold = a.cold;
  uint32_t *__restrict__ cold_sorted = a.cold_sorted;
  uint32_t *__restrict__ tile_off = a.tile_off;
  uint32_t *__restrict__ n_cold = a.n_cold;
  TileTotals *__restrict__ wtot = a.wtot;
  uint32_t *bins = pool;                      // [kHotWords] packed hot counters
  uint32_t *tab = bins + kHotWords;           // [kHotT]
  uint32_t *sorted = tab + kHotT;             // [kColdTile]
  uint32_t *bc = sorted + kColdTile;          // [kColdMaxBuckets]
  uint32_t *scan_tmp = bc + kColdMaxBuckets;  // [kHotThreads / kWave + 1]
  __shared__ uint32_t s_cur, s_valid, s_lat;
  const unsigned tid = threadIdx.x, lane = lane_id();
  const uint64_t r0 = (uint64_t)wg * per, r1 = min(r0 + per, n);
  // full steps below rf, then at most one partial step; three register
  // buffers in rotation (the first two issued before the set-up)
  const uint64_t rf = r0 + (r1 - r0) / kHotStep * kHotStep;
  uint64_t va[2 * kHotUnroll], vb[2 * kHotUnroll], vc[2 * kHotUnroll];
  auto issue = [&](uint64_t i0, uint64_t (&v)[2 * kHotUnroll]) {
    if (i0 < rf) hot_load<VEC, true>(rec, r1, i0, v);
  };
  issue(r0, va);
  issue(r0 + kHotStep, vb);
  for (uint32_t k = tid; k < kHotWords; k += kHotThreads) bins[k] = 0;
  for (uint32_t k = tid; k < kHotT; k += kHotThreads) tab[k] = hot_tab[k];
  if (tid == 0) {
    s_cur = 0;
    s_valid = 0;
    s_lat = 0;
  }
  lds_barrier();
  uint32_t *my_cold = cold + r0;
  // the wave's valid and latency records, counted from ballots (uniform)
  uint32_t w_valid = 0, w_lat = 0;
  // FULL: a step wholly below r1 (no index check); the table slots are in
  // range for any pc, so the lookups need no validity branch
  auto step = [&](auto full, uint64_t i0, const uint64_t (&cur)[2 * kHotUnroll]) {
    constexpr bool FULL = decltype(full)::value;
    uint32_t cmask = 0;
#pragma unroll
    for (int q = 0; q < 2 * kHotUnroll; ++q) {
      const uint64_t r = cur[q];
      const uint32_t pc = (uint32_t)r, hi = (uint32_t)(r >> 32);
      bool ok = pc < n_instr && hi < 0x200u && (hi & 0xFFu) < 12u;   // rec_valid
      if (!FULL) ok = ok && i0 + 2 * ((uint64_t)(q / 2) * kHotThreads + tid) + (q & 1) < r1;
      const uint32_t e1 = tab[hot_slot1(pc)], e2 = tab[hot_slot2(pc)];
      const uint32_t e = (e1 & kPcMask) == pc ? e1 : e2;   // an empty slot matches no pc
      const bool hot = ok && (e & kPcMask) == pc;
      if (hot) {
        const uint32_t w = (e >> kPcBits) * 12u + (hi & 0xFFu);
        const uint32_t sh = (hi >> 4) & 16u;   // the latency bit selects the high counter
        const uint32_t old = atomicAdd(&bins[w], 1u << sh);
        if (((old >> sh) & 0xFFFFu) == 0xFFFFu) hot_wrap(a.corr, w, sh, old);
      }
      w_valid += (uint32_t)__popcll(__ballot(ok));
      w_lat += (uint32_t)__popcll(__ballot(ok && ((hi >> 8) & 1u)));
      cmask |= (ok && !hot) ? 1u << q : 0u;
    }
    // the step's cold keys: one LDS reservation per wave
    const uint32_t c = __popc(cmask);
    const uint32_t inc = wave_incl_scan(c);
    const uint32_t wt = __shfl(inc, kWave - 1, kWave);
    if (wt) {
      uint32_t pos = 0;
      if (lane == kWave - 1) pos = atomicAdd(&s_cur, wt);
      pos = __shfl(pos, kWave - 1, kWave) + inc - c;
#pragma unroll
      for (int q = 0; q < 2 * kHotUnroll; ++q)
        if ((cmask >> q) & 1u) {
          const uint32_t hi = (uint32_t)(cur[q] >> 32);
          const uint32_t key = ((uint32_t)cur[q] << 5) | ((hi & 0xFFu) * 2u + ((hi >> 8) & 1u));
          if (pos < kColdTile) sorted[pos] = key;
          else my_cold[pos] = key;
          ++pos;
        }
    }
  };
  constexpr std::true_type kFull{};
  constexpr std::false_type kPart{};
  for (uint64_t i0 = r0; i0 < rf;) {
    issue(i0 + 2 * kHotStep, vc);
    step(kFull, i0, va);
    if ((i0 += kHotStep) >= rf) break;
    issue(i0 + 2 * kHotStep, va);
    step(kFull, i0, vb);
    if ((i0 += kHotStep) >= rf) break;
    issue(i0 + 2 * kHotStep, vb);
    step(kFull, i0, vc);
    i0 += kHotStep;
  }
  if (rf < r1) {
    hot_load<VEC, false>(rec, r1, rf, va);
    step(kPart, rf, va);
  }
  if (lane == 0) {
    atomicAdd(&s_valid, w_valid);
    atomicAdd(&s_lat, w_lat);
  }
  __syncthreads();
  {
    // the packed hot counters, merged with the corrections by the finish
    uint32_t *dst = a.partial + (size_t)wg * kHotWords;
    for (uint32_t k = tid; k < kHotWords; k += kHotThreads) dst[k] = bins[k];
  }
  if (tid == 0) {
    TileTotals t;
    t.valid = s_valid;
    t.latency = s_lat;
    t.dropped = (uint32_t)(r1 - r0) - s_valid;
    t.pad = 0;
    wtot[wg] = t;
    n_cold[wg] = s_cur;
  }
  const uint32_t nc = s_cur;   // the keys were written before the barrier above
  for (uint32_t t = 0; t * kColdTile < nc; ++t)
    sort_cold_tile(n_cb, r0 + t * kColdTile, min(kColdTile, nc - t * kColdTile),
                   t == 0 ? (const uint32_t *)sorted : my_cold + t * kColdTile, cold_sorted,
                   tile_off + ((size_t)wg * T + t) * (n_cb + 1), sorted, bc, scan_tmp);
}

// blocks [0, n_cb): the cold bins of one bucket; the next n_merge: hot bins
// summed over the pass's workgroups (none when the pass had one workgroup,
// which wrote its hot bins itself); the last: the totals
template <bool BATCH>
__global__ void __launch_bounds__(kHotThreads)
k_hot_finish(HotArgs one, const HotArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  HotArgs a;
  uint32_t bid;
  hot_item<BATCH>(one, many, items, a, bid);
  const uint32_t n_instr = a.n_instr, n_cb = a.n_cb, G = a.G, T = a.T;
  const uint32_t *__restrict__ hot_pc = a.hot_pc;
  const uint32_t *__restrict__ n_hot_p = a.n_hot;
  const uint32_t *__restrict__ partial = a.partial;
  const uint32_t *__restrict__ cold_sorted = a.cold_sorted;
  const uint32_t *__restrict__ tile_off = a.tile_off;
  const uint32_t *__restrict__ n_cold = a.n_cold;
  const TileTotals *__restrict__ wtot = a.wtot;
  uint32_t *__restrict__ counts = a.counts;
  unsigned long long *__restrict__ totals = a.totals;
  constexpr uint32_t kWaves = kHotThreads / kWave;
  static_assert(kHotGrid <= (uint32_t)kHotThreads, "one pass workgroup per thread");
  __shared__ __align__(16) uint32_t bins[kColdBins];
  __shared__ uint32_t hot_mark[kColdPCs / 32];
  __shared__ uint32_t rs[kMaxRuns], rp[kMaxRuns + 1];
  __shared__ uint32_t scan_tmp[kHotThreads / kWave + 1];
  const unsigned tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  const uint32_t n_hot = *n_hot_p;
  const uint32_t n_merge = a.n_merge;
  if (bid < n_cb) {
    const uint32_t b = bid, pc0 = b * kColdPCs;
    const uint32_t npc = min(kColdPCs, n_instr - pc0);
    for (uint32_t k = tid; k < kColdBins; k += kHotThreads) bins[k] = 0;
    if (tid < kColdPCs / 32) hot_mark[tid] = 0;
    // the bucket's runs, one per sorted tile (w, t), numbered by a scan over w
    const uint32_t nf = tid < G ? (n_cold[tid] + kColdTile - 1) / kColdTile : 0u;
    uint32_t n_runs;
    const uint32_t ex = block_excl_scan<kHotThreads>(nf, scan_tmp, &n_runs);
    if (tid < n_hot) {
      const uint32_t pl = hot_pc[tid] - pc0;
      if (pl < kColdPCs) atomicOr(&hot_mark[pl / 32], 1u << (pl % 32));
    }
    // up to kMaxRuns runs at a time: their starts and a prefix of their
    // lengths in LDS, then the concatenated keys walked flat, each wave a
    // contiguous share, lane-interleaved, eight loads in flight per lane
    for (uint32_t c0 = 0; c0 < n_runs; c0 += kMaxRuns) {
      const uint32_t m = min(kMaxRuns, n_runs - c0);
      for (uint32_t f = 0; f < nf; ++f)
        if (ex + f >= c0 && ex + f < c0 + m) {
          const uint32_t *off = tile_off + ((size_t)tid * T + f) * (n_cb + 1);
          const uint32_t st = off[b];
          rs[ex + f - c0] = st;
          rp[ex + f - c0] = off[b + 1] - st;   // the length, until the scan below
        }
      __syncthreads();
      {
        static_assert(kMaxRuns == 4 * (uint32_t)kHotThreads, "four runs per thread in the scan");
        uint32_t l[4], sum = 0;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
          l[i] = 4 * tid + i < m ? rp[4 * tid + i] : 0u;
          sum += l[i];
        }
        uint32_t total;
        uint32_t run = block_excl_scan<kHotThreads>(sum, scan_tmp, &total);
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
          if (4 * tid + i < m) rp[4 * tid + i] = run;
          run += l[i];
        }
        if (tid == 0) rp[m] = total;
      }
      __syncthreads();
      const uint32_t T_keys = rp[m];
      const uint32_t share = (T_keys + kWaves - 1) / kWaves;
      const uint32_t lo = min(wv * share, T_keys), hi = min(lo + share, T_keys);
      uint32_t k = lo + lane, r = 0;
      if (k < hi) {   // the run holding k: rp[r] <= k < rp[r + 1]
        uint32_t x = 0, z = m;
        while (z - x > 1) {
          const uint32_t mid = (x + z) / 2;
          if (rp[mid] <= k) x = mid;
          else z = mid;
        }
        r = x;
      }
      for (; k < hi; k += 8 * kWave) {
        uint32_t key[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
          const uint32_t kk = k + u * kWave;
          key[u] = kEmpty;
          if (kk < hi) {
            while (rp[r + 1] <= kk) ++r;   // ends: kk < rp[m]
            key[u] = cold_sorted[rs[r] + (kk - rp[r])];
          }
        }
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u)
          if (key[u] != kEmpty) atomicAdd(&bins[cold_local_bin(key[u])], 1u);
      }
      __syncthreads();
    }
    __syncthreads();   // the hot marks (and the cleared bins when there are no runs)
    for (uint32_t k = tid; k < npc * 24u; k += kHotThreads) {
      const uint32_t pl = k / 24u;
      if (!((hot_mark[pl / 32] >> (pl % 32)) & 1u)) {
        counts[(size_t)pc0 * 24u + k] = bins[k];
        if (k % 24u == 2 * GPA_ST_SELECTED) a.issued[pc0 + pl] = bins[k] + bins[k + 1];
      }
    }
  } else if (bid < n_cb + n_merge) {
    // the partial tables merged by word: a thread takes the two counters of
    // one word of the packed hot bins (or, in direct mode, one (lo, hi)
    // pair of the exact partials), kMergeWords words kHotThreads / S apart;
    // the pass's workgroups split over S slices (S a power of two, so that a
    // slice holds at most kMergeSlice partials), summed across slices in
    // LDS, and the hot bins' wrap corrections added
    const bool direct = a.direct != 0;
    const uint32_t S = a.merge_slices, wpb = kHotThreads / S;
    const uint32_t c = tid % wpb, sl = tid / wpb;
    const uint32_t n_words = (direct ? n_instr : n_hot) * 12u;
    const size_t width = direct ? (size_t)n_instr * 24u : (size_t)kHotWords;
    const uint32_t base = (bid - n_cb) * wpb * kMergeWords;
    for (uint32_t k = 0; k < kMergeWords; ++k) {
      const uint32_t word = base + k * wpb + c;
      const bool live = word < n_words;
      uint32_t lo = 0, hi = 0;
      if (live) {
        if (direct) {
#pragma unroll 4
          for (uint32_t w = sl; w < G; w += S) {
            const uint2 x = *(const uint2 *)(partial + (size_t)w * width + 2u * word);
            lo += x.x;
            hi += x.y;
          }
        } else {
#pragma unroll 4
          for (uint32_t w = sl; w < G; w += S) {
            const uint32_t x = partial[(size_t)w * width + word];
            lo += x & 0xFFFFu;
            hi += x >> 16;
          }
        }
      }
      if (S > 1) {
        bins[sl * wpb + c] = lo;
        bins[kHotThreads + sl * wpb + c] = hi;
        __syncthreads();
        if (sl == 0) {
          for (uint32_t q = 1; q < S; ++q) {
            lo += bins[q * wpb + c];
            hi += bins[kHotThreads + q * wpb + c];
          }
        }
        __syncthreads();
      }
      if (sl == 0 && live) {
        if (direct) {
          *(uint2 *)(counts + 2u * (size_t)word) = make_uint2(lo, hi);
          if (word % 12u == GPA_ST_SELECTED) a.issued[word / 12u] = lo + hi;
        } else {
          const uint2 cr = *(const uint2 *)(a.corr + 2u * word);
          const size_t at = (size_t)hot_pc[word / 12u] * 24u + 2u * (word % 12u);
          *(uint2 *)(counts + at) = make_uint2(lo + cr.x, hi + cr.y);
          if (word % 12u == GPA_ST_SELECTED) a.issued[at / 24u] = lo + cr.x + hi + cr.y;
        }
      }
    }
  } else {
    unsigned long long v = 0, l = 0, d = 0;
    if (tid < G) {
      v = wtot[tid].valid;
      l = wtot[tid].latency;
      d = wtot[tid].dropped;
    }
    v = wave_sum(v);
    l = wave_sum(l);
    d = wave_sum(d);
    unsigned long long *red = (unsigned long long *)bins;   // [3][kWaves]
    if (lane == 0) {
      red[wv] = v;
      red[kWaves + wv] = l;
      red[2 * kWaves + wv] = d;
    }
    __syncthreads();
    if (tid < 3) {
      unsigned long long a = 0;
      for (uint32_t k = 0; k < kWaves; ++k) a += red[tid * kWaves + k];
      totals[tid] = a;
    }
    if (tid == 3) totals[3] = 0;
  }
}

// The hot-set path, for programs of at most kHotMaxPCs instructions.
uint32_t hist_hot_max_pcs() { return kHotMaxPCs; }

// Direct mode for programs of at most kDirectPCs instructions, unless the
// environment sets GPA_HIST_HOTSET=1 (the hot/cold path for every program;
// the counts are the same).
static bool hot_direct(uint32_t n_instr) {
  if (n_instr > kDirectPCs) return false;
  const char *f = getenv("GPA_HIST_HOTSET");
  return !(f && f[0] == '1');
}

// The pass's workgroup ranges, each a multiple of 128 records (even, so the
// 16-byte loads stay aligned; finer than a whole step, so that the grid
// comes as close to its target as it can, a range's last step being partial
// where it must).
//   hot/cold: kHotGrid ranges at most; per_min, when given, is the least
//             range;
//   direct:   ranges of at least 96 (batched: 960) records per instruction,
//             so that the partial tables (96 bytes per instruction and
//             range) stay under a quarter (a fortieth) of the records'
//             bytes, and at most kDirectMaxPer records.  (On the
//             whole-application batch 960 measured best: 480 and 240 cost
//             2% and 6% more histogram time, 1,920 and more 15%, where a few
//             long ranges end last.)
struct HotShape {
  uint64_t per, run_stride;
  uint32_t G, T, n_cb, n_merge, merge_slices;
  bool direct;
};
static HotShape hot_shape(uint32_t n_instr, uint64_t n, uint64_t per_min = 0) {
  HotShape h;
  // (a profile of more than kHotGrid ranges of kDirectMaxPer records takes
  // the hot-set path, whose ranges have no bound)
  h.direct = hot_direct(n_instr) && n <= (uint64_t)kHotGrid * kDirectMaxPer;
  uint64_t per = std::max<uint64_t>((n + kHotGrid - 1) / kHotGrid, per_min);
  if (h.direct) {
    per = std::max<uint64_t>(per, (per_min ? 960ull : 96ull) * n_instr);
    per = std::min<uint64_t>(per, kDirectMaxPer);
  }
  h.per = (per + 2 * kWave - 1) / (2 * kWave) * (2 * kWave);
  if (h.per == 0) h.per = 2 * kWave;
  h.G = (uint32_t)((n + h.per - 1) / h.per);
  if (h.G > kHotGrid) fail(GPA_E_DEVICE, "histogram shape: %u ranges", h.G);
  h.n_cb = h.direct ? 0u : (n_instr + kColdPCs - 1) / kColdPCs;
  h.T = h.direct ? 0u : (uint32_t)((h.per + kColdTile - 1) / kColdTile);   // tiles per workgroup
  h.run_stride = n > kSelSample ? (n - kSelRun) / (kSelSample / kSelRun - 1) : 0;
  // merge: S slices of at most kMergeSlice of the G partials, kHotThreads / S
  // threads per slice, kMergeWords words per thread
  uint32_t S = 1;
  while (S * kMergeSlice < h.G) S <<= 1;
  h.merge_slices = S;
  const uint32_t words_per_wg = kHotThreads / S * kMergeWords;
  const uint32_t live_words = (h.direct ? n_instr : std::min<uint32_t>(kHotH, n_instr)) * 12u;
  // direct mode merges partials only when there are several; the hot bins
  // are always merged (packed counters and corrections to exact counts)
  h.n_merge = (h.G > 1 || !h.direct) ? (live_words + words_per_wg - 1) / words_per_wg : 0;
  return h;
}

static size_t blk256(size_t bytes) { return (bytes + 255) / 256 * 256; }

// element counts of a profile's scratch pieces, in the order hot_args takes
// them: lookup table, hot PCs, hot count, partial tables, cold keys, sorted
// cold keys, tile offsets, cold counts, wrap corrections (u32 each), then
// the range totals
struct HotPieces {
  size_t u32[9];
  size_t totals;
};
static HotPieces hot_pieces(const HotShape &h, uint32_t n_instr, uint64_t n) {
  HotPieces q;
  const bool d = h.direct;
  q.u32[0] = d ? 1 : kHotT;
  q.u32[1] = d ? 1 : kHotH;
  q.u32[2] = 1;
  q.u32[3] = d ? (h.G > 1 ? (size_t)h.G * n_instr * 24 : 1) : (size_t)h.G * kHotWords;
  q.u32[4] = d ? 1 : n;
  q.u32[5] = d ? 1 : n;
  q.u32[6] = d ? 1 : (size_t)h.G * h.T * (h.n_cb + 1);
  q.u32[7] = h.G;
  q.u32[8] = d ? 1 : kHotBins;
  q.totals = h.G;
  return q;
}

static size_t hot_scratch(const HotShape &h, uint32_t n_instr, uint64_t n) {
  const HotPieces q = hot_pieces(h, n_instr, n);
  size_t b = 0;
  for (size_t c : q.u32) b += blk256(4 * (c ? c : 1));
  return b + blk256(sizeof(TileTotals) * (q.totals ? q.totals : 1));
}

size_t hist_hot_scratch_bytes(uint32_t n_instr, uint64_t n) {
  if (n == 0) return 0;
  return hot_scratch(hot_shape(n_instr, n), n_instr, n);
}

// one profile's arguments, its scratch taken from the arena (in the order
// hot_scratch counts it)
static HotArgs hot_args(const HotShape &h, const uint64_t *rec, uint64_t n, uint32_t n_instr,
                        uint32_t *counts, uint32_t *issued, unsigned long long *totals,
                        Arena &ar) {
  const HotPieces q = hot_pieces(h, n_instr, n);
  HotArgs a;
  a.rec = rec;
  a.n = n;
  a.per = h.per;
  a.run_stride = h.run_stride;
  a.n_instr = n_instr;
  a.n_cb = h.n_cb;
  a.G = h.G;
  a.T = h.T;
  a.n_merge = h.n_merge;
  a.merge_slices = h.merge_slices;
  a.direct = h.direct ? 1u : 0u;
  a.pad = 0;
  a.hot_tab = ar.get<uint32_t>(q.u32[0]);
  a.hot_pc = ar.get<uint32_t>(q.u32[1]);
  a.n_hot = ar.get<uint32_t>(q.u32[2]);
  a.partial = ar.get<uint32_t>(q.u32[3]);
  a.cold = ar.get<uint32_t>(q.u32[4]);
  a.cold_sorted = ar.get<uint32_t>(q.u32[5]);
  a.tile_off = ar.get<uint32_t>(q.u32[6]);
  a.n_cold = ar.get<uint32_t>(q.u32[7]);
  a.corr = ar.get<uint32_t>(q.u32[8]);
  a.wtot = ar.get<TileTotals>(q.totals);
  a.counts = counts;
  a.issued = issued;
  a.totals = totals;
  return a;
}

// workgroups of the three launches for one profile: selection (hot/cold
// only), pass ranges, finish (cold buckets, merges and the totals; nothing
// in direct mode when one range wrote the counts and totals itself)
static void hot_blocks(const HotShape &h, uint32_t &n_sel, uint32_t &n_pass, uint32_t &n_fin) {
  n_sel = h.direct ? 0u : 1u;
  n_pass = h.G;
  n_fin = (h.direct && h.G == 1) ? 0u : h.n_cb + h.n_merge + 1;
}

// the selection's dynamic LDS limit, set once per device
static void set_select_lds() {
  static std::mutex mu;
  static std::vector<bool> done;
  int dev = 0;
  GPA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev < done.size() && done[dev]) return;
  const int lds_sel = (int)(kSelLdsWords * 4);
  GPA_HIP(hipFuncSetAttribute((const void *)k_hot_select<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_sel));
  GPA_HIP(hipFuncSetAttribute((const void *)k_hot_select<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_sel));
  if (done.size() <= (size_t)dev) done.resize((size_t)dev + 1, false);
  done[dev] = true;
}

static bool run_hist_hot(const gpa_program &p, const uint64_t *rec, uint64_t n, bool vec,
                         uint32_t *counts, uint32_t *issued, unsigned long long *totals,
                         hipStream_t s, Arena &ar, bool allow_partition) {
  const uint32_t n_instr = p.n_instr;
  if (n_instr > kHotMaxPCs) return false;
  const char *force = getenv("GPA_HIST_PARTITION");
  if (allow_partition && force && force[0] == '1') return false;
  const HotShape hs = hot_shape(n_instr, n);
  const HotArgs a = hot_args(hs, rec, n, n_instr, counts, issued, totals, ar);
  uint32_t n_sel, n_pass, n_fin;
  hot_blocks(hs, n_sel, n_pass, n_fin);
  if (n_sel) {
    set_select_lds();
    hipLaunchKernelGGL(k_hot_select<false>, dim3(n_sel), dim3(kHotThreads), kSelLdsWords * 4, s, a,
                       nullptr, nullptr);
    GPA_LAUNCH_CHECK();
  }
  if (vec)
    hipLaunchKernelGGL((k_hot_pass<true, false>), dim3(n_pass), dim3(kHotThreads), 0, s, a,
                       nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_hot_pass<false, false>), dim3(n_pass), dim3(kHotThreads), 0, s, a,
                       nullptr, nullptr);
  GPA_LAUNCH_CHECK();
  if (n_fin) {
    hipLaunchKernelGGL(k_hot_finish<false>, dim3(n_fin), dim3(kHotThreads), 0, s, a, nullptr,
                       nullptr);
    GPA_LAUNCH_CHECK();
  }
  return true;
}

// A batched histogram ready to launch: its argument table and work lists on
// the device (uploaded and expanded on the stream).
struct HistBatch {
  BatchPlan plan;
  const HotArgs *d_args = nullptr;
  uint32_t q_sel = 0, q_pass = 0, q_fin = 0;
  explicit HistBatch(uint32_t count) : plan(count) {}
};

static void prepare_hist_batch(HistBatch &hb, const HistEntry *e, uint32_t count, uint64_t per,
                               hipStream_t s, Arena &ar) {
  std::vector<HotArgs> args(count);
  std::vector<uint32_t> n_sel(count), n_pass(count), n_fin(count);
  std::vector<uint64_t> range(count);
  for (uint32_t k = 0; k < count; ++k) {
    if (e[k].n == 0 || e[k].n_instr > kHotMaxPCs || ((uintptr_t)e[k].samples % 16) != 0)
      fail(GPA_E_INVALID, "batched histogram entry %u: n > 0, at most %u instructions and "
           "16-byte aligned records are required", k, kHotMaxPCs);
    const HotShape h = hot_shape(e[k].n_instr, e[k].n, per);
    args[k] = hot_args(h, (const uint64_t *)e[k].samples, e[k].n, e[k].n_instr, e[k].counts,
                       e[k].issued, e[k].totals, ar);
    hot_blocks(h, n_sel[k], n_pass[k], n_fin[k]);
    range[k] = std::min<uint64_t>(h.per, e[k].n);
  }
  // the pass's workgroups longest range first (direct ranges can be several
  // times the others), so that the long ones do not start last
  std::vector<uint32_t> order(count);
  for (uint32_t k = 0; k < count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t x, uint32_t y) { return range[x] > range[y]; });
  hb.q_sel = hb.plan.add(n_sel);
  hb.q_pass = hb.plan.add(n_pass, &order);
  hb.q_fin = hb.plan.add(n_fin);
  Upload up;
  const size_t i_args = up.add(args), i_pre = up.add(hb.plan.pre);
  up.send(ar, s);
  hb.d_args = up.ptr<HotArgs>(i_args);
  hb.plan.d_pre = up.ptr<uint32_t>(i_pre);
  hb.plan.d_items = ar.get<WorkItem>(hb.plan.total_items());
  hb.plan.expand(s);
}

static void launch_hist_select(const HistBatch &hb, hipStream_t s) {
  if (!hb.plan.blocks(hb.q_sel)) return;
  HotArgs none{};
  set_select_lds();
  hipLaunchKernelGGL(k_hot_select<true>, dim3(hb.plan.blocks(hb.q_sel)), dim3(kHotThreads),
                     kSelLdsWords * 4, s, none, hb.d_args, hb.plan.items(hb.q_sel));
  GPA_LAUNCH_CHECK();
}

static void launch_hist_pass_finish(const HistBatch &hb, hipStream_t s) {
  HotArgs none{};
  hipLaunchKernelGGL((k_hot_pass<true, true>), dim3(hb.plan.blocks(hb.q_pass)), dim3(kHotThreads),
                     0, s, none, hb.d_args, hb.plan.items(hb.q_pass));
  GPA_LAUNCH_CHECK();
  if (hb.plan.blocks(hb.q_fin)) {
    hipLaunchKernelGGL(k_hot_finish<true>, dim3(hb.plan.blocks(hb.q_fin)), dim3(kHotThreads), 0, s,
                       none, hb.d_args, hb.plan.items(hb.q_fin));
    GPA_LAUNCH_CHECK();
  }
}

void run_hist_batch(const HistEntry *e, uint32_t count, uint64_t per, hipStream_t s, Arena &ar,
                    PhaseTimer *t) {
  if (count == 0) return;
  HistBatch hb(count);
  prepare_hist_batch(hb, e, count, per, s, ar);
  if (t) t->begin(kPhaseHist, s);
  launch_hist_select(hb, s);
  launch_hist_pass_finish(hb, s);
  if (t) t->end(s);
}

// ------------------------------------------------------------- autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, uint64_t> g_tuned;
constexpr uint64_t kPerCandidates[] = {32768, 65536, 131072, 262144, 524288};
constexpr uint64_t kPerDefault = 131072;

uint32_t log2_bucket(uint64_t v) {
  uint32_t b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}
}  // namespace

uint64_t batch_records_per_workgroup(const HistEntry *e, uint32_t count, hipStream_t s, Arena &ar,
                                     bool measure) {
  (void)ar;
  if (const char *f = getenv("GPA_BATCH_PER")) {
    const unsigned long long v = strtoull(f, nullptr, 10);
    if (v) return v;
  }
  if (count == 0) return kPerDefault;
  uint64_t total = 0, largest = 0;
  for (uint32_t k = 0; k < count; ++k) {
    total += e[k].n;
    largest = std::max(largest, e[k].n);
  }
  const auto key = std::make_tuple(log2_bucket(count), log2_bucket(total), log2_bucket(largest));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  const char *at = getenv("GPA_AUTOTUNE");
  if (!measure || (at && at[0] == '0')) return kPerDefault;
  hipEvent_t a = nullptr, b = nullptr;
  GPA_HIP(hipEventCreate(&a));
  GPA_HIP(hipEventCreate(&b));
  uint64_t best = kPerDefault;
  float best_ms = 0.f;
  bool have = false;
  try {
    // the first candidate runs twice: its first run pays for cold code and caches
    for (int rep = 0; rep < 2; ++rep) {
      for (uint64_t per : kPerCandidates) {
        if (rep == 1 && per != kPerCandidates[0]) continue;
        // each candidate's scratch goes back to the pool after it; only the
        // three launches are timed, not the host's preparation
        Arena trial(s);
        HistBatch hb(count);
        prepare_hist_batch(hb, e, count, per, s, trial);
        GPA_HIP(hipEventRecord(a, s));
        launch_hist_select(hb, s);
        launch_hist_pass_finish(hb, s);
        GPA_HIP(hipEventRecord(b, s));
        GPA_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        GPA_HIP(hipEventElapsedTime(&ms, a, b));
        if (rep == 1 || per != kPerCandidates[0]) {
          if (!have || ms < best_ms) {
            best_ms = ms;
            best = per;
            have = true;
          }
        }
      }
    }
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

__global__ void k_hist_empty(uint32_t *counts, uint32_t *issued, uint32_t n_instr,
                             unsigned long long *totals) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < (size_t)n_instr * 24;
       k += (size_t)gridDim.x * blockDim.x) {
    counts[k] = 0;
    if (k < n_instr) issued[k] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 4) totals[threadIdx.x] = 0;
}

// the issued samples from finished counts (the partition path)
__global__ void k_issued(const uint32_t *__restrict__ counts, uint32_t n_instr,
                         uint32_t *__restrict__ issued) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_instr; i += gridDim.x * blockDim.x)
    issued[i] = counts[(size_t)i * 24 + 2 * GPA_ST_SELECTED] +
                counts[(size_t)i * 24 + 2 * GPA_ST_SELECTED + 1];
}

void run_hist(const gpa_program &p, const gpa_sample *samples, uint64_t n, uint32_t *counts,
              uint32_t *issued, unsigned long long *totals, hipStream_t s, Arena &ar,
              bool allow_partition) {
  const uint32_t n_instr = p.n_instr;
  const uint32_t n_buckets = (n_instr + kBucketPCs - 1) / kBucketPCs;
  if (n_buckets > kMaxBuckets)
    fail(GPA_E_UNSUPPORTED, "histogram supports up to %d instructions", kMaxBuckets * kBucketPCs);
  if (n == 0) {
    hipLaunchKernelGGL(k_hist_empty, dim3(grid_for((size_t)n_instr * 24, 256, 4096)), dim3(256), 0,
                       s, counts, issued, n_instr, totals);
    GPA_LAUNCH_CHECK();
    return;
  }
  if (n >= 0x40000000ull) fail(GPA_E_UNSUPPORTED, "fewer than 2^30 samples per call are supported");
  const uint64_t *rec = (const uint64_t *)samples;
  const bool vec = ((uintptr_t)samples % 16) == 0;
  if (run_hist_hot(p, rec, n, vec, counts, issued, totals, s, ar, allow_partition)) return;
  if (!allow_partition)
    fail(GPA_E_UNSUPPORTED, "this path counts programs of up to %u instructions", kHotMaxPCs);
  const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
  // bucket regions from a sample of the records
  const uint64_t n_samp =
      (n + (uint64_t)kSampleStride * kSampleSlice - 1) / ((uint64_t)kSampleStride * kSampleSlice);
  const uint32_t n_slots = n_buckets * kSubs;
  // cleared by one fill: the sampled estimates (kSubs padded copies per
  // bucket) and the overflow count
  const size_t n_est = (size_t)n_slots * kCursorStride;
  uint32_t *ctl = ar.get<uint32_t>(n_est + 1);
  uint32_t *est = ctl, *ov_count = ctl + n_est;
  GPA_HIP(hipMemsetAsync(ctl, 0, 4 * (n_est + 1), s));
  uint32_t *cap = ar.get<uint32_t>(n_slots);
  uint32_t *region = ar.get<uint32_t>(n_slots);
  uint32_t *cursor = ar.get<uint32_t>((size_t)n_slots * kCursorStride);
  const size_t lds_count = (size_t)n_buckets * 4;
  hipLaunchKernelGGL(k_hsample, dim3((unsigned)n_samp), dim3(kHistThreads), lds_count, s, rec, n,
                     n_instr, n_buckets, est);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hregions, dim3(1), dim3(kHistThreads), 0, s, n_buckets, est, cap, region,
                     cursor);
  GPA_LAUNCH_CHECK();
  // the sub-regions hold at most 5/4 of the scaled sample plus the slack;
  // payload offsets stay below 2^31 (bit 31 marks the overflow area)
  const uint64_t max_region = n_samp * kSampleSlice * kSampleStride * 5 / 4 +
                              (uint64_t)n_slots * (kSubSlack + 1);
  if (max_region >= 0x80000000ull)
    fail(GPA_E_UNSUPPORTED, "histogram payload of %llu records exceeds 2^31",
         (unsigned long long)max_region);
  uint16_t *payload = ar.get<uint16_t>(max_region);
  uint32_t *ov_keys = ar.get<uint32_t>(n);
  TileTotals *tt = ar.get<TileTotals>(n_tiles);
  uint32_t *sfill = ar.get<uint32_t>(n_slots), *bfill = ar.get<uint32_t>(n_buckets);
  uint32_t *items = ar.get<uint32_t>(n_buckets);
  uint32_t *item_start = ar.get<uint32_t>(n_buckets);
  const size_t lds_part = partition_lds_words(n_buckets) * 4;
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
  hipLaunchKernelGGL(k_hplan, dim3(1), dim3(kHistThreads), 0, s, tt, n_tiles, totals, n_buckets,
                     cursor, cap, sfill, bfill, items, item_start);
  GPA_LAUNCH_CHECK();
  // items <= one per bucket plus one per kItemRecords records
  const uint64_t max_items = n_buckets + n / kItemRecords + 1;
  uint32_t *partial = ar.get<uint32_t>((size_t)max_items * kBucketBins);
  hipLaunchKernelGGL(k_count, dim3((unsigned)max_items), dim3(kCountThreads), 0, s, payload, region,
                     sfill, bfill, n_buckets, n_instr, items, item_start, counts, partial);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_merge, dim3(n_buckets, kBucketBins / kHistThreads), dim3(kHistThreads), 0,
                     s, partial, items, item_start, n_instr, counts);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hoverflow, dim3(256), dim3(256), 0, s, ov_keys, ov_count, counts);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_issued, dim3(grid_for(n_instr, 256, 4096)), dim3(256), 0, s, counts, n_instr,
                     issued);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
