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
  if (n >= 0x40000000ull) fail(GPA_E_UNSUPPORTED, "fewer than 2^30 samples per call are supported");
  const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
  const uint64_t *rec = (const uint64_t *)samples;
  const bool vec = ((uintptr_t)samples % 16) == 0;
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
}

}  // namespace gpa
