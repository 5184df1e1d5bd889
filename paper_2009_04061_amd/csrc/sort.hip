// Stable LSD radix sort of (key, value) u32 pairs, 8-bit digits (9-bit
// when that saves a pass).
// Each pass: per-chunk digit histograms in LDS (digit-major counts), one
// exclusive scan over them, and a stable scatter that ranks equal digits
// inside each wave by ballot matching and across waves by LDS counts.
// Used to group items by a key while keeping item order inside each group.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kRsThreads = 256;
constexpr int kRsChunk = 2048;

template <int D>
__global__ void __launch_bounds__(kRsThreads)
k_rs_hist(const uint32_t *keys, size_t n, uint32_t shift, uint32_t n_chunks, uint32_t *counts) {
  constexpr int kRsDigits = 1 << D;
  __shared__ uint32_t h[kRsDigits];
  for (int d = threadIdx.x; d < kRsDigits; d += kRsThreads) h[d] = 0;
  __syncthreads();
  const size_t a = (size_t)blockIdx.x * kRsChunk, b = min(a + kRsChunk, n);
  for (size_t i = a + threadIdx.x; i < b; i += kRsThreads)
    atomicAdd(&h[(keys[i] >> shift) & (kRsDigits - 1u)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kRsDigits; d += kRsThreads)
    counts[(size_t)d * n_chunks + blockIdx.x] = h[d];
}

template <int D>
__global__ void __launch_bounds__(kRsThreads)
k_rs_scatter(const uint32_t *keys, const uint32_t *vals, size_t n, uint32_t shift,
             uint32_t n_chunks, const uint32_t *offsets, uint32_t *keys_out, uint32_t *vals_out) {
  constexpr int kRsDigits = 1 << D;
  constexpr int NW = kRsThreads / kWave;
  __shared__ uint32_t cursor[kRsDigits];
  __shared__ uint32_t wcnt[NW][kRsDigits];
  const unsigned tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  for (int d = tid; d < kRsDigits; d += kRsThreads) {
    cursor[d] = offsets[(size_t)d * n_chunks + blockIdx.x];
    for (int v = 0; v < NW; ++v) wcnt[v][d] = 0;
  }
  __syncthreads();
  const size_t a = (size_t)blockIdx.x * kRsChunk, b = min(a + kRsChunk, n);
  for (size_t r0 = a; r0 < b; r0 += kRsThreads) {
    const size_t i = r0 + tid;
    const bool active = i < b;
    const uint32_t key = active ? keys[i] : 0u;
    const uint32_t dg = (key >> shift) & (kRsDigits - 1u);
    uint64_t peers = __ballot(active);
#pragma unroll
    for (uint32_t bit = 0; bit < (uint32_t)D; ++bit) {
      const uint64_t m = __ballot(active && ((dg >> bit) & 1u));
      peers &= ((dg >> bit) & 1u) ? m : ~m;
    }
    const uint64_t lower = peers & ((1ull << lane) - 1ull);
    if (active && lower == 0) wcnt[w][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (active) {
      uint32_t before = 0;
      for (unsigned v = 0; v < w; ++v) before += wcnt[v][dg];
      const uint32_t pos = cursor[dg] + before + (uint32_t)__popcll(lower);
      keys_out[pos] = key;
      vals_out[pos] = vals[i];
    }
    __syncthreads();
    if (active && lower == 0) {
      bool first = true;
      uint32_t tot = 0;
      for (int v = 0; v < NW; ++v) {
        tot += wcnt[v][dg];
        if ((unsigned)v < w && wcnt[v][dg]) first = false;
      }
      if (first) cursor[dg] += tot;
    }
    __syncthreads();
    if (active && lower == 0) wcnt[w][dg] = 0;
    __syncthreads();
  }
}

template <int D>
static void sort_passes(uint32_t *keys, uint32_t *vals, size_t n, uint32_t passes, hipStream_t s,
                        Arena &ar) {
  constexpr uint32_t kRsDigits = 1u << D;
  const uint32_t n_chunks = (uint32_t)((n + kRsChunk - 1) / kRsChunk);
  uint32_t *k2 = ar.get<uint32_t>(n), *v2 = ar.get<uint32_t>(n);
  uint32_t *counts = ar.get<uint32_t>((size_t)kRsDigits * n_chunks);
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  for (uint32_t p = 0; p < passes; ++p) {
    const uint32_t shift = D * p;
    hipLaunchKernelGGL(k_rs_hist<D>, dim3(n_chunks), dim3(kRsThreads), 0, s, ka, n, shift,
                       n_chunks, counts);
    GPA_LAUNCH_CHECK();
    exclusive_scan_u32(counts, counts, (size_t)kRsDigits * n_chunks, s, ar);
    hipLaunchKernelGGL(k_rs_scatter<D>, dim3(n_chunks), dim3(kRsThreads), 0, s, ka, va, n, shift,
                       n_chunks, counts, kb, vb);
    GPA_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    GPA_HIP(hipMemcpyAsync(keys, ka, n * 4, hipMemcpyDeviceToDevice, s));
    GPA_HIP(hipMemcpyAsync(vals, va, n * 4, hipMemcpyDeviceToDevice, s));
  }
}

void sort_pairs_u32(uint32_t *keys, uint32_t *vals, size_t n, uint32_t key_bits, hipStream_t s,
                    Arena &ar) {
  if (n <= 1 || key_bits == 0) return;
  // 17 or 18 bits take two 9-bit passes instead of three 8-bit ones
  if (key_bits > 16 && key_bits <= 18) sort_passes<9>(keys, vals, n, 2, s, ar);
  else sort_passes<8>(keys, vals, n, (key_bits + 7) / 8, s, ar);
}

__global__ void k_iota_keys(const uint32_t *key, size_t n, uint32_t none_key, uint32_t *k,
                            uint32_t *v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t x = key[i];
    k[i] = (x == GPA_NONE) ? none_key : x;
    v[i] = (uint32_t)i;
  }
}

// ptr[k] = first position of the sorted keys holding a key >= k, k <= n_keys
__global__ void k_key_bounds(size_t n, const uint32_t *sk, uint32_t n_keys, uint32_t *ptr) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p <= n;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t lo = (p == 0) ? 0u : sk[p - 1] + 1u;
    const uint32_t hi = (p == n) ? n_keys : sk[p];
    for (uint32_t k = lo; k <= hi && k <= n_keys; ++k) ptr[k] = (uint32_t)p;
  }
}

// ptr[n_keys+1] and perm: items with key k are perm[ptr[k] .. ptr[k+1]) in
// item order; items whose key is GPA_NONE are left out (they sort last).
void group_by_key(const uint32_t *key, size_t n, uint32_t n_keys, DBuf<uint32_t> &ptr,
                  DBuf<uint32_t> &perm, hipStream_t s, Arena &ar) {
  ptr.alloc((size_t)n_keys + 1);
  perm.alloc(n ? n : 1);
  uint32_t *k = ar.get<uint32_t>(n ? n : 1);
  if (n) {
    hipLaunchKernelGGL(k_iota_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, key, n, n_keys,
                       k, perm.p);
    GPA_LAUNCH_CHECK();
    uint32_t bits = 1;
    while (bits < 32 && (1ull << bits) <= n_keys) ++bits;
    sort_pairs_u32(k, perm.p, n, bits, s, ar);
  }
  hipLaunchKernelGGL(k_key_bounds, dim3(grid_for(n + 1, 256, 8192)), dim3(256), 0, s, n, k,
                     n_keys, ptr.p);
  GPA_LAUNCH_CHECK();
}

// Several groupings in one sort: group g's items take keys key_base[g] +
// key (GPA_NONE -> key_base[g] + n_keys[g], so they sort after the group's
// valid keys and before the next group) and carry their index inside the
// group.
struct GroupSet {
  const uint32_t *key[kMaxGroups];
  uint64_t item_base[kMaxGroups + 1];
  uint32_t key_base[kMaxGroups], n_keys[kMaxGroups];
  uint32_t n;
};

__global__ void k_iota_groups(GroupSet g, uint32_t *k, uint32_t *v) {
  const uint64_t total = g.item_base[g.n];
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t q = 0;
    while (i >= g.item_base[q + 1]) ++q;
    const uint64_t j = i - g.item_base[q];
    const uint32_t x = g.key[q][j];
    k[i] = g.key_base[q] + (x == GPA_NONE ? g.n_keys[q] : x);
    v[i] = (uint32_t)j;
  }
}

// ptr[k] = first position of the sorted keys holding a key >= k (one
// thread per key, a binary search), less the first position of key k's
// grouping, so that every grouping's ptr starts at 0 within its own stretch
// of perm (ptr[n_keys_all] is left absolute)
__global__ void k_key_bounds_groups(uint64_t n, const uint32_t *sk, GroupSet g,
                                    uint32_t n_keys_all, uint32_t *ptr) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= n_keys_all;
       k += gridDim.x * blockDim.x) {
    uint64_t lo = 0, hi = n;   // first position with sk >= k in [lo, hi]
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (sk[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    uint64_t base = 0;
    for (uint32_t q = 0; q < g.n; ++q)
      if (k >= g.key_base[q] && k <= g.key_base[q] + g.n_keys[q]) base = g.item_base[q];
    ptr[k] = (uint32_t)(lo - base);
  }
}

void group_by_keys(const GroupSpec *spec, int n_groups, DBuf<uint32_t> &ptr,
                   DBuf<uint32_t> &perm, uint32_t *ptr_base, uint64_t *item_base,
                   hipStream_t s, Arena &ar) {
  if (n_groups < 1 || n_groups > (int)kMaxGroups) fail(GPA_E_DEVICE, "bad grouping count");
  GroupSet g{};
  g.n = (uint32_t)n_groups;
  uint64_t items = 0, keys = 0;
  for (int q = 0; q < n_groups; ++q) {
    g.key[q] = spec[q].key;
    g.item_base[q] = items;
    g.key_base[q] = (uint32_t)keys;
    g.n_keys[q] = spec[q].n_keys;
    ptr_base[q] = (uint32_t)keys;
    item_base[q] = items;
    items += spec[q].n;
    keys += (uint64_t)spec[q].n_keys + 1;
  }
  g.item_base[n_groups] = items;
  if (items >= (1ull << 32) || keys >= (1ull << 31))
    fail(GPA_E_UNSUPPORTED, "groupings of %llu items over %llu keys", (unsigned long long)items,
         (unsigned long long)keys);
  const uint32_t n_keys_all = (uint32_t)keys;   // every key of the sort is < n_keys_all
  ptr.alloc((size_t)n_keys_all + 1);
  perm.alloc(items ? items : 1);
  uint32_t *k = ar.get<uint32_t>(items ? items : 1);
  if (items) {
    hipLaunchKernelGGL(k_iota_groups, dim3(grid_for(items, 256, 8192)), dim3(256), 0, s, g, k,
                       perm.p);
    GPA_LAUNCH_CHECK();
    uint32_t bits = 1;
    while (bits < 32 && (1ull << bits) < n_keys_all) ++bits;
    sort_pairs_u32(k, perm.p, items, bits, s, ar);
  }
  hipLaunchKernelGGL(k_key_bounds_groups, dim3(grid_for((size_t)n_keys_all + 1, 256, 8192)),
                     dim3(256), 0, s, items, k, g, n_keys_all, ptr.p);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
