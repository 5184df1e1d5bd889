// Program loading: descriptor validation and the derived structure every
// later step reads (Sec. 3: CFGs, program structure, architecture table).
//   - block -> function, instruction -> block, predecessor lists;
//   - def and use sites sorted by (function, location, instruction): the
//     per-location views the backward searches work on;
//   - per use site the condition its search must cover (Sec. 4, predicated
//     instructions);
//   - scope tree: kernel root, depth and preorder subtree end per scope.
#include "common.h"
#include "devutil.h"

namespace gpa {

enum : uint32_t {
  kErrOpClass = 1u << 0,
  kErrGuard = 1u << 1,
  kErrCsr = 1u << 2,
  kErrDef = 1u << 3,
  kErrUse = 1u << 4,
  kErrDupDef = 1u << 5,
  kErrBlocks = 1u << 6,
  kErrSucc = 1u << 7,
  kErrFuncs = 1u << 8,
  kErrFuncScope = 1u << 9,
  kErrScopes = 1u << 10,
  kErrInstrScope = 1u << 11,
};

static const char *kErrText[] = {
    "op_class out of range",
    "guard out of range (0, 1+2k or 2+2k with k < n_preds)",
    "def_ptr/use_ptr not a valid CSR",
    "def location or kind out of range",
    "use location or kind out of range",
    "a location appears twice in one instruction's def list",
    "block_begin not strictly increasing from 0 to n_instr",
    "successor out of range or outside its function",
    "func_block_begin not strictly increasing from 0 to n_blocks",
    "func_scope is not a FUNCTION scope with GPA_SF_HAS_CFG",
    "scope tree not in preorder with FUNCTION kernel roots",
    "instr_scope is not a LINE scope inside its own CFG function",
};

// ------------------------------------------------------------ validation
__device__ void val_instr_part(uint32_t t0_, uint32_t st_, uint32_t n_instr, uint32_t n_preds, uint32_t n_scopes, uint32_t n_defs,
                            uint32_t n_uses, const uint8_t *op_class, const uint8_t *guard,
                            const uint32_t *def_ptr, const uint32_t *use_ptr,
                            const uint32_t *def_loc, const uint32_t *instr_scope,
                            const uint8_t *scope_kind, uint32_t *err) {
  uint32_t e = 0;
  for (uint32_t i = t0_; i < n_instr;
       i += st_) {
    if (op_class[i] >= GPA_N_OP_CLASSES) e |= kErrOpClass;
    if (guard[i] > 2 * n_preds) e |= kErrGuard;
    if (def_ptr[i] > def_ptr[i + 1] || use_ptr[i] > use_ptr[i + 1] || def_ptr[i + 1] > n_defs ||
        use_ptr[i + 1] > n_uses) {
      e |= kErrCsr;
      continue;
    }
    for (uint32_t a = def_ptr[i]; a < def_ptr[i + 1]; ++a)
      for (uint32_t b = a + 1; b < def_ptr[i + 1]; ++b)
        if (def_loc[a] == def_loc[b]) e |= kErrDupDef;
    const uint32_t sc = instr_scope[i];
    if (sc >= n_scopes || scope_kind[sc] != GPA_SCOPE_LINE) e |= kErrInstrScope;
  }
  if (e) atomicOr(err, e);
}

__device__ void val_sites_part(uint32_t t0_, uint32_t st_, uint32_t n, const uint32_t *loc, const uint8_t *kind, uint32_t n_loc,
                            uint32_t max_kind, uint32_t bit, uint32_t *err) {
  uint32_t e = 0;
  for (uint32_t i = t0_; i < n; i += st_)
    if (loc[i] >= n_loc || kind[i] > max_kind) e = bit;
  if (e) atomicOr(err, e);
}

__global__ void k_val_ends(uint32_t n_instr, uint32_t n_blocks, uint32_t n_funcs,
                           const uint32_t *def_ptr, const uint32_t *use_ptr,
                           const uint32_t *block_begin, const uint32_t *succ_ptr,
                           const uint32_t *fbb, uint32_t *vals) {
  // first of the checks: it also clears the verdict words the others update
  uint32_t e = 0;
  if (def_ptr[0] != 0 || use_ptr[0] != 0) e |= kErrCsr;
  if (block_begin[0] != 0 || block_begin[n_blocks] != n_instr) e |= kErrBlocks;
  if (succ_ptr[0] != 0) e |= kErrSucc;
  if (fbb[0] != 0 || fbb[n_funcs] != n_blocks) e |= kErrFuncs;
  vals[0] = e;
  for (int q = 1; q < 8; ++q) vals[q] = 0;
}

__device__ void val_funcs_part(uint32_t t0_, uint32_t st_, uint32_t n_funcs, uint32_t n_scopes, const uint32_t *fbb,
                            const uint32_t *func_scope, const uint8_t *scope_kind,
                            const uint8_t *scope_flags, uint32_t *err) {
  uint32_t e = 0;
  for (uint32_t f = t0_; f < n_funcs;
       f += st_) {
    if (fbb[f] >= fbb[f + 1]) e |= kErrFuncs;
    const uint32_t s = func_scope[f];
    if (s >= n_scopes || scope_kind[s] != GPA_SCOPE_FUNCTION || !(scope_flags[s] & GPA_SF_HAS_CFG))
      e |= kErrFuncScope;
  }
  if (e) atomicOr(err, e);
}

__device__ void val_scopes_part(uint32_t t0_, uint32_t st_, uint32_t n_scopes, const uint32_t *parent, const uint8_t *kind,
                             const uint8_t *flags, uint32_t *err) {
  uint32_t e = 0;
  for (uint32_t s = t0_; s < n_scopes;
       s += st_) {
    const uint32_t p = parent[s];
    if (kind[s] > GPA_SCOPE_LINE) e |= kErrScopes;
    if (p == GPA_NONE) {
      if (kind[s] != GPA_SCOPE_FUNCTION || !(flags[s] & GPA_SF_KERNEL_ENTRY)) e |= kErrScopes;
    } else if (p >= s || kind[p] == GPA_SCOPE_LINE) {
      e |= kErrScopes;
    }
  }
  if (e) atomicOr(err, e);
}

// block structure: block -> function and instruction -> block by binary
// search over the range starts (always in bounds; the blocks' own check
// rejects a block_begin that is not strictly increasing)
__device__ void blocks_part(uint32_t t0_, uint32_t st_, uint32_t n_funcs, uint32_t n_blocks, uint32_t n_instr, const uint32_t *fbb,
                         const uint32_t *block_begin, uint32_t *block_of, uint32_t *func_of_block,
                         uint32_t *pred_cnt, uint32_t *err) {
  uint32_t e = 0;
  if (t0_ == 0) pred_cnt[n_blocks] = 0;
  for (uint32_t k = t0_; k < n_blocks + n_instr;
       k += st_) {
    if (k < n_blocks) {
      pred_cnt[k] = 0;
      func_of_block[k] = upper_index_u32(fbb, 0, n_funcs, k);
      const uint32_t i0 = block_begin[k], i1 = block_begin[k + 1];
      if (i0 >= i1 || i1 > n_instr) e |= kErrBlocks;
    } else {
      const uint32_t i = k - n_blocks;
      block_of[i] = upper_index_u32(block_begin, 0, n_blocks, i);
    }
  }
  if (e) atomicOr(err, e);
}

__device__ void val_succ_part(uint32_t t0_, uint32_t st_, uint32_t n_blocks, const uint32_t *succ_ptr, const uint32_t *succ,
                           uint32_t n_succ, const uint32_t *func_of_block, uint32_t *pred_cnt,
                           uint32_t *err) {
  uint32_t e = 0;
  for (uint32_t b = t0_; b < n_blocks;
       b += st_) {
    const uint32_t e0 = succ_ptr[b], e1 = succ_ptr[b + 1];
    if (e0 > e1 || e1 > n_succ) {
      e |= kErrSucc;
      continue;
    }
    for (uint32_t k = e0; k < e1; ++k) {
      const uint32_t t = succ[k];
      if (t >= n_blocks || func_of_block[t] != func_of_block[b]) {
        e |= kErrSucc;
        continue;
      }
      atomicAdd(&pred_cnt[t], 1u);
    }
  }
  if (e) atomicOr(err, e);
}

// pred lists filled from their ends: the remaining count of each list is
// its next free slot counted from the list start
__global__ void k_fill_pred(uint32_t n_blocks, const uint32_t *succ_ptr, const uint32_t *succ,
                            const uint32_t *pred_ptr, uint32_t *remaining, uint32_t *pred) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks;
       b += gridDim.x * blockDim.x)
    for (uint32_t k = succ_ptr[b]; k < succ_ptr[b + 1]; ++k) {
      const uint32_t t = succ[k];
      pred[pred_ptr[t] + atomicSub(&remaining[t], 1u) - 1u] = b;
    }
}

// Each pred list in ascending order, so that everything downstream is
// independent of the order in which the atomics above were served.
__global__ void k_sort_pred(uint32_t n_blocks, const uint32_t *pred_ptr, uint32_t *pred) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks;
       b += gridDim.x * blockDim.x) {
    const uint32_t p0 = pred_ptr[b], p1 = pred_ptr[b + 1];
    for (uint32_t i = p0 + 1; i < p1; ++i) {
      uint32_t v = pred[i], j = i;
      while (j > p0 && pred[j - 1] > v) {
        pred[j] = pred[j - 1];
        --j;
      }
      pred[j] = v;
    }
  }
}

// every instruction's LINE scope lies under its function's scope and under no
// other CFG function (scope ids are range-checked here: this runs before the
// other checks' verdict is known)
__device__ void val_instr_scope_part(uint32_t t0_, uint32_t st_, uint32_t n_instr, uint32_t n_scopes, const uint32_t *instr_scope,
                                  const uint32_t *block_of, const uint32_t *func_of_block,
                                  const uint32_t *func_scope, const uint32_t *parent,
                                  const uint8_t *kind, const uint8_t *flags, uint32_t *err) {
  uint32_t e = 0;
  for (uint32_t i = t0_; i < n_instr;
       i += st_) {
    const uint32_t want = func_scope[func_of_block[block_of[i]]];
    uint32_t s = instr_scope[i];
    uint32_t guard = 0;
    while (s < n_scopes && !(kind[s] == GPA_SCOPE_FUNCTION && (flags[s] & GPA_SF_HAS_CFG)) &&
           guard < 4096) {
      s = parent[s];
      ++guard;
    }
    if (s != want) e |= kErrInstrScope;
  }
  if (e) atomicOr(err, e);
}

// ------------------------------------------------- sites by (func, location)
// Sites (defs or uses) of function f occupy [site_ptr[i0], site_ptr[i1]) for
// its instruction range [i0, i1); they are processed in chunks of kChunk.
// Defs (set 0) and uses (set 1) are sorted by the same launches: grid row y
// or the chunk's set field picks the set.
constexpr int kSortThreads = 256;
constexpr int kChunk = 2048;

struct SiteChunk {
  uint32_t func, begin, end, set;
};

struct SiteSet {
  const uint32_t *site_ptr;   // [n_instr + 1]
  const uint32_t *key;        // location of each site
  uint32_t *fl_ptr;           // [n_funcs][n_loc + 1] list starts, closing entry last
  uint32_t *sorted;           // sites in (function, location, instruction) order
  uint32_t *rank_of;          // site -> its position in sorted
};
struct SiteSets {
  SiteSet set[2];
};

__device__ __forceinline__ void func_sites(const SiteSet &ss, const uint32_t *fbb,
                                           const uint32_t *block_begin, uint32_t f, uint32_t &s0,
                                           uint32_t &s1) {
  s0 = ss.site_ptr[block_begin[fbb[f]]];
  s1 = ss.site_ptr[block_begin[fbb[f + 1]]];
}

// nchunks[set * n_funcs + f]
__global__ void k_chunk_count(uint32_t n_funcs, const uint32_t *fbb, const uint32_t *block_begin,
                              SiteSets sets, uint32_t *nchunks) {
  const uint32_t y = blockIdx.y;
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < n_funcs;
       f += gridDim.x * blockDim.x) {
    uint32_t s0, s1;
    func_sites(sets.set[y], fbb, block_begin, f, s0, s1);
    nchunks[y * n_funcs + f] = (s1 - s0 + kChunk - 1) / kChunk;
  }
}

__global__ void k_chunk_fill(uint32_t n_funcs, const uint32_t *fbb, const uint32_t *block_begin,
                             SiteSets sets, const uint32_t *chunk_start, SiteChunk *chunks) {
  const uint32_t y = blockIdx.y;
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < n_funcs;
       f += gridDim.x * blockDim.x) {
    uint32_t s0, s1;
    func_sites(sets.set[y], fbb, block_begin, f, s0, s1);
    uint32_t c = chunk_start[y * n_funcs + f];
    for (uint32_t a = s0; a < s1; a += kChunk, ++c) {
      SiteChunk ch;
      ch.func = f;
      ch.begin = a;
      ch.end = min(a + kChunk, s1);
      ch.set = y;
      chunks[c] = ch;
    }
  }
}

// per chunk, the number of sites of each location
__global__ void __launch_bounds__(kSortThreads)
k_chunk_hist(const SiteChunk *chunks, const unsigned long long *n_chunks, SiteSets sets,
             uint32_t n_loc, uint32_t *chunk_cnt) {
  extern __shared__ uint32_t cnt[];
  if (blockIdx.x >= *n_chunks) return;
  const SiteChunk ch = chunks[blockIdx.x];
  const uint32_t *key = sets.set[ch.set].key;
  for (uint32_t x = threadIdx.x; x < n_loc; x += kSortThreads) cnt[x] = 0;
  __syncthreads();
  for (uint32_t s = ch.begin + threadIdx.x; s < ch.end; s += kSortThreads) atomicAdd(&cnt[key[s]], 1u);
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < n_loc; x += kSortThreads)
    chunk_cnt[(size_t)blockIdx.x * n_loc + x] = cnt[x];
}

// per (function, set): start of each (function, location) list (fl_ptr) and
// each chunk's offset inside its location's list (written over the
// per-chunk counts; k_chunk_scatter adds the list start).  Each thread takes
// up to 4 locations and walks their columns eight chunks per batch of loads.
// Every list start is written, also for functions without sites.
__global__ void __launch_bounds__(kSortThreads)
k_chunk_bases(uint32_t n_funcs, const uint32_t *fbb, const uint32_t *block_begin, SiteSets sets,
              const uint32_t *chunk_start, const uint32_t *nchunks, uint32_t n_loc,
              uint32_t *chunk_cnt) {
  __shared__ uint32_t tmp[kSortThreads / kWave + 1];
  const uint32_t f = blockIdx.x, y = blockIdx.y;
  const SiteSet &ss = sets.set[y];
  uint32_t s0, s1;
  func_sites(ss, fbb, block_begin, f, s0, s1);
  const uint32_t c0 = chunk_start[y * n_funcs + f], nc = nchunks[y * n_funcs + f];
  const uint32_t per = (n_loc + kSortThreads - 1) / kSortThreads;   // <= 4
  const uint32_t x0 = min(threadIdx.x * per, n_loc), x1 = min(x0 + per, n_loc);
  uint32_t tot[4] = {0, 0, 0, 0};
  uint32_t mytot = 0;
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    const uint32_t x = x0 + i;
    if (x >= x1) continue;
    uint32_t run = 0;
    for (uint32_t c = 0; c < nc; c += 8) {
      uint32_t v[8];
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j)
        v[j] = c + j < nc ? chunk_cnt[(size_t)(c0 + c + j) * n_loc + x] : 0u;
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        if (c + j < nc) chunk_cnt[(size_t)(c0 + c + j) * n_loc + x] = run;
        run += v[j];
      }
    }
    tot[i] = run;
    mytot += run;
  }
  uint32_t total;
  uint32_t base = block_excl_scan<kSortThreads>(mytot, tmp, &total) + s0;
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    const uint32_t x = x0 + i;
    if (x >= x1) continue;
    ss.fl_ptr[(size_t)f * (n_loc + 1) + x] = base;
    base += tot[i];
  }
  // the function's closing entry: one past its last site
  if (threadIdx.x == 0) ss.fl_ptr[(size_t)f * (n_loc + 1) + n_loc] = s0 + total;
}

// Stable scatter: rounds of kSortThreads consecutive sites; the rank of a
// site among equal keys of its round comes from ballot matching inside the
// wave plus per-wave counts in LDS; per-location cursors carry across rounds.
__global__ void __launch_bounds__(kSortThreads)
k_chunk_scatter(const SiteChunk *chunks, const unsigned long long *n_chunks, SiteSets sets,
                uint32_t n_loc, uint32_t key_bits, const uint32_t *chunk_base) {
  extern __shared__ uint32_t sh[];
  uint32_t *cursor = sh;                        // [n_loc]
  uint32_t *wcnt = sh + n_loc;                  // [4][n_loc]
  constexpr int NW = kSortThreads / kWave;
  if (blockIdx.x >= *n_chunks) return;
  const SiteChunk ch = chunks[blockIdx.x];
  const SiteSet &ss = sets.set[ch.set];
  const uint32_t *key = ss.key;
  const unsigned tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  for (uint32_t x = tid; x < n_loc; x += kSortThreads) {
    cursor[x] = chunk_base[(size_t)blockIdx.x * n_loc + x] + ss.fl_ptr[(size_t)ch.func * (n_loc + 1) + x];
    for (int k = 0; k < NW; ++k) wcnt[k * n_loc + x] = 0;
  }
  __syncthreads();
  for (uint32_t r0 = ch.begin; r0 < ch.end; r0 += kSortThreads) {
    const uint32_t s = r0 + tid;
    const bool active = s < ch.end;
    const uint32_t k = active ? key[s] : 0xFFFFFFFFu;
    // lanes of this wave holding the same key
    uint64_t peers = __ballot(active);
    for (uint32_t bit = 0; bit < key_bits; ++bit) {
      const uint64_t m = __ballot(active && ((k >> bit) & 1u));
      peers &= ((k >> bit) & 1u) ? m : ~m;
    }
    const uint64_t lower = peers & ((1ull << lane) - 1ull);
    const uint32_t in_wave = __popcll(lower);
    if (active && lower == 0) wcnt[w * n_loc + k] = __popcll(peers);
    __syncthreads();
    if (active) {
      uint32_t before = 0;
      for (unsigned v = 0; v < w; ++v) before += wcnt[v * n_loc + k];
      const uint32_t pos = cursor[k] + before + in_wave;
      ss.sorted[pos] = s;
      ss.rank_of[s] = pos;
    }
    __syncthreads();
    if (active && lower == 0) {
      uint32_t tot = 0;
      for (int v = 0; v < NW; ++v) tot += wcnt[v * n_loc + k];
      // only the first wave holding this key advances the cursor
      bool first = true;
      for (unsigned v = 0; v < w; ++v)
        if (wcnt[v * n_loc + k]) first = false;
      if (first) cursor[k] += tot;
    }
    __syncthreads();
    if (active && lower == 0) wcnt[w * n_loc + k] = 0;
    __syncthreads();
  }
}

// site -> instruction, grid row 0 for the defs, 1 for the uses
__global__ void k_site_instr(uint32_t n_instr, const uint32_t *def_ptr, uint32_t *def_instr,
                             const uint32_t *use_ptr, uint32_t *use_instr) {
  const uint32_t *site_ptr = blockIdx.y ? use_ptr : def_ptr;
  uint32_t *site_instr = blockIdx.y ? use_instr : def_instr;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_instr; i += gridDim.x * blockDim.x)
    for (uint32_t s = site_ptr[i]; s < site_ptr[i + 1]; ++s) site_instr[s] = i;
}

// A use's search must cover its condition: the instruction's guard for an
// operand use, `_` for a guard read or a wait.
__global__ void k_use_cond(uint32_t n_uses, const uint32_t *use_instr, const uint8_t *use_kind,
                           const uint8_t *guard, uint8_t *cond) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_uses; u += gridDim.x * blockDim.x)
    cond[u] = use_kind[u] == GPA_USE_OPND ? guard[use_instr[u]] : (uint8_t)0;
}

// ------------------------------------------------------------------ scopes
__global__ void k_scope_info(uint32_t n_scopes, const uint32_t *parent, uint32_t *root_of,
                             uint32_t *depth) {
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_scopes;
       s += gridDim.x * blockDim.x) {
    uint32_t a = s, d = 0;
    while (parent[a] != GPA_NONE) {
      a = parent[a];
      ++d;
    }
    root_of[s] = a;
    depth[s] = d;
  }
}

// Preorder subtree ends: index t closes scope t-1 and every ancestor of it
// whose depth is at least depth[t] (t = n_scopes closes everything left);
// every scope is closed exactly once.
__global__ void k_scope_end(uint32_t n_scopes, const uint32_t *parent, const uint32_t *depth,
                            uint32_t *scope_end) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x + 1; t <= n_scopes;
       t += gridDim.x * blockDim.x) {
    uint32_t cur = t - 1;
    while (cur != GPA_NONE && (t == n_scopes || depth[cur] >= depth[t])) {
      scope_end[cur] = t;
      cur = parent[cur];
    }
  }
}

// bit0: some FUNCTION scope above the instruction is a math function;
// bit1: some FUNCTION scope above it is a device function with its own CFG
__global__ void k_instr_tags(uint32_t n_instr, const uint32_t *instr_scope, const uint32_t *parent,
                             const uint8_t *kind, const uint8_t *flags, uint8_t *tags) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_instr;
       i += gridDim.x * blockDim.x) {
    uint8_t t = 0;
    for (uint32_t s = instr_scope[i]; s != GPA_NONE; s = parent[s]) {
      if (kind[s] != GPA_SCOPE_FUNCTION) continue;
      if (flags[s] & GPA_SF_MATH_FN) t |= 1;
      if ((flags[s] & GPA_SF_DEVICE_FN) && (flags[s] & GPA_SF_HAS_CFG)) t |= 2;
    }
    tags[i] = t;
  }
}

// kernel roots in ascending scope order, by one workgroup (ballot ranks
// within a wave, a running count across the waves of each round)
__global__ void __launch_bounds__(1024)
k_roots(uint32_t n_scopes, const uint32_t *parent, uint32_t *roots, uint32_t *n) {
  __shared__ uint32_t wcnt[1024 / kWave];
  uint32_t base = 0;
  const unsigned w = threadIdx.x / kWave, lane = lane_id();
  for (uint32_t s0 = 0; s0 < n_scopes; s0 += 1024) {
    const uint32_t s = s0 + threadIdx.x;
    const bool is_root = s < n_scopes && parent[s] == GPA_NONE;
    const uint64_t m = __ballot(is_root);
    if (lane == 0) wcnt[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = base, total = 0;
    for (unsigned v = 0; v < 1024 / kWave; ++v) {
      if (v < w) before += wcnt[v];
      total += wcnt[v];
    }
    if (is_root) roots[before + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = s;
    base += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n = base;
}

// largest function: blocks, and CFG edges
// mx = (largest block count, largest edge count, sum over functions of the
// squared block count as a 64-bit value in words 2-3)
// (function bounds are clamped: this runs before the validation verdict)
__device__ void max_func_blocks_part(uint32_t t0_, uint32_t st_, uint32_t n_funcs, uint32_t n_blocks, const uint32_t *fbb,
                                  const uint32_t *succ_ptr, uint32_t *mx) {
  uint32_t m = 0, e = 0;
  unsigned long long sq = 0;
  for (uint32_t f = t0_; f < n_funcs;
       f += st_) {
    const uint32_t a = min(fbb[f], n_blocks), b = min(fbb[f + 1], n_blocks);
    const uint32_t nb = b - a;
    m = max(m, nb);
    e = max(e, succ_ptr[b] - succ_ptr[a]);
    sq += (unsigned long long)nb * nb;
  }
  atomicMax(&mx[0], m);
  atomicMax(&mx[1], e);
  if (sq) atomicAdd((unsigned long long *)(mx + 2), sq);
}

// The checks and maps run as two launches, each grid cut into sections of
// workgroups, one per check (a section runs the check's grid-stride loop
// over its own workgroups): first everything that needs only the inputs,
// then what needs the block maps.
struct ValArgs {
  uint32_t n_instr, n_blocks, n_funcs, n_scopes, n_preds, n_defs, n_uses, n_succ, n_loc;
  const uint8_t *op_class, *guard, *def_kind, *use_kind, *scope_kind, *scope_flags;
  const uint32_t *def_ptr, *use_ptr, *def_loc, *use_loc, *instr_scope, *fbb, *func_scope,
      *scope_parent, *block_begin, *succ_ptr, *succ;
  uint32_t *block_of, *func_of_block, *pred_cnt, *err, *mx;
};
constexpr int kValSectionsA = 7, kValSectionsB = 2;
struct ValSections {
  uint32_t start[kValSectionsA + 1];   // cumulative workgroup offsets
};

__device__ __forceinline__ uint32_t val_section(const ValSections &sec, int n, uint32_t &t0,
                                                uint32_t &st) {
  uint32_t q = 0;
  while ((int)q + 1 < n && blockIdx.x >= sec.start[q + 1]) ++q;
  t0 = (blockIdx.x - sec.start[q]) * blockDim.x + threadIdx.x;
  st = (sec.start[q + 1] - sec.start[q]) * blockDim.x;
  return q;
}

__global__ void k_val_inputs(ValArgs a, ValSections sec) {
  uint32_t t0, st;
  switch (val_section(sec, kValSectionsA, t0, st)) {
    case 0:
      val_instr_part(t0, st, a.n_instr, a.n_preds, a.n_scopes, a.n_defs, a.n_uses, a.op_class,
                     a.guard, a.def_ptr, a.use_ptr, a.def_loc, a.instr_scope, a.scope_kind, a.err);
      break;
    case 1:
      val_sites_part(t0, st, a.n_defs, a.def_loc, a.def_kind, a.n_loc, (uint32_t)GPA_DEF_RBAR,
                     kErrDef, a.err);
      break;
    case 2:
      val_sites_part(t0, st, a.n_uses, a.use_loc, a.use_kind, a.n_loc, (uint32_t)GPA_USE_WAIT,
                     kErrUse, a.err);
      break;
    case 3:
      val_funcs_part(t0, st, a.n_funcs, a.n_scopes, a.fbb, a.func_scope, a.scope_kind,
                     a.scope_flags, a.err);
      break;
    case 4:
      val_scopes_part(t0, st, a.n_scopes, a.scope_parent, a.scope_kind, a.scope_flags, a.err);
      break;
    case 5:
      blocks_part(t0, st, a.n_funcs, a.n_blocks, a.n_instr, a.fbb, a.block_begin, a.block_of,
                  a.func_of_block, a.pred_cnt, a.err);
      break;
    default:
      max_func_blocks_part(t0, st, a.n_funcs, a.n_blocks, a.fbb, a.succ_ptr, a.mx);
      break;
  }
}

__global__ void k_val_maps(ValArgs a, ValSections sec) {
  uint32_t t0, st;
  if (val_section(sec, kValSectionsB, t0, st) == 0)
    val_succ_part(t0, st, a.n_blocks, a.succ_ptr, a.succ, a.n_succ, a.func_of_block, a.pred_cnt,
                  a.err);
  else
    val_instr_scope_part(t0, st, a.n_instr, a.n_scopes, a.instr_scope, a.block_of,
                         a.func_of_block, a.func_scope, a.scope_parent, a.scope_kind,
                         a.scope_flags, a.err);
}

static void raise_validation(uint32_t err) {
  std::string msg = "invalid program descriptor:";
  for (int b = 0; b < 12; ++b)
    if (err & (1u << b)) {
      msg += " ";
      msg += kErrText[b];
      msg += ";";
    }
  fail(GPA_E_INVALID, "%s", msg.c_str());
}

// defs and uses sorted by (function, location, instruction), both sets in
// the same launches
static void sort_sites(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t nf = p.n_funcs, nl = p.n_loc;
  p.def_site_sorted.alloc(p.n_defs);
  p.use_site_sorted.alloc(p.n_uses);
  p.fl_def_ptr.alloc((size_t)nf * (nl + 1));
  p.fl_use_ptr.alloc((size_t)nf * (nl + 1));
  SiteSets sets;
  sets.set[0] = SiteSet{p.def_ptr.p, p.def_loc.p, p.fl_def_ptr.p, p.def_site_sorted.p, p.def_rank.p};
  sets.set[1] = SiteSet{p.use_ptr.p, p.use_loc.p, p.fl_use_ptr.p, p.use_site_sorted.p, p.use_rank.p};
  uint32_t *nchunks = ar.get<uint32_t>(2 * (size_t)nf);
  uint32_t *cstart = ar.get<uint32_t>(2 * (size_t)nf);
  unsigned long long *ntot = ar.get<unsigned long long>(1);
  hipLaunchKernelGGL(k_chunk_count, dim3(grid_for(nf, 256), 2), dim3(256), 0, s, nf,
                     p.func_block_begin.p, p.block_begin.p, sets, nchunks);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(nchunks, cstart, 2 * (size_t)nf, s, ar, ntot);
  // chunks <= sites / kChunk + one partial chunk per (function, set); the
  // kernels read the exact count from device memory
  const uint32_t n_chunks = (uint32_t)((p.n_defs + p.n_uses) / kChunk + 2 * nf);
  SiteChunk *chunks = ar.get<SiteChunk>(n_chunks);
  hipLaunchKernelGGL(k_chunk_fill, dim3(grid_for(nf, 256), 2), dim3(256), 0, s, nf,
                     p.func_block_begin.p, p.block_begin.p, sets, cstart, chunks);
  GPA_LAUNCH_CHECK();
  uint32_t *ccnt = ar.get<uint32_t>((size_t)n_chunks * nl);
  hipLaunchKernelGGL(k_chunk_hist, dim3(n_chunks), dim3(kSortThreads), nl * 4, s, chunks, ntot, sets,
                     nl, ccnt);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_chunk_bases, dim3(nf, 2), dim3(kSortThreads), 0, s, nf, p.func_block_begin.p,
                     p.block_begin.p, sets, cstart, nchunks, nl, ccnt);
  GPA_LAUNCH_CHECK();
  uint32_t key_bits = 1;
  while ((1u << key_bits) < nl) ++key_bits;
  const size_t lds = (size_t)nl * 4 * (1 + kSortThreads / kWave);
  hipLaunchKernelGGL(k_chunk_scatter, dim3(n_chunks), dim3(kSortThreads), lds, s, chunks, ntot, sets,
                     nl, key_bits, ccnt);
  GPA_LAUNCH_CHECK();
}

void validate_and_build_structure(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t n = p.n_instr, nb = p.n_blocks, nf = p.n_funcs, ns = p.n_scopes;
  // Every check and the maps they need run before one read of the verdict;
  // each kernel stays in bounds on any input (ranges are checked or clamped
  // before they index).  vals: error bits, then the largest-function sizes
  // (words 2-5, see k_max_func_blocks).
  uint32_t *vals = ar.get<uint32_t>(8);
  uint32_t *err = vals, *mx = vals + 2;
  p.sync_words = vals;
  hipLaunchKernelGGL(k_val_ends, dim3(1), dim3(1), 0, s, n, nb, nf, p.def_ptr.p, p.use_ptr.p,
                     p.block_begin.p, p.succ_ptr.p, p.func_block_begin.p, vals);
  // function and block maps (binary searches, in bounds on any input)
  p.block_of.alloc(n);
  p.func_of_block.alloc(nb);
  uint32_t *pcnt = ar.get<uint32_t>(nb + 1);   // predecessor counts, cleared by blocks_part
  ValArgs va{n, nb, nf, ns, p.n_preds, p.n_defs, p.n_uses, p.n_succ, p.n_loc,
             p.op_class.p, p.guard.p, p.def_kind.p, p.use_kind.p, p.scope_kind.p, p.scope_flags.p,
             p.def_ptr.p, p.use_ptr.p, p.def_loc.p, p.use_loc.p, p.instr_scope.p,
             p.func_block_begin.p, p.func_scope.p, p.scope_parent.p, p.block_begin.p,
             p.succ_ptr.p, p.succ.p, p.block_of.p, p.func_of_block.p, pcnt, err, mx};
  ValSections sa{}, sb{};
  {
    const unsigned g[kValSectionsA] = {grid_for(n, 256, 2048), grid_for(p.n_defs, 256, 2048),
                                       grid_for(p.n_uses, 256, 2048), grid_for(nf, 256, 2048),
                                       grid_for(ns, 256, 2048),
                                       grid_for((size_t)nb + n, 256, 4096),
                                       grid_for(nf, 256, 1024)};
    for (int q = 0; q < kValSectionsA; ++q) sa.start[q + 1] = sa.start[q] + g[q];
    const unsigned h2[kValSectionsB] = {grid_for(nb, 256, 2048), grid_for(n, 256, 2048)};
    for (int q = 0; q < kValSectionsB; ++q) sb.start[q + 1] = sb.start[q] + h2[q];
  }
  hipLaunchKernelGGL(k_val_inputs, dim3(sa.start[kValSectionsA]), dim3(256), 0, s, va, sa);
  GPA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_val_maps, dim3(sb.start[kValSectionsB]), dim3(256), 0, s, va, sb);
  GPA_LAUNCH_CHECK();
  uint32_t h[6];
  GPA_HIP(hipMemcpyAsync(h, vals, sizeof(h), hipMemcpyDeviceToHost, s));
  GPA_HIP(hipStreamSynchronize(s));
  if (h[0]) raise_validation(h[0]);
  p.max_func_blocks = h[2];
  p.max_func_edges = h[3];
  p.dist_entries = (uint64_t)h[4] | ((uint64_t)h[5] << 32);
  if (p.max_func_blocks > 4096)
    fail(GPA_E_UNSUPPORTED, "a function has %u blocks; at most 4096 are supported",
         p.max_func_blocks);
  // predecessor lists (the successor lists are valid from here on)
  p.pred_ptr.alloc(nb + 1);
  p.pred.alloc(p.n_succ);
  exclusive_scan_u32(pcnt, p.pred_ptr.p, nb + 1, s, ar);
  hipLaunchKernelGGL(k_fill_pred, dim3(grid_for(nb, 256, 2048)), dim3(256), 0, s, nb, p.succ_ptr.p,
                     p.succ.p, p.pred_ptr.p, pcnt, p.pred.p);
  hipLaunchKernelGGL(k_sort_pred, dim3(grid_for(nb, 256, 2048)), dim3(256), 0, s, nb,
                     p.pred_ptr.p, p.pred.p);
  GPA_LAUNCH_CHECK();
}

void build_sites_and_scopes(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t n = p.n_instr, ns = p.n_scopes;
  // sites by (function, location, instruction)
  p.def_instr.alloc(p.n_defs);
  p.use_instr.alloc(p.n_uses);
  hipLaunchKernelGGL(k_site_instr, dim3(grid_for(n, 256, 2048), 2), dim3(256), 0, s, n,
                     p.def_ptr.p, p.def_instr.p, p.use_ptr.p, p.use_instr.p);
  GPA_LAUNCH_CHECK();
  p.def_rank.alloc(p.n_defs);
  p.use_rank.alloc(p.n_uses);
  sort_sites(p, s, ar);
  p.use_cond.alloc(p.n_uses);
  hipLaunchKernelGGL(k_use_cond, dim3(grid_for(p.n_uses, 256, 4096)), dim3(256), 0, s, p.n_uses,
                     p.use_instr.p, p.use_kind.p, p.guard.p, p.use_cond.p);
  GPA_LAUNCH_CHECK();
  // scope tree
  p.root_of.alloc(ns);
  p.scope_depth.alloc(ns);
  p.scope_end.alloc(ns);
  hipLaunchKernelGGL(k_scope_info, dim3(grid_for(ns, 256, 4096)), dim3(256), 0, s, ns,
                     p.scope_parent.p, p.root_of.p, p.scope_depth.p);
  hipLaunchKernelGGL(k_scope_end, dim3(grid_for(ns, 256, 4096)), dim3(256), 0, s, ns,
                     p.scope_parent.p, p.scope_depth.p, p.scope_end.p);
  p.instr_tags.alloc(n);
  hipLaunchKernelGGL(k_instr_tags, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n,
                     p.instr_scope.p, p.scope_parent.p, p.scope_kind.p, p.scope_flags.p,
                     p.instr_tags.p);
  p.roots.alloc(ns);
  // the count is read with the next host synchronization of the load (word
  // 4 of the synchronization words, free after the validation verdict)
  p.n_roots_dev = p.sync_words + 4;
  hipLaunchKernelGGL(k_roots, dim3(1), dim3(1024), 0, s, ns, p.scope_parent.p, p.roots.p,
                     p.n_roots_dev);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
