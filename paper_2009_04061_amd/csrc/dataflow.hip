// Reaching definitions and the dependency graph (Sec. 4, "Backward slicing",
// "Construct a dependency graph", dominator pruning).
//
// The immediate sources of a use are found as the paper finds them, by a
// backward search from the use that stops on every path at the first def
// that settles it, run in parallel over all uses:
//
//   * a search is keyed by location x and the condition c the use must cover
//     (its guard for an operand use, `_` for a guard read or a wait); a def
//     covers c iff its guard is `_` or c; a def that completes a
//     complementary pair with the previous def of x in its block ({Pi} with
//     {!Pi} covers `_`) stops the search after its partner;
//   * the use-blocked variant (dominator pruning) also stops at every
//     unpredicated instruction that uses x;
//   * the search runs over blocks: inside one whole block the defs that
//     survive to its end are one range of def ordinals (the defs of x in
//     instruction order), plus a flag saying whether the block stops the
//     search; a dense (location, block) index gives each block's def and use
//     ranges in one load;
//   * one thread follows one use (both variants) and ORs the surviving
//     ranges of the blocks it reaches into that use's IN bitsets; a search
//     that reaches more blocks than a thread keeps track of is handed to a
//     whole workgroup, which repeats it breadth-first with LDS bitsets.
// The per-use source lists then combine IN of the use's block (if nothing in
// the block before the use stops the search) with the in-block survivors.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr uint32_t kUnpred = 0x80000000u;
constexpr int kSearchThreads = 256;      // (use, variant) searches per workgroup
constexpr int kLongThreads = 256;
constexpr uint32_t kSearchCap = 64;      // blocks one thread tracks per search
constexpr uint32_t kLongGrid = 512;      // workgroups that take the long searches
constexpr uint32_t kStagePred = 16 * 1024;   // LDS for a function's predecessor lists
constexpr uint32_t kStageRows = 48 * 1024;   // LDS for (location, block) index rows
constexpr uint32_t kKill = 0x80000000u;

__device__ __forceinline__ bool covers(uint32_t g, uint32_t c) { return g == 0 || g == c; }
__device__ __forceinline__ uint32_t complement(uint32_t g) { return (g & 1u) ? g + 1 : g - 1; }

// first position in [lo, hi) whose instruction (low 31 bits) is >= key
__device__ __forceinline__ uint32_t lower_pos(const uint32_t *a, uint32_t lo, uint32_t hi,
                                              uint32_t key) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if ((a[mid] & ~kUnpred) < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------ sorted views
// def ordinal -> instruction and guard; use -> instruction | unpredicated flag
__global__ void k_sorted_views(uint32_t n_defs, uint32_t n_uses, const uint32_t *def_site_sorted,
                               const uint32_t *def_instr, const uint32_t *use_site_sorted,
                               const uint32_t *use_instr, const uint8_t *guard, uint32_t *dsi,
                               uint8_t *dsg, uint32_t *usi, uint32_t *scal) {
  const uint32_t tot = n_defs + n_uses;
  // the plan's largest word count and the long-search counter start at zero
  if (blockIdx.x == 0 && threadIdx.x < 2) scal[threadIdx.x] = 0;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < tot; k += gridDim.x * blockDim.x) {
    if (k < n_defs) {
      const uint32_t i = def_instr[def_site_sorted[k]];
      dsi[k] = i;
      dsg[k] = guard[i];
    } else {
      const uint32_t q = k - n_defs;
      const uint32_t i = use_instr[use_site_sorted[q]];
      usi[q] = i | (guard[i] == 0 ? kUnpred : 0u);
    }
  }
}

// ------------------------------------------------------------------ plan
// IN bitset words per use site of (function, x): one word per 64 defs of x,
// twice (plain, use-blocked); the largest word count sizes the LDS of the
// workgroup search.
__global__ void k_rd_plan(uint32_t n_funcs, uint32_t n_loc, const uint32_t *fl_def_ptr,
                          uint32_t *fl_words, uint32_t *fl_chunks, uint32_t *max_words) {
  const size_t total = (size_t)n_funcs * n_loc;
  uint32_t mx = 0;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    const uint32_t f = (uint32_t)(q / n_loc), x = (uint32_t)(q % n_loc);
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const uint32_t nd = fl_def_ptr[fi + 1] - fl_def_ptr[fi];
    const uint32_t nw = (nd + 63) / 64;
    fl_words[q] = 1;
    fl_chunks[q] = nw;
    mx = max(mx, nw);
  }
  mx = wave_max_u32(mx);
  if (lane_id() == 0 && mx) atomicMax(max_words, mx);
}

// IN words each use site receives: chunks * 2 * words (plain, blocked)
__global__ void k_use_slots(uint32_t n_uses, const uint32_t *use_instr, const uint32_t *use_loc,
                            const uint32_t *block_of, const uint32_t *func_of_block,
                            uint32_t n_loc, const uint32_t *fl_words, const uint32_t *fl_chunks,
                            const uint32_t *use_rank, uint32_t *slot_words) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_uses; u += gridDim.x * blockDim.x) {
    const uint32_t f = func_of_block[block_of[use_instr[u]]];
    const size_t q = (size_t)f * n_loc + use_loc[u];
    slot_words[use_rank[u]] = fl_chunks[q] * 2u * fl_words[q];
  }
}

// --------------------------------------------------- block and prefix rules
// Survivors of the defs of x at positions [lo, hi) of one block (all defs of
// x in an instruction range of the block), for condition c: the first
// surviving position g (survivors are [g, hi)) and whether something in the
// range stops everything before it (kill).  With `blocked`, unpredicated
// uses of x (positions [ulo, uhi) of the sorted uses) also stop the search.
struct Survive {
  uint32_t g, hi;
  bool kill;
};

__device__ Survive survivors_range(const uint32_t *dI, const uint8_t *dG, const uint32_t *uI,
                                   uint32_t lo, uint32_t hi, uint32_t ulo, uint32_t uhi,
                                   uint32_t c, bool blocked) {
  // last def in the range that stops the search, and its kind
  uint32_t qk = 0xFFFFFFFFu;
  bool pair = false;
  for (uint32_t q = hi; q-- > lo;) {
    const uint32_t g = dG[q];
    if (covers(g, c)) {
      qk = q;
      break;
    }
    if (g != 0 && q > lo && dG[q - 1] == complement(g)) {
      qk = q;
      pair = true;
      break;
    }
  }
  // last unpredicated use of x in the range
  uint32_t qb = 0xFFFFFFFFu;
  if (blocked) {
    for (uint32_t q = uhi; q-- > ulo;) {
      if (uI[q] & kUnpred) {
        qb = uI[q] & ~kUnpred;
        break;
      }
    }
  }
  Survive r;
  r.hi = hi;
  if (qk != 0xFFFFFFFFu) {
    const uint32_t ik = dI[qk];
    if (qb != 0xFFFFFFFFu && qb > ik) {
      // a use after the last stopping def: only defs at or after the use survive
      r.g = lower_pos(dI, qk, hi, qb);
      r.kill = true;
      return r;
    }
    if (pair) {
      const uint32_t ip = dI[qk - 1];
      // the partner survives unless an unpredicated use sits between the two
      r.g = (qb != 0xFFFFFFFFu && qb > ip) ? qk : qk - 1;
    } else {
      r.g = qk;
    }
    r.kill = true;
    return r;
  }
  if (qb != 0xFFFFFFFFu) {
    r.g = lower_pos(dI, lo, hi, qb);
    r.kill = true;
    return r;
  }
  r.g = lo;
  r.kill = false;
  return r;
}

__device__ __forceinline__ uint64_t range_word(uint32_t lo, uint32_t hi, uint32_t w0) {
  // bits [lo, hi) intersected with word [w0, w0+64), shifted to the word
  const uint32_t a = max(lo, w0), b = min(hi, w0 + 64);
  if (a >= b) return 0ull;
  const uint32_t len = b - a;
  const uint64_t m = (len == 64) ? ~0ull : ((1ull << len) - 1ull);
  return m << (a - w0);
}

// ------------------------------------------------ (location, block) index
// For location x and block b (row-major by location, so a search over one
// location reads one row):
//   t0 = (g plain | kill << 31, g blocked | kill << 31, def end, def begin)
//        where the g are the block's survivors for condition `_` (the
//        condition of most uses), so such a visit is a single load;
//   t1 = (use begin, use end) for the other conditions, which rescan.
// Positions are absolute in the sorted def and use arrays.
__global__ void k_loc_block_index(uint32_t n_blocks, uint32_t n_loc, const uint32_t *func_of_block,
                                  const uint32_t *block_begin, const uint32_t *fl_def_ptr,
                                  const uint32_t *fl_use_ptr, const uint32_t *dsi,
                                  const uint8_t *dsg, const uint32_t *usi, uint4 *t0, uint2 *t1) {
  const size_t total = (size_t)n_loc * n_blocks;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)(k / n_blocks), b = (uint32_t)(k % n_blocks);
    const size_t fi = (size_t)func_of_block[b] * (n_loc + 1) + x;
    const uint32_t d0 = fl_def_ptr[fi], d1 = fl_def_ptr[fi + 1];
    const uint32_t u0 = fl_use_ptr[fi], u1 = fl_use_ptr[fi + 1];
    const uint32_t i0 = block_begin[b], i1 = block_begin[b + 1];
    const uint32_t dlo = lower_pos(dsi, d0, d1, i0), dhi = lower_pos(dsi, dlo, d1, i1);
    const uint32_t ulo = lower_pos(usi, u0, u1, i0), uhi = lower_pos(usi, ulo, u1, i1);
    const Survive f = survivors_range(dsi, dsg, usi, dlo, dhi, ulo, uhi, 0, false);
    const Survive g = survivors_range(dsi, dsg, usi, dlo, dhi, ulo, uhi, 0, true);
    t0[k] = make_uint4(f.g | (f.kill ? kKill : 0u), g.g | (g.kill ? kKill : 0u), dhi, dlo);
    t1[k] = make_uint2(ulo, uhi);
  }
}

// survivors of a whole block for a use of condition c, from the index
__device__ __forceinline__ Survive block_step(const uint4 &r, const uint2 *t1, size_t k,
                                              const uint32_t *dsi, const uint8_t *dsg,
                                              const uint32_t *usi, uint32_t c, bool blocked) {
  if (c == 0) {
    const uint32_t v = blocked ? r.y : r.x;
    Survive s;
    s.g = v & ~kKill;
    s.hi = r.z;
    s.kill = (v & kKill) != 0;
    return s;
  }
  const uint2 u = t1[k];
  return survivors_range(dsi, dsg, usi, r.w, r.z, u.x, u.y, c, blocked);
}

// OR the def positions [g, hi) (absolute; the bitset starts at d0) into the
// words of one IN bitset whose word w sits at in[2 * w]
__device__ __forceinline__ void or_range(uint64_t *in, uint32_t d0, uint32_t g, uint32_t hi) {
  if (g >= hi) return;
  const uint32_t a = g - d0, b = hi - d0;
  for (uint32_t w = a / 64; w * 64 < b; ++w) in[2 * w] |= range_word(a, b, w * 64);
}

// ------------------------------------------------------- the searches
// One thread per (use site, variant): threads [0, n) take the plain search
// of the sorted use sites, threads [n, 2n) the use-blocked one, so a wave's
// uses share a location.  A breadth-first search backwards from the use's
// block over whole predecessor blocks; the blocks met are kept in a
// per-thread list in LDS (also the queue), with a 256-bit filter in
// registers to skip most list scans; a thread's list is contiguous (rows
// padded to 144 bytes, so that 16-byte reads of a wave's 16-lane groups hit
// distinct banks) and a scan reads eight entries per load.  A workgroup stages in LDS what most of
// its visits read: the predecessor lists of its function (the function of
// its first use) as local ids, and the index rows (survivors for condition
// `_` and def end, per block) of the (location, variant) of its first and of
// its last search; other visits read the index in global memory.  IN
// bitsets of up to kRegWords words are accumulated in registers and written
// once; longer ones are OR-ed in place.  A search that would meet more than
// kSearchCap blocks is left to k_rd_search_long.
constexpr uint32_t kRegWords = 8;
constexpr uint32_t kSeenStride = kSearchCap + 8;   // u16 entries per thread row
constexpr uint32_t kSearchStage = 8160;   // predecessor lists, bytes
constexpr uint32_t kRowStageBlocks = 2048;  // index rows are staged for functions up to this size

__global__ void __launch_bounds__(kSearchThreads)
k_rd_search(uint32_t n_uses, uint32_t n_blocks, uint32_t n_loc, uint32_t row_nb,
            const uint32_t *use_site_sorted, const uint32_t *use_instr, const uint32_t *use_loc,
            const uint8_t *use_cond, const uint32_t *block_of, const uint32_t *func_of_block,
            const uint32_t *fbb, const uint32_t *pred_ptr, const uint32_t *pred,
            const uint32_t *fl_def_ptr, const uint32_t *dsi, const uint8_t *dsg,
            const uint32_t *usi, const uint4 *t0, const uint2 *t1, const uint32_t *slot_start,
            uint64_t *rd_in, uint32_t *long_list, uint32_t *n_long) {
  __shared__ __align__(16) uint16_t seen[kSeenStride * kSearchThreads];
  __shared__ uint16_t stage[kSearchStage / 2];   // [nb + 1] list starts, then the lists
  extern __shared__ uint2 s_rows[];              // [2][row_nb]: (survivor | kill, def end)
  __shared__ uint32_t s_f, s_ok, s_key[2];
  const unsigned tid = threadIdx.x;
  const uint32_t t = blockIdx.x * kSearchThreads + tid;
  // (location | variant << 31) of search tt, whose function is f
  auto key_of = [&](uint32_t tt, uint32_t &f) {
    const uint32_t v = tt >= n_uses ? 1u : 0u;
    const uint32_t u = use_site_sorted[tt - v * n_uses];
    f = func_of_block[block_of[use_instr[u]]];
    return use_loc[u] | (v << 31);
  };
  // the workgroup's first thread is always a valid search
  if (tid == 0) {
    const uint32_t t_first = blockIdx.x * kSearchThreads;
    const uint32_t t_last = min(t_first + kSearchThreads, 2 * n_uses) - 1;
    uint32_t f, fl;
    const uint32_t ka = key_of(t_first, f), kb = key_of(t_last, fl);
    const uint32_t b0 = fbb[f], nb = fbb[f + 1] - b0;
    const uint32_t np = pred_ptr[b0 + nb] - pred_ptr[b0];
    s_f = f;
    s_ok = (nb + 1 + np) * 2u <= kSearchStage ? 1u : 0u;
    const bool rows = row_nb != 0 && nb <= row_nb;
    s_key[0] = rows ? ka : 0xFFFFFFFFu;
    s_key[1] = (rows && fl == f && kb != ka) ? kb : 0xFFFFFFFFu;
  }
  __syncthreads();
  const uint32_t sf = s_f;
  const bool staged = s_ok != 0;
  uint16_t *s_pp = stage, *s_pr = stage;
  {
    const uint32_t b0 = fbb[sf], nb = fbb[sf + 1] - b0;
    if (staged) {
      const uint32_t p0 = pred_ptr[b0], np = pred_ptr[b0 + nb] - p0;
      s_pr = stage + nb + 1;
      for (uint32_t q = tid; q <= nb; q += kSearchThreads) s_pp[q] = (uint16_t)(pred_ptr[b0 + q] - p0);
      for (uint32_t q = tid; q < np; q += kSearchThreads) s_pr[q] = (uint16_t)(pred[p0 + q] - b0);
    }
    for (int sl = 0; sl < 2; ++sl) {
      const uint32_t key = s_key[sl];
      if (key == 0xFFFFFFFFu) continue;
      const size_t rw = (size_t)(key & 0x7FFFFFFFu) * n_blocks + b0;
      const bool bl = (key >> 31) != 0;
      for (uint32_t q = tid; q < nb; q += kSearchThreads) {
        const uint4 r = t0[rw + q];
        s_rows[sl * row_nb + q] = make_uint2(bl ? r.y : r.x, r.z);
      }
    }
  }
  __syncthreads();
  if (t >= 2 * n_uses) return;
  const uint32_t var = t >= n_uses ? 1u : 0u;
  const uint32_t k = t - var * n_uses;
  const bool blocked = var == 1;
  const uint32_t u = use_site_sorted[k];
  const uint32_t j = use_instr[u], x = use_loc[u];
  const uint32_t b = block_of[j], f = func_of_block[b], b0 = fbb[f];
  const size_t fi = (size_t)f * (n_loc + 1) + x;
  const uint32_t d0 = fl_def_ptr[fi];
  const uint32_t nd = fl_def_ptr[fi + 1] - d0;
  if (nd == 0) return;
  const uint32_t nw = (nd + 63) / 64;
  const bool local = nw <= kRegWords;
  const bool mine = staged && f == sf;   // this thread's function is the staged one
  const uint32_t c = use_cond[u];
  const uint32_t my_key = x | (var << 31);
  // a staged index row serves this search when its key matches and the
  // condition is `_` (other conditions rescan the block's defs)
  const int slot = (c != 0 || f != sf) ? -1 : (my_key == s_key[0] ? 0 : (my_key == s_key[1] ? 1 : -1));
  const uint2 *my_row = s_rows + (slot < 0 ? 0 : slot) * row_nb;
  const size_t row = (size_t)x * n_blocks + b0;
  uint64_t *in = rd_in + slot_start[k] + var;
  uint64_t acc[kRegWords];
#pragma unroll
  for (uint32_t w = 0; w < kRegWords; ++w) acc[w] = 0ull;
  // every word of the slot is written by its own search: registers for a
  // short bitset, stored at the end; a long one is cleared here and built in
  // place (a search that overflows is redone whole by the long kernel)
  if (!local)
    for (uint32_t w = 0; w < nw; ++w) in[2 * w] = 0ull;
  uint32_t n_seen = 0, head = 0;
  uint64_t fl0 = 0, fl1 = 0, fl2 = 0, fl3 = 0;
  bool ok = true;
  uint16_t *my = seen + tid * kSeenStride;
  auto visit = [&](uint32_t pl) {
    const uint32_t h = (pl * 0x9E3779B1u) >> 24;
    const uint64_t bit = 1ull << (h & 63);
    const uint32_t hw = h >> 6;
    const uint64_t fl = hw == 0 ? fl0 : hw == 1 ? fl1 : hw == 2 ? fl2 : fl3;
    if (fl & bit) {
      for (uint32_t q0 = 0; q0 < n_seen; q0 += 8) {
        const uint4 v = *(const uint4 *)(my + q0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        bool hit = false;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
          const uint32_t e = (w[i / 2] >> (16 * (i & 1))) & 0xFFFFu;
          hit |= (q0 + i < n_seen) && e == pl;
        }
        if (hit) return;
      }
    }
    if (n_seen == kSearchCap) {
      ok = false;
      return;
    }
    fl0 |= hw == 0 ? bit : 0ull;
    fl1 |= hw == 1 ? bit : 0ull;
    fl2 |= hw == 2 ? bit : 0ull;
    fl3 |= hw == 3 ? bit : 0ull;
    my[n_seen++] = (uint16_t)pl;
  };
  // predecessors of local block pl: staged lists or the global CSR
  auto visit_preds = [&](uint32_t pl) {
    if (mine) {
      const uint32_t qa = s_pp[pl], qb = s_pp[pl + 1];
      for (uint32_t q = qa; q < qb && ok; ++q) visit(s_pr[q]);
    } else {
      const uint32_t qa = pred_ptr[b0 + pl], qb = pred_ptr[b0 + pl + 1];
      for (uint32_t q = qa; q < qb && ok; ++q) visit(pred[q] - b0);
    }
  };
  visit_preds(b - b0);
  while (ok && head < n_seen) {
    const uint32_t pl = my[head++];
    Survive sv;
    if (slot >= 0) {
      const uint2 e = my_row[pl];
      sv.g = e.x & ~kKill;
      sv.kill = (e.x & kKill) != 0;
      sv.hi = e.y;
    } else {
      const uint4 r = t0[row + pl];
      sv = block_step(r, t1, row + pl, dsi, dsg, usi, c, blocked);
    }
    if (sv.g < sv.hi) {
      const uint32_t lo = sv.g - d0, hi = sv.hi - d0;
      if (local) {
#pragma unroll
        for (uint32_t w = 0; w < kRegWords; ++w) acc[w] |= range_word(lo, hi, 64 * w);
      } else {
        for (uint32_t w = lo / 64; w * 64 < hi; ++w) in[2 * w] |= range_word(lo, hi, 64 * w);
      }
    }
    if (!sv.kill) visit_preds(pl);
  }
  if (!ok) {
    long_list[atomicAdd(n_long, 1u)] = k | (var << 31);
    return;
  }
  if (local) {
#pragma unroll
    for (uint32_t w = 0; w < kRegWords; ++w)
      if (w < nw) in[2 * w] = acc[w];
  }
}

__global__ void __launch_bounds__(kLongThreads)
k_rd_search_long(uint32_t n_blocks, uint32_t n_loc, uint32_t max_nb, uint32_t max_words,
                 const uint32_t *use_site_sorted, const uint32_t *use_instr,
                 const uint32_t *use_loc, const uint8_t *use_cond, const uint32_t *block_of,
                 const uint32_t *func_of_block, const uint32_t *fbb, const uint32_t *pred_ptr,
                 const uint32_t *pred, const uint32_t *fl_def_ptr, const uint32_t *dsi,
                 const uint8_t *dsg, const uint32_t *usi, const uint4 *t0, const uint2 *t1,
                 const uint32_t *slot_start, uint64_t *rd_in, const uint32_t *long_list,
                 const uint32_t *n_long) {
  extern __shared__ uint4 lds_l[];
  const uint32_t vis_words = (max_nb + 31) / 32;
  uint4 *s_row = lds_l;                                          // kStageRows bytes
  uint64_t *bits = (uint64_t *)(s_row + kStageRows / 16);        // [max_words]
  uint32_t *s_ptr = (uint32_t *)(bits + max_words);               // kStagePred bytes
  uint16_t *s_predl = nullptr;
  uint32_t *vis = (uint32_t *)((char *)s_ptr + kStagePred);       // [vis_words]
  uint16_t *q0 = (uint16_t *)(vis + vis_words);                   // [max_nb]
  uint16_t *q1 = q0 + max_nb;                                     // [max_nb]
  __shared__ uint32_t n_cur, n_next;
  const unsigned tid = threadIdx.x;
  const uint32_t nl = *n_long;
  for (uint32_t i = blockIdx.x; i < nl; i += gridDim.x) {
    const uint32_t k = long_list[i] & 0x7FFFFFFFu;
    const int var = (int)(long_list[i] >> 31);
    const uint32_t u = use_site_sorted[k];
    const uint32_t j = use_instr[u], x = use_loc[u];
    const uint32_t b = block_of[j], f = func_of_block[b], b0 = fbb[f];
    const uint32_t nb = fbb[f + 1] - b0;
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const uint32_t d0 = fl_def_ptr[fi], nd = fl_def_ptr[fi + 1] - d0;
    const uint32_t nw = (nd + 63) / 64;
    const uint32_t c = use_cond[u];
    const size_t row = (size_t)x * n_blocks;
    uint64_t *in = rd_in + slot_start[k];
    const uint32_t p0 = pred_ptr[b0], np = pred_ptr[b0 + nb] - p0;
    const bool sp = (nb + 1) * 4u + np * 2u <= kStagePred;
    const bool sr = nb * 16u <= kStageRows;
    __syncthreads();
    s_predl = (uint16_t *)(s_ptr + nb + 1);
    if (sp) {
      for (uint32_t q = tid; q <= nb; q += kLongThreads) s_ptr[q] = pred_ptr[b0 + q] - p0;
      for (uint32_t q = tid; q < np; q += kLongThreads) s_predl[q] = (uint16_t)(pred[p0 + q] - b0);
    }
    if (sr)
      for (uint32_t q = tid; q < nb; q += kLongThreads) s_row[q] = t0[row + b0 + q];
    {
      const bool blocked = var == 1;
      __syncthreads();
      for (uint32_t w = tid; w < nw; w += kLongThreads) bits[w] = 0ull;
      for (uint32_t w = tid; w < (nb + 31) / 32; w += kLongThreads) vis[w] = 0u;
      if (tid == 0) n_cur = 0;
      __syncthreads();
      auto claim = [&](uint32_t pl, uint16_t *queue, uint32_t *count) {
        if (!(atomicOr(&vis[pl / 32], 1u << (pl % 32)) & (1u << (pl % 32))))
          queue[atomicAdd(count, 1u)] = (uint16_t)pl;
      };
      const uint32_t bl = b - b0;
      const uint32_t qa = sp ? s_ptr[bl] : pred_ptr[b] - p0;
      const uint32_t qb = sp ? s_ptr[bl + 1] : pred_ptr[b + 1] - p0;
      for (uint32_t q = qa + tid; q < qb; q += kLongThreads)
        claim(sp ? s_predl[q] : pred[p0 + q] - b0, q0, &n_cur);
      __syncthreads();
      uint16_t *cur = q0, *nxt = q1;
      for (;;) {
        const uint32_t nc = n_cur;
        if (nc == 0) break;
        __syncthreads();
        if (tid == 0) n_next = 0;
        __syncthreads();
        for (uint32_t t = tid; t < nc; t += kLongThreads) {
          const uint32_t pl = cur[t];
          const uint4 r = sr ? s_row[pl] : t0[row + b0 + pl];
          const Survive s = block_step(r, t1, row + b0 + pl, dsi, dsg, usi, c, blocked);
          if (s.g < r.z) {
            const uint32_t a = s.g - d0, e = r.z - d0;
            for (uint32_t w = a / 64; w * 64 < e; ++w)
              atomicOr((unsigned long long *)&bits[w], (unsigned long long)range_word(a, e, w * 64));
          }
          if (!s.kill) {
            const uint32_t ra = sp ? s_ptr[pl] : pred_ptr[b0 + pl] - p0;
            const uint32_t rb = sp ? s_ptr[pl + 1] : pred_ptr[b0 + pl + 1] - p0;
            for (uint32_t q = ra; q < rb; ++q) claim(sp ? s_predl[q] : pred[p0 + q] - b0, nxt, &n_next);
          }
        }
        __syncthreads();
        if (tid == 0) n_cur = n_next;
        uint16_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        __syncthreads();
      }
      for (uint32_t w = tid; w < nw; w += kLongThreads) in[2 * w + var] = bits[w];
    }
  }
}

// ------------------------------------------------------ per-use extraction
// Pass 0 counts the sources of every use site, pass 1 writes them (ordinal
// order is instruction order) with the blocked bit and whether the def is
// anything but a read barrier.
__global__ void k_rd_lists(uint32_t n_uses, int fill, const uint32_t *use_instr,
                           const uint32_t *use_loc, const uint8_t *use_cond,
                           const uint32_t *block_of, const uint32_t *func_of_block,
                           const uint32_t *block_begin, const uint32_t *dsi, const uint8_t *dsg,
                           const uint32_t *usi, const uint32_t *def_site_sorted,
                           const uint8_t *def_kind, const uint32_t *fl_def_ptr,
                           const uint32_t *fl_use_ptr, uint32_t n_loc, const uint32_t *fl_words,
                           const uint32_t *fl_chunks, const uint32_t *use_rank,
                           const uint32_t *slot_start, const uint64_t *rd_in, uint32_t *rd_cnt,
                           const uint32_t *rd_ptr, uint32_t *rd_src, uint8_t *rd_blk,
                           uint8_t *rd_nonrbar, uint32_t n_blocks, const uint4 *t0,
                           const uint2 *t1) {
  // the count array's extra entry, so that its exclusive scan ends in the total
  if (!fill && blockIdx.x == 0 && threadIdx.x == 0) rd_cnt[n_uses] = 0;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_uses; u += gridDim.x * blockDim.x) {
    const uint32_t j = use_instr[u], x = use_loc[u];
    const uint32_t b = block_of[j], f = func_of_block[b];
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const uint32_t d0 = fl_def_ptr[fi], nd = fl_def_ptr[fi + 1] - d0;
    if (nd == 0) {
      if (!fill) rd_cnt[u] = 0;
      continue;
    }
    const size_t q = (size_t)f * n_loc + x;
    const uint32_t W = fl_words[q], chunks = fl_chunks[q];
    const uint64_t *in = rd_in + slot_start[use_rank[u]];
    const uint32_t c = use_cond[u];
    // the defs and uses of x in j's block before j, from the block's index
    // entry (absolute positions in the sorted arrays), then relative to d0
    const size_t tk = (size_t)x * n_blocks + b;
    const uint4 r = t0[tk];
    const uint2 ur = t1[tk];
    const uint32_t lo = r.w, hi = lower_pos(dsi, r.w, r.z, j);
    const uint32_t ulo = ur.x, uhi = lower_pos(usi, ur.x, ur.y, j);
    Survive sF = survivors_range(dsi, dsg, usi, lo, hi, ulo, uhi, c, false);
    Survive sB = survivors_range(dsi, dsg, usi, lo, hi, ulo, uhi, c, true);
    sF.g -= d0;
    sB.g -= d0;
    const uint32_t pj = hi - d0;
    uint32_t cnt = 0;
    uint32_t pos = fill ? rd_ptr[u] : 0;
    for (uint32_t k = 0; k < chunks; ++k) {
      for (uint32_t w = 0; w < W; ++w) {
        const uint32_t o0 = (k * W + w) * 64u;
        if (o0 >= nd) break;
        const uint64_t F = (sF.kill ? 0ull : in[(size_t)k * 2 * W + w]) | range_word(sF.g, pj, o0);
        const uint64_t B = (sB.kill ? 0ull : in[(size_t)k * 2 * W + W + w]) | range_word(sB.g, pj, o0);
        if (!fill) {
          cnt += __popcll(F);
          continue;
        }
        uint64_t m = F;
        while (m) {
          const uint32_t bit = __ffsll((long long)m) - 1;
          m &= m - 1;
          rd_src[pos] = dsi[d0 + o0 + bit];
          rd_blk[pos] = (uint8_t)((B >> bit) & 1ull);
          rd_nonrbar[pos] = (uint8_t)(def_kind[def_site_sorted[d0 + o0 + bit]] != GPA_DEF_RBAR);
          ++pos;
        }
      }
    }
    if (!fill) rd_cnt[u] = cnt;
  }
}

// ------------------------------------------------------------------ edges
__global__ void k_edge_sort(uint32_t n_instr, const uint32_t *use_ptr, const uint32_t *rd_ptr,
                            const uint32_t *rd_src, const uint8_t *rd_blk,
                            const uint8_t *rd_nonrbar, uint64_t *items, uint32_t *in_cnt) {
  if (blockIdx.x == 0 && threadIdx.x == 0) in_cnt[n_instr] = 0;   // the scan's extra entry
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_instr;
       j += gridDim.x * blockDim.x) {
    const uint32_t a = rd_ptr[use_ptr[j]], b = rd_ptr[use_ptr[j + 1]];
    for (uint32_t k = a; k < b; ++k) {
      const uint64_t v = ((uint64_t)rd_src[k] << 8) | ((uint64_t)rd_nonrbar[k] << 1) | rd_blk[k];
      uint32_t p = k;
      while (p > a && items[p - 1] > v) {
        items[p] = items[p - 1];
        --p;
      }
      items[p] = v;
    }
    uint32_t distinct = 0;
    for (uint32_t k = a; k < b; ++k)
      if (k == a || (items[k] >> 8) != (items[k - 1] >> 8)) ++distinct;
    in_cnt[j] = distinct;
  }
}

// One edge per (i, j): kept by dominance if any carrying location keeps it,
// write-after-read if every carrying location is a read barrier of i.
// The edge's source opcode class is kept beside it (e_cls), so that the
// blamer reads it with the edge instead of gathering it through the source.
__global__ void k_edge_fill(uint32_t n_instr, const uint32_t *use_ptr, const uint32_t *rd_ptr,
                            const uint64_t *items, const uint32_t *in_ptr,
                            const uint8_t *op_class, uint32_t *e_src, uint32_t *e_dst,
                            uint8_t *e_flags, uint8_t *e_cls) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_instr;
       j += gridDim.x * blockDim.x) {
    const uint32_t a = rd_ptr[use_ptr[j]], b = rd_ptr[use_ptr[j + 1]];
    uint32_t e = in_ptr[j];
    uint32_t k = a;
    while (k < b) {
      const uint32_t src = (uint32_t)(items[k] >> 8);
      uint32_t blk = 0, nonrbar = 0;
      while (k < b && (uint32_t)(items[k] >> 8) == src) {
        blk |= (uint32_t)(items[k] & 1ull);
        nonrbar |= (uint32_t)((items[k] >> 1) & 1ull);
        ++k;
      }
      e_src[e] = src;
      e_dst[e] = j;
      e_cls[e] = op_class[src];
      e_flags[e] = (uint8_t)((blk ? GPA_E_DOM_KEEP : 0) | (nonrbar ? 0 : GPA_E_WAR));
      ++e;
    }
  }
}

// ------------------------------------------------------------------ host
void build_reaching_defs(gpa_program &p, hipStream_t s, Arena &ar, PhaseTimer &t_search) {
  const uint32_t nf = p.n_funcs, nl = p.n_loc, nb = p.n_blocks;
  const size_t nfl = (size_t)nf * nl;
  uint32_t *dsi = ar.get<uint32_t>(p.n_defs), *usi = ar.get<uint32_t>(p.n_uses);
  uint8_t *dsg = ar.get<uint8_t>(p.n_defs);
  // synchronization words: [0, 2) the IN slot total, [2] the largest IN
  // bitset in words, [3] the long searches, [4] the kernel roots (k_roots)
  uint32_t *scal = p.sync_words + 2;
  hipLaunchKernelGGL(k_sorted_views, dim3(grid_for((size_t)p.n_defs + p.n_uses, 256, 8192)),
                     dim3(256), 0, s, p.n_defs, p.n_uses, p.def_site_sorted.p, p.def_instr.p,
                     p.use_site_sorted.p, p.use_instr.p, p.guard.p, dsi, dsg, usi, scal);
  GPA_LAUNCH_CHECK();
  uint32_t *fl_words = ar.get<uint32_t>(nfl), *fl_chunks = ar.get<uint32_t>(nfl);
  hipLaunchKernelGGL(k_rd_plan, dim3(grid_for(nfl, 256, 4096)), dim3(256), 0, s, nf, nl,
                     p.fl_def_ptr.p, fl_words, fl_chunks, scal);
  GPA_LAUNCH_CHECK();
  // IN slots per use site, in sorted-use order
  uint32_t *slot_words = ar.get<uint32_t>(p.n_uses);
  uint32_t *slot_start = ar.get<uint32_t>(p.n_uses);
  unsigned long long *nslot_d = (unsigned long long *)p.sync_words;
  hipLaunchKernelGGL(k_use_slots, dim3(grid_for(p.n_uses, 256, 4096)), dim3(256), 0, s, p.n_uses,
                     p.use_instr.p, p.use_loc.p, p.block_of.p, p.func_of_block.p, nl, fl_words,
                     fl_chunks, p.use_rank.p, slot_words);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(slot_words, slot_start, p.n_uses, s, ar, nslot_d);
  // the (location, block) index (the searches and the per-use lists read
  // it) is built while the host waits for the sizes
  uint4 *t0 = ar.get<uint4>((size_t)nl * nb);
  uint2 *t1 = ar.get<uint2>((size_t)nl * nb);
  hipLaunchKernelGGL(k_loc_block_index, dim3(grid_for((size_t)nl * nb, 256, 8192)), dim3(256), 0,
                     s, nb, nl, p.func_of_block.p, p.block_begin.p, p.fl_def_ptr.p,
                     p.fl_use_ptr.p, dsi, dsg, usi, t0, t1);
  GPA_LAUNCH_CHECK();
  uint32_t h[5];
  GPA_HIP(hipMemcpyAsync(h, p.sync_words, sizeof(h), hipMemcpyDeviceToHost, s));
  GPA_HIP(hipStreamSynchronize(s));
  const unsigned long long nslot = (unsigned long long)h[0] | ((unsigned long long)h[1] << 32);
  const uint32_t max_words = h[2];
  if (p.n_roots_dev) p.n_roots = h[4];
  p.n_roots_dev = nullptr;
  uint64_t *rd_in = ar.get<uint64_t>(nslot ? nslot : 1);
  if (nslot) {
    const size_t lds_long = kStageRows + 8u * (size_t)max_words + kStagePred +
                            4u * ((p.max_func_blocks + 31) / 32) + 4u * (size_t)p.max_func_blocks;
    if (lds_long > 160 * 1024)
      fail(GPA_E_UNSUPPORTED, "a location has %u defs in one function (too many for one search)",
           64u * max_words);
    uint32_t *long_list = ar.get<uint32_t>(p.n_uses);
    t_search.begin(kPhaseRdSearch, s);
    // two staged index rows per workgroup when the largest function fits
    const uint32_t row_nb = p.max_func_blocks <= kRowStageBlocks ? p.max_func_blocks : 0u;
    const size_t lds_rows = (size_t)2 * 8 * row_nb;
    GPA_HIP(hipFuncSetAttribute((const void *)k_rd_search,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_rows));
    hipLaunchKernelGGL(k_rd_search, dim3((2 * p.n_uses + kSearchThreads - 1) / kSearchThreads),
                       dim3(kSearchThreads), lds_rows, s, p.n_uses, nb, nl, row_nb,
                       p.use_site_sorted.p,
                       p.use_instr.p, p.use_loc.p, p.use_cond.p, p.block_of.p, p.func_of_block.p,
                       p.func_block_begin.p, p.pred_ptr.p, p.pred.p, p.fl_def_ptr.p, dsi, dsg, usi,
                       t0, t1, slot_start, rd_in, long_list, scal + 1);
    GPA_LAUNCH_CHECK();
    GPA_HIP(hipFuncSetAttribute((const void *)k_rd_search_long,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_long));
    hipLaunchKernelGGL(k_rd_search_long, dim3(kLongGrid), dim3(kLongThreads), lds_long, s, nb,
                       nl, p.max_func_blocks, max_words, p.use_site_sorted.p, p.use_instr.p,
                       p.use_loc.p, p.use_cond.p, p.block_of.p, p.func_of_block.p,
                       p.func_block_begin.p, p.pred_ptr.p, p.pred.p, p.fl_def_ptr.p, dsi, dsg, usi,
                       t0, t1, slot_start, rd_in, long_list, scal + 1);
    GPA_LAUNCH_CHECK();
    t_search.end(s);
  }
  // per-use source lists
  uint32_t *rd_cnt = ar.get<uint32_t>(p.n_uses + 1);
  hipLaunchKernelGGL(k_rd_lists, dim3(grid_for(p.n_uses, 256, 8192)), dim3(256), 0, s, p.n_uses, 0,
                     p.use_instr.p, p.use_loc.p, p.use_cond.p, p.block_of.p, p.func_of_block.p,
                     p.block_begin.p, dsi, dsg, usi, p.def_site_sorted.p, p.def_kind.p,
                     p.fl_def_ptr.p, p.fl_use_ptr.p, nl, fl_words, fl_chunks, p.use_rank.p,
                     slot_start, rd_in, rd_cnt, nullptr, nullptr, nullptr, nullptr, nb, t0, t1);
  GPA_LAUNCH_CHECK();
  p.rd_ptr.alloc(p.n_uses + 1);
  unsigned long long *nrd_d = ar.get<unsigned long long>(1);
  exclusive_scan_u32(rd_cnt, p.rd_ptr.p, p.n_uses + 1, s, ar, nrd_d);
  p.n_rd = read_scalar(nrd_d, s);
  p.rd_src.alloc(p.n_rd);
  p.rd_blk.alloc(p.n_rd);
  p.rd_nonrbar.alloc(p.n_rd);
  hipLaunchKernelGGL(k_rd_lists, dim3(grid_for(p.n_uses, 256, 8192)), dim3(256), 0, s, p.n_uses, 1,
                     p.use_instr.p, p.use_loc.p, p.use_cond.p, p.block_of.p, p.func_of_block.p,
                     p.block_begin.p, dsi, dsg, usi, p.def_site_sorted.p, p.def_kind.p,
                     p.fl_def_ptr.p, p.fl_use_ptr.p, nl, fl_words, fl_chunks, p.use_rank.p,
                     slot_start, rd_in, nullptr, p.rd_ptr.p, p.rd_src.p, p.rd_blk.p,
                     p.rd_nonrbar.p, nb, t0, t1);
  GPA_LAUNCH_CHECK();
}

void build_edges(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t n = p.n_instr;
  uint64_t *items = ar.get<uint64_t>(p.n_rd);
  uint32_t *in_cnt = ar.get<uint32_t>(n + 1);
  hipLaunchKernelGGL(k_edge_sort, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, p.use_ptr.p,
                     p.rd_ptr.p, p.rd_src.p, p.rd_blk.p, p.rd_nonrbar.p, items, in_cnt);
  GPA_LAUNCH_CHECK();
  p.in_ptr.alloc(n + 1);
  unsigned long long *ne_d = ar.get<unsigned long long>(1);
  exclusive_scan_u32(in_cnt, p.in_ptr.p, n + 1, s, ar, ne_d);
  p.n_edges = read_scalar(ne_d, s);
  const uint64_t ne = p.n_edges;
  p.e_src.alloc(ne);
  p.e_dst.alloc(ne);
  p.e_flags.alloc(ne);
  p.e_cls.alloc(ne);
  hipLaunchKernelGGL(k_edge_fill, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, p.use_ptr.p,
                     p.rd_ptr.p, items, p.in_ptr.p, p.op_class.p, p.e_src.p, p.e_dst.p,
                     p.e_flags.p, p.e_cls.p);
  GPA_LAUNCH_CHECK();
  // (the grouping by source instruction is built with the target scopes)
}

}  // namespace gpa
