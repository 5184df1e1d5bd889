// Reaching definitions and the dependency graph (Sec. 4, "Backward slicing",
// "Construct a dependency graph", dominator pruning).
//
// The backward slice of a use reaches exactly the defs from which a path to
// the use exists with no intermediate instruction that stops the search, so
// the same relation is computed forward as bit-vector reaching definitions:
//
//   * RD separates by location x and by the condition c the use must cover
//     (its guard for an operand use, `_` for a guard read or a wait): a def
//     covers c iff its guard is `_` or c.  Within one (x, c) the transfer of
//     a def is  S := {d}  if it covers c,  S := {d, partner} if it completes
//     a complementary pair with the previous def of x in the block
//     ({Pi} with {!Pi} covers `_`), and  S := S + {d}  otherwise.
//   * The use-blocked variant (dominator pruning) also empties S at every
//     unpredicated instruction that uses x, before that instruction's defs.
//   * Bits are the defs of x in instruction order (ordinals), split into
//     chunks of 64*W so that one chunk's OUT bitsets for every block of the
//     function fit in LDS.  A workgroup owns one (function, x, c, chunk) tile
//     and iterates OUT[b] = GEN[b] | (KILL[b] ? 0 : OR_{p in pred(b)} OUT[p])
//     to the least fixed point, each thread sweeping a contiguous run of
//     blocks in order (chaotic iteration; it stops after a sweep that changes
//     nothing anywhere, when every block satisfies its equation).
//   * Inside one block the effect of the defs (and blocking uses) is a
//     single range of ordinals that survives to the end, plus a kill flag.
// The per-use source lists then combine IN of the use's block (if nothing in
// the block before the use stops the search) with the in-block survivors.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kTileThreads = 256;
constexpr uint32_t kLdsBudget = 64 * 1024;
constexpr uint32_t kMaxWords = 16;

struct RdTile {
  uint32_t func, loc, chunk, cond;   // cond: guard byte the tile's uses must cover
  uint32_t words, n_blocks, block0, pad;
};

__device__ __forceinline__ bool covers(uint32_t g, uint32_t c) { return g == 0 || g == c; }
__device__ __forceinline__ uint32_t complement(uint32_t g) { return (g & 1u) ? g + 1 : g - 1; }

// ------------------------------------------------------------------ plan
__global__ void k_fl_plan(uint32_t n_funcs, uint32_t n_loc, const uint32_t *fbb,
                          const uint32_t *fl_def_ptr, const uint32_t *fl_use_ptr,
                          const uint32_t *use_site_sorted, const uint8_t *use_cond,
                          uint32_t *fl_words, uint32_t *fl_chunks, uint64_t *fl_condmask,
                          uint32_t *fl_tiles) {
  const size_t total = (size_t)n_funcs * n_loc;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    const uint32_t f = (uint32_t)(q / n_loc), x = (uint32_t)(q % n_loc);
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const uint32_t nd = fl_def_ptr[fi + 1] - fl_def_ptr[fi];
    const uint32_t u0 = fl_use_ptr[fi], u1 = fl_use_ptr[fi + 1];
    const uint32_t nb = fbb[f + 1] - fbb[f];
    uint32_t w = kLdsBudget / (nb * 24u);   // two u64 bitsets and one u64 summary per block
    if (w < 1) w = 1;
    if (w > kMaxWords) w = kMaxWords;
    const uint32_t need = (nd + 63) / 64;
    if (w > need) w = need ? need : 1;
    uint64_t mask = 0;   // guard bytes go up to 32
    for (uint32_t k = u0; k < u1; ++k) mask |= 1ull << use_cond[use_site_sorted[k]];
    const uint32_t chunks = (nd + 64 * w - 1) / (64 * w);
    fl_words[q] = w;
    fl_chunks[q] = chunks;
    fl_condmask[q] = (nd && u1 > u0) ? mask : 0ull;
    fl_tiles[q] = (nd && u1 > u0) ? chunks * (uint32_t)__popcll(mask) : 0u;
  }
}

__global__ void k_fl_tiles(uint32_t n_funcs, uint32_t n_loc, const uint32_t *fbb,
                           const uint32_t *fl_words, const uint32_t *fl_chunks,
                           const uint64_t *fl_condmask, const uint32_t *fl_tile_start,
                           RdTile *tiles) {
  const size_t total = (size_t)n_funcs * n_loc;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    uint64_t mask = fl_condmask[q];
    if (!mask) continue;
    const uint32_t f = (uint32_t)(q / n_loc), x = (uint32_t)(q % n_loc);
    uint32_t t = fl_tile_start[q];
    while (mask) {
      const uint32_t c = (uint32_t)__ffsll((long long)mask) - 1;
      mask &= mask - 1;
      for (uint32_t k = 0; k < fl_chunks[q]; ++k) {
        RdTile d;
        d.func = f;
        d.loc = x;
        d.chunk = k;
        d.cond = c;
        d.words = fl_words[q];
        d.block0 = fbb[f];
        d.n_blocks = fbb[f + 1] - fbb[f];
        d.pad = 0;
        tiles[t++] = d;
      }
    }
  }
}

// IN words each use site receives: chunks * 2 * words (full, blocked)
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
// View of the defs of one (function, location): ordinal -> instruction.
struct DefView {
  const uint32_t *sorted;   // def sites sorted by (function, location, instruction)
  const uint32_t *instr;    // def site -> instruction
  uint32_t base, n;         // this list: sorted[base .. base+n)
  __device__ uint32_t at(uint32_t o) const { return instr[sorted[base + o]]; }
  // first ordinal whose instruction is >= i
  __device__ uint32_t lower(uint32_t i) const {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) / 2;
      if (at(mid) < i) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  }
};

struct UseView {
  const uint32_t *sorted;
  const uint32_t *instr;
  uint32_t base, n;
  __device__ uint32_t at(uint32_t o) const { return instr[sorted[base + o]]; }
  __device__ uint32_t lower(uint32_t i) const {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) / 2;
      if (at(mid) < i) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  }
};

// Survivors of the defs of x among instructions [i_begin, i_end) of one
// block, for condition c.  Returns the first surviving ordinal g (survivors
// are [g, ord_end)) and whether something in the range stops everything
// that came before (kill).  With `blocked`, unpredicated uses of x in the
// range also stop the search.
struct Survive {
  uint32_t g;
  bool kill;
};

__device__ Survive survivors(const DefView &D, const UseView &U, const uint8_t *guard,
                             uint32_t i_begin, uint32_t i_end, uint32_t c, bool blocked) {
  const uint32_t lo = D.lower(i_begin), hi = D.lower(i_end);
  // last def in the range that stops the search, and its kind
  uint32_t qk = 0xFFFFFFFFu;
  bool pair = false;
  for (uint32_t q = hi; q-- > lo;) {
    const uint32_t g = guard[D.at(q)];
    if (covers(g, c)) {
      qk = q;
      break;
    }
    if (g != 0 && q > lo && guard[D.at(q - 1)] == complement(g)) {
      qk = q;
      pair = true;
      break;
    }
  }
  // last unpredicated use of x in the range
  uint32_t qb = 0xFFFFFFFFu;
  if (blocked) {
    const uint32_t ulo = U.lower(i_begin), uhi = U.lower(i_end);
    for (uint32_t q = uhi; q-- > ulo;) {
      const uint32_t ins = U.at(q);
      if (guard[ins] == 0) {
        qb = ins;
        break;
      }
    }
  }
  Survive r;
  if (qk != 0xFFFFFFFFu) {
    const uint32_t ik = D.at(qk);
    if (qb != 0xFFFFFFFFu && qb > ik) {
      // a use after the last stopping def: only defs at or after the use survive
      r.g = D.lower(qb);
      r.kill = true;
      return r;
    }
    if (pair) {
      const uint32_t ip = D.at(qk - 1);
      // the partner survives unless an unpredicated use sits between the two
      r.g = (qb != 0xFFFFFFFFu && qb > ip) ? qk : qk - 1;
    } else {
      r.g = qk;
    }
    r.kill = true;
    return r;
  }
  if (qb != 0xFFFFFFFFu) {
    r.g = D.lower(qb);
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

// ------------------------------------------------------------- the tiles
__global__ void __launch_bounds__(kTileThreads)
k_rd_tile(const RdTile *tiles, const uint32_t *block_begin, const uint32_t *pred_ptr,
          const uint32_t *pred, const uint8_t *guard, const uint32_t *def_site_sorted,
          const uint32_t *def_instr, const uint32_t *use_site_sorted, const uint32_t *use_instr,
          const uint32_t *fl_def_ptr, const uint32_t *fl_use_ptr, uint32_t n_loc,
          const uint8_t *use_cond, const uint32_t *block_of, const uint32_t *slot_start,
          uint64_t *rd_in) {
  extern __shared__ uint64_t lds[];
  const RdTile t = tiles[blockIdx.x];
  const uint32_t nb = t.n_blocks, W = t.words, b0 = t.block0;
  uint64_t *outF = lds;                      // [nb][W]
  uint64_t *outB = lds + (size_t)nb * W;     // [nb][W]
  uint64_t *summ = lds + 2 * (size_t)nb * W; // [nb]: genF lo|hi, genB lo|hi, kill bits
  const size_t fi = (size_t)t.func * (n_loc + 1) + t.loc;
  DefView D{def_site_sorted, def_instr, fl_def_ptr[fi], fl_def_ptr[fi + 1] - fl_def_ptr[fi]};
  UseView U{use_site_sorted, use_instr, fl_use_ptr[fi], fl_use_ptr[fi + 1] - fl_use_ptr[fi]};
  const uint32_t c0 = t.chunk * 64u * W, c1 = c0 + 64u * W;
  // block summaries, clipped to this chunk's ordinals
  for (uint32_t b = threadIdx.x; b < nb; b += kTileThreads) {
    const uint32_t i0 = block_begin[b0 + b], i1 = block_begin[b0 + b + 1];
    const uint32_t hi = D.lower(i1);
    const Survive sF = survivors(D, U, guard, i0, i1, t.cond, false);
    const Survive sB = survivors(D, U, guard, i0, i1, t.cond, true);
    auto clip = [&](uint32_t v) { return v < c0 ? 0u : (v > c1 ? c1 - c0 : v - c0); };
    uint64_t m = (uint64_t)clip(sF.g) | ((uint64_t)clip(hi) << 14) | ((uint64_t)clip(sB.g) << 28) |
                 ((uint64_t)sF.kill << 62) | ((uint64_t)sB.kill << 63);
    summ[b] = m;
    for (uint32_t w = 0; w < W; ++w) {
      outF[(size_t)b * W + w] = 0ull;
      outB[(size_t)b * W + w] = 0ull;
    }
  }
  __syncthreads();
  // each thread sweeps a contiguous run of blocks, in block order
  const uint32_t per = (nb + kTileThreads - 1) / kTileThreads;
  const uint32_t bb0 = min(threadIdx.x * per, nb), bb1 = min(bb0 + per, nb);
  for (;;) {
    int changed = 0;
    for (uint32_t b = bb0; b < bb1; ++b) {
      const uint64_t m = summ[b];
      const uint32_t gF = (uint32_t)(m & 0x3FFF), gE = (uint32_t)((m >> 14) & 0x3FFF);
      const uint32_t gB = (uint32_t)((m >> 28) & 0x3FFF);
      const bool kF = (m >> 62) & 1ull, kB = (m >> 63) & 1ull;
      const uint32_t p0 = pred_ptr[b0 + b], p1 = pred_ptr[b0 + b + 1];
      for (uint32_t w = 0; w < W; ++w) {
        uint64_t inF = 0, inB = 0;
        if (!kF || !kB) {
          for (uint32_t k = p0; k < p1; ++k) {
            const uint32_t pb = pred[k] - b0;
            inF |= outF[(size_t)pb * W + w];
            inB |= outB[(size_t)pb * W + w];
          }
        }
        const uint64_t nF = (kF ? 0ull : inF) | range_word(gF, gE, 64u * w);
        const uint64_t nB = (kB ? 0ull : inB) | range_word(gB, gE, 64u * w);
        if (nF != outF[(size_t)b * W + w]) {
          outF[(size_t)b * W + w] = nF;
          changed = 1;
        }
        if (nB != outB[(size_t)b * W + w]) {
          outB[(size_t)b * W + w] = nB;
          changed = 1;
        }
      }
    }
    if (!__syncthreads_or(changed)) break;
  }
  // IN of each use's block, for the uses of x whose condition is this tile's
  for (uint32_t k = threadIdx.x; k < U.n; k += kTileThreads) {
    const uint32_t site = use_site_sorted[U.base + k];
    if (use_cond[site] != t.cond) continue;
    const uint32_t b = block_of[use_instr[site]] - b0;
    const uint32_t p0 = pred_ptr[b0 + b], p1 = pred_ptr[b0 + b + 1];
    uint64_t *dst = rd_in + slot_start[U.base + k] + (size_t)t.chunk * 2u * W;
    for (uint32_t w = 0; w < W; ++w) {
      uint64_t inF = 0, inB = 0;
      for (uint32_t q = p0; q < p1; ++q) {
        const uint32_t pb = pred[q] - b0;
        inF |= outF[(size_t)pb * W + w];
        inB |= outB[(size_t)pb * W + w];
      }
      dst[w] = inF;
      dst[W + w] = inB;
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
                           const uint32_t *block_begin, const uint8_t *guard,
                           const uint32_t *def_site_sorted, const uint32_t *def_instr,
                           const uint8_t *def_kind, const uint32_t *use_site_sorted,
                           const uint32_t *fl_def_ptr, const uint32_t *fl_use_ptr, uint32_t n_loc,
                           const uint32_t *fl_words, const uint32_t *fl_chunks,
                           const uint32_t *use_rank, const uint32_t *slot_start,
                           const uint64_t *rd_in, uint32_t *rd_cnt, const uint32_t *rd_ptr,
                           uint32_t *rd_src, uint8_t *rd_blk, uint8_t *rd_nonrbar) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_uses; u += gridDim.x * blockDim.x) {
    const uint32_t j = use_instr[u], x = use_loc[u];
    const uint32_t b = block_of[j], f = func_of_block[b];
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const DefView D{def_site_sorted, def_instr, fl_def_ptr[fi], fl_def_ptr[fi + 1] - fl_def_ptr[fi]};
    if (D.n == 0) {
      if (!fill) rd_cnt[u] = 0;
      continue;
    }
    const UseView U{use_site_sorted, use_instr, fl_use_ptr[fi], fl_use_ptr[fi + 1] - fl_use_ptr[fi]};
    const size_t q = (size_t)f * n_loc + x;
    const uint32_t W = fl_words[q], chunks = fl_chunks[q];
    const uint64_t *in = rd_in + slot_start[use_rank[u]];
    const uint32_t c = use_cond[u], i0 = block_begin[b];
    const uint32_t pj = D.lower(j);
    const Survive sF = survivors(D, U, guard, i0, j, c, false);
    const Survive sB = survivors(D, U, guard, i0, j, c, true);
    uint32_t cnt = 0;
    uint32_t pos = fill ? rd_ptr[u] : 0;
    for (uint32_t k = 0; k < chunks; ++k) {
      for (uint32_t w = 0; w < W; ++w) {
        const uint32_t o0 = (k * W + w) * 64u;
        if (o0 >= D.n) break;
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
          const uint32_t site = def_site_sorted[D.base + o0 + bit];
          rd_src[pos] = def_instr[site];
          rd_blk[pos] = (uint8_t)((B >> bit) & 1ull);
          rd_nonrbar[pos] = (uint8_t)(def_kind[site] != GPA_DEF_RBAR);
          ++pos;
        }
      }
    }
    if (!fill) rd_cnt[u] = cnt;
  }
}

// ------------------------------------------------------------------ edges
// The sources of all uses of j, sorted by source instruction in place; the
// number of distinct sources is the number of edges into j.
__global__ void k_edge_sort(uint32_t n_instr, const uint32_t *use_ptr, const uint32_t *rd_ptr,
                            const uint32_t *rd_src, const uint8_t *rd_blk,
                            const uint8_t *rd_nonrbar, uint64_t *items, uint32_t *in_cnt) {
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
__global__ void k_edge_fill(uint32_t n_instr, const uint32_t *use_ptr, const uint32_t *rd_ptr,
                            const uint64_t *items, const uint32_t *in_ptr, uint32_t *e_src,
                            uint32_t *e_dst, uint8_t *e_flags) {
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
      e_flags[e] = (uint8_t)((blk ? GPA_E_DOM_KEEP : 0) | (nonrbar ? 0 : GPA_E_WAR));
      ++e;
    }
  }
}

// ------------------------------------------------------------------ host
void build_reaching_defs(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t nf = p.n_funcs, nl = p.n_loc;
  const size_t nfl = (size_t)nf * nl;
  uint32_t *fl_words = ar.get<uint32_t>(nfl), *fl_chunks = ar.get<uint32_t>(nfl);
  uint64_t *fl_mask = ar.get<uint64_t>(nfl);
  uint32_t *fl_tiles = ar.get<uint32_t>(nfl);
  uint32_t *fl_tstart = ar.get<uint32_t>(nfl);
  hipLaunchKernelGGL(k_fl_plan, dim3(grid_for(nfl, 256, 4096)), dim3(256), 0, s, nf, nl,
                     p.func_block_begin.p, p.fl_def_ptr.p, p.fl_use_ptr.p, p.use_site_sorted.p,
                     p.use_cond.p, fl_words, fl_chunks, fl_mask, fl_tiles);
  GPA_LAUNCH_CHECK();
  unsigned long long *ntiles_d = ar.get<unsigned long long>(1);
  exclusive_scan_u32(fl_tiles, fl_tstart, nfl, s, ar, ntiles_d);
  // IN slots per use site, in sorted-use order
  uint32_t *slot_words = ar.get<uint32_t>(p.n_uses);
  uint32_t *slot_start = ar.get<uint32_t>(p.n_uses);
  unsigned long long *nslot_d = ar.get<unsigned long long>(1);
  hipLaunchKernelGGL(k_use_slots, dim3(grid_for(p.n_uses, 256, 4096)), dim3(256), 0, s, p.n_uses,
                     p.use_instr.p, p.use_loc.p, p.block_of.p, p.func_of_block.p, nl, fl_words,
                     fl_chunks, p.use_rank.p, slot_words);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(slot_words, slot_start, p.n_uses, s, ar, nslot_d);
  const uint64_t ntiles = read_scalar(ntiles_d, s);
  const uint64_t nslot = read_scalar(nslot_d, s);
  uint64_t *rd_in = ar.get<uint64_t>(nslot);
  if (ntiles) {
    RdTile *tiles = ar.get<RdTile>(ntiles);
    hipLaunchKernelGGL(k_fl_tiles, dim3(grid_for(nfl, 256, 4096)), dim3(256), 0, s, nf, nl,
                       p.func_block_begin.p, fl_words, fl_chunks, fl_mask, fl_tstart, tiles);
    GPA_LAUNCH_CHECK();
    // LDS per tile: nb * (16 W + 8) bytes, at most max(budget, 24 nb) by the choice of W
    const size_t lds_cap = std::max<size_t>(kLdsBudget, (size_t)p.max_func_blocks * 24u);
    GPA_HIP(hipFuncSetAttribute((const void *)k_rd_tile, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_cap));
    hipLaunchKernelGGL(k_rd_tile, dim3((unsigned)ntiles), dim3(kTileThreads), lds_cap, s, tiles,
                       p.block_begin.p, p.pred_ptr.p, p.pred.p, p.guard.p, p.def_site_sorted.p,
                       p.def_instr.p, p.use_site_sorted.p, p.use_instr.p, p.fl_def_ptr.p,
                       p.fl_use_ptr.p, nl, p.use_cond.p, p.block_of.p, slot_start, rd_in);
    GPA_LAUNCH_CHECK();
  }
  // per-use source lists
  uint32_t *rd_cnt = ar.get<uint32_t>(p.n_uses + 1);
  GPA_HIP(hipMemsetAsync(rd_cnt + p.n_uses, 0, 4, s));
  hipLaunchKernelGGL(k_rd_lists, dim3(grid_for(p.n_uses, 256, 8192)), dim3(256), 0, s, p.n_uses, 0,
                     p.use_instr.p, p.use_loc.p, p.use_cond.p, p.block_of.p, p.func_of_block.p,
                     p.block_begin.p, p.guard.p, p.def_site_sorted.p, p.def_instr.p, p.def_kind.p,
                     p.use_site_sorted.p, p.fl_def_ptr.p, p.fl_use_ptr.p, nl, fl_words, fl_chunks,
                     p.use_rank.p, slot_start, rd_in, rd_cnt, nullptr, nullptr, nullptr, nullptr);
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
                     p.block_begin.p, p.guard.p, p.def_site_sorted.p, p.def_instr.p, p.def_kind.p,
                     p.use_site_sorted.p, p.fl_def_ptr.p, p.fl_use_ptr.p, nl, fl_words, fl_chunks,
                     p.use_rank.p, slot_start, rd_in, nullptr, p.rd_ptr.p, p.rd_src.p, p.rd_blk.p,
                     p.rd_nonrbar.p);
  GPA_LAUNCH_CHECK();
}

void build_edges(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t n = p.n_instr;
  uint64_t *items = ar.get<uint64_t>(p.n_rd);
  uint32_t *in_cnt = ar.get<uint32_t>(n + 1);
  GPA_HIP(hipMemsetAsync(in_cnt + n, 0, 4, s));
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
  hipLaunchKernelGGL(k_edge_fill, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, p.use_ptr.p,
                     p.rd_ptr.p, items, p.in_ptr.p, p.e_src.p, p.e_dst.p, p.e_flags.p);
  GPA_LAUNCH_CHECK();
  // by source instruction, in edge order inside each source
  group_by_key(p.e_src.p, ne, n, p.out_ptr, p.out_perm, s, ar);
}

}  // namespace gpa
