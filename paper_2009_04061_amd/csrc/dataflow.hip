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
//     single range of ordinals that survives to the end, plus a kill flag;
//     these block summaries are computed once per (function, x, c).
// The per-use source lists then combine IN of the use's block (if nothing in
// the block before the use stops the search) with the in-block survivors.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kTileThreads = 256;
constexpr uint32_t kLdsBudget = 96 * 1024;
constexpr uint32_t kMaxWords = 16;
constexpr uint32_t kStageMax = 4096;     // defs / uses of one (function, x) staged in LDS
constexpr uint32_t kUnpred = 0x80000000u;

struct RdTile {
  uint32_t func, loc, chunk, cond;   // cond: guard byte the tile's uses must cover
  uint32_t words, n_blocks, block0, summ;   // summ: first block summary of its problem
};

struct BlockSumm {
  uint32_t gF, gB, hi, kill;   // survivor ranges [gF, hi), [gB, hi); kill bit0 full, bit1 blocked
};

__device__ __forceinline__ bool covers(uint32_t g, uint32_t c) { return g == 0 || g == c; }
__device__ __forceinline__ uint32_t complement(uint32_t g) { return (g & 1u) ? g + 1 : g - 1; }

// first index in [0, n) whose instruction (low 31 bits) is >= key
__device__ __forceinline__ uint32_t lower_instr(const uint32_t *a, uint32_t n, uint32_t key) {
  uint32_t lo = 0, hi = n;
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
                               uint8_t *dsg, uint32_t *usi) {
  const uint32_t tot = n_defs + n_uses;
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
// conditions the uses of each (function, location) must cover
__global__ void k_use_condmask(uint32_t n_uses, uint32_t n_loc, const uint32_t *use_instr,
                               const uint32_t *use_loc, const uint32_t *block_of,
                               const uint32_t *func_of_block, const uint8_t *use_cond,
                               unsigned long long *mask) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_uses; u += gridDim.x * blockDim.x) {
    const size_t q = (size_t)func_of_block[block_of[use_instr[u]]] * n_loc + use_loc[u];
    atomicOr(&mask[q], 1ull << use_cond[u]);
  }
}

// tile LDS: nb*(16W + 12) + 2*npred + 4 bytes (bitsets, summaries, pred CSR)
__device__ __host__ __forceinline__ uint32_t tile_words(uint32_t nb, uint32_t npred) {
  const uint32_t fixed = nb * 12u + 2u * npred + 8u;
  uint32_t w = fixed < kLdsBudget ? (kLdsBudget - fixed) / (16u * nb) : 0u;
  if (w < 1) w = 1;
  if (w > kMaxWords) w = kMaxWords;
  return w;
}

__global__ void k_fl_plan(uint32_t n_funcs, uint32_t n_loc, const uint32_t *fbb,
                          const uint32_t *succ_ptr, const uint32_t *fl_def_ptr,
                          const uint32_t *fl_use_ptr, uint32_t *fl_words, uint32_t *fl_chunks,
                          uint64_t *fl_condmask, uint32_t *fl_tiles, uint32_t *fl_summ) {
  const size_t total = (size_t)n_funcs * n_loc;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    const uint32_t f = (uint32_t)(q / n_loc), x = (uint32_t)(q % n_loc);
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const uint32_t nd = fl_def_ptr[fi + 1] - fl_def_ptr[fi];
    const uint32_t nu = fl_use_ptr[fi + 1] - fl_use_ptr[fi];
    const uint32_t nb = fbb[f + 1] - fbb[f];
    uint32_t w = tile_words(nb, succ_ptr[fbb[f + 1]] - succ_ptr[fbb[f]]);
    const uint32_t need = (nd + 63) / 64;
    if (w > need) w = need ? need : 1;
    const uint64_t mask = fl_condmask[q];   // guard bytes go up to 32
    const uint32_t chunks = (nd + 64 * w - 1) / (64 * w);
    const bool live = nd && nu;
    fl_words[q] = w;
    fl_chunks[q] = chunks;
    if (!live) fl_condmask[q] = 0ull;
    fl_tiles[q] = live ? chunks * (uint32_t)__popcll(mask) : 0u;
    fl_summ[q] = live ? nb * (uint32_t)__popcll(mask) : 0u;
  }
}

__global__ void k_fl_tiles(uint32_t n_funcs, uint32_t n_loc, const uint32_t *fbb,
                           const uint32_t *fl_words, const uint32_t *fl_chunks,
                           const uint64_t *fl_condmask, const uint32_t *fl_tile_start,
                           const uint32_t *fl_summ_start, RdTile *tiles) {
  const size_t total = (size_t)n_funcs * n_loc;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    uint64_t mask = fl_condmask[q];
    if (!mask) continue;
    const uint32_t f = (uint32_t)(q / n_loc), x = (uint32_t)(q % n_loc);
    const uint32_t nb = fbb[f + 1] - fbb[f];
    uint32_t t = fl_tile_start[q];
    uint32_t summ = fl_summ_start[q];
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
        d.n_blocks = nb;
        d.summ = summ;
        tiles[t++] = d;
      }
      summ += nb;
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
// Survivors of the defs of x among instructions [i_begin, i_end) of one
// block, for condition c: the first surviving ordinal g (survivors are
// [g, ord_end)) and whether something in the range stops everything before
// it (kill).  With `blocked`, unpredicated uses of x also stop the search.
// dI/dG: instruction and guard per def ordinal; uI: use instructions with
// the unpredicated flag, sorted.
struct Survive {
  uint32_t g, hi;
  bool kill;
};

__device__ Survive survivors(const uint32_t *dI, const uint8_t *dG, uint32_t nd, const uint32_t *uI,
                             uint32_t nu, uint32_t i_begin, uint32_t i_end, uint32_t c,
                             bool blocked) {
  const uint32_t lo = lower_instr(dI, nd, i_begin), hi = lower_instr(dI, nd, i_end);
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
    const uint32_t ulo = lower_instr(uI, nu, i_begin), uhi = lower_instr(uI, nu, i_end);
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
      r.g = lower_instr(dI, nd, qb);
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
    r.g = lower_instr(dI, nd, qb);
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

// ------------------------------------------------------- block summaries
// One workgroup per (function, x, c): the def and use views of (function, x)
// staged in LDS, then one summary per block.
__global__ void __launch_bounds__(kTileThreads)
k_rd_summ(const RdTile *tiles, const uint32_t *block_begin, const uint32_t *fl_def_ptr,
          const uint32_t *fl_use_ptr, uint32_t n_loc, const uint32_t *dsi, const uint8_t *dsg,
          const uint32_t *usi, BlockSumm *summ) {
  __shared__ uint32_t sI[kStageMax];
  __shared__ uint32_t sU[kStageMax];
  __shared__ uint8_t sG[kStageMax];
  const RdTile t = tiles[blockIdx.x];
  if (t.chunk != 0) return;
  const size_t fi = (size_t)t.func * (n_loc + 1) + t.loc;
  const uint32_t d0 = fl_def_ptr[fi], nd = fl_def_ptr[fi + 1] - d0;
  const uint32_t u0 = fl_use_ptr[fi], nu = fl_use_ptr[fi + 1] - u0;
  const uint32_t *dI = dsi + d0;
  const uint8_t *dG = dsg + d0;
  const uint32_t *uI = usi + u0;
  if (nd <= kStageMax) {
    for (uint32_t k = threadIdx.x; k < nd; k += kTileThreads) {
      sI[k] = dI[k];
      sG[k] = dG[k];
    }
    dI = sI;
    dG = sG;
  }
  if (nu <= kStageMax) {
    for (uint32_t k = threadIdx.x; k < nu; k += kTileThreads) sU[k] = uI[k];
    uI = sU;
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < t.n_blocks; b += kTileThreads) {
    const uint32_t i0 = block_begin[t.block0 + b], i1 = block_begin[t.block0 + b + 1];
    const Survive sF = survivors(dI, dG, nd, uI, nu, i0, i1, t.cond, false);
    const Survive sB = survivors(dI, dG, nd, uI, nu, i0, i1, t.cond, true);
    BlockSumm m;
    m.gF = sF.g;
    m.gB = sB.g;
    m.hi = sF.hi;
    m.kill = (sF.kill ? 1u : 0u) | (sB.kill ? 2u : 0u);
    summ[t.summ + b] = m;
  }
}

// ------------------------------------------------------------- the tiles
__global__ void __launch_bounds__(kTileThreads)
k_rd_tile(const RdTile *tiles, const uint32_t *pred_ptr, const uint32_t *pred,
          const BlockSumm *summ, const uint32_t *use_site_sorted, const uint32_t *use_instr,
          const uint32_t *fl_use_ptr, uint32_t n_loc, const uint8_t *use_cond,
          const uint32_t *block_of, const uint32_t *slot_start, uint64_t *rd_in) {
  extern __shared__ uint64_t lds[];
  const RdTile t = tiles[blockIdx.x];
  const uint32_t nb = t.n_blocks, W = t.words, b0 = t.block0;
  uint64_t *outF = lds;                        // [nb][W]
  uint64_t *outB = lds + (size_t)nb * W;       // [nb][W]
  uint64_t *sm = lds + 2 * (size_t)nb * W;     // [nb] clipped summaries
  uint32_t *lptr = (uint32_t *)(sm + nb);      // [nb+1] predecessor CSR, local ids
  uint16_t *lpred = (uint16_t *)(lptr + nb + 1);
  const uint32_t p_base = pred_ptr[b0];
  const uint32_t c0 = t.chunk * 64u * W, c1 = c0 + 64u * W;
  auto clip = [&](uint32_t v) { return v < c0 ? 0u : (v > c1 ? c1 - c0 : v - c0); };
  for (uint32_t b = threadIdx.x; b < nb; b += kTileThreads) {
    const BlockSumm m = summ[t.summ + b];
    sm[b] = (uint64_t)clip(m.gF) | ((uint64_t)clip(m.hi) << 14) | ((uint64_t)clip(m.gB) << 28) |
            ((uint64_t)(m.kill & 1u) << 62) | ((uint64_t)((m.kill >> 1) & 1u) << 63);
    lptr[b] = pred_ptr[b0 + b] - p_base;
    for (uint32_t w = 0; w < W; ++w) {
      outF[(size_t)b * W + w] = 0ull;
      outB[(size_t)b * W + w] = 0ull;
    }
  }
  const uint32_t np = pred_ptr[b0 + nb] - p_base;
  if (threadIdx.x == 0) lptr[nb] = np;
  for (uint32_t k = threadIdx.x; k < np; k += kTileThreads) lpred[k] = (uint16_t)(pred[p_base + k] - b0);
  __syncthreads();
  // each thread sweeps a contiguous run of blocks, in block order
  const uint32_t per = (nb + kTileThreads - 1) / kTileThreads;
  const uint32_t bb0 = min(threadIdx.x * per, nb), bb1 = min(bb0 + per, nb);
  for (;;) {
    int changed = 0;
    for (uint32_t b = bb0; b < bb1; ++b) {
      const uint64_t m = sm[b];
      const uint32_t gF = (uint32_t)(m & 0x3FFF), gE = (uint32_t)((m >> 14) & 0x3FFF);
      const uint32_t gB = (uint32_t)((m >> 28) & 0x3FFF);
      const bool kF = (m >> 62) & 1ull, kB = (m >> 63) & 1ull;
      const uint32_t p0 = lptr[b], p1 = lptr[b + 1];
      for (uint32_t w = 0; w < W; ++w) {
        uint64_t inF = 0, inB = 0;
        if (!kF || !kB) {
          for (uint32_t k = p0; k < p1; ++k) {
            const uint32_t pb = lpred[k];
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
  const size_t fi = (size_t)t.func * (n_loc + 1) + t.loc;
  const uint32_t ub = fl_use_ptr[fi], un = fl_use_ptr[fi + 1] - ub;
  for (uint32_t k = threadIdx.x; k < un; k += kTileThreads) {
    const uint32_t site = use_site_sorted[ub + k];
    if (use_cond[site] != t.cond) continue;
    const uint32_t b = block_of[use_instr[site]] - b0;
    const uint32_t p0 = lptr[b], p1 = lptr[b + 1];
    uint64_t *dst = rd_in + slot_start[ub + k] + (size_t)t.chunk * 2u * W;
    for (uint32_t w = 0; w < W; ++w) {
      uint64_t inF = 0, inB = 0;
      for (uint32_t q = p0; q < p1; ++q) {
        const uint32_t pb = lpred[q];
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
                           const uint32_t *block_begin, const uint32_t *dsi, const uint8_t *dsg,
                           const uint32_t *usi, const uint32_t *def_site_sorted,
                           const uint8_t *def_kind, const uint32_t *fl_def_ptr,
                           const uint32_t *fl_use_ptr, uint32_t n_loc, const uint32_t *fl_words,
                           const uint32_t *fl_chunks, const uint32_t *use_rank,
                           const uint32_t *slot_start, const uint64_t *rd_in, uint32_t *rd_cnt,
                           const uint32_t *rd_ptr, uint32_t *rd_src, uint8_t *rd_blk,
                           uint8_t *rd_nonrbar) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_uses; u += gridDim.x * blockDim.x) {
    const uint32_t j = use_instr[u], x = use_loc[u];
    const uint32_t b = block_of[j], f = func_of_block[b];
    const size_t fi = (size_t)f * (n_loc + 1) + x;
    const uint32_t d0 = fl_def_ptr[fi], nd = fl_def_ptr[fi + 1] - d0;
    if (nd == 0) {
      if (!fill) rd_cnt[u] = 0;
      continue;
    }
    const uint32_t u0 = fl_use_ptr[fi], nu = fl_use_ptr[fi + 1] - u0;
    const size_t q = (size_t)f * n_loc + x;
    const uint32_t W = fl_words[q], chunks = fl_chunks[q];
    const uint64_t *in = rd_in + slot_start[use_rank[u]];
    const uint32_t c = use_cond[u], i0 = block_begin[b];
    const Survive sF = survivors(dsi + d0, dsg + d0, nd, usi + u0, nu, i0, j, c, false);
    const Survive sB = survivors(dsi + d0, dsg + d0, nd, usi + u0, nu, i0, j, c, true);
    const uint32_t pj = sF.hi;
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
  uint32_t *dsi = ar.get<uint32_t>(p.n_defs), *usi = ar.get<uint32_t>(p.n_uses);
  uint8_t *dsg = ar.get<uint8_t>(p.n_defs);
  hipLaunchKernelGGL(k_sorted_views, dim3(grid_for((size_t)p.n_defs + p.n_uses, 256, 8192)),
                     dim3(256), 0, s, p.n_defs, p.n_uses, p.def_site_sorted.p, p.def_instr.p,
                     p.use_site_sorted.p, p.use_instr.p, p.guard.p, dsi, dsg, usi);
  uint32_t *fl_words = ar.get<uint32_t>(nfl), *fl_chunks = ar.get<uint32_t>(nfl);
  uint64_t *fl_mask = ar.get<uint64_t>(nfl);
  uint32_t *fl_tiles = ar.get<uint32_t>(nfl), *fl_summ = ar.get<uint32_t>(nfl);
  uint32_t *fl_tstart = ar.get<uint32_t>(nfl), *fl_sstart = ar.get<uint32_t>(nfl);
  GPA_HIP(hipMemsetAsync(fl_mask, 0, 8 * nfl, s));
  hipLaunchKernelGGL(k_use_condmask, dim3(grid_for(p.n_uses, 256, 8192)), dim3(256), 0, s,
                     p.n_uses, nl, p.use_instr.p, p.use_loc.p, p.block_of.p, p.func_of_block.p,
                     p.use_cond.p, (unsigned long long *)fl_mask);
  hipLaunchKernelGGL(k_fl_plan, dim3(grid_for(nfl, 256, 4096)), dim3(256), 0, s, nf, nl,
                     p.func_block_begin.p, p.succ_ptr.p, p.fl_def_ptr.p, p.fl_use_ptr.p, fl_words,
                     fl_chunks, fl_mask, fl_tiles, fl_summ);
  GPA_LAUNCH_CHECK();
  unsigned long long *ntiles_d = ar.get<unsigned long long>(1);
  unsigned long long *nsumm_d = ar.get<unsigned long long>(1);
  exclusive_scan_u32(fl_tiles, fl_tstart, nfl, s, ar, ntiles_d);
  exclusive_scan_u32(fl_summ, fl_sstart, nfl, s, ar, nsumm_d);
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
  const uint64_t nsumm = read_scalar(nsumm_d, s);
  const uint64_t nslot = read_scalar(nslot_d, s);
  uint64_t *rd_in = ar.get<uint64_t>(nslot);
  if (ntiles) {
    RdTile *tiles = ar.get<RdTile>(ntiles);
    BlockSumm *summ = ar.get<BlockSumm>(nsumm);
    hipLaunchKernelGGL(k_fl_tiles, dim3(grid_for(nfl, 256, 4096)), dim3(256), 0, s, nf, nl,
                       p.func_block_begin.p, fl_words, fl_chunks, fl_mask, fl_tstart, fl_sstart,
                       tiles);
    hipLaunchKernelGGL(k_rd_summ, dim3((unsigned)ntiles), dim3(kTileThreads), 0, s, tiles,
                       p.block_begin.p, p.fl_def_ptr.p, p.fl_use_ptr.p, nl, dsi, dsg, usi, summ);
    GPA_LAUNCH_CHECK();
    const size_t lds = std::max<size_t>(kLdsBudget, (size_t)p.max_func_blocks * 28u +
                                                        2u * p.max_func_edges + 16u);
    GPA_HIP(hipFuncSetAttribute((const void *)k_rd_tile, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(k_rd_tile, dim3((unsigned)ntiles), dim3(kTileThreads), lds, s, tiles,
                       p.pred_ptr.p, p.pred.p, summ, p.use_site_sorted.p, p.use_instr.p,
                       p.fl_use_ptr.p, nl, p.use_cond.p, p.block_of.p, slot_start, rd_in);
    GPA_LAUNCH_CHECK();
  }
  // per-use source lists
  uint32_t *rd_cnt = ar.get<uint32_t>(p.n_uses + 1);
  GPA_HIP(hipMemsetAsync(rd_cnt + p.n_uses, 0, 4, s));
  hipLaunchKernelGGL(k_rd_lists, dim3(grid_for(p.n_uses, 256, 8192)), dim3(256), 0, s, p.n_uses, 0,
                     p.use_instr.p, p.use_loc.p, p.use_cond.p, p.block_of.p, p.func_of_block.p,
                     p.block_begin.p, dsi, dsg, usi, p.def_site_sorted.p, p.def_kind.p,
                     p.fl_def_ptr.p, p.fl_use_ptr.p, nl, fl_words, fl_chunks, p.use_rank.p,
                     slot_start, rd_in, rd_cnt, nullptr, nullptr, nullptr, nullptr);
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
