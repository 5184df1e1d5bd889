// Edge distances (Sec. 4: latency pruning uses the paths from i to j in the
// CFG, apportioning uses the longest of them) and the static target scopes
// the estimators roll matched samples into (Sec. 5).
//
// Distances count the instructions strictly between i and j along a walk.
// They are computed between blocks and combined with the in-block offsets:
//   same block, i before j:  j - i - 1 for both;
//   otherwise:  (|B_i| - o_i - 1) + D(B_i -> B_j) + o_j  where D sums the
//   sizes of the intermediate blocks: the shortest walk of at least one edge
//   for dmin; for dmax the longest walk in G', the CFG without the edges that
//   are retreating in a depth-first search from the entry (successors in
//   CSR order, then from every unvisited block in index order), or dmin when
//   G' has no such walk.
#include <cstring>

#include "common.h"
#include "devutil.h"

namespace gpa {

// ------------------------------------------------------------------ DFS
// One wave per function walks its CFG depth-first (the visiting order is
// sequential by definition).  Every lane executes the same walk, so the
// walk's values are wave-uniform; the visited and finished sets are bitsets
// spread over the lanes of two VGPRs each (bit v in word v/32, word w in
// lane w%64 of register w/64), so a membership test is one readlane instead
// of an LDS round trip.  Each block's edge range and first two successors
// are staged together, so most tree edges cost one LDS read and most other
// edges none; the stack holds (block, next edge, end, next successor).
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ bool bit_test(uint32_t r0, uint32_t r1, uint32_t v) {
  const uint32_t w = v >> 5;
  const uint32_t word = (w >> 6) ? __builtin_amdgcn_readlane(r1, w & 63)
                                 : __builtin_amdgcn_readlane(r0, w & 63);
  return (word >> (v & 31)) & 1u;
}

__device__ __forceinline__ void bit_set(uint32_t &r0, uint32_t &r1, uint32_t v) {
  const uint32_t w = v >> 5;
  const uint32_t m = (lane_id() == (w & 63)) ? (1u << (v & 31)) : 0u;
  if (w >> 6) r1 |= m;
  else r0 |= m;
}

constexpr uint32_t kNoSucc = 0xFFFFu;

// The first v >= from whose bit is set in (a & ~b), over the lane-spread
// bitsets (two VGPRs each), or 0xFFFFFFFF: words below from's word and the
// bits below from in that word are masked, then two ballots find the first
// word with a bit left.
__device__ __forceinline__ uint32_t first_set_from(uint32_t a0, uint32_t a1, uint32_t b0,
                                                   uint32_t b1, uint32_t from) {
  const uint32_t lane = lane_id();
  const uint32_t fw = from >> 5, fb = from & 31u;
  const uint32_t w0 = lane, w1 = lane + 64;
  uint32_t c0 = a0 & ~b0, c1 = a1 & ~b1;
  c0 = w0 < fw ? 0u : (w0 == fw ? c0 & (0xFFFFFFFFu << fb) : c0);
  c1 = w1 < fw ? 0u : (w1 == fw ? c1 & (0xFFFFFFFFu << fb) : c1);
  const uint64_t m0 = __ballot(c0 != 0u);
  if (m0) {
    const uint32_t l = (uint32_t)__builtin_ctzll(m0);
    return l * 32u + (uint32_t)__builtin_ctz(__builtin_amdgcn_readlane(c0, l));
  }
  const uint64_t m1 = __ballot(c1 != 0u);
  if (m1) {
    const uint32_t l = (uint32_t)__builtin_ctzll(m1);
    return (l + 64u) * 32u + (uint32_t)__builtin_ctz(__builtin_amdgcn_readlane(c1, l));
  }
  return 0xFFFFFFFFu;
}

// Chains: a block v whose only predecessor p has v as its only successor and
// comes before it (p < v) is a chain member behind p.  The walk enters such a
// v from p at once (v cannot be a root: p is reached no later than the root
// loop reaches v), no other edge leads to v, and v finishes right after
// everything behind it, so the walk only needs the chain heads, each with
// the edges of its chain's last block; the postorder is expanded afterwards.
__global__ void __launch_bounds__(64)
k_dfs(const uint32_t *fbb, const uint32_t *succ_ptr, const uint32_t *succ,
      const uint32_t *pred_ptr, const uint32_t *pred, uint8_t *retreat, uint32_t *rpo_pos,
      uint32_t *rpo_order) {
  extern __shared__ uint4 shq[];
  const uint32_t f = blockIdx.x;
  const uint32_t b0 = fbb[f], nb = fbb[f + 1] - b0;
  const uint32_t e0 = succ_ptr[b0], ne = succ_ptr[b0 + nb] - e0;
  const unsigned lane = lane_id();
  uint4 *stk = shq;                            // [nb] (head, next edge, end, next successor)
  uint2 *rng = (uint2 *)(stk + nb);            // [nb] edge range of the head's chain end
  uint32_t *s01 = (uint32_t *)(rng + nb);      // [nb] its first two successors
  uint16_t *nxt = (uint16_t *)(s01 + nb);      // [nb] next chain member or kNoSucc
  uint16_t *posth = nxt + nb;                  // [nb] heads in postorder
  uint16_t *lsucc = posth + nb;                // [ne]
  uint8_t *ret = (uint8_t *)(lsucc + ne);      // [ne]
  uint8_t *head = ret + ne;                    // [nb]
  for (uint32_t b = lane; b < nb; b += 64) nxt[b] = (uint16_t)kNoSucc;
  for (uint32_t e = lane; e < ne; e += 64) {
    lsucc[e] = (uint16_t)(succ[e0 + e] - b0);
    ret[e] = 0;
  }
  __syncthreads();
  for (uint32_t v = lane; v < nb; v += 64) {
    const uint32_t q0 = pred_ptr[b0 + v], q1 = pred_ptr[b0 + v + 1];
    bool member = false;
    if (q1 - q0 == 1) {
      const uint32_t pb = pred[q0] - b0;
      member = pb < v && succ_ptr[b0 + pb + 1] - succ_ptr[b0 + pb] == 1;
      if (member) nxt[pb] = (uint16_t)v;
    }
    head[v] = member ? 0 : 1;
  }
  __syncthreads();
  for (uint32_t h = lane; h < nb; h += 64) {
    if (!head[h]) continue;
    uint32_t t = h;
    while (nxt[t] != kNoSucc) t = nxt[t];
    const uint32_t lo = succ_ptr[b0 + t] - e0, hi = succ_ptr[b0 + t + 1] - e0;
    rng[h] = make_uint2(lo, hi);
    const uint32_t a0 = lo < hi ? succ[e0 + lo] - b0 : kNoSucc;
    const uint32_t a1 = lo + 1 < hi ? succ[e0 + lo + 1] - b0 : kNoSucc;
    s01[h] = a0 | (a1 << 16);
  }
  __syncthreads();
  uint32_t vis0 = 0, vis1 = 0, fin0 = 0, fin1 = 0;
  // the chain heads as a lane-spread bitset: 64 blocks per ballot, whose two
  // words go to lanes w and w + 1 of the register that holds them
  uint32_t hd0 = 0, hd1 = 0;
  for (uint32_t v0 = 0; v0 < nb; v0 += 64) {
    const uint32_t v = v0 + lane;
    const uint64_t m = __ballot(v < nb && head[v] != 0);
    const uint32_t w = v0 >> 5;   // even
    const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
    if ((w >> 6) == 0) {
      hd0 = lane == (w & 63) ? lo : hd0;
      hd0 = lane == ((w + 1) & 63) ? hi : hd0;
    } else {
      hd1 = lane == (w & 63) ? lo : hd1;
      hd1 = lane == ((w + 1) & 63) ? hi : hd1;
    }
  }
  uint32_t npost = 0;
  for (uint32_t root = first_set_from(hd0, hd1, vis0, vis1, 0); root < nb;
       root = first_set_from(hd0, hd1, vis0, vis1, root + 1)) {
    bit_set(vis0, vis1, root);
    uint32_t sp = 0, u = root;
    uint2 r = rng[root];
    uint32_t pair = uni(s01[root]);
    uint32_t k = uni(r.x), end = uni(r.y);
    // the successor at edge k when it is known without a read; `fresh` while
    // k is the first edge of u, whose second successor is staged too
    uint32_t nextv = k < end ? (pair & 0xFFFFu) : kNoSucc;
    uint32_t second = pair >> 16;
    bool fresh = true;
    for (;;) {
      if (k < end) {
        const uint32_t v = nextv != kNoSucc ? nextv : uni(lsucc[k]);
        const uint32_t k1 = k + 1;
        const uint32_t after = (fresh && k1 < end) ? second : kNoSucc;
        fresh = false;
        if (!bit_test(vis0, vis1, v)) {
          if (lane == 0) stk[sp] = make_uint4(u, k1, end, after);
          ++sp;
          bit_set(vis0, vis1, v);
          u = v;
          r = rng[v];
          pair = uni(s01[v]);
          k = uni(r.x);
          end = uni(r.y);
          nextv = k < end ? (pair & 0xFFFFu) : kNoSucc;
          second = pair >> 16;
          fresh = true;
        } else {
          if (!bit_test(fin0, fin1, v) && lane == 0) ret[k] = 1;
          k = k1;
          nextv = after;
        }
      } else {
        bit_set(fin0, fin1, u);
        if (lane == 0) posth[npost] = (uint16_t)u;
        ++npost;
        if (sp == 0) break;
        --sp;
        const uint4 t = stk[sp];
        u = uni(t.x);
        k = uni(t.y);
        end = uni(t.z);
        nextv = uni(t.w);
        fresh = false;
      }
    }
  }
  __syncthreads();
  for (uint32_t e = lane; e < ne; e += 64) retreat[e0 + e] = ret[e];
  // postorder: a finished head is followed by its chain's members from the
  // last to the head itself; positions by a running sum of chain lengths
  uint32_t carry = 0;
  for (uint32_t base = 0; base < npost; base += 64) {
    const uint32_t i = base + lane;
    uint32_t h = 0, len = 0;
    if (i < npost) {
      h = posth[i];
      for (uint32_t t = h; t != kNoSucc; t = nxt[t]) ++len;
    }
    const uint32_t incl = wave_incl_scan(len);
    const uint32_t first = carry + incl - len;   // postorder index of the chain's last block
    if (i < npost) {
      uint32_t o = 0;
      for (uint32_t t = h; t != kNoSucc; t = nxt[t], ++o) {
        const uint32_t post = first + (len - 1 - o);
        const uint32_t rp = nb - 1 - post;
        rpo_pos[b0 + t] = rp;
        rpo_order[b0 + rp] = b0 + t;
      }
    }
    carry += __shfl(incl, 63, 64);
  }
}

// ------------------------------------------------------------ distances
// Sweep streams.  For every block w of a function, in a sweep order (the
// DFS reverse postorder, whose forward edges are G'; or block order), one entry
// per predecessor edge v -> w (one entry with v = none for a block without
// predecessors): v and w as function-local ids, flags for the first and last
// entry of w and for a retreating edge, and the size of w beside it.  An edge
// v -> w is retreating exactly when w does not come after v in the order.
// The retreating edges are also listed on their own, for the convergence
// test of shortest walks.
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint32_t kLocalNone = 0x1FFFu;   // local block ids are < 4096
constexpr uint32_t kEntFirst = 1u << 26, kEntLast = 1u << 27, kEntRet = 1u << 28;
constexpr uint32_t kDistLds = 64 * 1024;   // distance tables of one workgroup

__global__ void k_sweep_count(uint32_t n_blocks, const uint32_t *fbb,
                              const uint32_t *func_of_block, const uint32_t *pred_ptr,
                              const uint32_t *pred, const uint32_t *rpo_pos, uint32_t *cnt,
                              uint32_t *rcnt) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks;
       b += gridDim.x * blockDim.x) {
    const uint32_t b0 = fbb[func_of_block[b]];
    const uint32_t pw = rpo_pos[b];
    const uint32_t q0 = pred_ptr[b], q1 = pred_ptr[b + 1];
    uint32_t r = 0;
    for (uint32_t q = q0; q < q1; ++q) r += (rpo_pos[pred[q]] >= pw) ? 1u : 0u;
    cnt[b0 + pw] = max(q1 - q0, 1u);
    rcnt[b0 + pw] = r;
    if (b == 0) {
      cnt[n_blocks] = 0;
      rcnt[n_blocks] = 0;
    }
  }
}

__global__ void k_sweep_fill(uint32_t n_blocks, const uint32_t *fbb,
                             const uint32_t *func_of_block, const uint32_t *block_begin,
                             const uint32_t *pred_ptr, const uint32_t *pred,
                             const uint32_t *rpo_pos, const uint32_t *ent_ptr,
                             const uint32_t *ret_ptr, uint32_t *ent, uint32_t *ent_w,
                             uint32_t *rent, uint32_t *rent_w, uint32_t *rent_e) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks;
       b += gridDim.x * blockDim.x) {
    const uint32_t b0 = fbb[func_of_block[b]];
    const uint32_t pw = rpo_pos[b], pos = b0 + pw, bl = b - b0;
    const uint32_t bs = block_begin[b + 1] - block_begin[b];
    const uint32_t q0 = pred_ptr[b], q1 = pred_ptr[b + 1];
    const uint32_t off = ent_ptr[pos];
    uint32_t roff = ret_ptr[pos];
    if (q0 == q1) {
      ent[off] = kLocalNone | (bl << 13) | kEntFirst | kEntLast;
      ent_w[off] = bs;
    }
    for (uint32_t q = q0; q < q1; ++q) {
      const uint32_t v = pred[q];
      const bool ret = rpo_pos[v] >= pw;
      ent[off + (q - q0)] = (v - b0) | (bl << 13) | (q == q0 ? kEntFirst : 0u) |
                            (q + 1 == q1 ? kEntLast : 0u) | (ret ? kEntRet : 0u);
      ent_w[off + (q - q0)] = bs;
      if (ret) {
        rent[roff] = (v - b0) | (bl << 13);
        rent_w[roff] = bs;
        rent_e[roff] = off;   // where the header's entries start
        ++roff;
      }
    }
  }
}

// One sweep over a function's stream in G' order.  Every lane follows its
// own source block s with the same (uniform) control flow; the table holds,
// per block w and lane, the walk length up to and including w:
//   shortest:  E[w] = min over edges v -> w of (v == s ? 0 : E[v]) + |w|,
//              saturating at kInf (no walk);
//   longest:   the same maximum over edges that are not retreating, stored
//              plus one so that 0 means no G' walk from s reaches w.
// The table has a spare row (written by entries that are not the last of
// their block) and a spare column (written by lanes without a source), so
// every entry is the same straight-line code.  Table reads run kPD entries
// ahead of their use and are issued before the writes of the kPD entries in
// between; those writes sit in a ring (slot = entry index mod kPD) and are
// forwarded (a block is written once per sweep, so at most one slot matches).
constexpr int kPD = 4;

template <bool kLongest, typename T>
__device__ void dist_sweep(T *D, uint32_t Lc, uint32_t col, uint32_t s, uint32_t spare_row,
                           const uint32_t *ent, const uint32_t *ent_w, uint32_t e_begin,
                           uint32_t e_end) {
  const unsigned lane = threadIdx.x;
  constexpr uint32_t kTInf = (uint32_t)(T)~0u;   // the entry type's "no walk" for shortest
  const uint32_t none = kLongest ? 0u : kTInf;
  const uint32_t at_s = kLongest ? 1u : 0u;       // a walk that starts at s
  uint32_t rw[kPD], re[kPD];
#pragma unroll
  for (int r = 0; r < kPD; ++r) {
    rw[r] = kLocalNone;
    re[r] = none;
  }
  uint32_t best = none;
  uint32_t idx = e_begin + lane;
  uint32_t vp = idx < e_end ? ent[idx] : kLocalNone;
  uint32_t vw = idx < e_end ? ent_w[idx] : 0u;
  for (uint32_t base = e_begin; base < e_end; base += 64) {
    const uint32_t nidx = base + 64 + lane;
    const uint32_t vp_next = nidx < e_end ? ent[nidx] : kLocalNone;
    const uint32_t vw_next = nidx < e_end ? ent_w[nidx] : 0u;
    uint32_t pre[kPD];
#pragma unroll
    for (int i = 0; i < kPD; ++i) {
      const uint32_t v = __builtin_amdgcn_readlane(vp, i) & kLocalNone;
      pre[i] = D[(v == kLocalNone ? spare_row : v) * Lc + col];
    }
    for (int i0 = 0; i0 < 64; i0 += 16) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = i0 + j;
        const uint32_t pk = __builtin_amdgcn_readlane(vp, i);
        const uint32_t bw = __builtin_amdgcn_readlane(vw, i);
        const uint32_t v = pk & kLocalNone;
        uint32_t c = pre[j % kPD];
        if (i + kPD < 64) {
          const uint32_t vn = __builtin_amdgcn_readlane(vp, i + kPD) & kLocalNone;
          pre[j % kPD] = D[(vn == kLocalNone ? spare_row : vn) * Lc + col];
        }
#pragma unroll
        for (int r = 0; r < kPD; ++r) c = (v == rw[r]) ? re[r] : c;
        c = (v == s) ? at_s : c;
        const bool use = v != kLocalNone && !(kLongest && (pk & kEntRet));
        best = (pk & kEntFirst) ? none : best;
        const uint32_t nb_ = kLongest ? max(best, c) : min(best, c);
        best = use ? nb_ : best;
        uint32_t e;
        if (kLongest) e = best ? best + bw : 0u;
        else if (sizeof(T) == 4) e = __builtin_elementwise_add_sat(best, bw);
        else e = min(best + bw, kTInf);   // walks stay below kTInf (checked on the host)
        const bool last = (pk & kEntLast) != 0;
        const uint32_t w = last ? (pk >> 13) & kLocalNone : spare_row;
        D[w * Lc + col] = (T)e;
        rw[j % kPD] = last ? w : kLocalNone;
        re[j % kPD] = e;
      }
    }
    vp = vp_next;
    vw = vw_next;
  }
}

// Walk tables of a group of L consecutive blocks, one lane per source block:
// for every block w of the source's function, the shortest walk
// (longest_tab = 0, any sweep order) or the longest G' walk (longest_tab = 1,
// the DFS reverse postorder) from the source to w, in the sweep table's
// terms (including |w|).  Shortest walks repeat the sweep until no
// retreating edge can shorten a walk (the sweep order settles every other
// edge); longest G' walks take one sweep.  The workgroup is one wave; the
// table is copied out to the source's row of the function's table.
template <typename T>
__global__ void __launch_bounds__(64)
k_dist_tables(uint32_t n_blocks, uint32_t n_funcs, uint32_t L, const uint32_t *fbb,
              const uint32_t *func_of_block, const uint32_t *ent_ptr, const uint32_t *ent,
              const uint32_t *ent_w, const uint32_t *ret_ptr, const uint32_t *rent,
              const uint32_t *rent_w, const uint32_t *rent_e, const uint32_t *rpo_pos,
              const uint32_t *tab_off, uint32_t *t_sp, uint32_t *t_lp, uint32_t longest_tab) {
  extern __shared__ uint4 dist_lds[];
  T *D = (T *)dist_lds;             // [blocks of the function + 1][L + 1]
  constexpr uint32_t kTInf = (uint32_t)(T)~0u;
  const unsigned lane = threadIdx.x;
  const bool longest = longest_tab != 0;
  const uint32_t c0 = blockIdx.x * L, c1 = min(c0 + L, n_blocks);
  if (c0 >= n_blocks) return;
  const uint32_t Lc = L + 1;
  const uint32_t col = lane < L ? lane : L;   // lanes without a source use the spare column
  for (uint32_t f = func_of_block[c0]; f < n_funcs && fbb[f] < c1; ++f) {
    const uint32_t b0 = fbb[f], b1 = fbb[f + 1], nb = b1 - b0;
    const uint32_t g0 = max(c0, b0), g1 = min(c1, b1);
    if (g0 >= g1) continue;
    const uint32_t sb = c0 + lane;
    const bool mine = lane < L && sb >= g0 && sb < g1;
    const uint32_t s = mine ? sb - b0 : 0xFFFFu;
    const uint32_t e_end = ent_ptr[b1];
    // Nothing before the earliest source (in the sweep order) is reached
    // without a retreating edge: the sweeps start there, a later shortest-walk sweep
    // at the earliest header whose retreating edge improved a walk.
    uint32_t pmin = mine ? rpo_pos[sb] : 0xFFFFFFFFu;
    for (int d = 32; d > 0; d >>= 1) pmin = min(pmin, (uint32_t)__shfl_xor((int)pmin, d, 64));
    const uint32_t e_src_start = ent_ptr[b0 + pmin];
    __syncthreads();
    const T none = longest ? (T)0 : (T)kTInf;
    for (uint32_t k = lane; k < (nb + 1) * Lc; k += 64) D[k] = none;
    __syncthreads();
    if (longest) {
      // every block is written before any later block reads it
      dist_sweep<true, T>(D, Lc, col, s, nb, ent, ent_w, e_src_start, e_end);
    } else {
      const uint32_t r_begin = ret_ptr[b0], r_end = ret_ptr[b1];
      uint32_t start = e_src_start;
      for (uint32_t sweep = 0; sweep <= nb; ++sweep) {
        dist_sweep<false, T>(D, Lc, col, s, nb, ent, ent_w, start, e_end);
        uint32_t restart = 0xFFFFFFFFu;
        for (uint32_t base = r_begin; base < r_end; base += 64) {
          const uint32_t idx = base + lane;
          const uint32_t rp = idx < r_end ? rent[idx] : kLocalNone;
          const uint32_t rw = idx < r_end ? rent_w[idx] : 0u;
          const uint32_t re = idx < r_end ? rent_e[idx] : 0u;
          const uint32_t cnt = min(64u, r_end - base);
          for (uint32_t i = 0; i < cnt; ++i) {
            const uint32_t pk = __builtin_amdgcn_readlane(rp, i);
            const uint32_t u = pk & kLocalNone, h = (pk >> 13) & kLocalNone;
            const uint32_t cu = (u == s) ? 0u : (uint32_t)D[u * Lc + col];
            const uint32_t bh = __builtin_amdgcn_readlane(rw, i);
            if (mine && cu != kTInf && cu + bh < (uint32_t)D[h * Lc + col])
              restart = min(restart, __builtin_amdgcn_readlane(re, i));
          }
        }
        for (int d = 32; d > 0; d >>= 1)
          restart = min(restart, (uint32_t)__shfl_xor((int)restart, d, 64));
        if (restart == 0xFFFFFFFFu) break;
        start = restart;
      }
    }
    __syncthreads();
    // rows (source - b0) of the function's table, nb entries each
    uint32_t *Tab = (longest ? t_lp : t_sp) + tab_off[f] + (size_t)(g0 - b0) * nb;
    const uint32_t l0 = g0 - c0, n_out = (g1 - g0) * nb;
    for (uint32_t k = lane; k < n_out; k += 64) {
      const uint32_t r = k / nb, w = k - r * nb;
      const uint32_t v = D[w * Lc + l0 + r];
      Tab[k] = (!longest && v == kTInf) ? kInf : v;
    }
  }
}

// Per edge i -> j: distances count the instructions strictly between them.
// Same block with i first: j - i - 1 both.  Otherwise, with the tables'
// walk lengths E (shortest) and E' (longest G', plus one) from B_i to B_j,
// which include |B_j|: dmin = E + (|B_i| - o_i - 1) + o_j - |B_j|, and dmax
// the same with E' - 1 when B_i != B_j and G' has such a walk, else dmin.
// The latency rule's flag is set when dmin is within the source's bound.
__global__ void k_edge_dist(uint64_t n_edges, const uint32_t *e_src, const uint32_t *e_dst,
                            const uint32_t *block_of, const uint32_t *func_of_block,
                            const uint32_t *fbb, const uint32_t *block_begin,
                            const uint8_t *op_class, LatTable lat_tab,
                            const uint32_t *tab_off, const uint32_t *t_sp, const uint32_t *t_lp,
                            uint32_t *e_dmin, uint32_t *e_dmax, uint8_t *e_flags) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n_edges;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t src = e_src[e], j = e_dst[e];
    const uint32_t sb = block_of[src], tb = block_of[j];
    const uint32_t oi = src - block_begin[sb], oj = j - block_begin[tb];
    uint32_t dmin, dmax;
    if (tb == sb && oi < oj) {
      dmin = dmax = oj - oi - 1;
    } else {
      const uint32_t f = func_of_block[sb];
      const uint32_t b0 = fbb[f], nb = fbb[f + 1] - b0;
      const uint32_t ss = block_begin[sb + 1] - block_begin[sb];
      const uint32_t bt = block_begin[tb + 1] - block_begin[tb];
      const uint32_t add = (ss - oi - 1) + oj - bt;   // mod 2^32; E >= |B_j|
      const size_t at = tab_off[f] + (size_t)(sb - b0) * nb + (tb - b0);
      const uint32_t Es = t_sp[at], El = t_lp[at];
      dmin = (Es == kInf) ? kInf : Es + add;
      dmax = (sb != tb && El != 0) ? (El - 1) + add : dmin;
    }
    e_dmin[e] = dmin;
    e_dmax[e] = dmax;
    if (dmin <= lat_tab.v[op_class[src] & 15]) e_flags[e] |= GPA_E_LAT_KEEP;
  }
}

// per function: its squared block count (the size of each of its tables)
__global__ void k_func_sq(uint32_t n_funcs, const uint32_t *fbb, uint32_t *sq) {
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < n_funcs;
       f += gridDim.x * blockDim.x) {
    const uint32_t nb = fbb[f + 1] - fbb[f];
    sq[f] = nb * nb;
  }
}

// the sweep streams of every function in the order given by pos (a block's
// position within its function)
static void build_sweep_plan(gpa_program &p, hipStream_t s, Arena &ar, const uint32_t *pos,
                             SweepPlan &plan) {
  const uint32_t nb = p.n_blocks;
  uint32_t *cnt = ar.get<uint32_t>((size_t)nb + 1), *rcnt = ar.get<uint32_t>((size_t)nb + 1);
  plan.ent_ptr = ar.get<uint32_t>((size_t)nb + 1);
  plan.ret_ptr = ar.get<uint32_t>((size_t)nb + 1);
  const size_t n_ent = (size_t)p.n_succ + nb;   // upper bound
  plan.ent = ar.get<uint32_t>(n_ent);
  plan.ent_w = ar.get<uint32_t>(n_ent);
  plan.rent = ar.get<uint32_t>(p.n_succ ? p.n_succ : 1);
  plan.rent_w = ar.get<uint32_t>(p.n_succ ? p.n_succ : 1);
  plan.rent_e = ar.get<uint32_t>(p.n_succ ? p.n_succ : 1);
  const uint32_t g = grid_for(nb, 256, 4096);
  hipLaunchKernelGGL(k_sweep_count, dim3(g), dim3(256), 0, s, nb, p.func_block_begin.p,
                     p.func_of_block.p, p.pred_ptr.p, p.pred.p, pos, cnt, rcnt);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(cnt, plan.ent_ptr, (size_t)nb + 1, s, ar);
  exclusive_scan_u32(rcnt, plan.ret_ptr, (size_t)nb + 1, s, ar);
  hipLaunchKernelGGL(k_sweep_fill, dim3(g), dim3(256), 0, s, nb, p.func_block_begin.p,
                     p.func_of_block.p, p.block_begin.p, p.pred_ptr.p, p.pred.p, pos,
                     plan.ent_ptr, plan.ret_ptr, plan.ent, plan.ent_w, plan.rent, plan.rent_w,
                     plan.rent_e);
  GPA_LAUNCH_CHECK();
}

void build_cfg_order(gpa_program &p, hipStream_t s, Arena &ar, SweepPlan &plan,
                     PhaseTimer &t_dfs) {
  const uint32_t nf = p.n_funcs, nb = p.n_blocks;
  const uint32_t max_ne = p.max_func_edges;
  const uint32_t max_nb = p.max_func_blocks;
  p.retreat.alloc(p.n_succ);
  p.rpo_pos.alloc(nb);
  p.rpo_order.alloc(nb);
  const size_t lds_dfs = 33u * (size_t)max_nb + 3u * (size_t)max_ne + 16;
  if (lds_dfs > 160 * 1024)
    fail(GPA_E_UNSUPPORTED, "a function's CFG (%u blocks, %u edges) exceeds the LDS staging",
         max_nb, max_ne);
  GPA_HIP(hipFuncSetAttribute((const void *)k_dfs, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_dfs));
  t_dfs.begin(kPhaseDfs, s);
  hipLaunchKernelGGL(k_dfs, dim3(nf), dim3(64), lds_dfs, s, p.func_block_begin.p, p.succ_ptr.p,
                     p.succ.p, p.pred_ptr.p, p.pred.p, p.retreat.p, p.rpo_pos.p, p.rpo_order.p);
  GPA_LAUNCH_CHECK();
  t_dfs.end(s);
  build_sweep_plan(p, s, ar, p.rpo_pos.p, plan);
}

// position of each block within its function in block order
__global__ void k_block_pos(uint32_t n_blocks, const uint32_t *fbb, const uint32_t *func_of_block,
                            uint32_t *pos) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks;
       b += gridDim.x * blockDim.x)
    pos[b] = b - fbb[func_of_block[b]];
}

void build_block_order_plan(gpa_program &p, hipStream_t s, Arena &ar, SweepPlan &plan,
                            uint32_t *&pos) {
  pos = ar.get<uint32_t>(p.n_blocks);
  hipLaunchKernelGGL(k_block_pos, dim3(grid_for(p.n_blocks, 256, 4096)), dim3(256), 0, s,
                     p.n_blocks, p.func_block_begin.p, p.func_of_block.p, pos);
  GPA_LAUNCH_CHECK();
  build_sweep_plan(p, s, ar, pos, plan);
}

void prepare_dist_tables(gpa_program &p, hipStream_t s, Arena &ar, DistTables &t) {
  const uint32_t nf = p.n_funcs;
  if (p.dist_entries >= (1ull << 32))
    fail(GPA_E_UNSUPPORTED, "walk tables of %llu entries; the sum over functions of the squared "
         "block count must stay below 2^32", (unsigned long long)p.dist_entries);
  t.off = ar.get<uint32_t>(nf);
  t.sp = ar.get<uint32_t>(p.dist_entries);
  t.lp = ar.get<uint32_t>(p.dist_entries);
  uint32_t *sq = ar.get<uint32_t>(nf);
  hipLaunchKernelGGL(k_func_sq, dim3(grid_for(nf, 256, 1024)), dim3(256), 0, s, nf,
                     p.func_block_begin.p, sq);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(sq, t.off, nf, s, ar);
}

void build_dist_tables(gpa_program &p, hipStream_t s, const SweepPlan &plan, const uint32_t *pos,
                       const DistTables &t, bool longest) {
  const uint32_t nf = p.n_funcs, nb = p.n_blocks;
  const uint32_t max_nb = p.max_func_blocks;
  // one table of (blocks + 1) x (L + 1) entries per workgroup, with L from
  // the u32 layout; 16-bit entries (half the LDS, so that more of the main
  // stream's workgroups fit beside) when every walk is shorter than 65,534
  // instructions: a walk of distinct blocks, or its length plus one, is at
  // most the instruction count plus one
  const uint32_t L = std::max<uint32_t>(
      1u, std::min<uint32_t>(63u, kDistLds / (4u * (max_nb + 1)) - 1u));
  const bool narrow = p.n_instr < 0xFFFEu;
  const size_t lds = (size_t)(narrow ? 2 : 4) * (L + 1) * (max_nb + 1);
  const void *kern = narrow ? (const void *)k_dist_tables<uint16_t>
                            : (const void *)k_dist_tables<uint32_t>;
  GPA_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (narrow)
    hipLaunchKernelGGL(k_dist_tables<uint16_t>, dim3((nb + L - 1) / L), dim3(64), lds, s, nb, nf,
                       L, p.func_block_begin.p, p.func_of_block.p, plan.ent_ptr, plan.ent,
                       plan.ent_w, plan.ret_ptr, plan.rent, plan.rent_w, plan.rent_e, pos, t.off,
                       t.sp, t.lp, longest ? 1u : 0u);
  else
    hipLaunchKernelGGL(k_dist_tables<uint32_t>, dim3((nb + L - 1) / L), dim3(64), lds, s, nb, nf,
                       L, p.func_block_begin.p, p.func_of_block.p, plan.ent_ptr, plan.ent,
                       plan.ent_w, plan.ret_ptr, plan.rent, plan.rent_w, plan.rent_e, pos, t.off,
                       t.sp, t.lp, longest ? 1u : 0u);
  GPA_LAUNCH_CHECK();
}

void build_distances(gpa_program &p, hipStream_t s, Arena &ar, const DistTables &t) {
  const uint64_t ne = p.n_edges;
  p.e_dmin.alloc(ne);
  p.e_dmax.alloc(ne);
  if (ne == 0) return;
  LatTable lat;
  static_assert(sizeof(lat.v) == sizeof(p.arch.lat), "latency table size");
  std::memcpy(lat.v, p.arch.lat, sizeof(lat.v));
  hipLaunchKernelGGL(k_edge_dist, dim3(grid_for(ne, 256, 8192)), dim3(256), 0, s, ne, p.e_src.p,
                     p.e_dst.p, p.block_of.p, p.func_of_block.p, p.func_block_begin.p,
                     p.block_begin.p, p.op_class.p, lat, t.off, t.sp, t.lp, p.e_dmin.p,
                     p.e_dmax.p, p.e_flags.p);
  GPA_LAUNCH_CHECK();
}

// --------------------------------------------------------- target scopes
__global__ void k_edge_scopes(uint64_t n_edges, const uint32_t *e_src, const uint32_t *e_dst,
                              const uint32_t *instr_scope, const uint32_t *parent,
                              const uint32_t *depth, const uint8_t *kind,
                              const uint32_t *block_of, const uint32_t *func_of_block,
                              const uint32_t *func_scope, uint32_t *e_lca, uint32_t *e_icl,
                              uint32_t *big_n) {
  // the big-segment counters of the roll-up lists, appended to later
  if (blockIdx.x == 0 && threadIdx.x < 4) big_n[threadIdx.x] = 0;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n_edges;
       e += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t a = instr_scope[e_src[e]], b = instr_scope[e_dst[e]];
    while (depth[a] > depth[b]) a = parent[a];
    while (depth[b] > depth[a]) b = parent[b];
    while (a != b) {
      a = parent[a];
      b = parent[b];
    }
    e_lca[e] = a;
    // innermost loop holding both, not above the instructions' CFG function
    const uint32_t fs = func_scope[func_of_block[block_of[e_src[e]]]];
    uint32_t l = a;
    while (l != GPA_NONE && kind[l] != GPA_SCOPE_LOOP && l != fs) l = parent[l];
    e_icl[e] = (l != GPA_NONE && kind[l] == GPA_SCOPE_LOOP) ? l : GPA_NONE;
  }
}

// segments of more than kSmallSeg elements, listed for a workgroup each;
// grid row g serves grouping g (the fourth lists scopes by their [l, end)
// ranges)
__global__ void k_big_segments(uint32_t n_seg, const uint32_t *ptr0, const uint32_t *ptr1,
                               const uint32_t *ptr2, const uint32_t *end, uint32_t *list,
                               uint32_t *n_list) {
  const uint32_t g = blockIdx.y;
  const uint32_t *ptr = g == 0 ? ptr0 : g == 1 ? ptr1 : g == 2 ? ptr2 : nullptr;
  uint32_t *lst = list + (size_t)g * n_seg;
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < n_seg; l += gridDim.x * blockDim.x) {
    const uint32_t a = ptr ? ptr[l] : l, b = ptr ? ptr[l + 1] : end[l];
    if (b - a > kSmallSeg) lst[atomicAdd(n_list + g, 1u)] = l;
  }
}

// One workgroup: for each of the four groupings, the first chunk of every
// listed big segment (chunks of kSegChunk elements, in list order) and the
// number of chunks.
__global__ void __launch_bounds__(1024)
k_big_chunks(uint32_t n_seg, const uint32_t *list, const uint32_t *n_list, const uint32_t *ptr0,
             const uint32_t *ptr1, const uint32_t *ptr2, const uint32_t *end,
             uint32_t *chunk_start, unsigned long long *totals) {
  __shared__ uint32_t tmp[1024 / kWave + 1];
  for (int g = 0; g < 4; ++g) {
    const uint32_t *ptr = g == 0 ? ptr0 : g == 1 ? ptr1 : g == 2 ? ptr2 : nullptr;
    const uint32_t *lst = list + (size_t)g * n_seg;
    const uint32_t nl = n_list[g];
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < nl; j0 += 1024) {
      const uint32_t j = j0 + threadIdx.x;
      uint32_t c = 0;
      if (j < nl) {
        const uint32_t l = lst[j];
        const uint32_t a = ptr ? ptr[l] : l, b = ptr ? ptr[l + 1] : end[l];
        c = (b - a + kSegChunk - 1) / kSegChunk;
      }
      uint32_t tot;
      const uint32_t run = block_excl_scan<1024>(c, tmp, &tot);
      if (j < nl) chunk_start[(size_t)g * n_seg + j] = carry + run;
      carry += tot;
    }
    if (threadIdx.x == 0) totals[g] = carry;
    __syncthreads();
  }
}

void build_scope_targets(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint64_t ne = p.n_edges;
  p.e_lca.alloc(ne);
  p.e_icl.alloc(ne);
  p.big_n.alloc(4);
  hipLaunchKernelGGL(k_edge_scopes, dim3(grid_for(ne, 256, 8192)), dim3(256), 0, s, ne, p.e_src.p,
                     p.e_dst.p, p.instr_scope.p, p.scope_parent.p, p.scope_depth.p,
                     p.scope_kind.p, p.block_of.p, p.func_of_block.p, p.func_scope.p, p.e_lca.p,
                     p.e_icl.p, p.big_n.p);
  GPA_LAUNCH_CHECK();
  // one stable sort for the four groupings: edges by source instruction, by
  // common scope and by common loop, instructions by line scope
  const GroupSpec spec[4] = {{p.e_src.p, ne, p.n_instr},
                             {p.e_lca.p, ne, p.n_scopes},
                             {p.e_icl.p, ne, p.n_scopes},
                             {p.instr_scope.p, p.n_instr, p.n_scopes}};
  uint32_t base[4];
  uint64_t ibase[4];
  group_by_keys(spec, 4, p.grp_ptr, p.grp_perm, base, ibase, s, ar);
  p.out_ptr = p.grp_ptr.p + base[0];
  p.lca_ptr = p.grp_ptr.p + base[1];
  p.icl_ptr = p.grp_ptr.p + base[2];
  p.line_ptr = p.grp_ptr.p + base[3];
  p.out_perm = p.grp_perm.p + ibase[0];
  p.lca_perm = p.grp_perm.p + ibase[1];
  p.icl_perm = p.grp_perm.p + ibase[2];
  p.line_perm = p.grp_perm.p + ibase[3];
  const uint32_t ns = p.n_scopes;
  p.big_list.alloc((size_t)4 * ns);
  const uint32_t *ptrs[3] = {p.line_ptr, p.icl_ptr, p.lca_ptr};
  hipLaunchKernelGGL(k_big_segments, dim3(grid_for(ns, 256, 4096), 4), dim3(256), 0, s, ns,
                     ptrs[0], ptrs[1], ptrs[2], p.scope_end.p, p.big_list.p, p.big_n.p);
  GPA_LAUNCH_CHECK();
  // the big segments' chunks: first chunk of each listed segment, and the
  // totals (read by the host with the load's last synchronization)
  p.big_chunk.alloc((size_t)4 * ns);
  p.big_chunk_tot.alloc(4);
  hipLaunchKernelGGL(k_big_chunks, dim3(1), dim3(1024), 0, s, ns, p.big_list.p, p.big_n.p, ptrs[0],
                     ptrs[1], ptrs[2], p.scope_end.p, p.big_chunk.p, p.big_chunk_tot.p);
  GPA_LAUNCH_CHECK();
}

}  // namespace gpa
