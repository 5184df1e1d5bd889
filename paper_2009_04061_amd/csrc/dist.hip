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
#include "common.h"
#include "devutil.h"

namespace gpa {

// ------------------------------------------------------------------ DFS
// One workgroup per function; its successor lists are staged in LDS and one
// lane walks them (the visiting order is sequential by definition).
__global__ void __launch_bounds__(64)
k_dfs(const uint32_t *fbb, const uint32_t *succ_ptr, const uint32_t *succ, uint8_t *retreat,
      uint32_t *rpo_pos, uint32_t *rpo_order) {
  extern __shared__ uint32_t sh[];
  const uint32_t f = blockIdx.x;
  const uint32_t b0 = fbb[f], nb = fbb[f + 1] - b0;
  const uint32_t e0 = succ_ptr[b0], ne = succ_ptr[b0 + nb] - e0;
  uint32_t *lptr = sh;                       // [nb+1]
  uint32_t *sk = lptr + nb + 1;              // [nb] saved edge cursors
  uint16_t *lsucc = (uint16_t *)(sk + nb);   // [ne]
  uint16_t *stk = lsucc + ne;                // [nb] saved blocks
  uint16_t *post = stk + nb;                 // [nb]
  uint8_t *state = (uint8_t *)(post + nb);   // [nb] 0 new, 1 on the stack, 2 done
  uint8_t *ret = state + nb;                 // [ne]
  for (uint32_t b = threadIdx.x; b <= nb; b += 64) lptr[b] = succ_ptr[b0 + b] - e0;
  for (uint32_t e = threadIdx.x; e < ne; e += 64) {
    lsucc[e] = (uint16_t)(succ[e0 + e] - b0);
    ret[e] = 0;
  }
  for (uint32_t b = threadIdx.x; b < nb; b += 64) state[b] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    // the block on top of the stack and its edge cursor live in registers;
    // the stack holds the blocks below it with their cursors
    uint32_t npost = 0;
    for (uint32_t root = 0; root < nb; ++root) {
      if (state[root]) continue;
      uint32_t sp = 0, u = root, k = lptr[root], end = lptr[root + 1];
      state[root] = 1;
      while (true) {
        if (k < end) {
          const uint32_t v = lsucc[k];
          const uint8_t sv = state[v];
          if (sv == 0) {
            stk[sp] = (uint16_t)u;
            sk[sp] = k + 1;
            ++sp;
            state[v] = 1;
            u = v;
            k = lptr[v];
            end = lptr[v + 1];
          } else {
            if (sv == 1) ret[k] = 1;
            ++k;
          }
        } else {
          state[u] = 2;
          post[npost++] = (uint16_t)u;
          if (sp == 0) break;
          --sp;
          u = stk[sp];
          k = sk[sp];
          end = lptr[u + 1];
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < ne; e += 64) retreat[e0 + e] = ret[e];
  for (uint32_t k = threadIdx.x; k < nb; k += 64) {
    const uint32_t b = post[nb - 1 - k];   // reverse postorder
    rpo_pos[b0 + b] = k;
    rpo_order[b0 + k] = b0 + b;
  }
}

// ------------------------------------------------------------ distances
// Sweep streams.  For every block w of a function, in the G' order, one entry
// per predecessor edge v -> w (one entry with v = none for a block without
// predecessors): v and w as function-local ids, flags for the first and last
// entry of w and for a retreating edge, and the size of w beside it.  An edge
// v -> w is retreating exactly when w does not come after v in the order
// (reverse postorder of the depth-first search).  The retreating edges are
// also listed on their own, for the convergence test of shortest walks.
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
                             uint32_t *rent, uint32_t *rent_w) {
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
        ++roff;
      }
    }
  }
}

// One sweep over a function's stream in G' order.  Every lane follows its
// own source block s with the same (uniform) control flow; the table holds,
// per block w and lane, the walk length up to and including w:
//   shortest:  E[w] = min over edges v -> w of (v == s ? 0 : E[v]) + |w|
//   longest:   the same maximum over edges that are not retreating, -1 for
//              blocks no G' walk from s reaches.
// The value of the block swept just before stays in a register, so a chain
// of single-predecessor blocks never waits on LDS.
template <bool kLongest>
__device__ void dist_sweep(uint32_t *D, uint32_t L, uint32_t li, bool writer, uint32_t s,
                           const uint32_t *ent, const uint32_t *ent_w, uint32_t e_begin,
                           uint32_t e_end) {
  const unsigned lane = threadIdx.x;
  uint32_t prev_w = kLocalNone, prev_e = kInf;
  uint32_t best = kInf;
  for (uint32_t base = e_begin; base < e_end; base += 64) {
    const uint32_t idx = base + lane;
    const uint32_t vp = idx < e_end ? ent[idx] : kLocalNone;
    const uint32_t vw = idx < e_end ? ent_w[idx] : 0u;
#pragma unroll 16
    for (int i = 0; i < 64; ++i) {
      const uint32_t pk = __builtin_amdgcn_readlane(vp, i);
      const uint32_t v = pk & kLocalNone;
      if (pk & kEntFirst) best = kInf;
      if (v != kLocalNone && !(kLongest && (pk & kEntRet))) {
        uint32_t c;
        if (v == prev_w) c = prev_e;
        else c = D[v * L + li];
        if (v == s) c = 0;
        // kInf reads as -1 for longest walks: no walk
        best = kLongest ? (uint32_t)max((int32_t)best, (int32_t)c) : min(best, c);
      }
      if (pk & kEntLast) {
        const uint32_t w = (pk >> 13) & kLocalNone;
        const uint32_t bw = __builtin_amdgcn_readlane(vw, i);
        const uint32_t e = (best == kInf) ? kInf : best + bw;
        if (writer) D[w * L + li] = e;
        prev_w = w;
        prev_e = e;
      }
    }
  }
}

// Distances of every edge out of a group of L consecutive source blocks, one
// lane per source.  Shortest walks repeat the sweep until no retreating edge
// can shorten a walk (the sweep order settles every other edge); longest G'
// walks take one sweep.  The workgroup is one wave.
__global__ void __launch_bounds__(64)
k_dist(uint32_t n_blocks, uint32_t n_funcs, uint32_t L, const uint32_t *fbb,
       const uint32_t *func_of_block, const uint32_t *block_begin, const uint32_t *block_of,
       const uint32_t *ent_ptr, const uint32_t *ent, const uint32_t *ent_w,
       const uint32_t *ret_ptr, const uint32_t *rent, const uint32_t *rent_w,
       const uint32_t *out_ptr, const uint32_t *out_perm, const uint32_t *e_src,
       const uint32_t *e_dst, const uint8_t *op_class, const uint16_t *lat_tab,
       uint32_t *e_dmin, uint32_t *e_dmax, uint8_t *e_flags) {
  extern __shared__ uint32_t D[];   // [blocks of the function][L]
  const unsigned lane = threadIdx.x;
  const uint32_t c0 = blockIdx.x * L, c1 = min(c0 + L, n_blocks);
  if (c0 >= n_blocks) return;
  const uint32_t li = lane < L ? lane : 0u;
  for (uint32_t f = func_of_block[c0]; f < n_funcs && fbb[f] < c1; ++f) {
    const uint32_t b0 = fbb[f], b1 = fbb[f + 1], nb = b1 - b0;
    const uint32_t g0 = max(c0, b0), g1 = min(c1, b1);
    if (g0 >= g1) continue;
    const uint32_t ea = out_ptr[block_begin[g0]], eb = out_ptr[block_begin[g1]];
    if (ea == eb) continue;
    const uint32_t sb = c0 + lane;
    const bool writer = lane < L;
    const bool mine = writer && sb >= g0 && sb < g1 &&
                      out_ptr[block_begin[sb]] < out_ptr[block_begin[sb + 1]];
    const uint32_t s = mine ? sb - b0 : 0xFFFFu;
    const uint32_t e_begin = ent_ptr[b0], e_end = ent_ptr[b1];
    const uint32_t r_begin = ret_ptr[b0], r_end = ret_ptr[b1];
    // shortest walks
    __syncthreads();
    for (uint32_t k = lane; k < nb * L; k += 64) D[k] = kInf;
    __syncthreads();
    for (uint32_t sweep = 0; sweep <= nb; ++sweep) {
      dist_sweep<false>(D, L, li, writer, s, ent, ent_w, e_begin, e_end);
      bool changed = false;
      for (uint32_t base = r_begin; base < r_end; base += 64) {
        const uint32_t idx = base + lane;
        const uint32_t rp = idx < r_end ? rent[idx] : kLocalNone;
        const uint32_t rw = idx < r_end ? rent_w[idx] : 0u;
        const uint32_t cnt = min(64u, r_end - base);
        for (uint32_t i = 0; i < cnt; ++i) {
          const uint32_t pk = __builtin_amdgcn_readlane(rp, i);
          const uint32_t u = pk & kLocalNone, h = (pk >> 13) & kLocalNone;
          const uint32_t cu = (u == s) ? 0u : D[u * L + li];
          const uint32_t bh = __builtin_amdgcn_readlane(rw, i);
          if (mine && cu != kInf && cu + bh < D[h * L + li]) changed = true;
        }
      }
      if (__ballot(changed) == 0) break;
    }
    __syncthreads();
    for (uint32_t k = ea + lane; k < eb; k += 64) {
      const uint32_t e = out_perm[k];
      const uint32_t src = e_src[e], j = e_dst[e];
      const uint32_t sbk = block_of[src], tb = block_of[j];
      const uint32_t sl = sbk - c0, t = tb - b0;
      const uint32_t i0 = block_begin[sbk], ss = block_begin[sbk + 1] - i0;
      const uint32_t tj0 = block_begin[tb], bt = block_begin[tb + 1] - tj0;
      const uint32_t oi = src - i0, oj = j - tj0;
      uint32_t dmin;
      if (tb == sbk && oi < oj) {
        dmin = oj - oi - 1;
      } else {
        const uint32_t Et = D[t * L + sl];
        dmin = (Et == kInf) ? kInf : (ss - oi - 1) + (Et - bt) + oj;
      }
      e_dmin[e] = dmin;
      if (dmin <= lat_tab[op_class[src]]) e_flags[e] |= GPA_E_LAT_KEEP;
    }
    // longest G' walks; every block is written before any later block reads it
    __syncthreads();
    dist_sweep<true>(D, L, li, writer, s, ent, ent_w, e_begin, e_end);
    __syncthreads();
    for (uint32_t k = ea + lane; k < eb; k += 64) {
      const uint32_t e = out_perm[k];
      const uint32_t src = e_src[e], j = e_dst[e];
      const uint32_t sbk = block_of[src], tb = block_of[j];
      const uint32_t sl = sbk - c0, t = tb - b0;
      const uint32_t i0 = block_begin[sbk], ss = block_begin[sbk + 1] - i0;
      const uint32_t tj0 = block_begin[tb], bt = block_begin[tb + 1] - tj0;
      const uint32_t oi = src - i0, oj = j - tj0;
      uint32_t dmax;
      if (tb == sbk && oi < oj) {
        dmax = oj - oi - 1;
      } else {
        const int32_t Et = (int32_t)D[t * L + sl];
        dmax = (tb != sbk && Et >= 0) ? (ss - oi - 1) + ((uint32_t)Et - bt) + oj : e_dmin[e];
      }
      e_dmax[e] = dmax;
    }
  }
}

void build_distances(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint32_t nf = p.n_funcs, nb = p.n_blocks;
  const uint32_t max_ne = p.max_func_edges;
  const uint32_t max_nb = p.max_func_blocks;
  p.retreat.alloc(p.n_succ);
  p.rpo_pos.alloc(nb);
  p.rpo_order.alloc(nb);
  const size_t lds_dfs = 4u * (2 * (size_t)max_nb + 1) + 2u * max_ne + 6u * max_nb + max_nb +
                         max_ne + 16;
  if (lds_dfs > 160 * 1024)
    fail(GPA_E_UNSUPPORTED, "a function's CFG (%u blocks, %u edges) exceeds the LDS staging",
         max_nb, max_ne);
  GPA_HIP(hipFuncSetAttribute((const void *)k_dfs, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_dfs));
  hipLaunchKernelGGL(k_dfs, dim3(nf), dim3(64), lds_dfs, s, p.func_block_begin.p, p.succ_ptr.p,
                     p.succ.p, p.retreat.p, p.rpo_pos.p, p.rpo_order.p);
  GPA_LAUNCH_CHECK();
  p.e_dmin.alloc(p.n_edges);
  p.e_dmax.alloc(p.n_edges);
  if (p.n_edges == 0) return;
  // sweep streams
  uint32_t *cnt = ar.get<uint32_t>((size_t)nb + 1), *rcnt = ar.get<uint32_t>((size_t)nb + 1);
  uint32_t *ent_ptr = ar.get<uint32_t>((size_t)nb + 1), *ret_ptr = ar.get<uint32_t>((size_t)nb + 1);
  const size_t n_ent = (size_t)p.n_succ + nb;   // upper bound
  uint32_t *ent = ar.get<uint32_t>(n_ent), *ent_w = ar.get<uint32_t>(n_ent);
  uint32_t *rent = ar.get<uint32_t>(p.n_succ ? p.n_succ : 1);
  uint32_t *rent_w = ar.get<uint32_t>(p.n_succ ? p.n_succ : 1);
  const uint32_t g = grid_for(nb, 256, 4096);
  hipLaunchKernelGGL(k_sweep_count, dim3(g), dim3(256), 0, s, nb, p.func_block_begin.p,
                     p.func_of_block.p, p.pred_ptr.p, p.pred.p, p.rpo_pos.p, cnt, rcnt);
  GPA_LAUNCH_CHECK();
  exclusive_scan_u32(cnt, ent_ptr, (size_t)nb + 1, s, ar);
  exclusive_scan_u32(rcnt, ret_ptr, (size_t)nb + 1, s, ar);
  hipLaunchKernelGGL(k_sweep_fill, dim3(g), dim3(256), 0, s, nb, p.func_block_begin.p,
                     p.func_of_block.p, p.block_begin.p, p.pred_ptr.p, p.pred.p, p.rpo_pos.p,
                     ent_ptr, ret_ptr, ent, ent_w, rent, rent_w);
  GPA_LAUNCH_CHECK();
  const uint32_t L = std::max<uint32_t>(1u, std::min<uint32_t>(64u, kDistLds / (4u * max_nb)));
  const size_t lds = (size_t)4 * L * max_nb;
  GPA_HIP(hipFuncSetAttribute((const void *)k_dist, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  uint16_t *lat = ar.get<uint16_t>(16);
  GPA_HIP(hipMemcpyAsync(lat, p.arch.lat, sizeof(p.arch.lat), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_dist, dim3((nb + L - 1) / L), dim3(64), lds, s, nb, nf, L,
                     p.func_block_begin.p, p.func_of_block.p, p.block_begin.p, p.block_of.p,
                     ent_ptr, ent, ent_w, ret_ptr, rent, rent_w, p.out_ptr.p, p.out_perm.p,
                     p.e_src.p, p.e_dst.p, p.op_class.p, lat, p.e_dmin.p, p.e_dmax.p,
                     p.e_flags.p);
  GPA_LAUNCH_CHECK();
}

// --------------------------------------------------------- target scopes
__global__ void k_edge_scopes(uint64_t n_edges, const uint32_t *e_src, const uint32_t *e_dst,
                              const uint32_t *instr_scope, const uint32_t *parent,
                              const uint32_t *depth, const uint8_t *kind,
                              const uint32_t *block_of, const uint32_t *func_of_block,
                              const uint32_t *func_scope, uint32_t *e_lca, uint32_t *e_icl) {
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

void build_scope_targets(gpa_program &p, hipStream_t s, Arena &ar) {
  const uint64_t ne = p.n_edges;
  p.e_lca.alloc(ne);
  p.e_icl.alloc(ne);
  if (ne)
    hipLaunchKernelGGL(k_edge_scopes, dim3(grid_for(ne, 256, 8192)), dim3(256), 0, s, ne,
                       p.e_src.p, p.e_dst.p, p.instr_scope.p, p.scope_parent.p, p.scope_depth.p,
                       p.scope_kind.p, p.block_of.p, p.func_of_block.p, p.func_scope.p, p.e_lca.p,
                       p.e_icl.p);
  GPA_LAUNCH_CHECK();
  group_by_key(p.e_lca.p, ne, p.n_scopes, p.lca_ptr, p.lca_perm, s, ar);
  group_by_key(p.e_icl.p, ne, p.n_scopes, p.icl_ptr, p.icl_perm, s, ar);
  p.n_icl = read_scalar(p.icl_ptr.p + p.n_scopes, s);
  group_by_key(p.instr_scope.p, p.n_instr, p.n_scopes, p.line_ptr, p.line_perm, s, ar);
}

}  // namespace gpa
