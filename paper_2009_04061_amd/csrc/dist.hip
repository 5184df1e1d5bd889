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
  uint32_t *it = lptr + nb + 1;              // [nb]
  uint16_t *lsucc = (uint16_t *)(it + nb);   // [ne]
  uint16_t *stk = lsucc + ne;                // [nb]
  uint16_t *post = stk + nb;                 // [nb]
  uint8_t *state = (uint8_t *)(post + nb);   // [nb]
  uint8_t *ret = state + nb;                 // [ne]
  for (uint32_t b = threadIdx.x; b <= nb; b += 64) lptr[b] = succ_ptr[b0 + b] - e0;
  for (uint32_t e = threadIdx.x; e < ne; e += 64) {
    lsucc[e] = (uint16_t)(succ[e0 + e] - b0);
    ret[e] = 0;
  }
  for (uint32_t b = threadIdx.x; b < nb; b += 64) state[b] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t npost = 0;
    for (uint32_t root = 0; root < nb; ++root) {
      if (state[root]) continue;
      uint32_t sp = 0;
      stk[sp++] = (uint16_t)root;
      state[root] = 1;
      it[root] = lptr[root];
      while (sp) {
        const uint32_t u = stk[sp - 1];
        const uint32_t k = it[u];
        if (k < lptr[u + 1]) {
          it[u] = k + 1;
          const uint32_t v = lsucc[k];
          const uint8_t sv = state[v];
          if (sv == 0) {
            state[v] = 1;
            it[v] = lptr[v];
            stk[sp++] = (uint16_t)v;
          } else if (sv == 1) {
            ret[k] = 1;
          }
        } else {
          state[u] = 2;
          post[npost++] = (uint16_t)u;
          --sp;
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
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint32_t kMaxTargets = 512;

// One wave walks source blocks with a grid stride; the CFG of the current
// function stays staged in LDS while consecutive sources share it.  For a
// source s: shortest walks by label-correcting relaxation over frontiers
// (bounded once every target has a distance), longest G' walks by dynamic
// programming over the G' order up to the last target after s.
__global__ void __launch_bounds__(64)
k_dist(uint32_t n_blocks, const uint32_t *fbb, const uint32_t *func_of_block,
       const uint32_t *block_begin, const uint32_t *block_of, const uint32_t *succ_ptr,
       const uint32_t *succ, const uint8_t *retreat, const uint32_t *rpo_pos,
       const uint32_t *rpo_order, const uint32_t *out_ptr, const uint32_t *out_perm,
       const uint32_t *e_src, const uint32_t *e_dst, const uint8_t *op_class,
       const uint16_t *lat_tab, uint32_t *e_dmin, uint32_t *e_dmax, uint8_t *e_flags) {
  extern __shared__ uint32_t sh[];
  __shared__ uint32_t tg[kMaxTargets];
  __shared__ uint32_t n_tg, n_cur, n_next, maxpos;
  __shared__ int overflow;
  const unsigned lane = threadIdx.x;
  uint32_t cur_f = 0xFFFFFFFFu, b0 = 0, nb = 0, ne = 0;
  uint32_t *dist = sh;
  int32_t *lp = nullptr;
  uint32_t *inq = nullptr, *lptr = nullptr, *bsize = nullptr;
  uint16_t *q0 = nullptr, *q1 = nullptr, *pos = nullptr, *order = nullptr,
           *lsucc = nullptr;
  uint8_t *ret = nullptr;
  for (uint32_t sblk = blockIdx.x; sblk < n_blocks; sblk += gridDim.x) {
    const uint32_t i0 = block_begin[sblk], i1 = block_begin[sblk + 1];
    const uint32_t ea = out_ptr[i0], eb = out_ptr[i1];
    if (ea == eb) continue;
    const uint32_t f = func_of_block[sblk];
    if (f != cur_f) {
      __syncthreads();
      cur_f = f;
      b0 = fbb[f];
      nb = fbb[f + 1] - b0;
      const uint32_t e0 = succ_ptr[b0];
      ne = succ_ptr[b0 + nb] - e0;
      dist = sh;                                   // [nb] u32
      lp = (int32_t *)(dist + nb);                 // [nb] i32
      inq = (uint32_t *)(lp + nb);                 // [nb] u32
      lptr = inq + nb;                             // [nb+1] u32
      bsize = lptr + nb + 1;                       // [nb] u32 block sizes
      q0 = (uint16_t *)(bsize + nb);               // [nb]
      q1 = q0 + nb;                                // [nb]
      pos = q1 + nb;                               // [nb] G' position
      order = pos + nb;                            // [nb]
      lsucc = order + nb;                          // [ne]
      ret = (uint8_t *)(lsucc + ne);               // [ne]
      for (uint32_t b = lane; b < nb; b += 64) {
        lptr[b] = succ_ptr[b0 + b] - e0;
        bsize[b] = block_begin[b0 + b + 1] - block_begin[b0 + b];
        pos[b] = (uint16_t)rpo_pos[b0 + b];
        order[b] = (uint16_t)(rpo_order[b0 + b] - b0);
      }
      if (lane == 0) lptr[nb] = ne;
      for (uint32_t e = lane; e < ne; e += 64) {
        lsucc[e] = (uint16_t)(succ[e0 + e] - b0);
        ret[e] = retreat[e0 + e];
      }
    }
    const uint32_t s = sblk - b0;
    for (uint32_t b = lane; b < nb; b += 64) {
      dist[b] = kInf;
      lp[b] = -1;
      inq[b] = 0;
    }
    if (lane == 0) {
      n_tg = 0;
      overflow = 0;
      maxpos = 0;
      n_cur = 0;
    }
    __syncthreads();
    // distinct target blocks of the edges leaving s
    for (uint32_t k = ea + lane; k < eb; k += 64) {
      const uint32_t t = block_of[e_dst[out_perm[k]]] - b0;
      if (atomicExch(&inq[t], 1u) == 0u) {
        const uint32_t slot = atomicAdd(&n_tg, 1u);
        if (slot < kMaxTargets) tg[slot] = t;
        else overflow = 1;
        if (pos[t] > pos[s]) atomicMax(&maxpos, (uint32_t)pos[t]);
      }
    }
    __syncthreads();
    for (uint32_t b = lane; b < nb; b += 64) inq[b] = 0;
    __syncthreads();
    // shortest walks: frontier = successors of s at distance 0
    for (uint32_t k = lptr[s] + lane; k < lptr[s + 1]; k += 64) {
      const uint32_t t = lsucc[k];
      dist[t] = 0;
      if (atomicExch(&inq[t], 1u) == 0u) q0[atomicAdd(&n_cur, 1u)] = (uint16_t)t;
    }
    __syncthreads();
    uint16_t *cur = q0, *nxt = q1;
    while (n_cur) {
      // once every target has a distance, walks longer than the largest of
      // them cannot shorten any target
      uint32_t bound = kInf;
      if (!overflow) {
        uint32_t m = 0;
        for (uint32_t k = 0; k < n_tg; ++k) m = max(m, dist[tg[k]]);
        bound = m;
      }
      const uint32_t nc = n_cur;
      for (uint32_t k = lane; k < nc; k += 64) inq[cur[k]] = 0;
      if (lane == 0) n_next = 0;
      __syncthreads();
      for (uint32_t k = lane; k < nc; k += 64) {
        const uint32_t v = cur[k];
        const uint32_t nd = dist[v] + bsize[v];
        if (bound != kInf && nd >= bound) continue;
        for (uint32_t q = lptr[v]; q < lptr[v + 1]; ++q) {
          const uint32_t w = lsucc[q];
          const uint32_t old = atomicMin(&dist[w], nd);
          if (nd < old && atomicExch(&inq[w], 1u) == 0u)
            nxt[atomicAdd(&n_next, 1u)] = (uint16_t)w;
        }
      }
      __syncthreads();
      if (lane == 0) n_cur = n_next;
      uint16_t *t = cur;
      cur = nxt;
      nxt = t;
      __syncthreads();
    }
    // longest G' walks over the G' order between s and the last target after it
    if (lane == 0 && maxpos > pos[s]) {
      const uint32_t mp = maxpos;
      for (uint32_t q = lptr[s]; q < lptr[s + 1]; ++q)
        if (!ret[q] && pos[lsucc[q]] <= mp && lp[lsucc[q]] < 0) lp[lsucc[q]] = 0;
      for (uint32_t ps = pos[s] + 1u; ps < mp; ++ps) {
        const uint32_t v = order[ps];
        const int32_t lv = lp[v];
        if (lv < 0) continue;
        const int32_t nv = lv + (int32_t)bsize[v];
        for (uint32_t q = lptr[v]; q < lptr[v + 1]; ++q) {
          const uint32_t w = lsucc[q];
          if (!ret[q] && pos[w] <= mp && lp[w] < nv) lp[w] = nv;
        }
      }
    }
    __syncthreads();
    const uint32_t ss = i1 - i0;
    for (uint32_t k = ea + lane; k < eb; k += 64) {
      const uint32_t e = out_perm[k];
      const uint32_t src = e_src[e], j = e_dst[e];
      const uint32_t t = block_of[j] - b0;
      const uint32_t oi = src - i0, oj = j - block_begin[b0 + t];
      uint32_t dmin, dmax;
      if (t == s && oi < oj) {
        dmin = dmax = oj - oi - 1;
      } else {
        dmin = (dist[t] == kInf) ? kInf : (ss - oi - 1) + dist[t] + oj;
        dmax = (t != s && lp[t] >= 0) ? (ss - oi - 1) + (uint32_t)lp[t] + oj : dmin;
      }
      e_dmin[e] = dmin;
      e_dmax[e] = dmax;
      if (dmin <= lat_tab[op_class[src]]) e_flags[e] |= GPA_E_LAT_KEEP;
    }
    __syncthreads();
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
  const size_t lds_dist = 4u * (5 * (size_t)max_nb + 1) + 8u * max_nb + 3u * max_ne + 16;
  if (lds_dfs > 160 * 1024 || lds_dist > 160 * 1024)
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
  GPA_HIP(hipFuncSetAttribute((const void *)k_dist, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_dist));
  uint16_t *lat = ar.get<uint16_t>(16);
  GPA_HIP(hipMemcpyAsync(lat, p.arch.lat, sizeof(p.arch.lat), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_dist, dim3(std::min<uint32_t>(nb, 2048)), dim3(64), lds_dist, s, nb,
                     p.func_block_begin.p, p.func_of_block.p, p.block_begin.p, p.block_of.p, p.succ_ptr.p, p.succ.p,
                     p.retreat.p, p.rpo_pos.p, p.rpo_order.p, p.out_ptr.p, p.out_perm.p, p.e_src.p,
                     p.e_dst.p,
                     p.op_class.p, lat, p.e_dmin.p, p.e_dmax.p, p.e_flags.p);
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
