// Code-optimization estimators (Sec. 5, Table 2, Eqs. (2), (4), (5)).
//
// Matched samples per optimizer are routed to a static target scope:
//   Register Reuse, Strength Reduction, Warp Balance (blamed part): the
//     source's line; Function Split, Fast Math, Memory Transaction
//     Reduction, Function Inlining, Warp Balance (kept part): the sampled
//     instruction's line;
//   Loop Unrolling: the innermost loop holding both ends of the edge;
//   Code Reordering: the lowest common scope of both ends.
// A scope's estimate uses the sums over its whole subtree (nested(l) in
// Eq. (5)): matched samples M, active samples A; T is its kernel's total.
//   stall elimination  S = T / (T - M)                     (Eq. 2)
//   latency hiding     S = T / (T - min(A, M))             (Eq. 5; Eq. 4 at a kernel)
// Subtree sums are direct sums over the contiguous preorder range of the
// subtree, never differences of prefix sums.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kNV = 11;  // 9 optimizers, active, total

__global__ void k_instr_contrib(uint32_t n_instr, uint32_t nbl, uint32_t blamable,
                                const uint32_t *counts, const double *blamed, const double *self_,
                                const uint8_t *op_class, const uint8_t *tags, double *iv) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_instr;
       k += gridDim.x * blockDim.x) {
    const uint32_t *C = counts + (size_t)k * 24;
    const double *Bl = blamed + (size_t)k * 24;
    const double *Sf = self_ + (size_t)k * 24;
    double act = 0.0, lat = 0.0, stalls = 0.0;
    for (int r = 0; r < 12; ++r) {
      act += (double)C[r * 2];
      lat += (double)C[r * 2 + 1];
      if (r != GPA_ST_SELECTED) stalls += (double)C[r * 2] + (double)C[r * 2 + 1];
    }
    const uint32_t cls = op_class[k];
    const uint8_t tg = tags[k];
    double v[kNV];
    v[GPA_O_REGISTER_REUSE] = (cls == GPA_OP_LOCAL_LOAD || cls == GPA_OP_LOCAL_STORE)
                                  ? Bl[GPA_ST_MEM_DEP * 2] + Bl[GPA_ST_MEM_DEP * 2 + 1]
                                  : 0.0;
    v[GPA_O_STRENGTH_REDUCTION] = (cls == GPA_OP_FP64 || cls == GPA_OP_LONG_ALU)
                                      ? Bl[GPA_ST_EXEC_DEP * 2] + Bl[GPA_ST_EXEC_DEP * 2 + 1]
                                      : 0.0;
    v[GPA_O_FUNCTION_SPLIT] = (double)C[GPA_ST_INST_FETCH * 2] + (double)C[GPA_ST_INST_FETCH * 2 + 1];
    v[GPA_O_FAST_MATH] = (tg & 1) ? stalls : 0.0;
    v[GPA_O_WARP_BALANCE] = Bl[GPA_ST_SYNC * 2] + Bl[GPA_ST_SYNC * 2 + 1] + Sf[GPA_ST_SYNC * 2] +
                            Sf[GPA_ST_SYNC * 2 + 1];
    v[GPA_O_MEM_TRANSACTION_REDUCTION] =
        (cls == GPA_OP_GLOBAL_LOAD || cls == GPA_OP_GLOBAL_STORE)
            ? (double)C[GPA_ST_MEM_THROTTLE * 2] + (double)C[GPA_ST_MEM_THROTTLE * 2 + 1]
            : 0.0;
    v[GPA_O_LOOP_UNROLLING] = 0.0;
    v[GPA_O_CODE_REORDERING] = 0.0;
    v[GPA_O_FUNCTION_INLINING] = (cls == GPA_OP_CALL || (tg & 2)) ? lat : 0.0;
    v[9] = act;
    v[10] = act + lat;
    for (int q = 0; q < kNV; ++q) iv[(size_t)k * kNV + q] = v[q];
  }
}

// latency samples of global-memory and execution dependency stalls carried
// by an edge (Loop Unrolling and Code Reordering)
__device__ __forceinline__ double edge_contrib(uint64_t e, uint32_t nbl, int s_mem, int s_exec,
                                               const uint32_t *e_src, const uint8_t *op_class,
                                               const double *share) {
  double v = 0.0;
  if (s_mem >= 0 && op_class[e_src[e]] == GPA_OP_GLOBAL_LOAD) v += share[(e * nbl + s_mem) * 2 + 1];
  if (s_exec >= 0) v += share[(e * nbl + s_exec) * 2 + 1];
  return v;
}

// the edge contributions straight into the common-loop and common-scope
// groupings' orders (edges without a common loop are left out of the first:
// its size is *n_icl)
__global__ void k_edge_gathered(uint64_t n_edges, uint32_t nbl, int s_mem, int s_exec,
                                const uint32_t *e_src, const uint8_t *op_class,
                                const double *share, const uint32_t *n_icl,
                                const uint32_t *icl_perm, const uint32_t *lca_perm, double *ev_icl,
                                double *ev_lca) {
  const uint64_t ni = min((uint64_t)*n_icl, n_edges);
  for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n_edges;
       k += (uint64_t)gridDim.x * blockDim.x) {
    ev_lca[k] = edge_contrib(lca_perm[k], nbl, s_mem, s_exec, e_src, op_class, share);
    if (k < ni) ev_icl[k] = edge_contrib(icl_perm[k], nbl, s_mem, s_exec, e_src, op_class, share);
  }
}

// values gathered into group order, so every group is a contiguous range;
// the grouped count is n, or *n_dev when given (items without a group are
// left out of the grouping)
template <int W>
__global__ void k_gather(size_t n, const uint32_t *n_dev, const uint32_t *perm, const double *src,
                         double *dst) {
  if (n_dev) n = min(n, (size_t)*n_dev);
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const double *x = src + (size_t)perm[k] * W;
#pragma unroll
    for (int q = 0; q < W; ++q) dst[k * W + q] = x[q];
  }
}

// Segmented sums over contiguous ranges [begin(l), end(l)), given either by
// ptr[l], ptr[l+1] (ptr mode) or by l, end[l] (subtree mode).  A segment of
// at most kSmallSeg elements is summed by one thread in element order; the
// longer ones (listed once at load, with their chunk counts) in chunks of
// kSegChunk by one workgroup each, every thread owning a fixed stride and the
// reduction a fixed shape, and the chunks then in order.  Either way the
// result does not depend on scheduling.  One launch serves up to two
// independent sets of segments (grid row y = set).
struct SegSet {
  const uint32_t *ptr, *end;          // segment bounds (ptr mode when ptr)
  const uint32_t *big_list, *big_n;   // the long segments
  const uint32_t *chunk_start;        // their first chunk
  uint32_t n_chunks;
  const double *data;
  double *out, *partial;
};
struct SegSets {
  SegSet set[2];
};

template <int W>
__global__ void k_seg_small(uint32_t n_seg, SegSets sets) {
  const SegSet &S = sets.set[blockIdx.y];
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < n_seg;
       l += gridDim.x * blockDim.x) {
    const uint32_t a = S.ptr ? S.ptr[l] : l;
    const uint32_t b = S.ptr ? S.ptr[l + 1] : S.end[l];
    if (b - a > kSmallSeg) continue;
    double v[W];
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = 0.0;
    for (uint32_t i = a; i < b; ++i)
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += S.data[(size_t)i * W + q];
#pragma unroll
    for (int q = 0; q < W; ++q) S.out[(size_t)l * W + q] = v[q];
  }
}

// Segments longer than kSmallSeg, in chunks of kSegChunk elements: one
// workgroup per chunk (element order within a thread's stride, then the
// waves' sums in a fixed shape), then per segment its chunks in order.
template <int W>
__global__ void __launch_bounds__(256)
k_seg_chunks(SegSets sets) {
  __shared__ double red[4][W];
  const SegSet &S = sets.set[blockIdx.y];
  const uint32_t nl = *S.big_n;
  for (uint32_t c = blockIdx.x; c < S.n_chunks; c += gridDim.x) {
    const uint32_t j = upper_index_u32(S.chunk_start, 0, nl, c);
    const uint32_t l = S.big_list[j];
    const uint32_t a0 = S.ptr ? S.ptr[l] : l, b0 = S.ptr ? S.ptr[l + 1] : S.end[l];
    const uint32_t a = a0 + (c - S.chunk_start[j]) * kSegChunk, b = min(a + kSegChunk, b0);
    const double *data = S.data;
    double v[W];
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = 0.0;
    uint32_t i = a + threadIdx.x;
    for (; i + 3 * 256 < b; i += 4 * 256) {
      double t0[W], t1[W], t2[W], t3[W];
#pragma unroll
      for (int q = 0; q < W; ++q) {
        t0[q] = data[(size_t)i * W + q];
        t1[q] = data[(size_t)(i + 256) * W + q];
        t2[q] = data[(size_t)(i + 512) * W + q];
        t3[q] = data[(size_t)(i + 768) * W + q];
      }
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += ((t0[q] + t1[q]) + (t2[q] + t3[q]));
    }
    for (; i < b; i += 256) {
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += data[(size_t)i * W + q];
    }
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = wave_sum(v[q]);
    const unsigned w = threadIdx.x / kWave;
    if (lane_id() == 0)
#pragma unroll
      for (int q = 0; q < W; ++q) red[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x < (unsigned)W)
      S.partial[(size_t)c * W + threadIdx.x] =
          (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    __syncthreads();
  }
}

template <int W>
__global__ void k_seg_combine(SegSets sets) {
  const SegSet &S = sets.set[blockIdx.y];
  const uint32_t nl = *S.big_n;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nl; j += gridDim.x * blockDim.x) {
    const uint32_t c0 = S.chunk_start[j], c1 = (j + 1 < nl) ? S.chunk_start[j + 1] : S.n_chunks;
    double v[W];
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = 0.0;
    for (uint32_t c = c0; c < c1; ++c)
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += S.partial[(size_t)c * W + q];
    const uint32_t l = S.big_list[j];
#pragma unroll
    for (int q = 0; q < W; ++q) S.out[(size_t)l * W + q] = v[q];
  }
}

// the sums of n_sets (1 or 2) sets of n_seg segments each
template <int W>
void seg_sum(uint32_t n_seg, SegSets sets, uint32_t n_sets, hipStream_t s, Arena &ar) {
  uint64_t max_chunks = 0;
  for (uint32_t y = 0; y < n_sets; ++y) {
    SegSet &S = sets.set[y];
    S.partial = S.n_chunks ? ar.get<double>((size_t)S.n_chunks * W) : nullptr;
    max_chunks = std::max<uint64_t>(max_chunks, S.n_chunks);
  }
  hipLaunchKernelGGL(k_seg_small<W>, dim3(grid_for(n_seg, 256, 8192), n_sets), dim3(256), 0, s,
                     n_seg, sets);
  if (max_chunks) {
    hipLaunchKernelGGL(k_seg_chunks<W>, dim3((unsigned)std::min<uint64_t>(max_chunks, 4096), n_sets),
                       dim3(256), 0, s, sets);
    hipLaunchKernelGGL(k_seg_combine<W>, dim3(grid_for(n_seg, 256, 1024), n_sets), dim3(256), 0, s,
                       sets);
  }
  GPA_LAUNCH_CHECK();
}

// own sums of the two edge optimizers, merged into the per-scope vectors
__global__ void k_merge_edge_own(uint32_t n_scopes, const double *own_icl, const double *own_lca,
                                 double *own) {
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < n_scopes;
       l += gridDim.x * blockDim.x) {
    own[(size_t)l * kNV + GPA_O_LOOP_UNROLLING] = own_icl[l];
    own[(size_t)l * kNV + GPA_O_CODE_REORDERING] = own_lca[l];
  }
}

// T / (T - y): 1 for an empty kernel; +inf once y reaches T (also when
// rounding in the share sums puts y a few ulps above T)
__device__ __forceinline__ double saturating_speedup(double T, double y) {
  return (T == 0.0) ? 1.0 : (y >= T ? __builtin_huge_val() : T / (T - y));
}

__global__ void k_speedup(uint32_t n_scopes, const uint32_t *parent, const uint32_t *root_of,
                          const double *sub, double *active, double *matched, double *speedup,
                          double *kernel_T, double *kernel_L, double *eq3) {
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < n_scopes;
       l += gridDim.x * blockDim.x) {
    const double *x = sub + (size_t)l * kNV;
    const double T = sub[(size_t)root_of[l] * kNV + 10];
    const double A = x[9];
    active[l] = A;
    for (int o = 0; o < GPA_N_OPT; ++o) {
      const double M = x[o];
      const double y = (o >= GPA_O_LOOP_UNROLLING) ? (A < M ? A : M) : M;
      matched[(size_t)l * GPA_N_OPT + o] = M;
      speedup[(size_t)l * GPA_N_OPT + o] = saturating_speedup(T, y);
    }
    const bool root = parent[l] == GPA_NONE;
    kernel_T[l] = root ? T : 0.0;
    kernel_L[l] = root ? T - A : 0.0;
    for (int h = 0; h < 3; ++h)
      eq3[(size_t)l * 3 + h] = root ? saturating_speedup(T, x[GPA_O_LOOP_UNROLLING + h]) : 0.0;
  }
}

// ------------------------------------------------------------------ top-k
// Two stages: a workgroup takes kTopChunk of one kernel's (scope, optimizer)
// items, 8 per thread kept sorted in registers, and picks its best 16 in 16
// rounds, each round selecting the best head over the workgroup (wave
// shuffles, then one exchange of the 4 wave winners in LDS) and popping it
// from its owner; one workgroup per kernel then does the same over its
// chunks' winners, carrying the best 16 across rounds of kTopChunk.  Order:
// speedup descending, then optimizer, then scope ascending (a total order,
// so the result is unique).
struct Cand {
  double s;
  uint32_t o, l;
};

// written with non-short-circuit operators so that it compiles to a few
// compares and mask operations rather than divergent branches
__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
  const uint64_t ka = ((uint64_t)a.o << 32) | a.l, kb = ((uint64_t)b.o << 32) | b.l;
  return (a.s > b.s) | ((a.s == b.s) & (ka < kb));
}

// the same item (bitwise: a winner is a copy of its owner's head)
__device__ __forceinline__ bool same(const Cand &a, const Cand &b) {
  return (__double_as_longlong(a.s) == __double_as_longlong(b.s)) & (a.o == b.o) & (a.l == b.l);
}

constexpr int kTopK = 16;
constexpr int kTopThreads = 256;
constexpr int kPerThread = 8;
constexpr uint32_t kTopChunk = kTopThreads * kPerThread;

__device__ __forceinline__ Cand cand_none() {
  Cand c;
  c.s = -1.0;
  c.o = 0xFFFFFFFFu;
  c.l = 0xFFFFFFFFu;
  return c;
}

__device__ __forceinline__ void cswap(Cand &a, Cand &b) {
  const bool sw = better(b, a);
  const Cand x = a, y = b;
  a.s = sw ? y.s : x.s;
  a.o = sw ? y.o : x.o;
  a.l = sw ? y.l : x.l;
  b.s = sw ? x.s : y.s;
  b.o = sw ? x.o : y.o;
  b.l = sw ? x.l : y.l;
}

// best first; a bitonic network on 8 with fixed register indices
__device__ __forceinline__ void sort8(Cand (&a)[kPerThread]) {
#pragma unroll
  for (int k = 2; k <= kPerThread; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < kPerThread; ++i) {
        const int ixj = i ^ j;
        if (ixj > i) {
          if ((i & k) == 0) cswap(a[i], a[ixj]);
          else cswap(a[ixj], a[i]);
        }
      }
}

// the workgroup's best kTopK of the threads' sorted lists, in order, into out.
// Real items are distinct and the order is total on them, so the round's
// winner has one owner, found by comparing it with the heads; when the lists
// are exhausted the winner is the empty candidate and popping an empty head
// changes nothing.
__device__ void select_top(Cand (&my)[kPerThread], Cand *out, Cand (*xch)[kTopThreads / kWave]) {
  const unsigned tid = threadIdx.x, w = tid / kWave;
  for (int r = 0; r < kTopK; ++r) {
    Cand c = my[0];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      Cand o;
      o.s = __shfl_xor(c.s, d, kWave);
      o.o = (uint32_t)__shfl_xor((int)c.o, d, kWave);
      o.l = (uint32_t)__shfl_xor((int)c.l, d, kWave);
      const bool take = better(o, c);
      c.s = take ? o.s : c.s;
      c.o = take ? o.o : c.o;
      c.l = take ? o.l : c.l;
    }
    if (lane_id() == 0) xch[r & 1][w] = c;
    __syncthreads();
    Cand best = xch[r & 1][0];
#pragma unroll
    for (int v = 1; v < kTopThreads / kWave; ++v) {
      const Cand o = xch[r & 1][v];
      const bool take = better(o, best);
      best.s = take ? o.s : best.s;
      best.o = take ? o.o : best.o;
      best.l = take ? o.l : best.l;
    }
    if (tid == 0) out[r] = best;
    const bool pop = same(my[0], best);
    const Cand none = cand_none();
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const Cand &nx = i + 1 < kPerThread ? my[i + 1] : none;
      my[i].s = pop ? nx.s : my[i].s;
      my[i].o = pop ? nx.o : my[i].o;
      my[i].l = pop ? nx.l : my[i].l;
    }
  }
}

__global__ void k_topk_plan(uint32_t n_roots, const uint32_t *roots, const uint32_t *scope_end,
                            uint32_t *nchunks) {
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n_roots; r += gridDim.x * blockDim.x) {
    const uint64_t items = (uint64_t)(scope_end[roots[r]] - roots[r]) * GPA_N_OPT;
    nchunks[r] = (uint32_t)((items + kTopChunk - 1) / kTopChunk);
  }
}

__global__ void __launch_bounds__(kTopThreads)
k_topk_chunks(uint32_t n_roots, const uint32_t *roots, const uint32_t *nchunks,
              const uint32_t *chunk_start, const uint32_t *scope_end, const double *speedup,
              Cand *cand) {
  __shared__ Cand xch[2][kTopThreads / kWave];
  const uint32_t c = blockIdx.x;
  const uint32_t total = chunk_start[n_roots - 1] + nchunks[n_roots - 1];
  if (c >= total) return;
  const uint32_t ri = upper_index_u32(chunk_start, 0, n_roots, c);
  const uint32_t r = roots[ri];
  const uint64_t n_items = (uint64_t)(scope_end[r] - r) * GPA_N_OPT;
  const uint64_t base = (uint64_t)(c - chunk_start[ri]) * kTopChunk;
  const double *sp = speedup + (size_t)r * GPA_N_OPT;
  Cand my[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const uint64_t it = base + (uint64_t)i * kTopThreads + threadIdx.x;
    Cand x = cand_none();
    if (it < n_items) {
      x.s = sp[it];
      x.l = r + (uint32_t)(it / GPA_N_OPT);
      x.o = (uint32_t)(it % GPA_N_OPT);
    }
    my[i] = x;
  }
  sort8(my);
  select_top(my, cand + (size_t)c * kTopK, xch);
}

__global__ void __launch_bounds__(kTopThreads)
k_topk_final(const uint32_t *nchunks, const uint32_t *chunk_start,
             const Cand *cand, uint32_t k, uint32_t *top_opt, uint32_t *top_scope,
             double *top_speed) {
  __shared__ Cand xch[2][kTopThreads / kWave];
  __shared__ Cand best[kTopK];
  const uint32_t ri = blockIdx.x;   // the ri-th kernel root; its row of the output
  const uint32_t n = nchunks[ri] * kTopK;
  const Cand *src = cand + (size_t)chunk_start[ri] * kTopK;
  // round 0 takes kTopChunk candidates; later rounds carry the best kTopK in
  // slots 0 .. kTopK-1 (item 0 of threads 0 .. 15) and take the rest anew
  uint32_t next = 0;
  for (uint32_t round = 0; round == 0 || next < n; ++round) {
    const uint32_t keep = round == 0 ? 0u : (uint32_t)kTopK;
    Cand my[kPerThread];
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const uint32_t slot = (uint32_t)i * kTopThreads + threadIdx.x;
      if (slot < keep) {
        my[i] = best[slot];
      } else {
        const uint32_t it = next + (slot - keep);
        my[i] = it < n ? src[it] : cand_none();
      }
    }
    next += kTopChunk - keep;
    __syncthreads();
    sort8(my);
    select_top(my, best, xch);
    __syncthreads();
  }
  for (uint32_t t = threadIdx.x; t < k; t += kTopThreads) {
    const Cand c = t < (uint32_t)kTopK ? best[t] : cand_none();
    top_opt[(size_t)ri * k + t] = c.o;
    top_scope[(size_t)ri * k + t] = c.l;
    top_speed[(size_t)ri * k + t] = c.o == 0xFFFFFFFFu ? 0.0 : c.s;
  }
}

void run_estimate(const gpa_program &p, const gpa_blame &b, gpa_advice &a, uint32_t k,
                  hipStream_t s, Arena &ar) {
  const uint32_t n = p.n_instr, ns = p.n_scopes, nbl = p.n_blamable;
  const uint32_t bl = p.arch.blamable;
  const int s_mem = ((bl >> GPA_ST_MEM_DEP) & 1) ? __builtin_popcount(bl & ((1u << GPA_ST_MEM_DEP) - 1)) : -1;
  const int s_exec =
      ((bl >> GPA_ST_EXEC_DEP) & 1) ? __builtin_popcount(bl & ((1u << GPA_ST_EXEC_DEP) - 1)) : -1;
  double *iv = ar.get<double>((size_t)n * kNV);
  double *own = ar.get<double>((size_t)ns * kNV);
  double *sub = ar.get<double>((size_t)ns * kNV);
  double *iv_g = ar.get<double>((size_t)n * kNV);
  double *ev_icl = ar.get<double>(p.n_edges), *ev_lca = ar.get<double>(p.n_edges);
  double *own_icl = ar.get<double>(ns), *own_lca = ar.get<double>(ns);
  hipLaunchKernelGGL(k_instr_contrib, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, nbl, bl,
                     b.counts.p, b.blamed.p, b.self_.p, p.op_class.p, p.instr_tags.p, iv);
  hipLaunchKernelGGL(k_gather<kNV>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, (size_t)n,
                     nullptr, p.line_perm, iv, iv_g);
  const uint32_t *big = p.big_list.p;
  const uint32_t *bch = p.big_chunk.p;
  // groupings g (0 line, 1 common loop, 2 common scope, 3 subtree): their
  // long-segment lists and chunk counts were made at load
  auto seg_set = [&](int g, const uint32_t *ptr, const uint32_t *end, const double *data,
                     double *out) {
    return SegSet{ptr, end, big + (size_t)g * ns, p.big_n.p + g, bch + (size_t)g * ns,
                  (uint32_t)p.seg_chunks[g], data, out, nullptr};
  };
  SegSets line{};
  line.set[0] = seg_set(0, p.line_ptr, nullptr, iv_g, own);
  seg_sum<kNV>(ns, line, 1, s, ar);
  if (p.n_edges)
    hipLaunchKernelGGL(k_edge_gathered, dim3(grid_for(p.n_edges, 256, 8192)), dim3(256), 0, s,
                       p.n_edges, nbl, s_mem, s_exec, p.e_src.p, p.op_class.p, b.share.p,
                       p.icl_ptr + ns, p.icl_perm, p.lca_perm, ev_icl, ev_lca);
  SegSets edges{};
  edges.set[0] = seg_set(1, p.icl_ptr, nullptr, ev_icl, own_icl);
  edges.set[1] = seg_set(2, p.lca_ptr, nullptr, ev_lca, own_lca);
  seg_sum<1>(ns, edges, 2, s, ar);
  hipLaunchKernelGGL(k_merge_edge_own, dim3(grid_for(ns, 256, 8192)), dim3(256), 0, s, ns, own_icl,
                     own_lca, own);
  SegSets subtree{};
  subtree.set[0] = seg_set(3, nullptr, p.scope_end.p, own, sub);
  seg_sum<kNV>(ns, subtree, 1, s, ar);
  GPA_LAUNCH_CHECK();
  a.active.alloc(ns);
  a.matched.alloc((size_t)ns * GPA_N_OPT);
  a.speedup.alloc((size_t)ns * GPA_N_OPT);
  a.kernel_T.alloc(ns);
  a.kernel_L.alloc(ns);
  a.eq3.alloc((size_t)ns * 3);
  hipLaunchKernelGGL(k_speedup, dim3(grid_for(ns, 256, 8192)), dim3(256), 0, s, ns,
                     p.scope_parent.p, p.root_of.p, sub, a.active.p, a.matched.p, a.speedup.p,
                     a.kernel_T.p, a.kernel_L.p, a.eq3.p);
  GPA_LAUNCH_CHECK();
  a.k = k;
  // one row of k per kernel root, in the order of p.roots (ascending scope)
  a.top_opt.alloc((size_t)p.n_roots * k);
  a.top_scope.alloc((size_t)p.n_roots * k);
  a.top_speed.alloc((size_t)p.n_roots * k);
  if (k) {
    if (p.n_roots) {
      uint32_t *nch = ar.get<uint32_t>(p.n_roots), *cst = ar.get<uint32_t>(p.n_roots);
      hipLaunchKernelGGL(k_topk_plan, dim3(grid_for(p.n_roots, 256, 1024)), dim3(256), 0, s,
                         p.n_roots, p.roots.p, p.scope_end.p, nch);
      exclusive_scan_u32(nch, cst, p.n_roots, s, ar);
      // every scope is in exactly one kernel's subtree: chunks <= items/chunk + roots
      const uint64_t max_chunks = ((uint64_t)ns * GPA_N_OPT) / kTopChunk + p.n_roots + 1;
      Cand *cand = ar.get<Cand>(max_chunks * kTopK);
      hipLaunchKernelGGL(k_topk_chunks, dim3((unsigned)max_chunks), dim3(kTopThreads), 0, s,
                         p.n_roots, p.roots.p, nch, cst, p.scope_end.p, a.speedup.p, cand);
      hipLaunchKernelGGL(k_topk_final, dim3(p.n_roots), dim3(kTopThreads), 0, s, nch, cst, cand,
                         k, a.top_opt.p, a.top_scope.p, a.top_speed.p);
    }
    GPA_LAUNCH_CHECK();
  }
}

}  // namespace gpa
