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
//
// Every kernel takes one profile's EstArgs by value, or, in a batched
// launch, reads the profile of its work item from a device table; each
// element is computed by the same code in the same order either way, so a
// profile's results do not depend on the batch it was advised in.
#include "common.h"
#include "devutil.h"

namespace gpa {

constexpr int kNV = 11;  // 9 optimizers, active, total
constexpr int kEstThreads = 256;
// scopes per wave tile of the line sums on the one-profile path (a batch
// takes 64)
constexpr uint32_t kLineTileOne = 16;

struct Cand {
  double s;
  uint32_t o, l;
};

// One profile's advise: its program's static groupings, its blame tables,
// the scratch of the roll-up and the advice's outputs.
struct EstArgs {
  uint32_t n_instr, ns, nbl, n_roots, k, tk_chunks;
  int32_t s_mem, s_exec, s_sync;   // slots of these reasons among the blamable ones, or -1
  uint64_t n_edges;
  const uint32_t *counts;
  const double *bl, *ec;
  const uint16_t *nocand;
  const uint8_t *op_class, *tags;
  const uint32_t *e_src, *line_ptr, *line_perm, *icl_ptr, *icl_perm, *lca_ptr, *lca_perm;
  const uint32_t *scope_end, *scope_parent, *root_of, *roots;
  const uint32_t *big_list, *big_n, *big_chunk;   // 4 groupings x ns
  uint32_t seg_chunks[4];
  const uint32_t *tk_nch, *tk_cst;                // top-k chunks per kernel root
  double *own, *sub;
  double *partial[4];
  Cand *cand;
  double *active, *matched, *speedup, *kernel_T, *kernel_L, *eq3;
  uint32_t *top_opt, *top_scope;
  double *top_speed;
};

// a thread's elements: element `local * blockDim.x + threadIdx.x` of a
// batched launch's profile, a grid-stride range of the one profile otherwise
#define EST_ITEM(COUNT, VAR)                                                     \
  const EstArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;                \
  const uint64_t first_ =                                                        \
      (uint64_t)(BATCH ? items[blockIdx.x].local : blockIdx.x) * blockDim.x + threadIdx.x; \
  const uint64_t count_ = (COUNT);                                               \
  const uint64_t stride_ = BATCH ? count_ : (uint64_t)gridDim.x * blockDim.x;    \
  for (uint64_t VAR = first_; VAR < count_; VAR += stride_)

// the contributions of the instruction at position kk of the line-grouped
// order to the nine optimizers (the two edge optimizers' come from the
// edges), its active and its total samples
__device__ __forceinline__ void line_value(const EstArgs &a, uint64_t kk, double (&v)[kNV]) {
  const uint32_t k = a.line_perm[kk];
  const uint32_t *C = a.counts + (size_t)k * 24;
  // blamed samples of the three blamable classes and the synchronization
  // samples kept on k (all of them when synchronization is not blamable,
  // none when a candidate took them)
  const double *Bk = a.bl + (size_t)k * a.nbl * 2;
  const double bm0 = a.s_mem >= 0 ? Bk[a.s_mem * 2] : 0.0;
  const double bm1 = a.s_mem >= 0 ? Bk[a.s_mem * 2 + 1] : 0.0;
  const double be0 = a.s_exec >= 0 ? Bk[a.s_exec * 2] : 0.0;
  const double be1 = a.s_exec >= 0 ? Bk[a.s_exec * 2 + 1] : 0.0;
  const double bs0 = a.s_sync >= 0 ? Bk[a.s_sync * 2] : 0.0;
  const double bs1 = a.s_sync >= 0 ? Bk[a.s_sync * 2 + 1] : 0.0;
  const bool sync_kept = a.s_sync < 0 || ((a.nocand[k] >> a.s_sync) & 1u);
  const double ks0 = sync_kept ? (double)C[GPA_ST_SYNC * 2] : 0.0;
  const double ks1 = sync_kept ? (double)C[GPA_ST_SYNC * 2 + 1] : 0.0;
  double act = 0.0, lat = 0.0, stalls = 0.0;
  for (int r = 0; r < 12; ++r) {
    act += (double)C[r * 2];
    lat += (double)C[r * 2 + 1];
    if (r != GPA_ST_SELECTED) stalls += (double)C[r * 2] + (double)C[r * 2 + 1];
  }
  const uint32_t cls = a.op_class[k];
  const uint8_t tg = a.tags[k];
  v[GPA_O_REGISTER_REUSE] = (cls == GPA_OP_LOCAL_LOAD || cls == GPA_OP_LOCAL_STORE) ? bm0 + bm1 : 0.0;
  v[GPA_O_STRENGTH_REDUCTION] = (cls == GPA_OP_FP64 || cls == GPA_OP_LONG_ALU) ? be0 + be1 : 0.0;
  v[GPA_O_FUNCTION_SPLIT] = (double)C[GPA_ST_INST_FETCH * 2] + (double)C[GPA_ST_INST_FETCH * 2 + 1];
  v[GPA_O_FAST_MATH] = (tg & 1) ? stalls : 0.0;
  v[GPA_O_WARP_BALANCE] = bs0 + bs1 + ks0 + ks1;
  v[GPA_O_MEM_TRANSACTION_REDUCTION] =
      (cls == GPA_OP_GLOBAL_LOAD || cls == GPA_OP_GLOBAL_STORE)
          ? (double)C[GPA_ST_MEM_THROTTLE * 2] + (double)C[GPA_ST_MEM_THROTTLE * 2 + 1]
          : 0.0;
  v[GPA_O_LOOP_UNROLLING] = 0.0;
  v[GPA_O_CODE_REORDERING] = 0.0;
  v[GPA_O_FUNCTION_INLINING] = (cls == GPA_OP_CALL || (tg & 2)) ? lat : 0.0;
  v[9] = act;
  v[10] = act + lat;
}

// latency samples of global-memory and execution dependency stalls carried
// by an edge (Loop Unrolling and Code Reordering)
// (written by the blamer with the shares: the latency-bit share of an
// execution dependency plus, from a global load, that of a memory
// dependency; two non-negative terms, so their order does not matter)
__device__ __forceinline__ double edge_contrib(const EstArgs &a, uint64_t e) { return a.ec[e]; }

// Segmented sums over contiguous ranges [begin(l), end(l)) of the four
// groupings g: 0 instructions by line (W = 11, into own), 1 edges by common
// loop and 2 edges by common scope (W = 1, into own's Loop Unrolling and
// Code Reordering columns, after grouping 0), 3 scope subtrees (ranges l to
// scope_end[l] of own, W = 11, into sub).  The elements of groupings 0-2 are
// the instructions' and edges' contributions, computed where they are summed
// (never stored); grouping 3 reads own.  A segment of at most kSmallSeg
// elements is summed by one thread in element order; the longer ones
// (listed once at load, with their chunk counts) in chunks of kSegChunk by
// one workgroup each, every thread owning a fixed stride and the reduction a
// fixed shape, and the chunks then in order.  Either way the result does not
// depend on scheduling.
struct SegView {
  const uint32_t *ptr, *end;          // segment bounds (ptr mode when ptr)
  const uint32_t *big_list, *big_n;   // the long segments
  const uint32_t *chunk_start;        // their first chunk
  uint32_t n_chunks, out_stride, out_off;
  const uint32_t *perm;               // edge groupings: the edge of each element
  const double *data;                 // grouping 3: the elements
  double *out, *partial;
};

template <int G>
__device__ __forceinline__ SegView seg_view(const EstArgs &a) {
  SegView v;
  v.ptr = G == 0 ? a.line_ptr : G == 1 ? a.icl_ptr : G == 2 ? a.lca_ptr : nullptr;
  v.end = G == 3 ? a.scope_end : nullptr;
  v.big_list = a.big_list + (size_t)G * a.ns;
  v.big_n = a.big_n + G;
  v.chunk_start = a.big_chunk + (size_t)G * a.ns;
  v.n_chunks = a.seg_chunks[G];
  v.perm = G == 1 ? a.icl_perm : G == 2 ? a.lca_perm : nullptr;
  v.data = G == 3 ? a.own : nullptr;
  v.out = G == 3 ? a.sub : a.own;
  v.out_stride = (G == 1 || G == 2) ? kNV : 1;
  v.out_off = G == 1 ? GPA_O_LOOP_UNROLLING : G == 2 ? GPA_O_CODE_REORDERING : 0;
  v.partial = a.partial[G];
  return v;
}

// grid row y picks grouping G0 + y when NG = 2 (the two edge groupings
// share launches)
template <int G0, int NG>
__device__ __forceinline__ SegView pick_view(const EstArgs &a) {
  if constexpr (NG == 2) {
    static_assert(G0 == 1, "the edge groupings");
    // field by field, so that no view is selected as a whole in memory
    const bool y = blockIdx.y != 0;
    SegView v;
    v.ptr = y ? a.lca_ptr : a.icl_ptr;
    v.end = nullptr;
    v.big_list = a.big_list + (size_t)(y ? 2 : 1) * a.ns;
    v.big_n = a.big_n + (y ? 2 : 1);
    v.chunk_start = a.big_chunk + (size_t)(y ? 2 : 1) * a.ns;
    v.n_chunks = y ? a.seg_chunks[2] : a.seg_chunks[1];
    v.out_stride = kNV;
    v.out_off = y ? GPA_O_CODE_REORDERING : GPA_O_LOOP_UNROLLING;
    v.perm = y ? a.lca_perm : a.icl_perm;
    v.data = nullptr;
    v.out = a.own;
    v.partial = y ? a.partial[2] : a.partial[1];
    return v;
  } else {
    return seg_view<G0>(a);
  }
}

// segment l's range: ptr mode for groupings 0-2, subtree mode for 3
template <int G0>
__device__ __forceinline__ uint32_t seg_lo(const SegView &S, uint32_t l) {
  if constexpr (G0 == 3) return l;
  else return S.ptr[l];
}
template <int G0>
__device__ __forceinline__ uint32_t seg_hi(const SegView &S, uint32_t l) {
  if constexpr (G0 == 3) return S.end[l];
  else return S.ptr[l + 1];
}

// element i of a grouping
template <int W, int G0>
__device__ __forceinline__ void seg_elem(const EstArgs &a, const SegView &S, uint32_t i,
                                         double (&t)[W]) {
  if constexpr (G0 == 0) {
    static_assert(W == kNV, "instruction contributions");
    line_value(a, i, t);
  } else if constexpr (G0 == 1 || G0 == 2) {
    static_assert(W == 1, "edge contributions");
    t[0] = edge_contrib(a, S.perm[i]);
  } else {
#pragma unroll
    for (int q = 0; q < W; ++q) t[q] = S.data[(size_t)i * W + q];
  }
}

template <int W>
__device__ __forceinline__ void seg_store(const SegView &S, uint32_t l, const double (&v)[W]) {
  double *o = S.out + ((size_t)l * W) * S.out_stride + S.out_off;
#pragma unroll
  for (int q = 0; q < W; ++q) o[q] = v[q];
}

template <int W, int G0, int NG, bool BATCH>
__global__ void __launch_bounds__(kEstThreads)
k_seg_small(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  EST_ITEM(a.ns, lw) {
    const uint32_t l = (uint32_t)lw;
    const SegView S = pick_view<G0, NG>(a);
    const uint32_t b0 = seg_lo<G0>(S, l), b1 = seg_hi<G0>(S, l);
    if (b1 - b0 <= kSmallSeg) {
      // (an instruction's contribution reads 30 values: two at a time)
      constexpr int kSmallU = G0 == 0 ? 2 : 4;
      double v[W];
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] = 0.0;
      // kSmallU elements' loads issued together, added in element order
      uint32_t i = b0;
      for (; i + kSmallU <= b1; i += kSmallU) {
        double t[kSmallU][W];
#pragma unroll
        for (int u = 0; u < kSmallU; ++u) seg_elem<W, G0>(a, S, i + u, t[u]);
#pragma unroll
        for (int u = 0; u < kSmallU; ++u)
#pragma unroll
          for (int q = 0; q < W; ++q) v[q] += t[u][q];
      }
      for (; i < b1; ++i) {
        double t[W];
        seg_elem<W, G0>(a, S, i, t);
#pragma unroll
        for (int q = 0; q < W; ++q) v[q] += t[q];
      }
      seg_store<W>(S, l, v);
    }
  }
}

// Grouping 0 (instructions by line), segments of at most kSmallSeg
// elements: one wave per tile of TW <= 64 consecutive scopes (lane l < TW
// owns scope l0 + l).  The tile's elements are contiguous in the line-grouped order and
// are computed 64 at a time by all lanes (their count rows read coalesced);
// each owner then adds its own elements, taken across lanes, in element
// order: the same additions in the same order as a loop over them.  (The
// elements of the longer segments, summed by k_seg_chunks, are computed
// here too and not used; lines that long are rare.)
template <bool BATCH, uint32_t TW>
__global__ void __launch_bounds__(kEstThreads)
k_line_tiles(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  static_assert(TW >= 1 && TW <= kWave, "tile width");
  constexpr uint32_t kWaves = kEstThreads / kWave;
  const EstArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t ns = a.ns, n_tiles = (ns + TW - 1) / TW;
  const uint32_t t0 = (BATCH ? items[blockIdx.x].local : blockIdx.x) * kWaves +
                      threadIdx.x / kWave;
  const uint32_t t_step = BATCH ? n_tiles : gridDim.x * kWaves;
  const SegView S = seg_view<0>(a);
  for (uint32_t t = t0; t < n_tiles; t += t_step) {
    const uint32_t l0 = t * TW, l = l0 + lane;
    const bool own = lane < TW && l < ns;
    const uint32_t b0 = own ? S.ptr[l] : 0u, b1 = own ? S.ptr[l + 1] : 0u;
    const bool mine = own && b1 - b0 <= kSmallSeg;
    const uint32_t P0 = S.ptr[l0], P1 = S.ptr[min(l0 + TW, ns)];
    double v[kNV];
#pragma unroll
    for (int q = 0; q < kNV; ++q) v[q] = 0.0;
    for (uint32_t base = P0; base < P1; base += kWave) {
      double x[kNV];
      line_value(a, base + lane < P1 ? base + lane : P0, x);
      const uint32_t lo = max(b0, base), hi = min(b1, base + kWave);
      const uint32_t cnt = (mine && hi > lo) ? hi - lo : 0u;
      const uint32_t rounds = wave_max_u32(cnt);
      for (uint32_t r = 0; r < rounds; ++r) {
        const int from = (int)(r < cnt ? lo - base + r : lane);
        double y[kNV];
#pragma unroll
        for (int q = 0; q < kNV; ++q) y[q] = __shfl(x[q], from, kWave);
        if (r < cnt)
#pragma unroll
          for (int q = 0; q < kNV; ++q) v[q] += y[q];
      }
    }
    if (mine) seg_store<kNV>(S, l, v);
  }
}

// Segments longer than kSmallSeg, in chunks of kSegChunk elements: one
// workgroup per chunk (element order within a thread's stride, then the
// waves' sums in a fixed shape), then per segment its chunks in order.
template <int W, int G0, int NG, bool BATCH>
__global__ void __launch_bounds__(kEstThreads)
k_seg_chunks(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  static_assert(kEstThreads == 256, "four waves");
  __shared__ double red[4][W];
  const EstArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;
  const SegView S = pick_view<G0, NG>(a);
  const uint32_t nl = *S.big_n;
  const uint32_t c0 = BATCH ? items[blockIdx.x].local : blockIdx.x;
  const uint32_t cstep = BATCH ? S.n_chunks : gridDim.x;
  for (uint32_t c = c0; c < S.n_chunks; c += cstep) {
    const uint32_t j = upper_index_u32(S.chunk_start, 0, nl, c);
    const uint32_t l = S.big_list[j];
    const uint32_t a0 = seg_lo<G0>(S, l), b0 = seg_hi<G0>(S, l);
    const uint32_t lo = a0 + (c - S.chunk_start[j]) * kSegChunk, hi = min(lo + kSegChunk, b0);
    double v[W];
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = 0.0;
    uint32_t i = lo + threadIdx.x;
    for (; i + 3 * 256 < hi; i += 4 * 256) {
      double t0[W], t1[W], t2[W], t3[W];
      seg_elem<W, G0>(a, S, i, t0);
      seg_elem<W, G0>(a, S, i + 256, t1);
      seg_elem<W, G0>(a, S, i + 512, t2);
      seg_elem<W, G0>(a, S, i + 768, t3);
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += ((t0[q] + t1[q]) + (t2[q] + t3[q]));
    }
    for (; i < hi; i += 256) {
      double t[W];
      seg_elem<W, G0>(a, S, i, t);
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += t[q];
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

template <int W, int G0, int NG, bool BATCH>
__global__ void __launch_bounds__(kEstThreads)
k_seg_combine(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  const EstArgs &a0 = BATCH ? many[items[blockIdx.x].entry] : one;
  const SegView S0 = pick_view<G0, NG>(a0);
  EST_ITEM(*S0.big_n, jw) {
    (void)a;   // the item's profile is a0's
    const SegView &S = S0;
    const uint32_t j = (uint32_t)jw, nl = *S.big_n;
    const uint32_t c0 = S.chunk_start[j], c1 = (j + 1 < nl) ? S.chunk_start[j + 1] : S.n_chunks;
    double v[W];
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = 0.0;
    for (uint32_t c = c0; c < c1; ++c)
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] += S.partial[(size_t)c * W + q];
    seg_store<W>(S, S.big_list[j], v);
  }
}

// T / (T - y): 1 for an empty kernel; +inf once y reaches T (also when
// rounding in the share sums puts y a few ulps above T)
__device__ __forceinline__ double saturating_speedup(double T, double y) {
  return (T == 0.0) ? 1.0 : (y >= T ? __builtin_huge_val() : T / (T - y));
}

// One thread per (scope, optimizer), in the output's order (consecutive
// threads write consecutive elements); the thread of optimizer 0 also writes
// the scope's active samples, its kernel totals and Eq. (3) at a root.
template <bool BATCH>
__global__ void __launch_bounds__(kEstThreads)
k_speedup(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  EST_ITEM((uint64_t)a.ns * GPA_N_OPT, ew) {
    const uint32_t l = (uint32_t)(ew / GPA_N_OPT), o = (uint32_t)(ew % GPA_N_OPT);
    const double *x = a.sub + (size_t)l * kNV;
    const double T = a.sub[(size_t)a.root_of[l] * kNV + 10];
    const double A = x[9];
    const double M = x[o];
    const double y = (o >= GPA_O_LOOP_UNROLLING) ? (A < M ? A : M) : M;
    a.matched[ew] = M;
    a.speedup[ew] = saturating_speedup(T, y);
    if (o == 0) {
      a.active[l] = A;
      const bool root = a.scope_parent[l] == GPA_NONE;
      a.kernel_T[l] = root ? T : 0.0;
      a.kernel_L[l] = root ? T - A : 0.0;
      for (int h = 0; h < 3; ++h)
        a.eq3[(size_t)l * 3 + h] = root ? saturating_speedup(T, x[GPA_O_LOOP_UNROLLING + h]) : 0.0;
    }
  }
}

// ------------------------------------------------------------------ top-k
// Two stages: a workgroup takes kTopChunk of one kernel's (scope, optimizer)
// items, 8 per thread kept sorted in registers, and picks its best 16 in 16
// rounds, each round selecting the best head over the workgroup (DPP moves
// within rows and lane reads across them, then one exchange of the 4 wave
// winners in LDS) and popping it
// from its owner; one workgroup per kernel then does the same over its
// chunks' winners, carrying the best 16 across rounds of kTopChunk.  Order:
// speedup descending, then optimizer, then scope ascending (a total order,
// so the result is unique).
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

// c becomes the better of itself and the candidate that DPP control CTRL
// brings from another lane of its row of 16 (every lane of the wave active)
template <int CTRL>
__device__ __forceinline__ void take_dpp(Cand &c) {
  const uint64_t sb = (uint64_t)__double_as_longlong(c.s);
  const uint32_t lo =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)sb, CTRL, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(sb >> 32), CTRL, 0xF, 0xF, false);
  Cand o;
  o.s = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  o.o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c.o, CTRL, 0xF, 0xF, false);
  o.l = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c.l, CTRL, 0xF, 0xF, false);
  const bool take = better(o, c);
  c.s = take ? o.s : c.s;
  c.o = take ? o.o : c.o;
  c.l = take ? o.l : c.l;
}

__device__ __forceinline__ Cand lane_cand(const Cand &c, int lane) {
  const uint64_t sb = (uint64_t)__double_as_longlong(c.s);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sb, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sb >> 32), lane);
  Cand r;
  r.s = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  r.o = (uint32_t)__builtin_amdgcn_readlane((int)c.o, lane);
  r.l = (uint32_t)__builtin_amdgcn_readlane((int)c.l, lane);
  return r;
}

// the best of the wave's candidates, the same in every lane: within each row
// of 16 lanes by exchanges with the lane at xor 1, xor 2, the mirror in 8 and
// the mirror in 16 (after which every lane of a row holds the row's best),
// then the four rows' winners read from lanes 0, 16, 32, 48
__device__ __forceinline__ Cand wave_best(Cand c) {
  take_dpp<0xB1>(c);    // quad_perm [1, 0, 3, 2]
  take_dpp<0x4E>(c);    // quad_perm [2, 3, 0, 1]
  take_dpp<0x141>(c);   // row_half_mirror
  take_dpp<0x140>(c);   // row_mirror
  Cand b = lane_cand(c, 0);
#pragma unroll
  for (int r = 1; r < kWave / 16; ++r) {
    const Cand o = lane_cand(c, 16 * r);
    const bool take = better(o, b);
    b.s = take ? o.s : b.s;
    b.o = take ? o.o : b.o;
    b.l = take ? o.l : b.l;
  }
  return b;
}

// the workgroup's best kTopK of the threads' sorted lists, in order, into out.
// Real items are distinct and the order is total on them, so the round's
// winner has one owner, found by comparing it with the heads; when the lists
// are exhausted the winner is the empty candidate and popping an empty head
// changes nothing.
__device__ void select_top(Cand (&my)[kPerThread], Cand *out, Cand (*xch)[kTopThreads / kWave]) {
  const unsigned tid = threadIdx.x, w = tid / kWave;
  for (int r = 0; r < kTopK; ++r) {
    const Cand c = wave_best(my[0]);
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

// chunk c of a profile's kernels (c < tk_chunks): the best kTopK of its items
template <bool BATCH>
__global__ void __launch_bounds__(kTopThreads)
k_topk_chunks(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  __shared__ Cand xch[2][kTopThreads / kWave];
  const EstArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;
  const uint32_t c = BATCH ? items[blockIdx.x].local : blockIdx.x;
  if (c >= a.tk_chunks) return;
  const uint32_t ri = upper_index_u32(a.tk_cst, 0, a.n_roots, c);
  const uint32_t r = a.roots[ri];
  const uint64_t n_items = (uint64_t)(a.scope_end[r] - r) * GPA_N_OPT;
  const uint64_t base = (uint64_t)(c - a.tk_cst[ri]) * kTopChunk;
  const double *sp = a.speedup + (size_t)r * GPA_N_OPT;
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
  select_top(my, a.cand + (size_t)c * kTopK, xch);
}

// one workgroup per kernel root (the ri-th, its row of the output)
template <bool BATCH>
__global__ void __launch_bounds__(kTopThreads)
k_topk_final(EstArgs one, const EstArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  __shared__ Cand xch[2][kTopThreads / kWave];
  __shared__ Cand best[kTopK];
  const EstArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;
  const uint32_t ri = BATCH ? items[blockIdx.x].local : blockIdx.x;
  const uint32_t k = a.k;
  const uint32_t n = a.tk_nch[ri] * kTopK;
  const Cand *src = a.cand + (size_t)a.tk_cst[ri] * kTopK;
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
    a.top_opt[(size_t)ri * k + t] = c.o;
    a.top_scope[(size_t)ri * k + t] = c.l;
    a.top_speed[(size_t)ri * k + t] = c.o == 0xFFFFFFFFu ? 0.0 : c.s;
  }
}

// ------------------------------------------------------------------- host
void build_topk_plan(gpa_program &p, hipStream_t s, Arena &ar) {
  if (p.n_roots_dev) {
    p.n_roots = read_scalar(p.n_roots_dev, s);
    p.n_roots_dev = nullptr;
  }
  p.tk_nch.alloc(p.n_roots);
  p.tk_cst.alloc(p.n_roots);
  p.tk_total_dev = nullptr;
  if (p.n_roots == 0) return;
  hipLaunchKernelGGL(k_topk_plan, dim3(grid_for(p.n_roots, 256, 1024)), dim3(256), 0, s,
                     p.n_roots, p.roots.p, p.scope_end.p, p.tk_nch.p);
  GPA_LAUNCH_CHECK();
  p.tk_total_dev = ar.get<unsigned long long>(1);
  exclusive_scan_u32(p.tk_nch.p, p.tk_cst.p, p.n_roots, s, ar, p.tk_total_dev);
}

static int reason_slot(uint32_t bl, int r) {
  return ((bl >> r) & 1) ? __builtin_popcount(bl & ((1u << r) - 1)) : -1;
}

// the arguments of one profile's advise; scratch from the arena, outputs
// allocated in the advice handle
// one profile's kernel arguments: scratch from `ar`; the advice's outputs
// carved from `sh` in a batched call, their own blocks otherwise
static EstArgs est_args(const gpa_program &p, const gpa_blame &b, gpa_advice &adv, uint32_t k,
                        Arena &ar, SharedBlocks *sh = nullptr) {
  const uint32_t n = p.n_instr, ns = p.n_scopes;
  EstArgs a{};
  a.n_instr = n;
  a.ns = ns;
  a.nbl = p.n_blamable;
  a.n_roots = p.n_roots;
  a.k = k;
  a.tk_chunks = p.tk_chunks;
  a.s_mem = reason_slot(p.arch.blamable, GPA_ST_MEM_DEP);
  a.s_exec = reason_slot(p.arch.blamable, GPA_ST_EXEC_DEP);
  a.s_sync = reason_slot(p.arch.blamable, GPA_ST_SYNC);
  a.n_edges = p.n_edges;
  a.counts = b.counts.p;
  a.bl = b.bl.p;
  a.nocand = b.nocand.p;
  a.ec = b.ec.p;
  a.op_class = p.op_class.p;
  a.tags = p.instr_tags.p;
  a.e_src = p.e_src.p;
  a.line_ptr = p.line_ptr;
  a.line_perm = p.line_perm;
  a.icl_ptr = p.icl_ptr;
  a.icl_perm = p.icl_perm;
  a.lca_ptr = p.lca_ptr;
  a.lca_perm = p.lca_perm;
  a.scope_end = p.scope_end.p;
  a.scope_parent = p.scope_parent.p;
  a.root_of = p.root_of.p;
  a.roots = p.roots.p;
  a.big_list = p.big_list.p;
  a.big_n = p.big_n.p;
  a.big_chunk = p.big_chunk.p;
  for (int g = 0; g < 4; ++g) a.seg_chunks[g] = (uint32_t)p.seg_chunks[g];
  a.tk_nch = p.tk_nch.p;
  a.tk_cst = p.tk_cst.p;

  a.own = ar.get<double>((size_t)ns * kNV);
  a.sub = ar.get<double>((size_t)ns * kNV);
  for (int g = 0; g < 4; ++g)
    a.partial[g] = ar.get<double>((size_t)a.seg_chunks[g] * (g == 0 || g == 3 ? kNV : 1));
  a.cand = ar.get<Cand>((size_t)p.tk_chunks * kTopK);
  auto out = [&](auto &d, size_t count) {
    if (sh) sh->carve(d, count);
    else d.alloc(count);
  };
  out(adv.active, ns);
  out(adv.matched, (size_t)ns * GPA_N_OPT);
  out(adv.speedup, (size_t)ns * GPA_N_OPT);
  out(adv.kernel_T, ns);
  out(adv.kernel_L, ns);
  out(adv.eq3, (size_t)ns * 3);
  adv.k = k;
  // one row of k per kernel root, in the order of p.roots (ascending scope)
  out(adv.top_opt, (size_t)p.n_roots * k);
  out(adv.top_scope, (size_t)p.n_roots * k);
  out(adv.top_speed, (size_t)p.n_roots * k);
  a.active = adv.active.p;
  a.matched = adv.matched.p;
  a.speedup = adv.speedup.p;
  a.kernel_T = adv.kernel_T.p;
  a.kernel_L = adv.kernel_L.p;
  a.eq3 = adv.eq3.p;
  a.top_opt = adv.top_opt.p;
  a.top_scope = adv.top_scope.p;
  a.top_speed = adv.top_speed.p;
  return a;
}

// launches over one profile (BATCH = false: grid-stride, args by value) or
// over a batch (work lists per stage, args from the device table)
struct EstLaunch {
  hipStream_t s;
  EstArgs one;
  const EstArgs *many = nullptr;
  template <typename K>
  void operator()(K kern, unsigned gx, unsigned gy, const WorkItem *items) {
    if (gx == 0) return;
    hipLaunchKernelGGL(kern, dim3(gx, gy), dim3(kEstThreads), 0, s, one, many, items);
    GPA_LAUNCH_CHECK();
  }
};

void run_estimate(const gpa_program &p, const gpa_blame &b, gpa_advice &adv, uint32_t k,
                  hipStream_t s, Arena &ar) {
  EstLaunch L{s, est_args(p, b, adv, k, ar)};
  const EstArgs &a = L.one;
  const uint32_t ns = p.n_scopes;
  const unsigned gs = grid_for(ns, kEstThreads, 8192);
  auto chunks = [](uint32_t c) { return (unsigned)std::min<uint32_t>(c, 4096); };
  auto combine = [&](uint32_t c) { return c ? grid_for(c, kEstThreads, 1024) : 0u; };
  L(k_line_tiles<false, kLineTileOne>,
    grid_for((ns + kLineTileOne - 1) / kLineTileOne, kEstThreads / kWave, 8192), 1, nullptr);
  L(k_seg_chunks<kNV, 0, 1, false>, chunks(a.seg_chunks[0]), 1, nullptr);
  L(k_seg_combine<kNV, 0, 1, false>, combine(a.seg_chunks[0]), 1, nullptr);
  L(k_seg_small<1, 1, 2, false>, gs, 2, nullptr);
  const uint32_t ce = std::max(a.seg_chunks[1], a.seg_chunks[2]);
  L(k_seg_chunks<1, 1, 2, false>, chunks(ce), 2, nullptr);
  L(k_seg_combine<1, 1, 2, false>, combine(ce), 2, nullptr);
  L(k_seg_small<kNV, 3, 1, false>, gs, 1, nullptr);
  L(k_seg_chunks<kNV, 3, 1, false>, chunks(a.seg_chunks[3]), 1, nullptr);
  L(k_seg_combine<kNV, 3, 1, false>, combine(a.seg_chunks[3]), 1, nullptr);
  L(k_speedup<false>, grid_for((size_t)ns * GPA_N_OPT, kEstThreads, 8192), 1, nullptr);
  if (k && p.n_roots) {
    hipLaunchKernelGGL(k_topk_chunks<false>, dim3(std::max(p.tk_chunks, 1u)), dim3(kTopThreads), 0,
                       s, L.one, nullptr, nullptr);
    GPA_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_topk_final<false>, dim3(p.n_roots), dim3(kTopThreads), 0, s, L.one,
                       nullptr, nullptr);
    GPA_LAUNCH_CHECK();
  }
}

void run_estimate_batch(const gpa_blame *const *b, gpa_advice *const *adv, uint32_t count,
                        uint32_t k, hipStream_t s, Arena &ar, PhaseTimer *t) {
  std::vector<EstArgs> args(count);
  // per-entry workgroups of each stage: scopes, chunks of each grouping and
  // their long segments, top-k chunks, kernel roots
  std::vector<uint32_t> w_scope(count), w_opt(count), w_ch[3], w_cb[3], w_tkc(count),
      w_tkf(count);
  for (int g = 0; g < 3; ++g) {
    w_ch[g].resize(count);
    w_cb[g].resize(count);
  }
  auto tiles = [](uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); };
  // the advice outputs of the whole batch share one set of pool chunks
  auto sh = std::make_shared<SharedBlocks>();
  for (uint32_t e = 0; e < count; ++e) {
    const gpa_program &p = *b[e]->prog;
    adv[e]->shared = sh;
    args[e] = est_args(p, *b[e], *adv[e], k, ar, sh.get());
    const EstArgs &a = args[e];
    w_scope[e] = tiles(p.n_scopes, kEstThreads);
    w_opt[e] = tiles((uint64_t)p.n_scopes * GPA_N_OPT, kEstThreads);
    const uint32_t nc[3] = {a.seg_chunks[0], std::max(a.seg_chunks[1], a.seg_chunks[2]),
                            a.seg_chunks[3]};
    for (int g = 0; g < 3; ++g) {
      w_ch[g][e] = nc[g];
      w_cb[g][e] = tiles(nc[g], kEstThreads);   // long segments <= chunks
    }
    w_tkc[e] = (k && p.n_roots) ? p.tk_chunks : 0u;
    w_tkf[e] = (k && p.n_roots) ? p.n_roots : 0u;
  }
  BatchPlan plan(count);
  const uint32_t q_scope = plan.add(w_scope), q_opt = plan.add(w_opt);
  uint32_t q_ch[3], q_cb[3];
  for (int g = 0; g < 3; ++g) {
    q_ch[g] = plan.add(w_ch[g]);
    q_cb[g] = plan.add(w_cb[g]);
  }
  const uint32_t q_tkc = plan.add(w_tkc), q_tkf = plan.add(w_tkf);
  Upload up;
  const size_t i_args = up.add(args), i_pre = up.add(plan.pre);
  send_plan_beside(up, i_pre, plan, ar, s);
  EstLaunch L{s, EstArgs{}, up.ptr<EstArgs>(i_args)};
  auto run = [&](auto kern, uint32_t q, unsigned gy) { L(kern, plan.blocks(q), gy, plan.items(q)); };
  if (t) t->begin(kPhaseAdvise, s);
  run(k_line_tiles<true, kWave>, q_scope, 1);
  run(k_seg_chunks<kNV, 0, 1, true>, q_ch[0], 1);
  run(k_seg_combine<kNV, 0, 1, true>, q_cb[0], 1);
  run(k_seg_small<1, 1, 2, true>, q_scope, 2);
  run(k_seg_chunks<1, 1, 2, true>, q_ch[1], 2);
  run(k_seg_combine<1, 1, 2, true>, q_cb[1], 2);
  run(k_seg_small<kNV, 3, 1, true>, q_scope, 1);
  run(k_seg_chunks<kNV, 3, 1, true>, q_ch[2], 1);
  run(k_seg_combine<kNV, 3, 1, true>, q_cb[2], 1);
  run(k_speedup<true>, q_opt, 1);
  if (plan.blocks(q_tkc)) {
    hipLaunchKernelGGL(k_topk_chunks<true>, dim3(plan.blocks(q_tkc)), dim3(kTopThreads), 0, s,
                       EstArgs{}, L.many, plan.items(q_tkc));
    GPA_LAUNCH_CHECK();
  }
  if (plan.blocks(q_tkf)) {
    hipLaunchKernelGGL(k_topk_final<true>, dim3(plan.blocks(q_tkf)), dim3(kTopThreads), 0, s,
                       EstArgs{}, L.many, plan.items(q_tkf));
    GPA_LAUNCH_CHECK();
  }
  if (t) t->end(s);
}

}  // namespace gpa
