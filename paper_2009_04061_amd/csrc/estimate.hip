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
__global__ void k_edge_contrib(uint64_t n_edges, uint32_t nbl, int s_mem, int s_exec,
                               const uint32_t *e_src, const uint8_t *op_class, const double *share,
                               double *ev) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n_edges;
       e += (uint64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (s_mem >= 0 && op_class[e_src[e]] == GPA_OP_GLOBAL_LOAD) v += share[(e * nbl + s_mem) * 2 + 1];
    if (s_exec >= 0) v += share[(e * nbl + s_exec) * 2 + 1];
    ev[e] = v;
  }
}

// own sums of each scope: its instructions, then the edges targeting it
__global__ void k_scope_own(uint32_t n_scopes, const uint32_t *line_ptr, const uint32_t *line_perm,
                            const uint32_t *icl_ptr, const uint32_t *icl_perm,
                            const uint32_t *lca_ptr, const uint32_t *lca_perm, const double *iv,
                            const double *ev, double *own) {
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < n_scopes;
       l += gridDim.x * blockDim.x) {
    double v[kNV];
    for (int q = 0; q < kNV; ++q) v[q] = 0.0;
    for (uint32_t k = line_ptr[l]; k < line_ptr[l + 1]; ++k) {
      const double *x = iv + (size_t)line_perm[k] * kNV;
      for (int q = 0; q < kNV; ++q) v[q] += x[q];
    }
    for (uint32_t k = icl_ptr[l]; k < icl_ptr[l + 1]; ++k) v[GPA_O_LOOP_UNROLLING] += ev[icl_perm[k]];
    for (uint32_t k = lca_ptr[l]; k < lca_ptr[l + 1]; ++k) v[GPA_O_CODE_REORDERING] += ev[lca_perm[k]];
    for (int q = 0; q < kNV; ++q) own[(size_t)l * kNV + q] = v[q];
  }
}

// one wave per scope: sum of `own` over the preorder range [l, end(l))
__global__ void __launch_bounds__(256)
k_subtree(uint32_t n_scopes, const uint32_t *scope_end, const double *own, double *sub) {
  const uint32_t l = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (l >= n_scopes) return;
  const unsigned lane = lane_id();
  const uint32_t end = scope_end[l];
  double v[kNV];
  for (int q = 0; q < kNV; ++q) v[q] = 0.0;
  for (uint32_t s = l + lane; s < end; s += kWave) {
    const double *x = own + (size_t)s * kNV;
    for (int q = 0; q < kNV; ++q) v[q] += x[q];
  }
  for (int q = 0; q < kNV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
    for (int q = 0; q < kNV; ++q) sub[(size_t)l * kNV + q] = v[q];
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
      speedup[(size_t)l * GPA_N_OPT + o] = (T == 0.0) ? 1.0 : T / (T - y);
    }
    const bool root = parent[l] == GPA_NONE;
    kernel_T[l] = root ? T : 0.0;
    kernel_L[l] = root ? T - A : 0.0;
    for (int h = 0; h < 3; ++h)
      eq3[(size_t)l * 3 + h] =
          root ? ((T == 0.0) ? 1.0 : T / (T - x[GPA_O_LOOP_UNROLLING + h])) : 0.0;
  }
}

// ------------------------------------------------------------------ top-k
struct Cand {
  double s;
  uint32_t o, l;
};

__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
  if (a.s != b.s) return a.s > b.s;
  if (a.o != b.o) return a.o < b.o;
  return a.l < b.l;
}

constexpr int kTopMax = 16;
constexpr int kTopThreads = 256;

__global__ void __launch_bounds__(kTopThreads)
k_topk(const uint32_t *roots, const uint32_t *scope_end, const double *speedup, uint32_t k,
       uint32_t *top_opt, uint32_t *top_scope, double *top_speed) {
  __shared__ Cand red[kTopThreads];
  const uint32_t r = roots[blockIdx.x];
  const uint32_t end = scope_end[r];
  const uint64_t n_items = (uint64_t)(end - r) * GPA_N_OPT;
  Cand mine[kTopMax];
  uint32_t nm = 0;
  for (uint64_t it = threadIdx.x; it < n_items; it += kTopThreads) {
    Cand c;
    c.l = r + (uint32_t)(it / GPA_N_OPT);
    c.o = (uint32_t)(it % GPA_N_OPT);
    c.s = speedup[(size_t)c.l * GPA_N_OPT + c.o];
    if (nm == k && !better(c, mine[k - 1])) continue;
    uint32_t p = (nm < k) ? nm++ : k - 1;
    while (p > 0 && better(c, mine[p - 1])) {
      mine[p] = mine[p - 1];
      --p;
    }
    mine[p] = c;
  }
  uint32_t head = 0;
  for (uint32_t t = 0; t < k; ++t) {
    Cand c;
    c.s = -1.0;
    c.o = 0xFFFFFFFFu;
    c.l = 0xFFFFFFFFu;
    if (head < nm) c = mine[head];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = kTopThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w && better(red[threadIdx.x + w], red[threadIdx.x]))
        red[threadIdx.x] = red[threadIdx.x + w];
      __syncthreads();
    }
    const Cand best = red[0];
    __syncthreads();
    if (best.o == 0xFFFFFFFFu) break;
    if (head < nm && mine[head].o == best.o && mine[head].l == best.l) ++head;
    if (threadIdx.x == 0) {
      top_opt[(size_t)r * k + t] = best.o;
      top_scope[(size_t)r * k + t] = best.l;
      top_speed[(size_t)r * k + t] = best.s;
    }
  }
}

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f64(double *p, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void run_estimate(const gpa_program &p, const gpa_blame &b, gpa_advice &a, uint32_t k,
                  hipStream_t s, Arena &ar) {
  const uint32_t n = p.n_instr, ns = p.n_scopes, nbl = p.n_blamable;
  const uint32_t bl = p.arch.blamable;
  const int s_mem = ((bl >> GPA_ST_MEM_DEP) & 1) ? __builtin_popcount(bl & ((1u << GPA_ST_MEM_DEP) - 1)) : -1;
  const int s_exec =
      ((bl >> GPA_ST_EXEC_DEP) & 1) ? __builtin_popcount(bl & ((1u << GPA_ST_EXEC_DEP) - 1)) : -1;
  double *iv = ar.get<double>((size_t)n * kNV);
  double *ev = ar.get<double>(p.n_edges);
  double *own = ar.get<double>((size_t)ns * kNV);
  double *sub = ar.get<double>((size_t)ns * kNV);
  hipLaunchKernelGGL(k_instr_contrib, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, nbl, bl,
                     b.counts.p, b.blamed.p, b.self_.p, p.op_class.p, p.instr_tags.p, iv);
  if (p.n_edges)
    hipLaunchKernelGGL(k_edge_contrib, dim3(grid_for(p.n_edges, 256, 8192)), dim3(256), 0, s,
                       p.n_edges, nbl, s_mem, s_exec, p.e_src.p, p.op_class.p, b.share.p, ev);
  hipLaunchKernelGGL(k_scope_own, dim3(grid_for(ns, 256, 8192)), dim3(256), 0, s, ns, p.line_ptr.p,
                     p.line_perm.p, p.icl_ptr.p, p.icl_perm.p, p.lca_ptr.p, p.lca_perm.p, iv, ev,
                     own);
  hipLaunchKernelGGL(k_subtree, dim3((ns + 3) / 4), dim3(256), 0, s, ns, p.scope_end.p, own, sub);
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
  a.top_opt.alloc((size_t)ns * k);
  a.top_scope.alloc((size_t)ns * k);
  a.top_speed.alloc((size_t)ns * k);
  if (k) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((size_t)ns * k, 256, 4096)), dim3(256), 0, s,
                       a.top_opt.p, (size_t)ns * k, GPA_NONE);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((size_t)ns * k, 256, 4096)), dim3(256), 0, s,
                       a.top_scope.p, (size_t)ns * k, GPA_NONE);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((size_t)ns * k, 256, 4096)), dim3(256), 0, s,
                       a.top_speed.p, (size_t)ns * k, 0.0);
    if (p.n_roots)
      hipLaunchKernelGGL(k_topk, dim3(p.n_roots), dim3(kTopThreads), 0, s, p.roots.p,
                         p.scope_end.p, a.speedup.p, k, a.top_opt.p, a.top_scope.p,
                         a.top_speed.p);
    GPA_LAUNCH_CHECK();
  }
}

}  // namespace gpa
