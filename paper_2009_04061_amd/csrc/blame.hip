// The instruction blamer's attribution step (Sec. 4, "Attribute stalls").
//
// For a sampled instruction j, a blamable reason r and a latency bit l with
// S = C[j][r][l] > 0, the candidates are j's incoming edges that survived
// dominator and latency pruning and whose source opcode class may cause r
// (opcode pruning).  Eq. (1) splits S over them with weights
//   R_issue(i) * R_path(i)  ~  issued(i) / (dmax(i, j) + 1)
// (more issued samples, more blame; longer longest path, less blame); when
// no candidate issued anything the path term alone decides.  Without a
// candidate the samples stay on j, as do all samples of other reasons; the
// rule applies the same way to latency samples.
//
// k_blame_dst takes the destinations by wave tiles, each lane owning one
// destination's sums, and writes every edge's shares (and its estimator
// contribution); k_blame_src owns one source per thread and sums its
// outgoing shares in edge order.  Every FP64 sum has a fixed order and no
// floating-point atomics are used.
//
// The per-instruction results are kept compact on the device: the blamed
// samples of the blamable reasons only (bl, [n_instr][n_blamable][2]), one
// bit per blamable reason telling whether its samples stayed on the
// instruction for want of a candidate (nocand), and the execution-dependency
// split into WAR and other sources plus the samples of blamable reasons
// outside the memory / execution / synchronization classes (fx, 6 per
// instruction).  Everything else of the full tables follows from these and
// the counts; k_blame_expand writes the full tables when they are asked for.
#include <algorithm>

#include "common.h"
#include "devutil.h"

namespace gpa {

// One profile's blame: its program's edges and classes, its counts and its
// output tables.  A launch for one profile takes it by value; a batched
// launch reads it from a device table per workgroup (a work item names the
// profile and a tile of kBlameThreads instructions).
struct BlameArgs {
  uint32_t n_instr, nbl, blamable;
  uint16_t allowed[12];
  const uint32_t *counts, *issued, *in_ptr, *e_src, *e_dst, *e_dmax, *out_ptr, *out_perm;
  const uint8_t *e_flags, *e_cls;
  double *share, *ec, *bl, *fx;   // ec may be null
  uint16_t *nocand;
};
constexpr int kBlameThreads = 128;

// the instructions a thread takes: one per tile in a batched launch, a
// grid-stride range otherwise
#define BLAME_ITEM(VAR)                                                          \
  const BlameArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;              \
  const uint32_t first_ = (BATCH ? items[blockIdx.x].local : blockIdx.x) * blockDim.x + threadIdx.x; \
  const uint32_t stride_ = BATCH ? a.n_instr : gridDim.x * blockDim.x;           \
  for (uint32_t VAR = first_; VAR < a.n_instr; VAR += stride_)

// One wave per tile of TW <= 64 consecutive destinations; lane l < TW owns
// destination j = d0 + l (narrow tiles give one profile more waves).  The
// tile's in-edges (contiguous: edges are sorted by
// destination) are read 64 at a time by all lanes, coalesced, each lane one
// edge with its source's issued samples.
//   Pass 1: every owner takes the weights of its own edges in the chunk from
//   the lanes holding them (cross-lane reads), in edge order, and sums, per
//   blamable reason, the issued-based and the path-only weights of the
//   candidates (as Eq. (1) is written; the same additions in the same order
//   as a loop over j's edges).
//   Pass 2: each lane takes one edge again, its owner's sums and counts from
//   the owner lane, and writes the edge's share slots (consecutive lanes,
//   consecutive edges).
// Reasons are unrolled, so the per-reason sums stay in registers.
constexpr uint32_t kTileWaves = 4;   // tiles (waves) per workgroup
// destinations per wave tile on the one-profile path and in a batch
constexpr uint32_t kDstTileOne = 16;
constexpr uint32_t kDstTileBatch = 32;

struct EdgeW {
  double wi, wp;    // issued / length, 1 / length
  uint32_t cls;     // the source's opcode class
  bool kept;        // survives dominator and latency pruning
};

// edge e of the range [e0, e1) (an edge past the range reads edge e0 and
// is not kept)
__device__ __forceinline__ EdgeW blame_edge(const BlameArgs &a, uint32_t e0, uint32_t e1,
                                            uint32_t e) {
  const bool in = e < e1;
  const uint32_t x = in ? e : e0;
  const uint8_t fl = a.e_flags[x];
  EdgeW w;
  w.kept = in && (fl & GPA_E_DOM_KEEP) && (fl & GPA_E_LAT_KEEP);
  w.cls = a.e_cls[x];
  const uint32_t i = a.e_src[x];
  const double len = (double)a.e_dmax[x] + 1.0;
  const double issued = (double)a.issued[i];
  w.wi = issued / len;
  w.wp = 1.0 / len;
  return w;
}

// NB: blamable reasons the kernel keeps sums for (the arch's blamable set
// has at most NB reasons; slot s is the s-th blamable reason ascending);
// TW: destinations per wave tile (at most kWave; the owners are lanes
// [0, TW), every lane takes edges)
template <bool BATCH, int NB, uint32_t TW>
__global__ void __launch_bounds__(kWave * kTileWaves)
k_blame_dst(BlameArgs one, const BlameArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  static_assert(TW >= 1 && TW <= kWave, "tile width");
  const BlameArgs &a = BATCH ? many[items[blockIdx.x].entry] : one;
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t n = a.n_instr, nbl = a.nbl;
  const uint32_t n_tiles = (n + TW - 1) / TW;
  // a batched workgroup takes its kTileWaves tiles once; otherwise a grid
  // stride over the tiles
  const uint32_t t0 = (BATCH ? items[blockIdx.x].local : blockIdx.x) * kTileWaves +
                      threadIdx.x / kWave;
  const uint32_t t_step = BATCH ? n_tiles : gridDim.x * kTileWaves;
  // the blamable reasons by slot, and the opcode classes each allows (slot
  // q takes the lowest blamable reason left, so every slot has a fixed
  // register; slots past the set read reason 0 and allow nothing)
  uint32_t rs[NB], allow[NB];
  {
    uint32_t m = a.blamable & 0xFFFu;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const uint32_t r = m ? (uint32_t)__builtin_ctz(m) : 0u;
      rs[q] = r;
      allow[q] = m ? a.allowed[r] : 0u;
      m &= m - 1u;
    }
  }
  for (uint32_t t = t0; t < n_tiles; t += t_step) {
    const uint32_t d0 = t * TW, j = d0 + lane;
    const bool own = lane < TW && j < n;
    const uint32_t e0 = own ? a.in_ptr[j] : 0u, e1 = own ? a.in_ptr[j + 1] : 0u;
    const uint32_t E0 = a.in_ptr[d0], E1 = a.in_ptr[min(d0 + TW, n)];
    double Wi[NB], Wp[NB];
    bool any[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      Wi[q] = 0.0;
      Wp[q] = 0.0;
      any[q] = false;
    }
    // pass 1
    for (uint32_t base = E0; base < E1; base += kWave) {
      const EdgeW w = blame_edge(a, E0, E1, base + lane);
      const uint32_t packed = (w.kept ? 1u : 0u) | (w.cls << 1);
      const uint32_t lo = max(e0, base), hi = min(e1, base + kWave);
      const uint32_t cnt = hi > lo ? hi - lo : 0u;
      const uint32_t rounds = wave_max_u32(cnt);
      for (uint32_t k = 0; k < rounds; ++k) {
        const int from = (int)(k < cnt ? lo - base + k : lane);
        const double wi = __shfl(w.wi, from, kWave), wp = __shfl(w.wp, from, kWave);
        const uint32_t pk = (uint32_t)__shfl((int)packed, from, kWave);
        if (k < cnt) {
          const bool kept = (pk & 1u) != 0;
          const uint32_t cls = pk >> 1;
#pragma unroll
          for (int q = 0; q < NB; ++q) {
            const bool cand = kept && ((allow[q] >> cls) & 1u);
            Wi[q] = cand ? Wi[q] + wi : Wi[q];
            Wp[q] = cand ? Wp[q] + wp : Wp[q];
            any[q] = any[q] || cand;
          }
        }
      }
    }
    // the owner's samples of the blamable reasons
    uint32_t S[NB][2];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int l = 0; l < 2; ++l)
        S[q][l] = (own && (uint32_t)q < nbl) ? a.counts[(size_t)j * 24 + rs[q] * 2 + l] : 0u;
    // pass 2
    for (uint32_t base = E0; base < E1; base += kWave) {
      const uint32_t e = base + lane;
      const bool in = e < E1;
      const EdgeW w = blame_edge(a, E0, E1, e);
      const int o = (int)(in ? a.e_dst[e] - d0 : lane);   // the owner lane
      double *sh = a.share + (size_t)(in ? e : 0u) * 2 * nbl;
      // the edge's estimator contribution: its latency samples of an
      // execution dependency and, from a global load, of a memory dependency
      double ecv = 0.0;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const double wiq = __shfl(Wi[q], o, kWave), wpq = __shfl(Wp[q], o, kWave);
        const uint32_t s0 = (uint32_t)__shfl((int)S[q][0], o, kWave);
        const uint32_t s1 = (uint32_t)__shfl((int)S[q][1], o, kWave);
        if (in && (uint32_t)q < nbl) {
          const bool cand = w.kept && ((allow[q] >> w.cls) & 1u);
          const bool by_path = (wiq == 0.0);
          const double wt = by_path ? w.wp : w.wi;
          const double W = by_path ? wpq : wiq;
          sh[q * 2] = (cand && s0 != 0) ? (double)s0 * wt / W : 0.0;
          const double v1 = (cand && s1 != 0) ? (double)s1 * wt / W : 0.0;
          sh[q * 2 + 1] = v1;
          if (rs[q] == GPA_ST_EXEC_DEP || (rs[q] == GPA_ST_MEM_DEP && w.cls == GPA_OP_GLOBAL_LOAD))
            ecv += v1;
        }
      }
      if (in && a.ec) a.ec[e] = ecv;
    }
    if (own) {
      uint32_t mask = 0;
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if ((uint32_t)q < nbl && !any[q]) mask |= 1u << q;
      a.nocand[j] = (uint16_t)mask;
    }
  }
}

// One thread per source i: sums its outgoing shares in edge order, per
// blamable reason, and the execution-dependency shares split by the WAR flag
// of the edge (the fine classes of a memory dependency and of a non-WAR
// execution dependency follow from i's opcode class alone).  The edges are
// read two at a time (their loads issued together) and summed in order.
constexpr uint32_t kBlameSrcU = 2;

template <bool BATCH, int NB>
__global__ void __launch_bounds__(kBlameThreads)
k_blame_src(BlameArgs one, const BlameArgs *__restrict__ many, const WorkItem *__restrict__ items) {
  BLAME_ITEM(i) {
    const uint32_t nbl = a.nbl;
    const uint32_t *__restrict__ out_perm = a.out_perm;
    const uint8_t *__restrict__ e_flags = a.e_flags;
    const double *__restrict__ share = a.share;
    uint32_t rs[NB];   // the blamable reasons by slot (12 past the set)
    {
      uint32_t m = a.blamable & 0xFFFu;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        rs[q] = m ? (uint32_t)__builtin_ctz(m) : 12u;
        m &= m - 1u;
      }
    }
    double acc[2 * NB];
#pragma unroll
    for (int q = 0; q < 2 * NB; ++q) acc[q] = 0.0;
    double war0 = 0.0, war1 = 0.0, nwar0 = 0.0, nwar1 = 0.0, oth0 = 0.0, oth1 = 0.0;
    const uint32_t k0 = a.out_ptr[i], k1 = a.out_ptr[i + 1];
    for (uint32_t k = k0; k < k1; k += kBlameSrcU) {
      double sv[kBlameSrcU][2 * NB];
      bool war[kBlameSrcU], in[kBlameSrcU];
#pragma unroll
      for (uint32_t u = 0; u < kBlameSrcU; ++u) {
        in[u] = k + u < k1;
        const uint32_t e = out_perm[in[u] ? k + u : k0];
        war[u] = (e_flags[e] & GPA_E_WAR) != 0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const bool live = (uint32_t)q < nbl;
          sv[u][2 * q] = live ? share[((size_t)e * nbl + q) * 2] : 0.0;
          sv[u][2 * q + 1] = live ? share[((size_t)e * nbl + q) * 2 + 1] : 0.0;
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < kBlameSrcU; ++u) {
        if (!in[u]) continue;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if ((uint32_t)q >= nbl) continue;
          const double s0 = sv[u][2 * q], s1 = sv[u][2 * q + 1];
          acc[2 * q] += s0;
          acc[2 * q + 1] += s1;
          if (rs[q] == GPA_ST_EXEC_DEP) {
            if (war[u]) {
              war0 += s0;
              war1 += s1;
            } else {
              nwar0 += s0;
              nwar1 += s1;
            }
          } else if (rs[q] != GPA_ST_MEM_DEP && rs[q] != GPA_ST_SYNC) {
            oth0 += s0;
            oth1 += s1;
          }
        }
      }
    }
    double *bl = a.bl + (size_t)i * nbl * 2;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if ((uint32_t)q >= nbl) continue;
      bl[q * 2] = acc[2 * q];
      bl[q * 2 + 1] = acc[2 * q + 1];
    }
    double *fx = a.fx + (size_t)i * kBlameFx;
    fx[0] = war0;
    fx[1] = war1;
    fx[2] = nwar0;
    fx[3] = nwar1;
    fx[4] = oth0;
    fx[5] = oth1;
  }
}

// The full per-instruction tables of the C-ABI from the compact ones, one
// thread per instruction:
//   blamed[j][r][l] = bl[j][slot(r)][l] for a blamable r, else 0;
//   self_[j][r][l]  = C[j][r][l] for a reason that is not blamable or whose
//                     samples found no candidate, else 0;
//   fine[j]         = the memory dependency blamed on j in the class of j's
//                     opcode (local, constant, global), the execution
//                     dependency split into WAR and the rest (shared-memory
//                     or arithmetic by j's opcode), synchronization, and the
//                     other blamable reasons.
__global__ void __launch_bounds__(256)
k_blame_expand(uint32_t n_instr, uint32_t nbl, uint32_t blamable, const uint32_t *__restrict__ counts,
               const uint8_t *__restrict__ op_class, const double *__restrict__ bl_all,
               const double *__restrict__ fx_all, const uint16_t *__restrict__ nocand,
               double *__restrict__ blamed, double *__restrict__ self_, double *__restrict__ fine) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_instr;
       j += gridDim.x * blockDim.x) {
    const uint32_t *C = counts + (size_t)j * 24;
    const double *bl = bl_all + (size_t)j * nbl * 2;
    const double *fx = fx_all + (size_t)j * kBlameFx;
    const uint32_t nc = nocand[j];
    double mem0 = 0.0, mem1 = 0.0, sync0 = 0.0, sync1 = 0.0;
    uint32_t slot = 0;
    for (uint32_t r = 0; r < 12; ++r) {
      const bool blam = (blamable >> r) & 1u;
      double b0 = 0.0, b1 = 0.0;
      bool kept = true;
      if (blam) {
        b0 = bl[slot * 2];
        b1 = bl[slot * 2 + 1];
        kept = (nc >> slot) & 1u;
        ++slot;
      }
      if (r == GPA_ST_MEM_DEP) {
        mem0 = b0;
        mem1 = b1;
      } else if (r == GPA_ST_SYNC) {
        sync0 = b0;
        sync1 = b1;
      }
      if (blamed) {
        blamed[(size_t)j * 24 + r * 2] = b0;
        blamed[(size_t)j * 24 + r * 2 + 1] = b1;
      }
      if (self_) {
        self_[(size_t)j * 24 + r * 2] = kept ? (double)C[r * 2] : 0.0;
        self_[(size_t)j * 24 + r * 2 + 1] = kept ? (double)C[r * 2 + 1] : 0.0;
      }
    }
    if (!fine) continue;
    const uint32_t cls = op_class[j];
    const uint32_t fm = (cls == GPA_OP_LOCAL_LOAD || cls == GPA_OP_LOCAL_STORE) ? GPA_F_MEM_LOCAL
                        : (cls == GPA_OP_CONST_LOAD)                           ? GPA_F_MEM_CONST
                                                                               : GPA_F_MEM_GLOBAL;
    const uint32_t fe = (cls == GPA_OP_SHARED_LOAD) ? GPA_F_EXEC_SHARED : GPA_F_EXEC_ARITH;
    double *dst = fine + (size_t)j * GPA_N_FINE * 2;
    for (int q = 0; q < GPA_N_FINE * 2; ++q) dst[q] = 0.0;
    dst[fm * 2] = mem0;
    dst[fm * 2 + 1] = mem1;
    dst[GPA_F_EXEC_WAR * 2] = fx[0];
    dst[GPA_F_EXEC_WAR * 2 + 1] = fx[1];
    dst[fe * 2] = fx[2];
    dst[fe * 2 + 1] = fx[3];
    dst[GPA_F_SYNC * 2] = sync0;
    dst[GPA_F_SYNC * 2 + 1] = sync1;
    dst[GPA_F_OTHER * 2] = fx[4];
    dst[GPA_F_OTHER * 2 + 1] = fx[5];
  }
}

void run_blame(const gpa_program &p, gpa_blame &b, hipStream_t s, Arena &ar) {
  (void)ar;
  const uint32_t n = p.n_instr;
  b.share.alloc(p.n_edges * p.n_blamable * 2);
  b.ec.alloc(p.n_edges);
  b.bl.alloc((size_t)n * p.n_blamable * 2);
  b.fx.alloc((size_t)n * kBlameFx);
  b.nocand.alloc(n);
  launch_blame(p, b.counts.p, b.issued.p, b.share.p, b.ec.p, b.bl.p, b.fx.p, b.nocand.p, s);
}

static BlameArgs blame_args(const gpa_program &p, const uint32_t *counts, const uint32_t *issued,
                            double *share, double *ec, double *bl, double *fx,
                            uint16_t *nocand) {
  BlameArgs a;
  a.n_instr = p.n_instr;
  a.nbl = p.n_blamable;
  a.blamable = p.arch.blamable;
  for (int r = 0; r < 12; ++r) a.allowed[r] = p.arch.allowed[r];
  a.counts = counts;
  a.issued = issued;
  a.in_ptr = p.in_ptr.p;
  a.e_src = p.e_src.p;
  a.e_dst = p.e_dst.p;
  a.e_dmax = p.e_dmax.p;
  a.out_ptr = p.out_ptr;
  a.out_perm = p.out_perm;
  a.e_flags = p.e_flags.p;
  a.e_cls = p.e_cls.p;
  a.share = share;
  a.ec = ec;
  a.bl = bl;
  a.fx = fx;
  a.nocand = nocand;
  return a;
}

void launch_blame(const gpa_program &p, const uint32_t *counts, const uint32_t *issued,
                  double *share, double *ec, double *bl, double *fx, uint16_t *nocand,
                  hipStream_t s) {
  const BlameArgs a = blame_args(p, counts, issued, share, ec, bl, fx, nocand);
  const unsigned g = grid_for(p.n_instr, kBlameThreads, 8192);
  const unsigned gd = grid_for((p.n_instr + kDstTileOne - 1) / kDstTileOne, kTileWaves, 8192);
  const dim3 bd(kWave * kTileWaves);
  if (p.n_blamable <= 4)
    hipLaunchKernelGGL((k_blame_dst<false, 4, kDstTileOne>), dim3(gd), bd, 0, s, a, nullptr,
                       nullptr);
  else
    hipLaunchKernelGGL((k_blame_dst<false, 12, kDstTileOne>), dim3(gd), bd, 0, s, a, nullptr,
                       nullptr);
  GPA_LAUNCH_CHECK();
  if (p.n_blamable <= 4)
    hipLaunchKernelGGL((k_blame_src<false, 4>), dim3(g), dim3(kBlameThreads), 0, s, a, nullptr,
                       nullptr);
  else
    hipLaunchKernelGGL((k_blame_src<false, 12>), dim3(g), dim3(kBlameThreads), 0, s, a, nullptr,
                       nullptr);
  GPA_LAUNCH_CHECK();
}

void expand_blame_tables(const gpa_program &p, const uint32_t *counts, const double *bl,
                         const double *fx, const uint16_t *nocand, double *blamed, double *self_,
                         double *fine, hipStream_t s) {
  if (p.n_instr == 0) return;
  hipLaunchKernelGGL(k_blame_expand, dim3(grid_for(p.n_instr, 256, 8192)), dim3(256), 0, s,
                     p.n_instr, p.n_blamable, (uint32_t)p.arch.blamable, counts, p.op_class.p, bl,
                     fx, nocand, blamed, self_, fine);
  GPA_LAUNCH_CHECK();
}

void run_blame_batch(const gpa_program *const *progs, gpa_blame *const *b, uint32_t count,
                     hipStream_t s, Arena &ar, SharedBlocks &sh, PhaseTimer *t) {
  std::vector<BlameArgs> args(count);
  std::vector<uint32_t> tiles(count), dst_groups(count);
  for (uint32_t k = 0; k < count; ++k) {
    const gpa_program &p = *progs[k];
    const uint32_t n = p.n_instr;
    sh.carve(b[k]->share, p.n_edges * p.n_blamable * 2);
    sh.carve(b[k]->ec, p.n_edges);
    sh.carve(b[k]->bl, (size_t)n * p.n_blamable * 2);
    sh.carve(b[k]->fx, (size_t)n * kBlameFx);
    sh.carve(b[k]->nocand, n);
    args[k] = blame_args(p, b[k]->counts.p, b[k]->issued.p, b[k]->share.p, b[k]->ec.p, b[k]->bl.p,
                         b[k]->fx.p, b[k]->nocand.p);
    tiles[k] = (n + kBlameThreads - 1) / kBlameThreads;
    dst_groups[k] = ((n + kDstTileBatch - 1) / kDstTileBatch + kTileWaves - 1) / kTileWaves;
  }
  BatchPlan plan(count);
  const uint32_t q = plan.add(tiles), qd = plan.add(dst_groups);
  if (plan.blocks(q) == 0) return;
  Upload up;
  const size_t i_args = up.add(args), i_pre = up.add(plan.pre);
  send_plan_beside(up, i_pre, plan, ar, s);
  const BlameArgs *d_args = up.ptr<BlameArgs>(i_args);
  BlameArgs none{};
  const unsigned g = plan.blocks(q);
  if (t) t->begin(kPhaseBlame, s);
  uint32_t max_nbl = 0;
  for (uint32_t k = 0; k < count; ++k) max_nbl = std::max(max_nbl, progs[k]->n_blamable);
  const unsigned gd = plan.blocks(qd);
  const dim3 bd(kWave * kTileWaves);
  if (max_nbl <= 4)
    hipLaunchKernelGGL((k_blame_dst<true, 4, kDstTileBatch>), dim3(gd), bd, 0, s, none, d_args,
                       plan.items(qd));
  else
    hipLaunchKernelGGL((k_blame_dst<true, 12, kDstTileBatch>), dim3(gd), bd, 0, s, none, d_args,
                       plan.items(qd));
  GPA_LAUNCH_CHECK();
  if (max_nbl <= 4)
    hipLaunchKernelGGL((k_blame_src<true, 4>), dim3(g), dim3(kBlameThreads), 0, s, none, d_args,
                       plan.items(q));
  else
    hipLaunchKernelGGL((k_blame_src<true, 12>), dim3(g), dim3(kBlameThreads), 0, s, none, d_args,
                       plan.items(q));
  GPA_LAUNCH_CHECK();
  if (t) t->end(s);
}

}  // namespace gpa
