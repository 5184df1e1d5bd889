// The advice report (Sec. 3: GPA's raw advice is ASCII text; Sec. 7: each
// optimizer lists hotspots, a def and use location with their distance; Sec.
// 6: single dependency coverage before and after pruning).
//
// Single dependency coverage: an instruction is a single-dependency node
// when none of its use sites has two or more sources (each incoming edge is
// then a dependency of its own); before pruning every reaching definition
// counts, after pruning only sources that survive the dominator rule for
// that use and the latency rule for their edge.  The opcode rule depends on
// the stall reason and is not applied here.
//
// Hotspots of an optimizer in one kernel: the edges (def, use) or the
// instructions carrying its matched samples, largest first (ties by def,
// then use), with the same matching as the estimators.  They are gathered
// on the host from the blame handle's tables: a report is made once per
// profile, off the analysis path.
#include <algorithm>
#include <cstring>
#include <string>

#include "common.h"
#include "devutil.h"

namespace gpa {

// one thread per instruction: is it a single-dependency node before and
// after pruning; two integer counts
__global__ void __launch_bounds__(256)
k_coverage(uint32_t n_instr, const uint32_t *__restrict__ use_ptr,
           const uint32_t *__restrict__ rd_ptr, const uint32_t *__restrict__ rd_src,
           const uint8_t *__restrict__ rd_blk, const uint32_t *__restrict__ in_ptr,
           const uint32_t *__restrict__ e_src, const uint8_t *__restrict__ e_flags,
           unsigned long long *__restrict__ out) {
  uint32_t before = 0, after = 0;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_instr;
       j += gridDim.x * blockDim.x) {
    bool sb = true, sa = true;
    for (uint32_t u = use_ptr[j]; u < use_ptr[j + 1]; ++u) {
      const uint32_t a = rd_ptr[u], b = rd_ptr[u + 1];
      if (b - a > 1) sb = false;
      uint32_t kept = 0;
      for (uint32_t q = a; q < b; ++q) {
        if (!rd_blk[q]) continue;
        // the edge (rd_src[q], j): edges into j are sorted by source
        const uint32_t e = lower_bound_u32(e_src, in_ptr[j], in_ptr[j + 1], rd_src[q]);
        if (e < in_ptr[j + 1] && e_src[e] == rd_src[q] && (e_flags[e] & GPA_E_LAT_KEEP)) ++kept;
      }
      if (kept > 1) sa = false;
    }
    before += sb;
    after += sa;
  }
  before = wave_sum(before);
  after = wave_sum(after);
  if (lane_id() == 0) {
    if (before) atomicAdd(&out[0], (unsigned long long)before);
    if (after) atomicAdd(&out[1], (unsigned long long)after);
  }
}

__global__ void k_zero2(unsigned long long *p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

namespace {

template <typename T>
std::vector<T> fetch(const DBuf<T> &d, size_t n) {
  std::vector<T> h(n);
  if (n) GPA_HIP(hipMemcpy(h.data(), d.p, n * sizeof(T), hipMemcpyDeviceToHost));
  return h;
}

// host copies of what the hotspots of a blame handle need
struct HostView {
  const gpa_program *p;
  uint32_t nbl = 0;
  int s_mem = -1, s_exec = -1, s_sync = -1;
  std::vector<uint32_t> counts, e_src, e_dst, e_dmin, e_dmax, e_icl, instr_scope, root_of, roots;
  std::vector<double> share;
  std::vector<uint16_t> nocand;
  std::vector<uint8_t> op_class, tags;

  explicit HostView(const gpa_blame &b) : p(b.prog) {
    const gpa_program &P = *p;
    nbl = P.n_blamable;
    auto slot = [&](int r) {
      return ((P.arch.blamable >> r) & 1) ? __builtin_popcount(P.arch.blamable & ((1u << r) - 1))
                                           : -1;
    };
    s_mem = slot(GPA_ST_MEM_DEP);
    s_exec = slot(GPA_ST_EXEC_DEP);
    s_sync = slot(GPA_ST_SYNC);
    counts = fetch(b.counts, (size_t)P.n_instr * 24);
    share = fetch(b.share, P.n_edges * nbl * 2);
    nocand = fetch(b.nocand, P.n_instr);
    e_src = fetch(P.e_src, P.n_edges);
    e_dst = fetch(P.e_dst, P.n_edges);
    e_dmin = fetch(P.e_dmin, P.n_edges);
    e_dmax = fetch(P.e_dmax, P.n_edges);
    e_icl = fetch(P.e_icl, P.n_edges);
    instr_scope = fetch(P.instr_scope, P.n_instr);
    root_of = fetch(P.root_of, P.n_scopes);
    roots = fetch(P.roots, P.n_roots);
    op_class = fetch(P.op_class, P.n_instr);
    tags = fetch(P.instr_tags, P.n_instr);
  }
  double sh(uint64_t e, int slot, int l) const {
    return slot < 0 ? 0.0 : share[(e * nbl + (uint32_t)slot) * 2 + l];
  }
  uint32_t C(uint32_t j, int r, int l) const { return counts[(size_t)j * 24 + r * 2 + l]; }
  // synchronization samples kept on j: all of them when synchronization is
  // not blamable, else those that found no candidate
  double kept_sync(uint32_t j, int l) const {
    const bool kept = s_sync < 0 || ((nocand[j] >> s_sync) & 1u);
    return kept ? (double)C(j, GPA_ST_SYNC, l) : 0.0;
  }

  std::vector<gpa_hotspot> hotspots(uint32_t root_index, uint32_t opt, uint32_t k) const {
    const uint32_t root = roots[root_index];
    std::vector<gpa_hotspot> all;
    auto in_kernel = [&](uint32_t j) { return root_of[instr_scope[j]] == root; };
    auto add = [&](uint32_t src, uint32_t dst, uint32_t dmin, uint32_t dmax, double v) {
      if (v > 0.0) all.push_back(gpa_hotspot{src, dst, dmin, dmax, v});
    };
    const uint32_t n = p->n_instr;
    for (uint64_t e = 0; e < p->n_edges; ++e) {
      const uint32_t i = e_src[e], j = e_dst[e];
      if (!in_kernel(j)) continue;
      const uint8_t ci = op_class[i];
      double v = 0.0;
      switch (opt) {
        case GPA_O_REGISTER_REUSE:
          if (ci == GPA_OP_LOCAL_LOAD || ci == GPA_OP_LOCAL_STORE) v = sh(e, s_mem, 0) + sh(e, s_mem, 1);
          break;
        case GPA_O_STRENGTH_REDUCTION:
          if (ci == GPA_OP_FP64 || ci == GPA_OP_LONG_ALU) v = sh(e, s_exec, 0) + sh(e, s_exec, 1);
          break;
        case GPA_O_WARP_BALANCE:
          v = sh(e, s_sync, 0) + sh(e, s_sync, 1);
          break;
        case GPA_O_LOOP_UNROLLING:
        case GPA_O_CODE_REORDERING:
          if (opt == GPA_O_LOOP_UNROLLING && e_icl[e] == GPA_NONE) break;
          v = (ci == GPA_OP_GLOBAL_LOAD ? sh(e, s_mem, 1) : 0.0) + sh(e, s_exec, 1);
          break;
        default:
          break;
      }
      add(i, j, e_dmin[e], e_dmax[e], v);
    }
    for (uint32_t j = 0; j < n; ++j) {
      if (!in_kernel(j)) continue;
      const uint8_t cj = op_class[j];
      double v = 0.0;
      switch (opt) {
        case GPA_O_FUNCTION_SPLIT:
          v = (double)C(j, GPA_ST_INST_FETCH, 0) + C(j, GPA_ST_INST_FETCH, 1);
          break;
        case GPA_O_FAST_MATH:
          if (tags[j] & 1)
            for (int r = 1; r < 12; ++r) v += (double)C(j, r, 0) + C(j, r, 1);
          break;
        case GPA_O_WARP_BALANCE:
          v = kept_sync(j, 0) + kept_sync(j, 1);
          break;
        case GPA_O_MEM_TRANSACTION_REDUCTION:
          if (cj == GPA_OP_GLOBAL_LOAD || cj == GPA_OP_GLOBAL_STORE)
            v = (double)C(j, GPA_ST_MEM_THROTTLE, 0) + C(j, GPA_ST_MEM_THROTTLE, 1);
          break;
        case GPA_O_FUNCTION_INLINING:
          if (cj == GPA_OP_CALL || (tags[j] & 2))
            for (int r = 0; r < 12; ++r) v += (double)C(j, r, 1);
          break;
        default:
          break;
      }
      add(GPA_NONE, j, 0, 0, v);
    }
    // largest first; ties by def (instruction items, GPA_NONE, last) then use
    auto before = [](const gpa_hotspot &a, const gpa_hotspot &b) {
      if (a.samples != b.samples) return a.samples > b.samples;
      if (a.src != b.src) return a.src < b.src;
      return a.dst < b.dst;
    };
    const size_t m = std::min<size_t>(k, all.size());
    std::partial_sort(all.begin(), all.begin() + m, all.end(), before);
    all.resize(m);
    return all;
  }
};

const char *kOptNames[GPA_N_OPT] = {"Register Reuse",       "Strength Reduction",
                                    "Function Split",       "Fast Math",
                                    "Warp Balance",         "Memory Transaction Reduction",
                                    "Loop Unrolling",       "Code Reordering",
                                    "Function Inlining"};

}  // namespace

}  // namespace gpa

using namespace gpa;

extern "C" {

gpa_status gpa_program_coverage(const gpa_program *p, uint64_t *single_before,
                                uint64_t *single_after) {
  if (!p) {
    set_error("gpa_program_coverage: NULL program");
    return GPA_E_INVALID;
  }
  try {
    hipStream_t s = nullptr;
    Arena ar(s);
    unsigned long long *d = ar.get<unsigned long long>(2);
    hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_coverage, dim3(grid_for(p->n_instr, 256, 4096)), dim3(256), 0, s,
                       p->n_instr, p->use_ptr.p, p->rd_ptr.p, p->rd_src.p, p->rd_blk.p,
                       p->in_ptr.p, p->e_src.p, p->e_flags.p, d);
    GPA_LAUNCH_CHECK();
    unsigned long long h[2];
    GPA_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s));
    GPA_HIP(hipStreamSynchronize(s));
    if (single_before) *single_before = h[0];
    if (single_after) *single_after = h[1];
    return GPA_OK;
  } catch (const Error &e) {
    return e.code;
  } catch (...) {
    set_error("gpa_program_coverage: unexpected failure");
    return GPA_E_DEVICE;
  }
}

gpa_status gpa_blame_hotspots(const gpa_blame *b, uint32_t root_index, uint32_t opt, uint32_t k,
                              gpa_hotspot *out, uint32_t *n_out) {
  if (!b || !n_out || (k && !out)) {
    set_error("gpa_blame_hotspots: NULL argument");
    return GPA_E_INVALID;
  }
  if (opt >= GPA_N_OPT || root_index >= b->prog->n_roots) {
    set_error("gpa_blame_hotspots: optimizer %u or kernel root %u out of range", opt, root_index);
    return GPA_E_INVALID;
  }
  try {
    const HostView v(*b);
    const std::vector<gpa_hotspot> h = v.hotspots(root_index, opt, k);
    std::copy(h.begin(), h.end(), out);
    *n_out = (uint32_t)h.size();
    return GPA_OK;
  } catch (const Error &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return GPA_E_NOMEM;
  }
}

gpa_status gpa_report(const gpa_advice *a, const gpa_blame *b, uint32_t top_optimizers,
                      uint32_t hotspots, char *buf, size_t *len) {
  if (!a || !b || !len || a->prog != b->prog) {
    set_error("gpa_report: NULL argument, or advice and blame of different programs");
    return GPA_E_INVALID;
  }
  try {
    const gpa_program &P = *a->prog;
    const HostView v(*b);
    const std::vector<double> sp = fetch(a->speedup, (size_t)P.n_scopes * GPA_N_OPT);
    const std::vector<double> kT = fetch(a->kernel_T, P.n_scopes);
    const std::vector<double> kL = fetch(a->kernel_L, P.n_scopes);
    uint64_t cb = 0, ca = 0;
    gpa_status st = gpa_program_coverage(&P, &cb, &ca);
    if (st != GPA_OK) return st;
    std::string out;
    char line[512];
    snprintf(line, sizeof line,
             "GPA advice: %u kernels, %u instructions, %llu dependency edges\n"
             "single dependency coverage: %.3f before pruning, %.3f after\n",
             P.n_roots, P.n_instr, (unsigned long long)P.n_edges,
             P.n_instr ? (double)cb / P.n_instr : 0.0, P.n_instr ? (double)ca / P.n_instr : 0.0);
    out += line;
    for (uint32_t ri = 0; ri < P.n_roots; ++ri) {
      const uint32_t r = v.roots[ri];
      snprintf(line, sizeof line, "\nkernel (scope %u): %.0f samples, %.0f latency samples\n", r,
               kT[r], kL[r]);
      out += line;
      // the optimizers ranked by their speedup at the kernel
      uint32_t order[GPA_N_OPT];
      for (uint32_t o = 0; o < GPA_N_OPT; ++o) order[o] = o;
      std::stable_sort(order, order + GPA_N_OPT, [&](uint32_t x, uint32_t y) {
        return sp[(size_t)r * GPA_N_OPT + x] > sp[(size_t)r * GPA_N_OPT + y];
      });
      for (uint32_t t = 0; t < std::min<uint32_t>(top_optimizers, GPA_N_OPT); ++t) {
        const uint32_t o = order[t];
        const double s = sp[(size_t)r * GPA_N_OPT + o];
        if (!(s > 1.0)) break;
        snprintf(line, sizeof line, "  %u. %s: estimated speedup %.4fx\n", t + 1, kOptNames[o], s);
        out += line;
        for (const gpa_hotspot &h : v.hotspots(ri, o, hotspots)) {
          if (h.src == GPA_NONE)
            snprintf(line, sizeof line, "       at instruction %u: %.1f samples\n", h.dst,
                     h.samples);
          else
            snprintf(line, sizeof line,
                     "       def %u -> use %u, distance %u..%u instructions: %.1f samples\n",
                     h.src, h.dst, h.dmin, h.dmax, h.samples);
          out += line;
        }
      }
    }
    const size_t need = out.size() + 1;
    if (buf && *len >= need) memcpy(buf, out.c_str(), need);
    *len = need;
    return GPA_OK;
  } catch (const Error &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return GPA_E_NOMEM;
  }
}

}  // extern "C"
