// The parallel optimizers of Table 2 (Block Increase, Thread Increase) and
// their estimate, Sec. 5.2 Eqs. (6)-(10): active warps per warp scheduler W
// before and after the change, the schedulers' issue probability
// I = 1 - (1 - R_I)^W with R_I the kernel's ratio of issued samples, and
// S = (1 / C_W) * C_I * f with C_W = W_new / W and C_I = I_new / I.
//
// Readings taken where the paper leaves the model open:
//   occupancy   resident blocks per SM = the smallest of the block cap, the
//               warp cap, the register file and the shared memory over one
//               block's needs, and of the blocks the grid gives each SM;
//               W = resident blocks x warps per block / schedulers per SM;
//   Block Increase (matched when blocks < SMs): the kernel's threads are
//               spread over one block per SM, W_new = W x blocks / SMs (each
//               scheduler's share of the work shrinks the same way); f = 1,
//               or, once W_new < 1 (fewer warps on an SM than schedulers),
//               T / (T - pipeline-busy - throttle - not-selected samples):
//               those contention stalls are taken to vanish;
//   Thread Increase (matched when the block cap is the smallest limit and
//               leaves warp slots free): threads per block grow until the
//               warps, registers or shared memory limit residency (and no
//               further than the grid's warps per SM); the kernel's warps
//               are the same, so each scheduler's work is too: f = C_W and
//               S = C_I.
// The kernel's sample sums come from the blame handle's counts on the
// device; everything after that is a handful of scalars on the host.
#include <cmath>

#include "common.h"
#include "devutil.h"

namespace gpa {

// per stall reason, the samples of the instructions under kernel root `root`
__global__ void __launch_bounds__(256)
k_root_reason_sums(uint32_t n_instr, uint32_t root, const uint32_t *__restrict__ instr_scope,
                   const uint32_t *__restrict__ root_of, const uint32_t *__restrict__ counts,
                   unsigned long long *__restrict__ sums) {
  unsigned long long v[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) v[r] = 0;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_instr;
       j += gridDim.x * blockDim.x) {
    if (root_of[instr_scope[j]] != root) continue;
    const uint32_t *C = counts + (size_t)j * 24;
#pragma unroll
    for (int r = 0; r < 12; ++r) v[r] += (unsigned long long)C[2 * r] + C[2 * r + 1];
  }
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    const unsigned long long w = wave_sum(v[r]);
    if (lane_id() == 0 && w) atomicAdd(&sums[r], w);
  }
}

__global__ void k_zero_u64(unsigned long long *p, uint32_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

namespace {

struct Occupancy {
  double W;            // active warps per scheduler
  uint32_t warps_per_block, resident_blocks, limit_blocks, limit_warps, limit_regs, limit_shared;
};

uint32_t div_or_max(uint64_t a, uint64_t b) {
  return b ? (uint32_t)std::min<uint64_t>(a / b, 0xFFFFFFFFu) : 0xFFFFFFFFu;
}

Occupancy occupancy(const gpa_launch &L, const gpa_device &D, uint32_t threads) {
  Occupancy o;
  o.warps_per_block = (threads + D.warp_size - 1) / D.warp_size;
  o.limit_blocks = D.max_blocks_per_sm;
  o.limit_warps = div_or_max(D.max_warps_per_sm, o.warps_per_block);
  o.limit_regs = L.regs_per_thread
                     ? div_or_max(D.regs_per_sm, (uint64_t)L.regs_per_thread * D.warp_size *
                                                     o.warps_per_block)
                     : 0xFFFFFFFFu;
  o.limit_shared = L.shared_per_block ? div_or_max(D.shared_per_sm, L.shared_per_block)
                                      : 0xFFFFFFFFu;
  const uint32_t per_sm = std::min(std::min(o.limit_blocks, o.limit_warps),
                                   std::min(o.limit_regs, o.limit_shared));
  const uint32_t grid_per_sm = (uint32_t)(((uint64_t)L.blocks + D.n_sm - 1) / D.n_sm);
  o.resident_blocks = std::min(per_sm, grid_per_sm);
  o.W = (double)o.resident_blocks * o.warps_per_block / D.schedulers_per_sm;
  return o;
}

double issue_prob(double R_I, double W) { return 1.0 - std::pow(1.0 - R_I, W); }

void finish(gpa_parallel_estimate &e, double T) {
  e.I = issue_prob(e.R_I, e.W);
  e.I_new = issue_prob(e.R_I, e.W_new);
  e.C_W = e.W > 0.0 ? e.W_new / e.W : 1.0;
  e.C_I = e.I > 0.0 ? e.I_new / e.I : 1.0;
  e.speedup = (e.matched && T > 0.0 && e.I > 0.0 && e.C_W > 0.0) ? e.C_I / e.C_W * e.f : 1.0;
}

}  // namespace

}  // namespace gpa

using namespace gpa;

extern "C" gpa_status gpa_parallel_advise(const gpa_blame *b, uint32_t root_index,
                                          const gpa_launch *launch, const gpa_device *device,
                                          gpa_parallel_estimate *out) {
  if (!b || !launch || !device || !out) {
    set_error("gpa_parallel_advise: NULL argument");
    return GPA_E_INVALID;
  }
  const gpa_program &p = *b->prog;
  if (root_index >= p.n_roots) {
    set_error("gpa_parallel_advise: kernel root %u of %u", root_index, p.n_roots);
    return GPA_E_INVALID;
  }
  const gpa_device &D = *device;
  const gpa_launch &L = *launch;
  if (!D.n_sm || !D.schedulers_per_sm || !D.warp_size || !D.max_warps_per_sm ||
      !D.max_blocks_per_sm || !D.max_threads_per_block || !L.blocks || !L.threads_per_block ||
      L.threads_per_block > D.max_threads_per_block) {
    set_error("gpa_parallel_advise: zero device or launch field, or a block larger than the "
              "device allows");
    return GPA_E_INVALID;
  }
  return [&]() -> gpa_status {
    try {
      hipStream_t s = nullptr;
      Arena ar(s);
      uint32_t root = 0;
      GPA_HIP(hipMemcpyAsync(&root, p.roots.p + root_index, 4, hipMemcpyDeviceToHost, s));
      GPA_HIP(hipStreamSynchronize(s));
      unsigned long long *d = ar.get<unsigned long long>(12);
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, d, 12u);
      hipLaunchKernelGGL(k_root_reason_sums, dim3(grid_for(p.n_instr, 256, 2048)), dim3(256), 0, s,
                         p.n_instr, root, p.instr_scope.p, p.root_of.p, b->counts.p, d);
      GPA_LAUNCH_CHECK();
      unsigned long long sums[12];
      GPA_HIP(hipMemcpyAsync(sums, d, sizeof(sums), hipMemcpyDeviceToHost, s));
      GPA_HIP(hipStreamSynchronize(s));
      double T = 0.0;
      for (int r = 0; r < 12; ++r) T += (double)sums[r];
      const double issued = (double)sums[GPA_ST_SELECTED];
      const double contention = (double)sums[GPA_ST_PIPE_BUSY] +
                                (double)sums[GPA_ST_MEM_THROTTLE] +
                                (double)sums[GPA_ST_NOT_SELECTED];
      const double R_I = T > 0.0 ? issued / T : 0.0;
      const Occupancy o = occupancy(L, D, L.threads_per_block);
      // Block Increase
      gpa_parallel_estimate bi{};
      bi.R_I = R_I;
      bi.W = o.W;
      bi.matched = L.blocks < D.n_sm;
      bi.W_new = bi.matched ? o.W * (double)L.blocks / D.n_sm : o.W;
      bi.f = (bi.matched && bi.W_new < 1.0 && T > contention) ? T / (T - contention) : 1.0;
      finish(bi, T);
      // Thread Increase
      gpa_parallel_estimate ti{};
      ti.R_I = R_I;
      ti.W = o.W;
      const uint32_t others = std::min(o.limit_warps, std::min(o.limit_regs, o.limit_shared));
      const uint64_t warps_now = (uint64_t)o.resident_blocks * o.warps_per_block;
      ti.matched = o.limit_blocks < others && o.resident_blocks == o.limit_blocks &&
                   warps_now < D.max_warps_per_sm;
      if (ti.matched) {
        // warps an SM could hold with larger blocks: the warp cap, the
        // register file and the shared memory (per warp), and the grid's
        // warps per SM
        uint64_t cap = D.max_warps_per_sm;
        if (L.regs_per_thread)
          cap = std::min<uint64_t>(cap, D.regs_per_sm / ((uint64_t)L.regs_per_thread * D.warp_size));
        if (L.shared_per_block)
          cap = std::min<uint64_t>(cap, (uint64_t)D.shared_per_sm * o.warps_per_block /
                                            L.shared_per_block);
        const uint64_t grid_warps =
            ((uint64_t)L.blocks * o.warps_per_block + D.n_sm - 1) / D.n_sm;
        cap = std::min(cap, grid_warps);
        ti.W_new = std::max((double)warps_now, (double)cap) / D.schedulers_per_sm;
      } else {
        ti.W_new = o.W;
      }
      ti.f = ti.W > 0.0 ? ti.W_new / ti.W : 1.0;
      finish(ti, T);
      out[0] = bi;
      out[1] = ti;
      return GPA_OK;
    } catch (const Error &e) {
      return e.code;
    } catch (...) {
      set_error("gpa_parallel_advise: unexpected failure");
      return GPA_E_DEVICE;
    }
  }();
}
