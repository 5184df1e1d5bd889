// Work lists of the batched launches, expanded on the device from per-entry
// block counts: a workgroup of stage q's launch reads one WorkItem (its
// entry and its block index within that entry's share).
#include "common.h"

namespace gpa {

uint32_t BatchPlan::add(const std::vector<uint32_t> &blocks, const std::vector<uint32_t> *order) {
  if (t.n_stages >= kMaxStages) fail(GPA_E_DEVICE, "too many stages in one batched launch chain");
  if (blocks.size() != t.count || (order && order->size() != t.count))
    fail(GPA_E_DEVICE, "stage with a wrong number of entries");
  const uint32_t q = t.n_stages++;
  t.pre_off[q] = (uint32_t)pre.size();
  uint64_t run = 0;
  pre.push_back(0);
  for (uint32_t k = 0; k < t.count; ++k) {
    const uint32_t e = order ? (*order)[k] : k;
    if (e >= t.count) fail(GPA_E_DEVICE, "stage order out of range");
    run += blocks[e];
    if (run >= (1ull << 31)) fail(GPA_E_UNSUPPORTED, "a batched launch of 2^31 workgroups or more");
    pre.push_back((uint32_t)run);
  }
  t.ord_off[q] = ~0u;
  if (order) {
    t.ord_off[q] = (uint32_t)pre.size();
    pre.insert(pre.end(), order->begin(), order->end());
  }
  t.item_off[q + 1] = t.item_off[q] + run;
  return q;
}

// item i of the concatenated stages: its stage (a short scan of the table),
// then the position p with pre[p] <= i' < pre[p + 1] by bisection (positions
// without blocks have pre[p] == pre[p + 1] and are never chosen), and the
// entry at that position of the stage's order
__global__ void __launch_bounds__(256) k_expand_items(const uint32_t *__restrict__ pre, StageTable t,
                                                      WorkItem *__restrict__ items) {
  const uint64_t total = t.item_off[t.n_stages];
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t q = 0;
    while (i >= t.item_off[q + 1]) ++q;
    const uint32_t li = (uint32_t)(i - t.item_off[q]);
    const uint32_t *P = pre + t.pre_off[q];
    uint32_t lo = 0, hi = t.count;   // P[lo] <= li < P[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (P[mid] <= li) lo = mid;
      else hi = mid;
    }
    const uint32_t e = t.ord_off[q] == ~0u ? lo : pre[t.ord_off[q] + lo];
    items[i] = WorkItem{e, li - P[lo]};
  }
}

void BatchPlan::expand(hipStream_t s) {
  const uint64_t total = total_items();
  if (total == 0) return;
  hipLaunchKernelGGL(k_expand_items, dim3(grid_for(total, 256, 4096)), dim3(256), 0, s, d_pre, t,
                     d_items);
  GPA_LAUNCH_CHECK();
}

void send_plan_beside(Upload &up, size_t i_pre, BatchPlan &plan, Arena &ar, hipStream_t s) {
  const hipStream_t c = side_stream(1);
  ar.add_stream(c);
  up.send(ar, c);
  plan.d_pre = up.ptr<uint32_t>(i_pre);
  plan.d_items = ar.get<WorkItem>(plan.total_items());
  plan.expand(c);
  hipEvent_t e = nullptr;
  GPA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const hipError_t r1 = hipEventRecord(e, c);
  const hipError_t r2 = r1 == hipSuccess ? hipStreamWaitEvent(s, e, 0) : r1;
  (void)hipEventDestroy(e);
  GPA_HIP(r2);
}

}  // namespace gpa
