// The C-ABI entry points of libgpa (declared in include/gpa.h): argument
// checks, descriptor upload, the order of the device steps, copy-out.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>

#include "common.h"

namespace gpa {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[2048];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

void fail(gpa_status code, const char *fmt, ...) {
  char buf[2048];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  throw Error{code};
}

// ------------------------------------------------------------------ pool
// Per device: free lists by size class, and the bytes handed out and held
// in the free lists.  A block is returned to the free list of the device it
// was allocated on.
namespace {
std::mutex g_mu;
struct DevPool {
  std::map<size_t, std::vector<void *>> free;   // size class -> cached blocks
  uint64_t in_use = 0, cached = 0;
};
std::map<int, DevPool> g_pools;
struct BlockInfo {
  int dev;
  size_t cls;
};
std::unordered_map<void *, BlockInfo> g_blocks;

size_t size_class(size_t b) {
  if (b <= 4096) return 4096;
  if (b <= (size_t)1 << 24) {
    size_t r = 4096;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t mb = (size_t)1 << 20;
  return (b + mb - 1) / mb * mb;
}

// frees the cached blocks of one device (that device must be current)
void release_cached_locked(int dev) {
  DevPool &P = g_pools[dev];
  for (auto &kv : P.free)
    for (void *p : kv.second) {
      (void)hipFree(p);
      g_blocks.erase(p);
    }
  P.free.clear();
  P.cached = 0;
}
}  // namespace

void *dev_alloc(size_t bytes) {
  const size_t c = size_class(bytes);
  int dev = 0;
  GPA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  DevPool &P = g_pools[dev];
  auto it = P.free.find(c);
  if (it != P.free.end() && !it->second.empty()) {
    void *p = it->second.back();
    it->second.pop_back();
    P.cached -= c;
    P.in_use += c;
    return p;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, c);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_cached_locked(dev);
    e = hipMalloc(&p, c);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed: %s", c, hipGetErrorString(e));
    throw Error{GPA_E_NOMEM};
  }
  g_blocks[p] = BlockInfo{dev, c};
  P.in_use += c;
  return p;
}

void dev_free(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_blocks.find(p);
  if (it == g_blocks.end()) return;
  DevPool &P = g_pools[it->second.dev];
  P.free[it->second.cls].push_back(p);
  P.in_use -= it->second.cls;
  P.cached += it->second.cls;
}

namespace {
std::mutex g_pin_mu;
std::multimap<size_t, void *> g_pinned;   // capacity -> free pinned block
}  // namespace

void *pinned_take(size_t bytes, size_t *cap) {
  size_t c = 64 << 10;
  while (c < bytes) c <<= 1;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pinned.lower_bound(c);
    if (it != g_pinned.end() && it->first <= 4 * c) {
      void *p = it->second;
      *cap = it->first;
      g_pinned.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  const hipError_t e = hipHostMalloc(&p, c);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    set_error("pinned host allocation of %zu bytes failed: %s", c, hipGetErrorString(e));
    throw Error{GPA_E_NOMEM};
  }
  *cap = c;
  return p;
}

void pinned_give(void *p, size_t cap) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pinned.emplace(cap, p);
}

void pool_stats(uint64_t *in_use, uint64_t *cached) {
  int dev = 0;
  GPA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  DevPool &P = g_pools[dev];
  if (in_use) *in_use = P.in_use;
  if (cached) *cached = P.cached;
}

void pool_trim() {
  int dev = 0;
  GPA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  release_cached_locked(dev);
}

// ------------------------------------------------------------- timing
namespace {
std::mutex g_tmu;
bool g_timing = false;
double g_ms[kNumPhases] = {0};
uint64_t g_calls[kNumPhases] = {0};
// events are reused, per device: creating and destroying two per timed
// phase on every call would put host work between the launches it times
std::map<int, std::vector<hipEvent_t>> g_events;

hipEvent_t take_event(int dev) {
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    auto &v = g_events[dev];
    if (!v.empty()) {
      hipEvent_t e = v.back();
      v.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  GPA_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

void PhaseTimer::begin(int ph, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return;
  }
  GPA_HIP(hipGetDevice(&dev));
  phase = ph;
  a = take_event(dev);
  b = take_event(dev);
  GPA_HIP(hipEventRecord(a, s));
}

void PhaseTimer::end(hipStream_t s) {
  if (phase < 0) return;
  GPA_HIP(hipEventRecord(b, s));
}

void PhaseTimer::collect() {
  if (phase < 0) return;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_ms[phase] += ms;
    g_calls[phase] += 1;
  }
  phase = -1;
}

PhaseTimer::~PhaseTimer() {
  // back to the device's pool (an event still pending is simply recorded
  // again by its next user)
  std::lock_guard<std::mutex> lk(g_tmu);
  if (a) g_events[dev].push_back(a);
  if (b) g_events[dev].push_back(b);
}

// ------------------------------------------------------- side streams
namespace {
std::mutex g_smu;
std::vector<hipStream_t> g_side;   // per device, two each
}  // namespace

hipStream_t side_stream(int which) {
  int dev = 0;
  GPA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_smu);
  const size_t k = 2 * (size_t)dev + (which ? 1 : 0);
  if (k >= g_side.size()) g_side.resize(k + 1, nullptr);
  if (!g_side[k]) GPA_HIP(hipStreamCreateWithFlags(&g_side[k], hipStreamNonBlocking));
  return g_side[k];
}

// a synchronization-only event, destroyed with its scope
struct Event {
  hipEvent_t e = nullptr;
  Event() { GPA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
  Event(const Event &) = delete;
  Event &operator=(const Event &) = delete;
};

// Device-resident descriptor arrays are copied by one kernel launch for all
// of them (a job per array, a row of workgroups per job); host arrays go
// through the runtime's copies.
constexpr int kMaxCopyJobs = 24;
struct CopyJobs {
  void *dst[kMaxCopyJobs];
  const void *src[kMaxCopyJobs];
  uint64_t bytes[kMaxCopyJobs];
  uint32_t n;
};

__global__ void __launch_bounds__(256) k_multi_copy(CopyJobs jobs) {
  const uint32_t j = blockIdx.y;
  const uint64_t nb = jobs.bytes[j];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uintptr_t a = (uintptr_t)jobs.dst[j] | (uintptr_t)jobs.src[j];
  if ((a & 3) == 0) {
    const uint32_t *src = (const uint32_t *)jobs.src[j];
    uint32_t *dst = (uint32_t *)jobs.dst[j];
    for (uint64_t k = t; k < nb / 4; k += stride) dst[k] = src[k];
    for (uint64_t k = (nb & ~3ull) + t; k < nb; k += stride)
      ((uint8_t *)dst)[k] = ((const uint8_t *)src)[k];
  } else {
    const uint8_t *src = (const uint8_t *)jobs.src[j];
    uint8_t *dst = (uint8_t *)jobs.dst[j];
    for (uint64_t k = t; k < nb; k += stride) dst[k] = src[k];
  }
}

struct Uploader {
  bool on_device;
  hipStream_t s;
  CopyJobs jobs{};
  uint64_t max_bytes = 0;
  template <typename T>
  void operator()(DBuf<T> &dst, const T *src, size_t n) {
    dst.alloc(n);
    if (n == 0) return;
    if (!src) fail(GPA_E_INVALID, "a descriptor array is NULL");
    if (!on_device) {
      GPA_HIP(hipMemcpyAsync(dst.p, src, n * sizeof(T), hipMemcpyHostToDevice, s));
      return;
    }
    // only memory the runtime knows as device memory of this device is read
    // by the kernel; anything else goes through the runtime's copy
    hipPointerAttribute_t at{};
    int cur = -1;
    const bool known = hipPointerGetAttributes(&at, src) == hipSuccess &&
                       hipGetDevice(&cur) == hipSuccess && at.device == cur &&
                       (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
                        at.type == hipMemoryTypeUnified);
    (void)hipGetLastError();   // a failed attribute query must not linger
    if (!known) {
      GPA_HIP(hipMemcpyAsync(dst.p, src, n * sizeof(T), hipMemcpyDefault, s));
      return;
    }
    if (jobs.n == kMaxCopyJobs) flush();
    jobs.dst[jobs.n] = dst.p;
    jobs.src[jobs.n] = src;
    jobs.bytes[jobs.n] = n * sizeof(T);
    max_bytes = std::max<uint64_t>(max_bytes, n * sizeof(T));
    ++jobs.n;
  }
  void flush() {
    if (jobs.n == 0) return;
    const unsigned gx = grid_for(max_bytes / 4 + 1, 256, 256);
    hipLaunchKernelGGL(k_multi_copy, dim3(gx, jobs.n), dim3(256), 0, s, jobs);
    GPA_LAUNCH_CHECK();
    jobs.n = 0;
    max_bytes = 0;
  }
};

template <typename F>
static gpa_status guarded(F &&body) {
  try {
    body();
    return GPA_OK;
  } catch (const Error &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return GPA_E_NOMEM;
  } catch (...) {
    set_error("unexpected failure");
    return GPA_E_DEVICE;
  }
}

template <typename T>
static void copy_out(T *host, const DBuf<T> &src, size_t n, hipStream_t s) {
  if (!host || n == 0) return;
  GPA_HIP(hipMemcpyAsync(host, src.p, n * sizeof(T), hipMemcpyDeviceToHost, s));
}

void enqueue_attribute_batch(gpa_program *const *progs, const gpa_sample *const *ds,
                             const uint64_t *n, uint32_t count, hipStream_t s, Arena &ar,
                             gpa_blame **b, unsigned long long *dtot, bool measure_tuning,
                             PhaseTimer *t_hist, PhaseTimer *t_blame) {
  std::vector<HistEntry> batched;
  std::vector<uint32_t> single;
  const char *force = getenv("GPA_HIST_PARTITION");
  const bool forced = force && force[0] == '1';
  // the tables of every handle of the batch come from one shared set of
  // pool chunks, returned with the last of the handles
  auto sh = std::make_shared<SharedBlocks>();
  for (uint32_t k = 0; k < count; ++k) {
    b[k] = new gpa_blame(progs[k]);
    b[k]->shared = sh;
    sh->carve(b[k]->counts, (size_t)progs[k]->n_instr * 24);
    sh->carve(b[k]->issued, progs[k]->n_instr);
    const bool fits = n[k] > 0 && progs[k]->n_instr <= hist_hot_max_pcs() && !forced &&
                      ((uintptr_t)ds[k] % 16) == 0;
    if (fits)
      batched.push_back({ds[k], n[k], progs[k]->n_instr, b[k]->counts.p, b[k]->issued.p, dtot + 4 * k});
    else single.push_back(k);
  }
  const uint64_t per = batch_records_per_workgroup(batched.data(), (uint32_t)batched.size(), s, ar,
                                                   measure_tuning);
  // the phase timer brackets the batched launches; when some entries take
  // the per-profile histogram, it brackets everything from the batch's
  // preparation to the last of those
  if (single.empty()) {
    run_hist_batch(batched.data(), (uint32_t)batched.size(), per, s, ar, t_hist);
  } else {
    if (t_hist) t_hist->begin(kPhaseHist, s);
    run_hist_batch(batched.data(), (uint32_t)batched.size(), per, s, ar);
    for (uint32_t k : single)
      run_hist(*progs[k], ds[k], n[k], b[k]->counts.p, b[k]->issued.p, dtot + 4 * k, s, ar);
    if (t_hist) t_hist->end(s);
  }
  run_blame_batch(progs, b, count, s, ar, *sh, t_blame);
}

}  // namespace gpa

void *gpa_blame::operator new(size_t n) {
  if (n != sizeof(gpa_blame)) return ::operator new(n);
  return gpa::handle_alloc<sizeof(gpa_blame)>();
}
void gpa_blame::operator delete(void *p, size_t n) {
  if (n != sizeof(gpa_blame)) ::operator delete(p);
  else gpa::handle_free<sizeof(gpa_blame)>(p);
}
gpa_blame::gpa_blame(const gpa_program *p) : prog(p) { gpa::program_retain(p); }
gpa_blame::~gpa_blame() {
  // the buffers go back to the pool before the program can go
  counts.release();
  issued.release();
  dtotals.release();
  share.release();
  ec.release();
  bl.release();
  fx.release();
  nocand.release();
  shared.reset();
  gpa::program_release(prog);
}
void *gpa_advice::operator new(size_t n) {
  if (n != sizeof(gpa_advice)) return ::operator new(n);
  return gpa::handle_alloc<sizeof(gpa_advice)>();
}
void gpa_advice::operator delete(void *p, size_t n) {
  if (n != sizeof(gpa_advice)) ::operator delete(p);
  else gpa::handle_free<sizeof(gpa_advice)>(p);
}
gpa_advice::gpa_advice(const gpa_program *p) : prog(p) { gpa::program_retain(p); }
gpa_advice::~gpa_advice() {
  active.release();
  matched.release();
  speedup.release();
  kernel_T.release();
  kernel_L.release();
  eq3.release();
  top_opt.release();
  top_scope.release();
  top_speed.release();
  shared.reset();
  gpa::program_release(prog);
}

using namespace gpa;

extern "C" {

const char *gpa_last_error(void) { return g_err.c_str(); }

gpa_status gpa_pool_stats(uint64_t *in_use, uint64_t *cached) {
  return guarded([&] { pool_stats(in_use, cached); });
}

gpa_status gpa_pool_trim(void) {
  return guarded([&] { pool_trim(); });
}

void gpa_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = on != 0;
}

uint32_t gpa_timing_read(double *ms, uint64_t *calls, uint32_t max_phases, int reset) {
  std::lock_guard<std::mutex> lk(g_tmu);
  const uint32_t n = max_phases < (uint32_t)kNumPhases ? max_phases : (uint32_t)kNumPhases;
  for (uint32_t k = 0; k < n; ++k) {
    if (ms) ms[k] = g_ms[k];
    if (calls) calls[k] = g_calls[k];
  }
  if (reset)
    for (int k = 0; k < kNumPhases; ++k) {
      g_ms[k] = 0.0;
      g_calls[k] = 0;
    }
  return (uint32_t)kNumPhases;
}

gpa_status gpa_load_program(const gpa_program_desc *d, void *stream, gpa_program **out) {
  if (!d || !out) {
    set_error("gpa_load_program: NULL argument");
    return GPA_E_INVALID;
  }
  *out = nullptr;
  gpa_program *p = nullptr;
  hipStream_t s = (hipStream_t)stream;
  gpa_status st = guarded([&] {
    if (d->n_instr == 0 || d->n_blocks == 0 || d->n_funcs == 0 || d->n_scopes == 0)
      fail(GPA_E_INVALID, "empty program: n_instr, n_blocks, n_funcs and n_scopes must be > 0");
    if (d->n_instr >= 0x80000000u) fail(GPA_E_UNSUPPORTED, "n_instr must be below 2^31");
    if (d->n_preds > 16) fail(GPA_E_UNSUPPORTED, "n_preds must be at most 16");
    const uint64_t n_loc = (uint64_t)d->n_regs + d->n_preds + d->n_bars;
    if (n_loc == 0 || n_loc > 1024)
      fail(GPA_E_UNSUPPORTED, "n_regs + n_preds + n_bars must be in [1, 1024]");
    if (d->arch.blamable & ~0xFFFu) fail(GPA_E_INVALID, "arch.blamable has bits above 11");
    if (d->n_blocks > d->n_instr) fail(GPA_E_INVALID, "more blocks than instructions");
    if (d->n_funcs > d->n_blocks) fail(GPA_E_INVALID, "more functions than blocks");
    const bool dev = d->on_device != 0;
    p = new gpa_program();
    p->n_instr = d->n_instr;
    p->n_blocks = d->n_blocks;
    p->n_funcs = d->n_funcs;
    p->n_scopes = d->n_scopes;
    p->n_regs = d->n_regs;
    p->n_preds = d->n_preds;
    p->n_bars = d->n_bars;
    p->n_loc = (uint32_t)n_loc;
    p->arch = d->arch;
    p->n_blamable = (uint32_t)__builtin_popcount(d->arch.blamable & 0xFFFu);
    if (!d->def_ptr || !d->use_ptr || !d->succ_ptr) fail(GPA_E_INVALID, "a descriptor array is NULL");
    if (dev) {
      uint32_t sizes[3];
      GPA_HIP(hipMemcpyAsync(&sizes[0], d->def_ptr + d->n_instr, 4, hipMemcpyDeviceToHost, s));
      GPA_HIP(hipMemcpyAsync(&sizes[1], d->use_ptr + d->n_instr, 4, hipMemcpyDeviceToHost, s));
      GPA_HIP(hipMemcpyAsync(&sizes[2], d->succ_ptr + d->n_blocks, 4, hipMemcpyDeviceToHost, s));
      GPA_HIP(hipStreamSynchronize(s));
      p->n_defs = sizes[0];
      p->n_uses = sizes[1];
      p->n_succ = sizes[2];
    } else {
      p->n_defs = d->def_ptr[d->n_instr];
      p->n_uses = d->use_ptr[d->n_instr];
      p->n_succ = d->succ_ptr[d->n_blocks];
    }
    const uint32_t n = p->n_instr, nb = p->n_blocks;
    Uploader up{dev, s};
    up(p->op_class, d->op_class, n);
    up(p->guard, d->guard, n);
    up(p->def_ptr, d->def_ptr, (size_t)n + 1);
    up(p->def_loc, d->def_loc, p->n_defs);
    up(p->def_kind, d->def_kind, p->n_defs);
    up(p->use_ptr, d->use_ptr, (size_t)n + 1);
    up(p->use_loc, d->use_loc, p->n_uses);
    up(p->use_kind, d->use_kind, p->n_uses);
    up(p->block_begin, d->block_begin, (size_t)nb + 1);
    up(p->succ_ptr, d->succ_ptr, (size_t)nb + 1);
    up(p->succ, d->succ, p->n_succ);
    up(p->func_block_begin, d->func_block_begin, (size_t)p->n_funcs + 1);
    up(p->func_scope, d->func_scope, p->n_funcs);
    up(p->instr_scope, d->instr_scope, n);
    up(p->scope_parent, d->scope_parent, p->n_scopes);
    up(p->scope_kind, d->scope_kind, p->n_scopes);
    up(p->scope_flags, d->scope_flags, p->n_scopes);
    up.flush();
    const hipStream_t side = side_stream(0), side2 = side_stream(1);
    // outlive the arena, whose end waits for all three streams
    Event ev_struct, ev_order, ev_short;
    Arena ar(s);
    ar.add_stream(side);
    ar.add_stream(side2);
    PhaseTimer t_load, t_rd, t_dist, t_dist_long, t_dfs, t_search, t_val, t_sites, t_edges,
        t_targets;
    t_load.begin(kPhaseLoad, s);
    t_val.begin(kPhaseValidate, s);
    validate_and_build_structure(*p, s, ar);
    t_val.end(s);
    DistTables tables;
    prepare_dist_tables(*p, s, ar, tables);
    // the walk tables need only the CFG: the longest G' tables follow the DFS
    // order on one side stream, the shortest-walk tables (which any sweep
    // order settles) run in block order on the other, while the main stream
    // sorts the sites and builds the reaching definitions and edges
    GPA_HIP(hipEventRecord(ev_struct.e, s));
    GPA_HIP(hipStreamWaitEvent(side, ev_struct.e, 0));
    GPA_HIP(hipStreamWaitEvent(side2, ev_struct.e, 0));
    SweepPlan plan, plan_blocks;
    uint32_t *block_pos = nullptr;
    build_block_order_plan(*p, side2, ar, plan_blocks, block_pos);
    t_dist.begin(kPhaseDist, side2);
    build_dist_tables(*p, side2, plan_blocks, block_pos, tables, false);
    t_dist.end(side2);
    GPA_HIP(hipEventRecord(ev_short.e, side2));
    build_cfg_order(*p, side, ar, plan, t_dfs);
    t_dist_long.begin(kPhaseDistLong, side);
    build_dist_tables(*p, side, plan, p->rpo_pos.p, tables, true);
    t_dist_long.end(side);
    GPA_HIP(hipEventRecord(ev_order.e, side));
    t_sites.begin(kPhaseSites, s);
    build_sites_and_scopes(*p, s, ar);
    t_sites.end(s);
    t_rd.begin(kPhaseRd, s);
    build_reaching_defs(*p, s, ar, t_search);
    t_edges.begin(kPhaseEdges, s);
    build_edges(*p, s, ar);
    t_edges.end(s);
    t_rd.end(s);
    t_targets.begin(kPhaseTargets, s);
    build_scope_targets(*p, s, ar);
    GPA_HIP(hipStreamWaitEvent(s, ev_order.e, 0));
    GPA_HIP(hipStreamWaitEvent(s, ev_short.e, 0));
    build_distances(*p, s, ar, tables);
    build_topk_plan(*p, s, ar);
    t_targets.end(s);
    t_load.end(s);
    if (p->n_roots_dev)   // not read by an earlier synchronization
      GPA_HIP(hipMemcpyAsync(&p->n_roots, p->n_roots_dev, 4, hipMemcpyDeviceToHost, s));
    GPA_HIP(hipMemcpyAsync(p->seg_chunks, p->big_chunk_tot.p, sizeof(p->seg_chunks),
                           hipMemcpyDeviceToHost, s));
    unsigned long long tk_total = 0;
    if (p->tk_total_dev)
      GPA_HIP(hipMemcpyAsync(&tk_total, p->tk_total_dev, sizeof(tk_total), hipMemcpyDeviceToHost, s));
    GPA_HIP(hipStreamSynchronize(s));
    p->tk_chunks = (uint32_t)tk_total;
    p->tk_total_dev = nullptr;   // arena memory, returned with this call
    p->n_roots_dev = nullptr;
    p->sync_words = nullptr;   // arena memory, returned with this call
    t_load.collect();
    t_val.collect();
    t_sites.collect();
    t_edges.collect();
    t_targets.collect();
    t_rd.collect();
    t_dist.collect();
    t_dist_long.collect();
    t_dfs.collect();
    t_search.collect();
  });
  if (st != GPA_OK) {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    delete p;
    return st;
  }
  p->stream = s;
  *out = p;
  return GPA_OK;
}

void gpa_program_free(gpa_program *p) { program_release(p); }

gpa_status gpa_program_get_info(const gpa_program *p, gpa_program_info *info) {
  if (!p || !info) {
    set_error("gpa_program_get_info: NULL argument");
    return GPA_E_INVALID;
  }
  info->n_instr = p->n_instr;
  info->n_blocks = p->n_blocks;
  info->n_funcs = p->n_funcs;
  info->n_scopes = p->n_scopes;
  info->n_defs = p->n_defs;
  info->n_uses = p->n_uses;
  info->n_rd = p->n_rd;
  info->n_edges = p->n_edges;
  info->n_blamable = p->n_blamable;
  info->n_roots = p->n_roots;
  return GPA_OK;
}

gpa_status gpa_program_roots(const gpa_program *p, uint32_t *roots) {
  if (!p) {
    set_error("gpa_program_roots: NULL program");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    copy_out(roots, p->roots, p->n_roots, s);
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_program_rd(const gpa_program *p, uint32_t *rd_ptr, uint32_t *rd_src,
                          uint8_t *rd_blocked) {
  if (!p) {
    set_error("gpa_program_rd: NULL program");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    copy_out(rd_ptr, p->rd_ptr, (size_t)p->n_uses + 1, s);
    copy_out(rd_src, p->rd_src, p->n_rd, s);
    copy_out(rd_blocked, p->rd_blk, p->n_rd, s);
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_program_edges(const gpa_program *p, uint32_t *src, uint32_t *dst, uint8_t *flags,
                             uint32_t *dmin, uint32_t *dmax) {
  if (!p) {
    set_error("gpa_program_edges: NULL program");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    copy_out(src, p->e_src, p->n_edges, s);
    copy_out(dst, p->e_dst, p->n_edges, s);
    copy_out(flags, p->e_flags, p->n_edges, s);
    copy_out(dmin, p->e_dmin, p->n_edges, s);
    copy_out(dmax, p->e_dmax, p->n_edges, s);
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_attribute(gpa_program *p, const gpa_sample *samples, uint64_t n,
                         int samples_on_device, void *stream, gpa_blame **out) {
  if (!p || !out || (n && !samples)) {
    set_error("gpa_attribute: NULL argument");
    return GPA_E_INVALID;
  }
  *out = nullptr;
  gpa_blame *b = nullptr;
  hipStream_t s = (hipStream_t)stream;
  gpa_status st = guarded([&] {
    b = new gpa_blame(p);
    Arena ar(s);
    const gpa_sample *dsamp = samples;
    if (n && !samples_on_device) {
      gpa_sample *tmp = ar.get<gpa_sample>(n);
      GPA_HIP(hipMemcpyAsync(tmp, samples, n * sizeof(gpa_sample), hipMemcpyHostToDevice, s));
      dsamp = tmp;
    }
    b->counts.alloc((size_t)p->n_instr * 24);
    b->issued.alloc(p->n_instr);
    b->dtotals.alloc(4);
    PhaseTimer t_hist, t_blame;
    t_hist.begin(kPhaseHist, s);
    run_hist(*p, dsamp, n, b->counts.p, b->issued.p, b->dtotals.p, s, ar);
    t_hist.end(s);
    t_blame.begin(kPhaseBlame, s);
    run_blame(*p, *b, s, ar);
    t_blame.end(s);
    GPA_HIP(hipMemcpyAsync(b->totals, b->dtotals.p, sizeof(b->totals), hipMemcpyDeviceToHost, s));
    GPA_HIP(hipStreamSynchronize(s));
    t_hist.collect();
    t_blame.collect();
  });
  if (st != GPA_OK) {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    delete b;
    return st;
  }
  *out = b;
  return GPA_OK;
}

gpa_status gpa_attribute_batch(gpa_program *const *progs, const gpa_sample *const *samples,
                               const uint64_t *n, uint32_t count, int samples_on_device,
                               void *stream, gpa_blame **out) {
  if (!out || (count && (!progs || !samples || !n))) {
    set_error("gpa_attribute_batch: NULL argument");
    return GPA_E_INVALID;
  }
  for (uint32_t k = 0; k < count; ++k) {
    out[k] = nullptr;
    if (!progs[k] || (n[k] && !samples[k])) {
      set_error("gpa_attribute_batch: entry %u has a NULL program or sample array", k);
      return GPA_E_INVALID;
    }
    if (n[k] >= 0x40000000ull) {
      set_error("gpa_attribute_batch: entry %u has 2^30 samples or more", k);
      return GPA_E_UNSUPPORTED;
    }
  }
  std::vector<gpa_blame *> b(count, nullptr);
  hipStream_t s = (hipStream_t)stream;
  gpa_status st = guarded([&] {
    Arena ar(s);
    std::vector<const gpa_sample *> dptr(count, nullptr);
    for (uint32_t k = 0; k < count; ++k) {
      dptr[k] = samples[k];
      if (n[k] && !samples_on_device) {
        gpa_sample *tmp = ar.get<gpa_sample>(n[k]);
        GPA_HIP(hipMemcpyAsync(tmp, samples[k], n[k] * sizeof(gpa_sample), hipMemcpyHostToDevice, s));
        dptr[k] = tmp;
      }
    }
    unsigned long long *dtot = ar.get<unsigned long long>((size_t)count * 4);
    PhaseTimer t_hist, t_blame;
    enqueue_attribute_batch(progs, dptr.data(), n, count, s, ar, b.data(), dtot, true, &t_hist,
                            &t_blame);
    // the totals come back through pinned staging (a direct DMA, no
    // pageable bounce), returned with the arena
    unsigned long long *tot = nullptr;
    if (count) {
      const size_t bytes = sizeof(unsigned long long) * 4 * (size_t)count;
      tot = static_cast<unsigned long long *>(ar.stage(bytes));
      GPA_HIP(hipMemcpyAsync(tot, dtot, bytes, hipMemcpyDeviceToHost, s));
    }
    GPA_HIP(hipStreamSynchronize(s));
    t_hist.collect();
    t_blame.collect();
    for (uint32_t k = 0; k < count; ++k)
      for (int q = 0; q < 4; ++q) b[k]->totals[q] = tot[4 * (size_t)k + q];
  });
  if (st != GPA_OK) {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    for (gpa_blame *x : b) delete x;
    return st;
  }
  for (uint32_t k = 0; k < count; ++k) out[k] = b[k];
  return GPA_OK;
}

void gpa_blame_free(gpa_blame *b) { delete b; }

gpa_status gpa_blame_counts(const gpa_blame *b, uint32_t *counts, uint64_t *totals) {
  if (!b) {
    set_error("gpa_blame_counts: NULL blame");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    copy_out(counts, b->counts, (size_t)b->prog->n_instr * 24, s);
    if (totals) memcpy(totals, b->totals, sizeof(b->totals));
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_blame_shares(const gpa_blame *b, double *share) {
  if (!b) {
    set_error("gpa_blame_shares: NULL blame");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    copy_out(share, b->share, b->prog->n_edges * b->prog->n_blamable * 2, s);
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_blame_table(const gpa_blame *b, double *blamed, double *self_, double *fine) {
  if (!b) {
    set_error("gpa_blame_table: NULL blame");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    const size_t n = b->prog->n_instr;
    // the full tables are expanded from the compact ones into scratch
    Arena ar(s);
    double *d_blamed = blamed ? ar.get<double>(n * 24) : nullptr;
    double *d_self = self_ ? ar.get<double>(n * 24) : nullptr;
    double *d_fine = fine ? ar.get<double>(n * GPA_N_FINE * 2) : nullptr;
    expand_blame_tables(*b->prog, b->counts.p, b->bl.p, b->fx.p, b->nocand.p, d_blamed, d_self,
                        d_fine, s);
    if (blamed && n) GPA_HIP(hipMemcpyAsync(blamed, d_blamed, n * 24 * 8, hipMemcpyDeviceToHost, s));
    if (self_ && n) GPA_HIP(hipMemcpyAsync(self_, d_self, n * 24 * 8, hipMemcpyDeviceToHost, s));
    if (fine && n)
      GPA_HIP(hipMemcpyAsync(fine, d_fine, n * GPA_N_FINE * 2 * 8, hipMemcpyDeviceToHost, s));
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_advise(const gpa_blame *b, void *stream, gpa_advice **out) {
  if (!b || !out) {
    set_error("gpa_advise: NULL argument");
    return GPA_E_INVALID;
  }
  *out = nullptr;
  gpa_advice *a = nullptr;
  hipStream_t s = (hipStream_t)stream;
  gpa_status st = guarded([&] {
    a = new gpa_advice(b->prog);
    Arena ar(s);
    PhaseTimer t_adv;
    t_adv.begin(kPhaseAdvise, s);
    run_estimate(*b->prog, *b, *a, 16, s, ar);
    t_adv.end(s);
    GPA_HIP(hipStreamSynchronize(s));
    t_adv.collect();
  });
  if (st != GPA_OK) {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    delete a;
    return st;
  }
  *out = a;
  return GPA_OK;
}

gpa_status gpa_advise_batch(const gpa_blame *const *blames, uint32_t count, void *stream,
                            gpa_advice **out) {
  if (!out || (count && !blames)) {
    set_error("gpa_advise_batch: NULL argument");
    return GPA_E_INVALID;
  }
  for (uint32_t k = 0; k < count; ++k) {
    out[k] = nullptr;
    if (!blames[k]) {
      set_error("gpa_advise_batch: entry %u is NULL", k);
      return GPA_E_INVALID;
    }
  }
  std::vector<gpa_advice *> a(count, nullptr);
  hipStream_t s = (hipStream_t)stream;
  gpa_status st = guarded([&] {
    for (uint32_t k = 0; k < count; ++k) a[k] = new gpa_advice(blames[k]->prog);
    Arena ar(s);
    PhaseTimer t_adv;
    run_estimate_batch(blames, a.data(), count, 16, s, ar, &t_adv);
    GPA_HIP(hipStreamSynchronize(s));
    t_adv.collect();
  });
  if (st != GPA_OK) {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    for (gpa_advice *x : a) delete x;
    return st;
  }
  for (uint32_t k = 0; k < count; ++k) out[k] = a[k];
  return GPA_OK;
}

void gpa_advice_free(gpa_advice *a) { delete a; }

gpa_status gpa_analyze_batch(gpa_program *const *progs, const gpa_sample *const *samples,
                             const uint64_t *n, uint32_t count, int samples_on_device, void *stream,
                             gpa_blame **blames, gpa_advice **advices) {
  if (!blames || !advices || (count && (!progs || !samples || !n))) {
    set_error("gpa_analyze_batch: NULL argument");
    return GPA_E_INVALID;
  }
  for (uint32_t k = 0; k < count; ++k) {
    blames[k] = nullptr;
    advices[k] = nullptr;
    if (!progs[k] || (n[k] && !samples[k])) {
      set_error("gpa_analyze_batch: entry %u has a NULL program or sample array", k);
      return GPA_E_INVALID;
    }
    if (n[k] >= 0x40000000ull) {
      set_error("gpa_analyze_batch: entry %u has 2^30 samples or more", k);
      return GPA_E_UNSUPPORTED;
    }
  }
  std::vector<gpa_blame *> b(count, nullptr);
  std::vector<gpa_advice *> a(count, nullptr);
  hipStream_t s = (hipStream_t)stream;
  gpa_status st = guarded([&] {
    Arena ar(s);
    std::vector<const gpa_sample *> dptr(count, nullptr);
    for (uint32_t k = 0; k < count; ++k) {
      dptr[k] = samples[k];
      if (n[k] && !samples_on_device) {
        gpa_sample *tmp = ar.get<gpa_sample>(n[k]);
        GPA_HIP(hipMemcpyAsync(tmp, samples[k], n[k] * sizeof(gpa_sample), hipMemcpyHostToDevice, s));
        dptr[k] = tmp;
      }
    }
    unsigned long long *dtot = ar.get<unsigned long long>((size_t)count * 4);
    PhaseTimer t_hist, t_blame, t_adv;
    enqueue_attribute_batch(progs, dptr.data(), n, count, s, ar, b.data(), dtot, true, &t_hist,
                            &t_blame);
    for (uint32_t k = 0; k < count; ++k) a[k] = new gpa_advice(b[k]->prog);
    run_estimate_batch(b.data(), a.data(), count, 16, s, ar, &t_adv);
    // the totals come back through pinned staging (a direct DMA, no
    // pageable bounce), returned with the arena
    unsigned long long *tot = nullptr;
    if (count) {
      const size_t bytes = sizeof(unsigned long long) * 4 * (size_t)count;
      tot = static_cast<unsigned long long *>(ar.stage(bytes));
      GPA_HIP(hipMemcpyAsync(tot, dtot, bytes, hipMemcpyDeviceToHost, s));
    }
    GPA_HIP(hipStreamSynchronize(s));
    t_hist.collect();
    t_blame.collect();
    t_adv.collect();
    for (uint32_t k = 0; k < count; ++k)
      for (int q = 0; q < 4; ++q) b[k]->totals[q] = tot[4 * (size_t)k + q];
  });
  if (st != GPA_OK) {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    for (gpa_advice *x : a) delete x;
    for (gpa_blame *x : b) delete x;
    return st;
  }
  for (uint32_t k = 0; k < count; ++k) {
    blames[k] = b[k];
    advices[k] = a[k];
  }
  return GPA_OK;
}

void gpa_batch_free(gpa_blame *const *blames, gpa_advice *const *advices, uint32_t count) {
  for (uint32_t k = 0; k < count; ++k) {
    if (advices) delete advices[k];
    if (blames) delete blames[k];
  }
}

gpa_status gpa_advice_get(const gpa_advice *a, double *active, double *matched, double *speedup,
                          double *kernel_T, double *kernel_L, double *eq3) {
  if (!a) {
    set_error("gpa_advice_get: NULL advice");
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    const size_t ns = a->prog->n_scopes;
    copy_out(active, a->active, ns, s);
    copy_out(matched, a->matched, ns * GPA_N_OPT, s);
    copy_out(speedup, a->speedup, ns * GPA_N_OPT, s);
    copy_out(kernel_T, a->kernel_T, ns, s);
    copy_out(kernel_L, a->kernel_L, ns, s);
    copy_out(eq3, a->eq3, ns * 3, s);
    GPA_HIP(hipStreamSynchronize(s));
  });
}

gpa_status gpa_advice_topk(const gpa_advice *a, uint32_t k, uint32_t *opt, uint32_t *scope,
                           double *speedup) {
  if (!a) {
    set_error("gpa_advice_topk: NULL advice");
    return GPA_E_INVALID;
  }
  if (k == 0 || k > a->k) {
    set_error("gpa_advice_topk: k must be in [1, %u]", a->k);
    return GPA_E_INVALID;
  }
  return guarded([&] {
    hipStream_t s = nullptr;
    const size_t ns = a->prog->n_roots;
    if (ns == 0) return;
    std::vector<uint32_t> o(ns * a->k), sc(ns * a->k);
    std::vector<double> sp(ns * a->k);
    GPA_HIP(hipMemcpyAsync(o.data(), a->top_opt.p, 4 * o.size(), hipMemcpyDeviceToHost, s));
    GPA_HIP(hipMemcpyAsync(sc.data(), a->top_scope.p, 4 * sc.size(), hipMemcpyDeviceToHost, s));
    GPA_HIP(hipMemcpyAsync(sp.data(), a->top_speed.p, 8 * sp.size(), hipMemcpyDeviceToHost, s));
    GPA_HIP(hipStreamSynchronize(s));
    for (size_t r = 0; r < ns; ++r)
      for (uint32_t t = 0; t < k; ++t) {
        if (opt) opt[r * k + t] = o[r * a->k + t];
        if (scope) scope[r * k + t] = sc[r * a->k + t];
        if (speedup) speedup[r * k + t] = sp[r * a->k + t];
      }
  });
}

}  // extern "C"
