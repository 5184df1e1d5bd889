// Internal declarations of libgpa: handle layouts, error reporting, the
// device memory pool and the launch helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <memory>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gpa.h"

namespace gpa {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);

struct Error {
  gpa_status code;
};

#define GPA_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::gpa::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                       __FILE__, __LINE__);                                        \
      throw ::gpa::Error{e_ == hipErrorOutOfMemory ? GPA_E_NOMEM : GPA_E_DEVICE};  \
    }                                                                              \
  } while (0)

#define GPA_LAUNCH_CHECK() GPA_HIP(hipGetLastError())

[[noreturn]] void fail(gpa_status code, const char *fmt, ...);

// ------------------------------------------------------------ device memory
// A caching allocator, per device: freed blocks go back to their device's
// per-size-class free list and are reused by later allocations; cached
// blocks are returned to the runtime when an allocation fails or on
// pool_trim.  Blocks are 256-byte aligned.
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// bytes of the current device's blocks handed out and cached in free lists
void pool_stats(uint64_t *in_use, uint64_t *cached);
// frees the current device's cached blocks
void pool_trim();

// Pinned host staging for uploads (hipHostMalloc), pooled process-wide:
// a copy from pinned memory is asynchronous, where one from pageable memory
// can hold the host until the stream has caught up with it.  A block goes
// back to the pool only when the stream work reading it is complete.
void *pinned_take(size_t bytes, size_t *cap);
void pinned_give(void *p, size_t cap);

template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  bool borrowed = false;   // carved from a block someone else returns to the pool
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    p = static_cast<T *>(dev_alloc((count ? count : 1) * sizeof(T)));
  }
  void carve(void *q, size_t count) {
    release();
    n = count;
    p = static_cast<T *>(q);
    borrowed = true;
  }
  void release() {
    if (p && !borrowed) dev_free(p);
    p = nullptr;
    n = 0;
    borrowed = false;
  }
};

// Pieces of at least 256-byte alignment carved from pool chunks, so that a
// call making thousands of small tables takes a handful of blocks from the
// pool.  Chunks grow from 1 MiB, doubling up to kChunkBytes (so a small
// call leaves little of its last chunk unused); a request of a quarter of
// kChunkBytes or more gets a block of its own.  Every piece keeps 256 bytes
// of slack behind it, as a block of its own would.  The chunks are listed
// in `chunks` for their owner to return.
constexpr size_t kChunkBytes = (size_t)32 << 20;
struct ChunkCarver {
  std::vector<void *> chunks;
  char *cur = nullptr;
  size_t left = 0, next = (size_t)1 << 20;
  void *take(size_t bytes) {
    const size_t need = ((bytes ? bytes : 1) + 255) / 256 * 256 + 256;
    if (need >= kChunkBytes / 4) {
      void *b = dev_alloc(need);
      chunks.push_back(b);
      return b;
    }
    if (need > left) {
      while (next < need) next *= 2;
      void *c = dev_alloc(next);
      chunks.push_back(c);
      cur = static_cast<char *>(c);
      left = next;
      next = std::min(2 * next, kChunkBytes);
    }
    void *q = cur;
    cur += need;
    left -= need;
    return q;
  }
  void release() {
    for (void *c : chunks) dev_free(c);
    chunks.clear();
    cur = nullptr;
    left = 0;
    next = (size_t)1 << 20;
  }
};

// Device memory shared by the handles one batched call returns (their
// counts, shares, tables, estimates): each handle holds a reference, and the
// chunks go back to the pool with the last of them.
struct SharedBlocks {
  ChunkCarver carver;
  ~SharedBlocks() { carver.release(); }
  template <typename T>
  void carve(DBuf<T> &d, size_t count) {
    d.carve(carver.take(count * sizeof(T)), count);
  }
};

// Per-call scratch.  Pool mode: every block is returned to the pool when the
// arena is destroyed, after the streams the call launched work on have
// finished (also when the call fails part-way through).  Fixed mode: blocks
// are carved, 256-byte aligned, from a caller-given device region of `cap`
// bytes; nothing is allocated, synchronized or returned, and a request
// beyond the region fails with GPA_E_UNSUPPORTED.
struct Arena {
  ChunkCarver carver;
  std::vector<hipStream_t> streams;
  // pinned host staging of uploads, kept until the streams have finished
  // with them
  std::vector<std::pair<void *, size_t>> pinned;
  char *fixed = nullptr;
  size_t cap = 0, used = 0;
  explicit Arena(hipStream_t s) { streams.push_back(s); }
  Arena(void *region, size_t bytes) : fixed(static_cast<char *>(region)), cap(bytes) {}
  Arena(const Arena &) = delete;
  Arena &operator=(const Arena &) = delete;
  void add_stream(hipStream_t s) { streams.push_back(s); }
  // the streams' work that used the blocks is known to be complete (an
  // event was observed): the destructor returns them without synchronizing
  void work_done() { streams.clear(); }
  ~Arena() {
    if (fixed) return;
    for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
    carver.release();
    for (auto &b : pinned) pinned_give(b.first, b.second);
  }
  // a pinned staging block of at least `bytes`, returned with the arena
  void *stage(size_t bytes) {
    size_t got = 0;
    void *p = pinned_take(bytes, &got);
    pinned.emplace_back(p, got);
    return p;
  }
  template <typename T>
  T *get(size_t count) {
    const size_t bytes = (count ? count : 1) * sizeof(T);
    if (fixed) {
      const size_t at = (used + 255) / 256 * 256;
      if (at > cap || bytes > cap - at) {
        set_error("scratch region of %zu bytes is too small (%zu more bytes needed)", cap,
                  at + bytes - cap);
        throw Error{GPA_E_UNSUPPORTED};
      }
      used = at + bytes;
      return reinterpret_cast<T *>(fixed + at);
    }
    return static_cast<T *>(carver.take(bytes));
  }
};

// ------------------------------------------------------------------ handles
}  // namespace gpa

struct gpa_program {
  // one reference for the caller's handle and one per blame or advice handle
  // made from it: the program's memory goes when the last of them is freed
  std::atomic<int> refs{1};
  // sizes
  uint32_t n_instr = 0, n_blocks = 0, n_funcs = 0, n_scopes = 0;
  uint32_t n_regs = 0, n_preds = 0, n_bars = 0, n_loc = 0;
  uint32_t n_defs = 0, n_uses = 0, n_succ = 0;
  uint32_t max_func_blocks = 0, max_func_edges = 0;
  uint64_t dist_entries = 0;   // sum over functions of (blocks)^2
  gpa_arch arch{};
  uint32_t n_blamable = 0;
  // device copies of the descriptor
  gpa::DBuf<uint8_t> op_class, guard, def_kind, use_kind, scope_kind, scope_flags;
  gpa::DBuf<uint32_t> def_ptr, def_loc, use_ptr, use_loc, block_begin, succ_ptr, succ;
  gpa::DBuf<uint32_t> func_block_begin, func_scope, instr_scope, scope_parent;
  // derived structure
  gpa::DBuf<uint32_t> block_of, func_of_block, pred_ptr, pred;
  gpa::DBuf<uint32_t> def_site_sorted, fl_def_ptr;   // def sites by (function, location, instr)
  gpa::DBuf<uint32_t> use_site_sorted, fl_use_ptr;   // use sites by (function, location, instr)
  gpa::DBuf<uint32_t> def_instr, use_instr;          // site -> instruction
  gpa::DBuf<uint32_t> def_rank, use_rank;            // site -> position in the sorted array
  gpa::DBuf<uint8_t> use_cond;                       // use site -> effective condition
  // reaching definitions
  uint64_t n_rd = 0;
  gpa::DBuf<uint32_t> rd_ptr, rd_src;
  gpa::DBuf<uint8_t> rd_blk, rd_nonrbar;
  // dependency graph
  uint64_t n_edges = 0;
  gpa::DBuf<uint32_t> in_ptr;                  // [n_instr+1] edges into j
  gpa::DBuf<uint32_t> e_src, e_dst, e_dmin, e_dmax;
  gpa::DBuf<uint8_t> e_flags, e_cls;           // flags; the source's opcode class
  // stable groupings, built by one sort after the edges: edges by source
  // instruction (out), by common scope (lca), by common loop (icl), and
  // instructions by line scope (line); each view is laid out as if grouped
  // alone: its ptr starts at 0 and indexes its own stretch of grp_perm
  gpa::DBuf<uint32_t> grp_ptr, grp_perm;
  const uint32_t *out_ptr = nullptr, *lca_ptr = nullptr, *icl_ptr = nullptr, *line_ptr = nullptr;
  const uint32_t *out_perm = nullptr, *lca_perm = nullptr, *icl_perm = nullptr,
                 *line_perm = nullptr;
  gpa::DBuf<uint32_t> rpo_pos, rpo_order;      // per block: topological position in G'
  gpa::DBuf<uint8_t> retreat;                  // per successor edge
  // scope structure for the estimators
  gpa::DBuf<uint32_t> scope_end, root_of, scope_depth;
  gpa::DBuf<uint32_t> e_lca, e_icl;            // per edge target scopes
  gpa::DBuf<uint8_t> instr_tags;               // bit0 in math fn, bit1 in device fn with CFG

  // segments longer than a thread sums alone, per grouping (own sums by
  // scope, edges by common loop, edges by common scope, subtrees), each list
  // n_scopes long, counts in big_n[4]
  gpa::DBuf<uint32_t> big_list, big_n;
  // their kSegChunk-element chunks: first chunk of each listed segment (4
  // lists of n_scopes) and the chunk totals (device; host copy seg_chunks)
  gpa::DBuf<uint32_t> big_chunk;
  gpa::DBuf<unsigned long long> big_chunk_tot;
  unsigned long long seg_chunks[4] = {0, 0, 0, 0};
  gpa::DBuf<uint32_t> roots;                   // kernel root scope ids
  uint32_t n_roots = 0;
  // top-k plan: chunks of (scope, optimizer) items per kernel root, their
  // starts, and the total (device copy during the load)
  gpa::DBuf<uint32_t> tk_nch, tk_cst;
  uint32_t tk_chunks = 0;
  unsigned long long *tk_total_dev = nullptr;
  uint32_t *n_roots_dev = nullptr;   // during the load: device copy of n_roots
  // during the load: 8 device words read back together at each host
  // synchronization (validation verdict, then the reaching-definition sizes)
  uint32_t *sync_words = nullptr;
  hipStream_t stream = nullptr;
};

namespace gpa {
// Blame and advice handles come from a small per-thread cache of fixed-size
// blocks: a batched call makes and frees hundreds of them, and the heap's
// small allocations cost more host time than the call's launches.  A block
// freed on another thread joins that thread's cache; each cache keeps at
// most kHandleCache blocks and returns them to the heap when its thread
// ends.
constexpr size_t kHandleCache = 8192;
template <size_t Size>
struct HandleCache {
  std::vector<void *> free;
  ~HandleCache() {
    for (void *p : free) ::operator delete(p);
  }
  static HandleCache &mine() {
    thread_local HandleCache c;
    return c;
  }
};
template <size_t Size>
void *handle_alloc() {
  HandleCache<Size> &c = HandleCache<Size>::mine();
  if (c.free.empty()) return ::operator new(Size);
  void *p = c.free.back();
  c.free.pop_back();
  return p;
}
template <size_t Size>
void handle_free(void *p) {
  if (!p) return;
  HandleCache<Size> &c = HandleCache<Size>::mine();
  if (c.free.size() < kHandleCache) c.free.push_back(p);
  else ::operator delete(p);
}
}  // namespace gpa

struct gpa_blame {
  static void *operator new(size_t n);
  static void operator delete(void *p, size_t n);
  const gpa_program *prog = nullptr;   // holds a reference
  std::shared_ptr<gpa::SharedBlocks> shared;   // the tables' memory, when made by a batched call
  uint64_t totals[4] = {0, 0, 0, 0};
  gpa::DBuf<uint32_t> counts;          // [n_instr*24]
  gpa::DBuf<uint32_t> issued;          // [n_instr] issued samples (SELECTED, both latency bits)
  gpa::DBuf<unsigned long long> dtotals;
  gpa::DBuf<double> share;             // [n_edges*n_blamable*2]
  // [n_edges] each edge's latency samples of global-memory and execution
  // dependencies (its Loop Unrolling and Code Reordering contribution)
  gpa::DBuf<double> ec;
  // compact per-instruction results (the full tables are expanded on request)
  gpa::DBuf<double> bl;                // [n_instr*n_blamable*2] blamed, blamable reasons
  gpa::DBuf<double> fx;                // [n_instr*kBlameFx] WAR / other / rest splits
  gpa::DBuf<uint16_t> nocand;          // [n_instr] blamable reasons kept for want of a candidate
  explicit gpa_blame(const gpa_program *p);
  ~gpa_blame();
};

struct gpa_advice {
  static void *operator new(size_t n);
  static void operator delete(void *p, size_t n);
  const gpa_program *prog = nullptr;   // holds a reference
  std::shared_ptr<gpa::SharedBlocks> shared;   // the outputs' memory, when made by a batched call
  gpa::DBuf<double> active, matched, speedup, kernel_T, kernel_L, eq3;
  gpa::DBuf<uint32_t> top_opt, top_scope;
  gpa::DBuf<double> top_speed;
  uint32_t k = 0;
  explicit gpa_advice(const gpa_program *p);
  ~gpa_advice();
};

namespace gpa {

// reference counting of programs by their blame and advice handles
inline void program_retain(const gpa_program *p) {
  const_cast<gpa_program *>(p)->refs.fetch_add(1, std::memory_order_relaxed);
}
inline void program_release(const gpa_program *p) {
  if (p && const_cast<gpa_program *>(p)->refs.fetch_sub(1, std::memory_order_acq_rel) == 1)
    delete const_cast<gpa_program *>(p);
}

// ------------------------------------------------------------ device steps
// scan.hip: exclusive prefix sum of n u32 values into out (out may alias
// in); returns the total through *total_dev (a device u64) when not null.
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n, hipStream_t s, Arena &ar,
                        unsigned long long *total_dev = nullptr);

// sort.hip: stable radix sort of (key, value) pairs over the low key_bits
// bits, and grouping of n items by key (GPA_NONE keys left out).
void sort_pairs_u32(uint32_t *keys, uint32_t *vals, size_t n, uint32_t key_bits, hipStream_t s,
                    Arena &ar);
// One stable sort for several groupings (see group_by_key): grouping q is
// ptr.p + ptr_base[q] (n_keys + 1 entries) over perm.p + item_base[q], as if
// it had been grouped alone; perm's entries are item indices inside the
// grouping.
constexpr uint32_t kMaxGroups = 4;
struct GroupSpec {
  const uint32_t *key;
  uint64_t n;
  uint32_t n_keys;
};
void group_by_keys(const GroupSpec *spec, int n_groups, DBuf<uint32_t> &ptr,
                   DBuf<uint32_t> &perm, uint32_t *ptr_base, uint64_t *item_base,
                   hipStream_t s, Arena &ar);
void group_by_key(const uint32_t *key, size_t n, uint32_t n_keys, DBuf<uint32_t> &ptr,
                  DBuf<uint32_t> &perm, hipStream_t s, Arena &ar);

// A workgroup of a batched launch: the profile it works on and its block
// index within that profile's grid.
struct WorkItem {
  uint32_t entry, local;
};

// The work lists of a batched launch chain, expanded on the device: stage q
// gives entry e blocks[q][e] workgroups; its items are those of entry 0,
// then entry 1, and so on (or of the entries in a given order).  The host
// keeps only per-entry counts and their prefix sums (and the order); the
// tables go into the call's one upload, then expand() writes every stage's
// items in one launch.
constexpr uint32_t kMaxStages = 16;
struct StageTable {
  uint32_t n_stages, count;
  uint32_t pre_off[kMaxStages];          // offset of stage q's prefix sums (count + 1)
  uint32_t ord_off[kMaxStages];          // offset of its entry order, or ~0u for 0, 1, ...
  uint64_t item_off[kMaxStages + 1];     // offset of stage q's items
};
struct BatchPlan {
  std::vector<uint32_t> pre;
  StageTable t{};
  explicit BatchPlan(uint32_t count) { t.count = count; }
  // a stage (its entries in the given order, a permutation of 0..count-1,
  // when one is given); returns its index
  uint32_t add(const std::vector<uint32_t> &blocks, const std::vector<uint32_t> *order = nullptr);
  uint32_t blocks(uint32_t q) const { return (uint32_t)(t.item_off[q + 1] - t.item_off[q]); }
  uint64_t total_items() const { return t.item_off[t.n_stages]; }
  // the device prefix sums and items once placed and expanded
  const uint32_t *d_pre = nullptr;
  WorkItem *d_items = nullptr;
  const WorkItem *items(uint32_t q) const { return d_items + t.item_off[q]; }
  void expand(hipStream_t s);
};

// One host-to-device copy for a batched call's tables: each part is
// appended (256-byte aligned) and gets its device address once sent.
struct Upload {
  std::vector<char> host;
  std::vector<size_t> at;
  char *dev = nullptr;
  template <typename T>
  size_t add(const std::vector<T> &v) {
    const size_t o = (host.size() + 255) / 256 * 256;
    host.resize(o + sizeof(T) * v.size());
    if (!v.empty()) memcpy(host.data() + o, v.data(), sizeof(T) * v.size());
    at.push_back(o);
    return at.size() - 1;
  }
  template <typename T>
  T *ptr(size_t part) const { return reinterpret_cast<T *>(dev + at[part]); }
  // copies the parts to one block of the call's arena on `s` (the host
  // buffer is kept by the arena until the stream is done with it)
  void send(Arena &ar, hipStream_t s) {
    dev = ar.get<char>(host.size());
    if (host.empty()) return;
    void *pin = ar.stage(host.size());
    memcpy(pin, host.data(), host.size());
    const hipError_t e = hipMemcpyAsync(dev, pin, host.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      set_error("upload of %zu bytes failed: %s", host.size(), hipGetErrorString(e));
      throw Error{GPA_E_DEVICE};
    }
  }
};

// plan.hip: sends `up` (whose part i_pre is plan.pre) and expands the plan's
// work list on a side stream, and makes `s` wait for both (an event), so
// that the copy and the expansion overlap what `s` is still running; the
// side stream joins the arena's streams.
void send_plan_beside(Upload &up, size_t i_pre, BatchPlan &plan, Arena &ar, hipStream_t s);

// hist.hip.  allow_partition = false keeps to the hot-set path (programs of
// up to hist_hot_max_pcs() instructions; GPA_E_UNSUPPORTED beyond), which
// issues no memset and no host synchronization.
// Besides the counts, every path writes issued[i] = C[i][SELECTED][0] +
// C[i][SELECTED][1], the sum the blamer gathers per source.
void run_hist(const gpa_program &p, const gpa_sample *samples, uint64_t n, uint32_t *counts,
              uint32_t *issued, unsigned long long *totals, hipStream_t s, Arena &ar,
              bool allow_partition = true);
uint32_t hist_hot_max_pcs();
// One profile of a batched histogram: n records at `samples` (device, 16-byte
// aligned) of a program of n_instr <= hist_hot_max_pcs() instructions.
struct HistEntry {
  const gpa_sample *samples;
  uint64_t n;
  uint32_t n_instr;
  uint32_t *counts;
  uint32_t *issued;   // [n_instr]: the issued (SELECTED) samples, both latency bits
  unsigned long long *totals;
};
// The hot-set histogram of many profiles in three launches (selection,
// pass, finish), each workgroup taking one profile's share; `per` is the
// records per pass workgroup (rounded up to a multiple of 128, and raised
// where a profile would need more than 256 workgroups).  Entries must have
// n > 0.  The counts equal run_hist's for each profile.
struct PhaseTimer;
// (t, when given, brackets the three launches only, not the host's
// preparation of the argument tables and work lists)
void run_hist_batch(const HistEntry *e, uint32_t count, uint64_t per, hipStream_t s, Arena &ar,
                    PhaseTimer *t = nullptr);
// The autotuner of the batched histogram: records per pass workgroup for
// this batch's shape bucket (profile count, total and largest record count,
// each to a power of two), measured once per bucket and process by timing
// the candidates on the batch itself (every candidate computes the same
// counts), then reused.  GPA_BATCH_PER=<records> fixes it; GPA_AUTOTUNE=0
// takes the default without measuring; so does measure = false (for callers
// that must not synchronize) when the bucket has not been measured yet.
uint64_t batch_records_per_workgroup(const HistEntry *e, uint32_t count, hipStream_t s, Arena &ar,
                                     bool measure = true);
// scratch bytes the hot-set path takes for n records of a program of n_instr
// instructions (256-byte aligned blocks)
size_t hist_hot_scratch_bytes(uint32_t n_instr, uint64_t n);

// load.hip
void validate_and_build_structure(gpa_program &p, hipStream_t s, Arena &ar);
void build_sites_and_scopes(gpa_program &p, hipStream_t s, Arena &ar);
// dataflow.hip
struct PhaseTimer;
void build_reaching_defs(gpa_program &p, hipStream_t s, Arena &ar, PhaseTimer &t_search);
void build_edges(gpa_program &p, hipStream_t s, Arena &ar);
// dist.hip
// Per device, a second stream (default priority, non-blocking) for load work
// that only needs the CFG and can overlap the reaching definitions.
hipStream_t side_stream(int which = 0);   // per device: 0 and 1

// The G' sweep streams the distance kernel reads (built with the DFS order).
struct SweepPlan {
  uint32_t *ent_ptr = nullptr, *ent = nullptr, *ent_w = nullptr;
  uint32_t *ret_ptr = nullptr, *rent = nullptr, *rent_w = nullptr, *rent_e = nullptr;
};
void build_cfg_order(gpa_program &p, hipStream_t s, Arena &ar, SweepPlan &plan,
                     PhaseTimer &t_dfs);
// the sweep plan in block order (position = block index within its function)
void build_block_order_plan(gpa_program &p, hipStream_t s, Arena &ar, SweepPlan &plan,
                            uint32_t *&pos);
// Block-to-block walk tables of every function (shortest and longest G'
// walks from each block to each block of its function), from the CFG alone.
// per-opcode-class latency bounds, passed to a kernel by value
struct LatTable {
  uint16_t v[16];
};

struct DistTables {
  uint32_t *off = nullptr;   // [n_funcs] first entry of the function's tables
  uint32_t *sp = nullptr;    // shortest walk lengths, kInf-saturated
  uint32_t *lp = nullptr;    // longest G' walk lengths + 1, 0 = none
};
// table offsets and storage, before either table is built
void prepare_dist_tables(gpa_program &p, hipStream_t s, Arena &ar, DistTables &t);
// the shortest-walk tables (any sweep order: pos and plan in block order) or
// the longest G' tables (pos = reverse postorder of the DFS, plan from it)
void build_dist_tables(gpa_program &p, hipStream_t s, const SweepPlan &plan, const uint32_t *pos,
                       const DistTables &t, bool longest);
// per edge: dmin, dmax and the latency rule's flag from the tables
void build_distances(gpa_program &p, hipStream_t s, Arena &ar, const DistTables &t);
// per instruction: execution dependency from WAR and from other sources,
// other blamable reasons (each for both latency bits)
constexpr uint32_t kBlameFx = 6;
constexpr uint32_t kSmallSeg = 64;   // longest segment one thread sums alone
constexpr uint32_t kSegChunk = 4096; // elements of a longer segment per workgroup
void build_scope_targets(gpa_program &p, hipStream_t s, Arena &ar);
// blame.hip: run_blame allocates the blame handle's tables and calls
// launch_blame, which writes caller-given device arrays and allocates nothing
void run_blame(const gpa_program &p, gpa_blame &b, hipStream_t s, Arena &ar);
// (ec may be NULL: the edges' estimator contributions are then not written)
void launch_blame(const gpa_program &p, const uint32_t *counts, const uint32_t *issued,
                  double *share, double *ec, double *bl, double *fx, uint16_t *nocand,
                  hipStream_t s);
// the full tables of the C-ABI (blamed, self_: [n_instr*24]; fine:
// [n_instr*GPA_N_FINE*2]; any may be NULL) from the compact ones, on s
void expand_blame_tables(const gpa_program &p, const uint32_t *counts, const double *bl,
                         const double *fx, const uint16_t *nocand, double *blamed, double *self_,
                         double *fine, hipStream_t s);
struct PhaseTimer;
// The histogram and blame of `count` profiles whose records are on the
// device at ds[k]: creates b[k] with its tables, totals to dtot[4k..4k+3]
// (device).  With measure_tuning the autotuner may time candidates (it
// synchronizes then); otherwise nothing synchronizes.  The phase timers,
// when given, bracket the histogram and the blame on s (the caller collects
// them after synchronizing).
void enqueue_attribute_batch(gpa_program *const *progs, const gpa_sample *const *ds,
                             const uint64_t *n, uint32_t count, hipStream_t s, Arena &ar,
                             gpa_blame **b, unsigned long long *dtot, bool measure_tuning,
                             PhaseTimer *t_hist = nullptr, PhaseTimer *t_blame = nullptr);

// device bytes one request of n records against program p takes from
// admission to completion (staged records when host_records, histogram
// scratch, blame and advise tables), an upper estimate
uint64_t request_device_bytes(const gpa_program &p, uint64_t n, bool host_records);

// the blame of many profiles (their counts already in b[k]->counts) in two
// launches; each handle's tables are carved from `sh`
void run_blame_batch(const gpa_program *const *progs, gpa_blame *const *b, uint32_t count,
                     hipStream_t s, Arena &ar, SharedBlocks &sh, PhaseTimer *t = nullptr);
// estimate.hip
void run_estimate(const gpa_program &p, const gpa_blame &b, gpa_advice &a, uint32_t k,
                  hipStream_t s, Arena &ar);
// the advise of many profiles, each stage one launch over all of them
void run_estimate_batch(const gpa_blame *const *b, gpa_advice *const *adv, uint32_t count,
                        uint32_t k, hipStream_t s, Arena &ar, PhaseTimer *t = nullptr);
// at load: the top-k chunks of every kernel root (static)
void build_topk_plan(gpa_program &p, hipStream_t s, Arena &ar);

// Opt-in phase timing with hipEvents on the caller's stream (gpa_timing_*):
// a phase records an event pair; the pair's elapsed time is accumulated when
// the API call that launched it has synchronized its stream.
enum Phase {
  kPhaseHist = 0, kPhaseBlame, kPhaseLoad, kPhaseAdvise, kPhaseRd, kPhaseDist, kPhaseDfs,
  kPhaseRdSearch, kPhaseValidate, kPhaseSites, kPhaseEdges, kPhaseTargets, kPhaseDistLong,
  kNumPhases
};
struct PhaseTimer {
  hipEvent_t a = nullptr, b = nullptr;   // from a per-device pool
  int phase = -1, dev = 0;
  void begin(int ph, hipStream_t s);
  void end(hipStream_t s);
  void collect();   // after the stream has been synchronized
  ~PhaseTimer();
};

// read a few device words synchronously
template <typename T>
T read_scalar(const T *dev, hipStream_t s) {
  T v{};
  GPA_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  GPA_HIP(hipStreamSynchronize(s));
  return v;
}

// read two device values with one synchronization
template <typename A, typename B>
void read_scalars(const A *da, A &a, const B *db, B &b, hipStream_t s) {
  GPA_HIP(hipMemcpyAsync(&a, da, sizeof(A), hipMemcpyDeviceToHost, s));
  GPA_HIP(hipMemcpyAsync(&b, db, sizeof(B), hipMemcpyDeviceToHost, s));
  GPA_HIP(hipStreamSynchronize(s));
}

inline unsigned grid_for(size_t n, unsigned block, unsigned cap = 1u << 20) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace gpa
