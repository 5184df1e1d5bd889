/* gpa.h -- C-ABI of the MI355X GPA hot-path library (libgpa.so).
 *
 * The library implements, as hand-written HIP kernels for gfx950, the
 * data-parallel hot path of GPA, the instruction-sampling GPU performance
 * advisor of Zhou, Meng, Sai and Mellor-Crummey:
 *   - aggregation of PC samples into per-instruction stall-reason counts
 *     (Sec. 2.1, the "raw PC sampling report" of Sec. 2.3);
 *   - reaching definitions over each function's CFG with predicates and
 *     virtual barrier registers (Sec. 4, backward slicing);
 *   - the instruction blamer: dependency graph, opcode / dominator / latency
 *     pruning and the apportioning rule Eq. (1) (Sec. 4);
 *   - the code-optimization estimators of Table 2 with Eqs. (2), (4) and (5),
 *     rolled up the line -> loop -> function scope tree (Sec. 5).
 *
 * Conventions for every call:
 *   - Return value: GPA_OK (0) or a negative gpa_status; the thread-local
 *     message of the last failure is returned by gpa_last_error().
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     synchronous with respect to the host unless stated otherwise: on
 *     return, results are complete and host inputs may be reused.
 *   - Inputs are borrowed for the duration of the call and copied; handles
 *     own their device memory until the matching *_free call.  A program is
 *     read-only after loading and may back any number of blame handles.
 *     Blame and advice handles hold a reference to their program: after
 *     gpa_program_free the program's memory stays until the last blame and
 *     advice handle made from it is freed, so the handles may be freed in
 *     any order.
 *   - Copy-out getters write to host buffers; passing NULL for an optional
 *     buffer skips it.
 */
#ifndef GPA_H
#define GPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gpa_status;
#define GPA_OK 0
#define GPA_E_INVALID (-1)      /* malformed argument or descriptor */
#define GPA_E_NOMEM (-2)        /* device or host allocation failed */
#define GPA_E_DEVICE (-3)       /* a HIP runtime call failed */
#define GPA_E_STATE (-4)        /* handle used with a mismatching program, or a server shutting down */
#define GPA_E_BUSY (-5)         /* a served request is still waiting or running */
#define GPA_E_UNSUPPORTED (-6)  /* input beyond the limits documented below */

/* ---------------------------------------------------------------------
 * Encodings shared by inputs and outputs.
 * ------------------------------------------------------------------- */
/* opcode classes */
enum { GPA_OP_ALU = 0, GPA_OP_FP64, GPA_OP_LONG_ALU, GPA_OP_GLOBAL_LOAD, GPA_OP_SHARED_LOAD,
       GPA_OP_LOCAL_LOAD, GPA_OP_CONST_LOAD, GPA_OP_GLOBAL_STORE, GPA_OP_SHARED_STORE,
       GPA_OP_LOCAL_STORE, GPA_OP_BRANCH, GPA_OP_BARRIER, GPA_OP_CALL, GPA_N_OP_CLASSES };
/* stall reasons (Sec. 2.1; the blamed ones are listed in Sec. 4) */
enum { GPA_ST_SELECTED = 0, GPA_ST_INST_FETCH, GPA_ST_EXEC_DEP, GPA_ST_MEM_DEP, GPA_ST_TEXTURE,
       GPA_ST_SYNC, GPA_ST_CONST_MEM_DEP, GPA_ST_PIPE_BUSY, GPA_ST_MEM_THROTTLE,
       GPA_ST_NOT_SELECTED, GPA_ST_OTHER, GPA_ST_SLEEPING, GPA_N_STALLS };
/* def kinds: register, predicate, write barrier, read barrier (Sec. 4) */
enum { GPA_DEF_REG = 0, GPA_DEF_PRED, GPA_DEF_WBAR, GPA_DEF_RBAR };
/* use kinds: operand (carries the instruction's guard), guard read, wait mask */
enum { GPA_USE_OPND = 0, GPA_USE_GUARD, GPA_USE_WAIT };
enum { GPA_SCOPE_FUNCTION = 0, GPA_SCOPE_LOOP, GPA_SCOPE_LINE };
enum { GPA_SF_KERNEL_ENTRY = 1, GPA_SF_DEVICE_FN = 2, GPA_SF_MATH_FN = 4, GPA_SF_HAS_CFG = 8 };
/* fine classes of blamed stalls (Sec. 4, Fig. 5) */
enum { GPA_F_MEM_GLOBAL = 0, GPA_F_MEM_LOCAL, GPA_F_MEM_CONST, GPA_F_EXEC_SHARED,
       GPA_F_EXEC_ARITH, GPA_F_EXEC_WAR, GPA_F_SYNC, GPA_F_OTHER, GPA_N_FINE };
/* the nine code optimizers of Table 2 */
enum { GPA_O_REGISTER_REUSE = 0, GPA_O_STRENGTH_REDUCTION, GPA_O_FUNCTION_SPLIT,
       GPA_O_FAST_MATH, GPA_O_WARP_BALANCE, GPA_O_MEM_TRANSACTION_REDUCTION,
       GPA_O_LOOP_UNROLLING, GPA_O_CODE_REORDERING, GPA_O_FUNCTION_INLINING, GPA_N_OPT };
/* edge flags */
enum { GPA_E_DOM_KEEP = 1, GPA_E_LAT_KEEP = 2, GPA_E_WAR = 4 };
#define GPA_NONE 0xFFFFFFFFu

/* One PC sample (8 bytes, little endian).  flags bit 0: latency sample
 * (the warp scheduler issued nothing, Sec. 2.1).  A record with
 * pc >= n_instr, stall >= 12, any other flag bit or reserved != 0 is not
 * counted; it is counted as dropped instead. */
typedef struct {
  uint32_t pc;
  uint8_t stall;
  uint8_t flags;
  uint16_t reserved;
} gpa_sample;

/* Architectural features (Sec. 3, static analyzer). */
typedef struct {
  uint16_t lat[16];      /* per opcode class: latency in instruction slots (pruning rule 3) */
  uint16_t allowed[12];  /* per stall reason: bitmask of opcode classes that may cause it (rule 1) */
  uint16_t blamable;     /* bitmask of stall reasons attributed to source instructions */
  uint16_t pad;
} gpa_arch;

/* A program: instructions, basic blocks, one CFG per function, and the
 * scope tree (Sec. 3, "Control flow graphs" and "Program structure").
 * All arrays are borrowed for the call.  If on_device != 0 every array
 * pointer is a device pointer, otherwise a host pointer.
 *
 *  locations : [0,n_regs) registers, then n_preds predicates, then n_bars
 *              virtual barrier registers;
 *  guard     : 0 = unpredicated ("_"), 1+2k = Pk, 2+2k = !Pk (k < n_preds);
 *  def/use   : CSR over instructions (def_ptr[n_instr+1] etc.); a location
 *              appears at most once in an instruction's def list;
 *  blocks    : block b holds instructions [block_begin[b], block_begin[b+1]),
 *              block_begin[0] = 0, block_begin[n_blocks] = n_instr, no block
 *              is empty; successors are a CSR over blocks (succ_ptr, succ);
 *  functions : function f holds blocks [func_block_begin[f],
 *              func_block_begin[f+1]); its first block is the entry; every
 *              successor stays inside its function; func_scope[f] is a
 *              FUNCTION scope with GPA_SF_HAS_CFG;
 *  scopes    : numbered in preorder (scope_parent[s] < s, GPA_NONE for a
 *              root); roots are kernels (FUNCTION with GPA_SF_KERNEL_ENTRY);
 *              instr_scope[i] is a LINE scope inside func_scope of i's
 *              function and below no other CFG function.
 * Limits: n_instr < 2^31, n_preds <= 16, n_regs+n_preds+n_bars <= 1024,
 * at most 4096 blocks in one function, and the sum over functions of the
 * squared block count below 2^32 (the block-to-block walk tables). */
typedef struct {
  uint32_t n_instr, n_blocks, n_funcs, n_scopes;
  uint32_t n_regs, n_preds, n_bars;
  int32_t on_device;
  const uint8_t *op_class;         /* [n_instr] */
  const uint8_t *guard;            /* [n_instr] */
  const uint32_t *def_ptr;         /* [n_instr+1] */
  const uint32_t *def_loc;         /* [n_defs] */
  const uint8_t *def_kind;         /* [n_defs] */
  const uint32_t *use_ptr;         /* [n_instr+1] */
  const uint32_t *use_loc;         /* [n_uses] */
  const uint8_t *use_kind;         /* [n_uses] */
  const uint32_t *block_begin;     /* [n_blocks+1] */
  const uint32_t *succ_ptr;        /* [n_blocks+1] */
  const uint32_t *succ;            /* [n_succ] */
  const uint32_t *func_block_begin;/* [n_funcs+1] */
  const uint32_t *func_scope;      /* [n_funcs] */
  const uint32_t *instr_scope;     /* [n_instr] */
  const uint32_t *scope_parent;    /* [n_scopes] */
  const uint8_t *scope_kind;       /* [n_scopes] */
  const uint8_t *scope_flags;      /* [n_scopes] */
  gpa_arch arch;
} gpa_program_desc;

typedef struct gpa_program gpa_program;
typedef struct gpa_blame gpa_blame;
typedef struct gpa_advice gpa_advice;

typedef struct {
  uint64_t n_instr, n_blocks, n_funcs, n_scopes, n_defs, n_uses;
  uint64_t n_rd;       /* total size of the per-use source lists */
  uint64_t n_edges;    /* dependency-graph edges (i, j) */
  uint32_t n_blamable; /* popcount(arch.blamable) */
  uint32_t n_roots;    /* kernel root scopes (scope_parent == GPA_NONE) */
} gpa_program_info;

/* Load a program and build its static analysis on the device: reaching
 * definitions per use site with and without the use-blocked variant
 * (dominator pruning, Sec. 4 rule 2), the dependency-graph edges (Sec. 4,
 * Fig. 4b) with their flags, the shortest and longest instruction distance
 * of every edge (rules 2 and 3, heuristic 2), and the static target scopes
 * used by the estimators.  Errors: GPA_E_INVALID on a malformed descriptor
 * (details in gpa_last_error), GPA_E_UNSUPPORTED beyond the limits. */
gpa_status gpa_load_program(const gpa_program_desc *desc, void *stream, gpa_program **out);
void gpa_program_free(gpa_program *p);
gpa_status gpa_program_get_info(const gpa_program *p, gpa_program_info *info);

/* The kernel root scopes in ascending order: roots[n_roots] (host). */
gpa_status gpa_program_roots(const gpa_program *p, uint32_t *roots);
/* Per use site (in def/use CSR order) the sorted source instructions:
 * rd_ptr[n_uses+1], rd_src[n_rd], rd_blocked[n_rd] (1 if the source also
 * survives the use-blocked search). */
gpa_status gpa_program_rd(const gpa_program *p, uint32_t *rd_ptr, uint32_t *rd_src,
                          uint8_t *rd_blocked);
/* Edges sorted by (dst, src): src, dst, flags (GPA_E_*), dmin, dmax [n_edges]. */
gpa_status gpa_program_edges(const gpa_program *p, uint32_t *src, uint32_t *dst, uint8_t *flags,
                             uint32_t *dmin, uint32_t *dmax);

/* Attribute one profile (one kernel launch context, Sec. 3) of n samples.
 * samples_on_device != 0: `samples` is a device pointer that must stay
 * valid until the call returns.  Counts the samples (Sec. 2.1) and runs
 * the instruction blamer (Sec. 4, Eq. 1).  At most 2^30 - 1 samples per
 * call and 2^22 instructions in the program (GPA_E_UNSUPPORTED beyond).
 * Programs of up to 2^17 instructions are counted by a hot-set pass, larger
 * ones by a bucket partition; the environment variable GPA_HIST_PARTITION=1
 * selects the partition for every program (the counts are the same). */
gpa_status gpa_attribute(gpa_program *p, const gpa_sample *samples, uint64_t n,
                         int samples_on_device, void *stream, gpa_blame **out);
void gpa_blame_free(gpa_blame *b);
/* counts[n_instr*24] (index (pc*12+stall)*2+latency); totals[4] =
 * {valid samples, latency samples, dropped records, 0}. */
gpa_status gpa_blame_counts(const gpa_blame *b, uint32_t *counts, uint64_t *totals);
/* Per edge, per blamable reason (ascending) and latency bit: the share of
 * the destination's samples attributed along the edge, Eq. (1).
 * share[n_edges * n_blamable * 2]. */
gpa_status gpa_blame_shares(const gpa_blame *b, double *share);
/* blamed[n_instr*24]: samples attributed to i as a source; self_[n_instr*24]:
 * samples kept by the sampled instruction; fine[n_instr*GPA_N_FINE*2]. */
gpa_status gpa_blame_table(const gpa_blame *b, double *blamed, double *self_, double *fine);

/* Estimate the speedup of each code optimizer at each scope: Eq. (2) for
 * stall elimination, Eq. (5) for latency hiding (Eq. (4) at a kernel).
 * A kernel without samples gives 1; an optimizer whose matched (or, for
 * hiding, hidden) samples reach the kernel's total gives +inf, also when
 * rounding in the share sums puts them a few ulps above it. */
gpa_status gpa_advise(const gpa_blame *b, void *stream, gpa_advice **out);
void gpa_advice_free(gpa_advice *a);
/* active[n_scopes], matched[n_scopes*9], speedup[n_scopes*9],
 * kernel_T / kernel_L [n_scopes] (set at roots, 0 elsewhere),
 * eq3[n_scopes*3] (kernel-level Eq. (3) for the three hiding optimizers). */
gpa_status gpa_advice_get(const gpa_advice *a, double *active, double *matched, double *speedup,
                          double *kernel_T, double *kernel_L, double *eq3);
/* Top-k (k <= 16) per kernel root, speedup descending then optimizer then
 * scope ascending: arrays of n_roots*k, row r for the r-th kernel root in
 * ascending scope order (gpa_program_roots), GPA_NONE padded (speedup 0)
 * where a kernel has fewer than k candidates. */
gpa_status gpa_advice_topk(const gpa_advice *a, uint32_t k, uint32_t *opt, uint32_t *scope,
                           double *speedup);

/* The advice report (Sec. 3: raw advice as ASCII text; Sec. 7: hotspots as
 * def and use locations with their distance; Sec. 6: single dependency
 * coverage).
 * gpa_program_coverage: the instructions that are single-dependency nodes
 *   (no use site with two or more sources) before pruning (every reaching
 *   definition) and after it (sources that survive the dominator rule for
 *   that use and the latency rule for their edge).
 * gpa_blame_hotspots: for optimizer `opt` (GPA_O_*) and the kernel root
 *   with index root_index, the k largest carriers of its matched samples:
 *   edges (src = def, dst = use, their shortest and longest distance) for
 *   the blamed-stall and edge optimizers, instructions (src = GPA_NONE, dst
 *   = the instruction, distances 0) for the others; samples descending,
 *   ties by src then dst.  *n_out = the number written (<= k).
 * gpa_report: the whole report as text: coverage, then per kernel its
 *   optimizers with estimated speedup above 1, best first (at most
 *   top_optimizers), each with up to `hotspots` hotspots.  *len is the
 *   buffer size on entry and the size needed (with the final NUL) on
 *   return; buf may be NULL to ask for the size. */
typedef struct {
  uint32_t src, dst, dmin, dmax;
  double samples;
} gpa_hotspot;
gpa_status gpa_program_coverage(const gpa_program *p, uint64_t *single_before,
                                uint64_t *single_after);
gpa_status gpa_blame_hotspots(const gpa_blame *b, uint32_t root_index, uint32_t opt, uint32_t k,
                              gpa_hotspot *out, uint32_t *n_out);
gpa_status gpa_report(const gpa_advice *a, const gpa_blame *b, uint32_t top_optimizers,
                      uint32_t hotspots, char *buf, size_t *len);

/* The parallel optimizers of Table 2 and their estimate (Sec. 5.2, Eqs.
 * (6)-(10)): Block Increase (matched when the grid has fewer blocks than the
 * device has SMs / CUs) and Thread Increase (matched when the per-SM block
 * cap, not warps, registers or shared memory, limits residency).  For the
 * kernel root with index root_index in gpa_program_roots order, from its
 * samples in `b`, the launch and the device description:
 *   W     = resident blocks per SM x warps per block / schedulers per SM;
 *   R_I   = issued samples / all samples of the kernel;
 *   I     = 1 - (1 - R_I)^W, I_new likewise with W_new    (Eqs. (8), (9));
 *   C_W   = W_new / W, C_I = I_new / I                     (Eqs. (6), (7));
 *   S     = C_I / C_W x f                                  (Eq. (10)).
 * Block Increase: W_new = W x blocks / SMs (the threads spread over one block
 * per SM); f = 1, or T / (T - pipeline busy - memory throttle - not selected
 * samples) once W_new < 1.  Thread Increase: W_new = the warps an SM holds
 * once larger blocks lift the block cap (warp cap, registers, shared
 * memory, and the grid's warps per SM), over the schedulers; f = C_W, so
 * S = C_I.  (The paper leaves f and the new configurations open: these are
 * this library's readings.)  out[0] is Block Increase, out[1] Thread
 * Increase; speedup = 1 when not matched or when the kernel has no issued
 * sample.  GPA_E_INVALID for a zero field or threads_per_block above the
 * device's maximum. */
typedef struct {
  uint32_t blocks, threads_per_block;
  uint32_t regs_per_thread;    /* 32-bit registers per thread; 0 = not limiting */
  uint32_t shared_per_block;   /* bytes; 0 = not limiting */
} gpa_launch;
typedef struct {
  uint32_t n_sm, schedulers_per_sm, warp_size;
  uint32_t max_warps_per_sm, max_blocks_per_sm, max_threads_per_block;
  uint32_t regs_per_sm, shared_per_sm;   /* 32-bit registers; bytes */
} gpa_device;
typedef struct {
  uint32_t matched, pad;
  double W, W_new, R_I, I, I_new, C_W, C_I, f, speedup;
} gpa_parallel_estimate;
gpa_status gpa_parallel_advise(const gpa_blame *b, uint32_t root_index, const gpa_launch *launch,
                               const gpa_device *device, gpa_parallel_estimate *out);

/* Batching (Sec. 3: every kernel launch context is analyzed on its own, so
 * many of them can share each device step).  gpa_attribute_batch does for
 * each entry k what gpa_attribute(progs[k], samples[k], n[k], ...) does,
 * with one launch of each histogram and blame kernel for the whole batch
 * (every workgroup takes one entry's share from a device work list), and
 * returns one blame handle per entry in out[k].  A program may appear in
 * several entries.  The results are bit for bit those of gpa_attribute.
 * Entries whose program has more than 2^17 instructions, or whose device
 * records are not 16-byte aligned, are counted by gpa_attribute's own path
 * inside the same call.  The records per histogram workgroup are picked by
 * an autotuner per batch shape (see GPA_BATCH_PER / GPA_AUTOTUNE in the
 * library's notes).  On failure no handle is returned (all out[k] NULL). */
gpa_status gpa_attribute_batch(gpa_program *const *progs, const gpa_sample *const *samples,
                               const uint64_t *n, uint32_t count, int samples_on_device,
                               void *stream, gpa_blame **out);
/* gpa_attribute_batch followed by gpa_advise_batch in one call: the
 * estimators' launches follow the blamer's on the stream without a return
 * to the host in between, and the call synchronizes once.  blames[k] and
 * advices[k] are what the two calls would return, bit for bit.  On failure
 * no handle is returned.
 * gpa_batch_free frees the handles of a batch (either array may be NULL;
 * NULL entries are skipped), advice before blame. */
gpa_status gpa_analyze_batch(gpa_program *const *progs, const gpa_sample *const *samples,
                             const uint64_t *n, uint32_t count, int samples_on_device, void *stream,
                             gpa_blame **blames, gpa_advice **advices);
void gpa_batch_free(gpa_blame *const *blames, gpa_advice *const *advices, uint32_t count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): what
 * gpa_attribute computes for one profile, written to caller-given device
 * arrays, with no allocation of any kind.  The histogram's scratch is a
 * fixed array of gpa_noalloc_scratch_bytes() bytes inside the library, one
 * per GPU, held from the library's first use on that GPU until the process
 * ends.
 *   samples : device, n records (8-byte aligned; 16-byte alignment is
 *             faster), borrowed until the stream's work is done;
 *   counts  : device u32 [n_instr*24], totals: device u64 [4] (as
 *             gpa_blame_counts); share: device f64 [n_edges*n_blamable*2]
 *             (may be NULL when that size is 0); blamed, self_: device f64
 *             [n_instr*24]; fine: device f64 [n_instr*GPA_N_FINE*2] (as
 *             gpa_blame_shares and gpa_blame_table).  Every element is
 *             written; nothing needs clearing beforehand.
 * The call only enqueues work on `stream` and returns; results are ready
 * when the stream's work is.  All calls on one GPU share its scratch array:
 * calls that overlap on one GPU (different streams or threads without
 * ordering between them) race; calls on one stream are ordered.
 * GPA_E_UNSUPPORTED, before anything is launched, for programs above 2^17
 * instructions or inputs whose scratch would exceed the fixed size.  The
 * scratch of a program of at most 3,072 instructions does not grow with the
 * records (at most 76 MB); a larger program's takes about 8 bytes per record
 * plus 13 MB to 26 MB with the program's size (some 23M records for a
 * program of 3,073 instructions, 21M for one of 2^17). */
uint64_t gpa_noalloc_scratch_bytes(void);
gpa_status gpa_attribute_noalloc(const gpa_program *p, const gpa_sample *samples, uint64_t n,
                                 void *stream, uint32_t *counts, uint64_t *totals, double *share,
                                 double *blamed, double *self_, double *fine);

/* gpa_advise for every blame handle of the batch, each estimate stage one
 * launch over all of them; out[k] as gpa_advise(blames[k]) would return,
 * bit for bit. */
gpa_status gpa_advise_batch(const gpa_blame *const *blames, uint32_t count, void *stream,
                            gpa_advice **out);

/* Serving (Sec. 3: analysis per kernel launch context, so requests against
 * resident programs are independent).  A server admits submitted requests
 * in arrival order as long as the device bytes they need (records staged
 * from the host, histogram scratch, blame and advice tables; an upper
 * estimate) fit in its budget together with the requests still running,
 * and runs what has been admitted in batches through the batched kernels of
 * gpa_attribute_batch / gpa_advise_batch, on two streams of its own so that
 * consecutive batches overlap on the device; requests that arrive while
 * others run join the next batch.  A request's results are bit for bit
 * those of gpa_attribute + gpa_advise on the same records.
 *
 * gpa_server_create: budget_bytes > 0; a worker thread is started; the
 *   server belongs to the device current at creation.
 * gpa_server_submit: enqueues one request (never blocks on the GPU).  The
 *   program must be loaded; the server holds a reference to it until the
 *   request completes.  `samples` (host, or device when samples_on_device)
 *   is borrowed until the request completes (its ticket polls done or
 *   failed).  GPA_E_NOMEM, with nothing enqueued, when the request alone
 *   needs more than the budget; GPA_E_STATE while the server shuts down.
 * gpa_server_poll: GPA_E_BUSY while the request waits or runs; then once
 *   GPA_OK with the request's advice (and, when blame is not NULL, its
 *   blame handle; otherwise the blame is freed), or the request's failure
 *   status with its message in gpa_last_error; the ticket is forgotten
 *   after that.  GPA_E_INVALID for an unknown ticket.
 * gpa_server_wait: blocks until a request has finished that no wait has
 *   returned yet and no poll has collected, then returns GPA_OK with its
 *   ticket (finished requests come back in the order they finished; poll
 *   then collects the results without waiting); GPA_E_BUSY when none
 *   finishes within timeout_us microseconds.  For callers that would
 *   otherwise poll in a loop: the caller wakes when a batch completes.
 * gpa_server_free: waits for every submitted request to finish, frees the
 *   results nobody polled and stops the worker. */
typedef struct gpa_server gpa_server;
typedef struct {
  uint64_t submitted, admitted, completed, failed;
  uint64_t batches, max_batch;      /* batches launched, most requests in one */
  uint64_t peak_reserved, reserved, budget;   /* admitted bytes: peak, now; the budget */
  uint64_t queued, inflight_batches;          /* now */
} gpa_server_stats;
gpa_status gpa_server_create(uint64_t budget_bytes, gpa_server **out);
gpa_status gpa_server_submit(gpa_server *server, gpa_program *p, const gpa_sample *samples,
                             uint64_t n, int samples_on_device, uint64_t *ticket);
gpa_status gpa_server_poll(gpa_server *server, uint64_t ticket, gpa_blame **blame,
                           gpa_advice **advice);
gpa_status gpa_server_wait(gpa_server *server, uint64_t timeout_us, uint64_t *ticket);
gpa_status gpa_server_stats_get(gpa_server *server, gpa_server_stats *stats);
void gpa_server_free(gpa_server *server);

/* Instrumentation (for benchmarks and profiling tools).  When enabled, the
 * library records a hipEvent pair around each phase on the stream the phase
 * runs on (the caller's, or for phases 5, 6 and 12 one of the library's two
 * per-device side streams) and accumulates the elapsed device time once the
 * call has synchronized.
 * Phases: 0 sample aggregation, 1 blame, 2 whole program load, 3 advise,
 * 4 reaching definitions and edges, 5 shortest-walk tables of the CFGs,
 * 6 depth-first order of the CFGs, 7 the backward searches, 8 descriptor
 * validation and derived CFG structure, 9 definition and use sites and scope
 * structure, 10 def-use edges, 11 edge distances and target scopes,
 * 12 longest-walk tables of the CFGs.  gpa_timing_read copies
 * up to max_phases accumulated milliseconds and call counts (either pointer
 * may be NULL), optionally resets them, and returns the number of phases. */
void gpa_timing_enable(int on);
uint32_t gpa_timing_read(double *ms, uint64_t *calls, uint32_t max_phases, int reset);

/* The library's device memory on the current device: bytes handed out to
 * live handles and scratch (in_use) and bytes cached for reuse (cached).
 * Either pointer may be NULL. */
gpa_status gpa_pool_stats(uint64_t *in_use, uint64_t *cached);
/* Return the current device's cached blocks to the HIP runtime. */
gpa_status gpa_pool_trim(void);

/* Thread-local description of the last failure on this thread. */
const char *gpa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
