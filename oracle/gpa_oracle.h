/* gpa_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the GPA hot path
 * (Zhou et al., "GPA: A GPU Performance Advisor Based on Instruction
 * Sampling"): sample counting (Sec. 2.1), immediate dependency sources by
 * backward slicing with virtual barrier registers and predicate coverage
 * (Sec. 4), the dependency graph and its three pruning rules (Sec. 4), the
 * apportioning rule Eq. (1), and the code-optimization estimators Eqs. (2),
 * (4), (5) over the scope tree (Sec. 5).
 *
 * It shares no code, header, table or helper with the HIP library; it is
 * loaded only by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark.  Every data-format constant below is restated here on purpose.
 */
#ifndef GPA_ORACLE_H
#define GPA_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* opcode classes */
enum { ORC_ALU, ORC_FP64, ORC_LONG_ALU, ORC_GLOBAL_LOAD, ORC_SHARED_LOAD, ORC_LOCAL_LOAD,
       ORC_CONST_LOAD, ORC_GLOBAL_STORE, ORC_SHARED_STORE, ORC_LOCAL_STORE, ORC_BRANCH,
       ORC_BARRIER, ORC_CALL };
/* stall reasons */
enum { ORC_SELECTED, ORC_INST_FETCH, ORC_EXEC_DEP, ORC_MEM_DEP, ORC_TEXTURE, ORC_SYNC,
       ORC_CONST_MEM_DEP, ORC_PIPE_BUSY, ORC_MEM_THROTTLE, ORC_NOT_SELECTED, ORC_OTHER,
       ORC_SLEEPING, ORC_N_STALLS };
enum { ORC_DEF_REG, ORC_DEF_PRED, ORC_DEF_WBAR, ORC_DEF_RBAR };
enum { ORC_USE_OPND, ORC_USE_GUARD, ORC_USE_WAIT };
enum { ORC_SCOPE_FUNCTION, ORC_SCOPE_LOOP, ORC_SCOPE_LINE };
enum { ORC_SF_KERNEL = 1, ORC_SF_DEVICE = 2, ORC_SF_MATH = 4, ORC_SF_CFG = 8 };
/* fine classes of blamed stalls (Sec. 4, Fig. 5) */
enum { ORC_F_MEM_GLOBAL, ORC_F_MEM_LOCAL, ORC_F_MEM_CONST, ORC_F_EXEC_SHARED,
       ORC_F_EXEC_ARITH, ORC_F_EXEC_WAR, ORC_F_SYNC, ORC_F_OTHER, ORC_N_FINE };
/* code optimizers of Table 2 */
enum { ORC_O_REG_REUSE, ORC_O_STRENGTH, ORC_O_FUNC_SPLIT, ORC_O_FAST_MATH, ORC_O_WARP_BAL,
       ORC_O_MEM_TRANS, ORC_O_LOOP_UNROLL, ORC_O_REORDER, ORC_O_INLINE, ORC_N_OPT };
/* edge flags */
enum { ORC_E_DOM_KEEP = 1, ORC_E_LAT_KEEP = 2, ORC_E_WAR = 4 };

#define ORC_NONE 0xFFFFFFFFu

typedef struct {
  uint32_t n_instr, n_blocks, n_funcs, n_scopes;
  uint32_t n_regs, n_preds, n_bars;
  const uint8_t *op_class, *guard;
  const uint32_t *def_ptr, *def_loc;
  const uint8_t *def_kind;
  const uint32_t *use_ptr, *use_loc;
  const uint8_t *use_kind;
  const uint32_t *block_begin, *succ_ptr, *succ;
  const uint32_t *func_block_begin, *func_scope;
  const uint32_t *instr_scope, *scope_parent;
  const uint8_t *scope_kind, *scope_flags;
  const uint16_t *lat;      /* [16] per opcode class, in instruction slots */
  const uint16_t *allowed;  /* [12] per stall reason, bitmask of opcode classes */
  uint32_t blamable;        /* bitmask of stall reasons blamed on sources */
} orc_prog;

/* Sample counting (Sec. 2.1): C[(pc*12+stall)*2+latency] over valid
 * records; a record is valid iff pc < n_instr, stall < 12, flags has no bit
 * other than bit 0 and reserved == 0.  Invalid records are counted in
 * *dropped. */
void orc_count(uint32_t n_instr, const uint8_t *records, uint64_t n, uint32_t *C,
               uint64_t *dropped);

typedef struct orc_ctx orc_ctx;
orc_ctx *orc_ctx_new(const orc_prog *p);
void orc_ctx_free(orc_ctx *c);

/* Immediate sources of one use site (index into the use CSR): the def
 * instructions reached by the backward search of Sec. 4; blocked != 0 also
 * stops at unpredicated uses of the same location (dominator pruning).
 * Returns the number of sources; writes up to cap of them, ascending. */
uint32_t orc_sources(orc_ctx *c, uint32_t use_idx, int blocked, uint32_t *out, uint32_t cap);

/* Instructions strictly between i and j on the shortest CFG walk (dmin) and
 * on the longest walk of the CFG without retreating edges (dmax; dmin when
 * no such walk exists).  Returns 0 if j is unreachable from i. */
int orc_dist(orc_ctx *c, uint32_t i, uint32_t j, uint32_t *dmin, uint32_t *dmax);

/* Whole-program analysis: per-use source lists and the pruned-edge table. */
typedef struct orc_analysis orc_analysis;
orc_analysis *orc_analyze(orc_ctx *c);
void orc_analysis_free(orc_analysis *a);
void orc_analysis_sizes(const orc_analysis *a, uint64_t *n_rd, uint64_t *n_edges);
/* rd_ptr[n_uses+1], rd_src[n_rd], rd_blocked[n_rd] */
void orc_analysis_rd(const orc_analysis *a, uint32_t *rd_ptr, uint32_t *rd_src, uint8_t *rd_blocked);
/* edges sorted by (dst, src) */
void orc_analysis_edges(const orc_analysis *a, uint32_t *src, uint32_t *dst, uint8_t *flags,
                        uint32_t *dmin, uint32_t *dmax);

/* Blame (Eq. 1).  C from orc_count.  Outputs (doubles):
 *   share[n_edges * nb * 2]   nb = popcount(blamable), reasons ascending
 *   blamed[n_instr*24], self_[n_instr*24], fine[n_instr*ORC_N_FINE*2]      */
void orc_blame(const orc_analysis *a, const uint32_t *C, double *share, double *blamed,
               double *self_, double *fine);

/* Estimates (Eqs. 2, 4, 5).  Outputs:
 *   active[n_scopes], matched[n_scopes*9], speedup[n_scopes*9],
 *   root_of[n_scopes], kernel_T/L[n_scopes] (valid at roots),
 *   eq3[n_scopes*3] (kernel-level Eq. 3 for the 3 hiding optimizers, at roots),
 *   top_opt/top_scope/top_speed[n_scopes*k] (per root, ORC_NONE padded)      */
void orc_estimate(const orc_analysis *a, const uint32_t *C, const double *share,
                  const double *blamed, const double *self_, double *active, double *matched,
                  double *speedup, uint32_t *root_of, double *kernel_T, double *kernel_L,
                  double *eq3, uint32_t k, uint32_t *top_opt, uint32_t *top_scope,
                  double *top_speed);

/* Parallel optimizers (Sec. 5.2, Eqs. (6)-(10)) for kernel root scope
 * `root`: launch[4], device[8] and out[22] as documented in gpa_oracle.c. */
void orc_parallel(const orc_analysis *a, const uint32_t *C, uint32_t root, const uint32_t *launch,
                  const uint32_t *device, double *out);

/* Single dependency coverage (Sec. 6): instructions with no use site of two
 * or more sources, before and after pruning. */
void orc_coverage(const orc_analysis *a, uint64_t *before, uint64_t *after);
/* Hotspots of one optimizer in one kernel (root scope): up to k rows of
 * {src, dst, dmin, dmax, samples}; returns the number of rows. */
uint32_t orc_hotspots(const orc_analysis *a, const uint32_t *C, const double *share,
                      const double *self_, uint32_t root, uint32_t opt, uint32_t k, double *out);

#ifdef __cplusplus
}
#endif
#endif
