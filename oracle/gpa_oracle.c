/* gpa_oracle.c -- TEST INFRASTRUCTURE ONLY (see gpa_oracle.h).
 *
 * Plain definitions, written for a reader holding the paper:
 *   counting          Sec. 2.1 (active / latency / stall samples)
 *   sources           Sec. 4 "Backward slicing": per use, walk the CFG
 *                     backwards and stop once the predicates of the defs met
 *                     on the path cover the use's predicate; barriers are
 *                     virtual registers (write/read barrier = def, wait = use)
 *   graph + pruning   Sec. 4 "Construct a dependency graph", "Prune cold
 *                     edges" (opcode, dominator and latency rules)
 *   apportioning      Sec. 4 "Attribute stalls", Eq. (1), applied per stall
 *                     reason and separately to latency samples
 *   estimates         Sec. 5: Table 2 matching, Eq. (2), Eq. (4), Eq. (5)
 * Readings of points the paper leaves open are listed in the design notes
 * of the repository; the ones that shape code are restated where used.
 * No blocking, fusion or reordering beyond these definitions.
 */
#include "gpa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ counts */
void orc_count(uint32_t n_instr, const uint8_t *rec, uint64_t n, uint32_t *C, uint64_t *dropped) {
  uint64_t bad = 0;
  memset(C, 0, sizeof(uint32_t) * (size_t)n_instr * 24u);
  for (uint64_t r = 0; r < n; ++r) {
    const uint8_t *b = rec + 8 * r;
    uint32_t pc = (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) |
                  ((uint32_t)b[3] << 24);
    uint32_t stall = b[4], flags = b[5];
    uint32_t reserved = (uint32_t)b[6] | ((uint32_t)b[7] << 8);
    if (pc < n_instr && stall < 12 && (flags & ~1u) == 0 && reserved == 0)
      C[((size_t)pc * 12 + stall) * 2 + (flags & 1u)] += 1;
    else
      bad += 1;
  }
  *dropped = bad;
}

/* ----------------------------------------------------------------- context */
struct orc_ctx {
  orc_prog p;
  uint32_t n_succ;
  uint32_t *block_of;      /* instruction -> block */
  uint32_t *func_of_block; /* block -> function */
  uint32_t *pred_ptr, *pred;
  uint8_t *retreat;        /* per successor-CSR edge: retreating in the DFS */
  uint32_t *tpos;          /* instruction -> position in the function's G' order */
  uint32_t *topo;          /* position -> instruction */
  /* scratch */
  uint32_t *stamp, cur;
  uint32_t *stack, stack_cap;
  int32_t *len;
  uint32_t *queue, *qd;
};

static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) abort();
  return p;
}

static uint32_t first_of(const orc_ctx *c, uint32_t b) { return c->p.block_begin[b]; }
static uint32_t last_of(const orc_ctx *c, uint32_t b) { return c->p.block_begin[b + 1] - 1; }

/* Depth-first search over the blocks of one function, from its entry block
 * and then from every block still unvisited in index order, successors in
 * CSR order.  An edge to a block that is still on the DFS stack (an ancestor
 * or the block itself) is retreating.  Reverse postorder of the forest is a
 * topological order of the CFG without its retreating edges (G'). */
static void dfs_function(orc_ctx *c, uint32_t f) {
  const orc_prog *p = &c->p;
  uint32_t b0 = p->func_block_begin[f], b1 = p->func_block_begin[f + 1];
  uint32_t nb = b1 - b0;
  uint8_t *state = (uint8_t *)calloc(nb ? nb : 1, 1);
  uint32_t *it = (uint32_t *)xmalloc(sizeof(uint32_t) * (nb + 1));
  uint32_t *stk = (uint32_t *)xmalloc(sizeof(uint32_t) * (nb + 1));
  uint32_t *post = (uint32_t *)xmalloc(sizeof(uint32_t) * (nb + 1));
  uint32_t npost = 0;
  for (uint32_t root = b0; root < b1; ++root) {
    if (state[root - b0]) continue;
    uint32_t sp = 0;
    stk[sp++] = root;
    state[root - b0] = 1;
    it[root - b0] = p->succ_ptr[root];
    while (sp) {
      uint32_t u = stk[sp - 1];
      if (it[u - b0] < p->succ_ptr[u + 1]) {
        uint32_t e = it[u - b0]++;
        uint32_t v = p->succ[e];
        if (state[v - b0] == 0) {
          state[v - b0] = 1;
          it[v - b0] = p->succ_ptr[v];
          stk[sp++] = v;
        } else if (state[v - b0] == 1) {
          c->retreat[e] = 1;
        }
      } else {
        state[u - b0] = 2;
        post[npost++] = u;
        --sp;
      }
    }
  }
  uint32_t pos = p->block_begin[b0];
  for (uint32_t k = npost; k-- > 0;) {
    uint32_t b = post[k];
    for (uint32_t ins = first_of(c, b); ins <= last_of(c, b); ++ins) {
      c->topo[pos] = ins;
      c->tpos[ins] = pos;
      ++pos;
    }
  }
  free(state);
  free(it);
  free(stk);
  free(post);
}

orc_ctx *orc_ctx_new(const orc_prog *p) {
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->p = *p;
  uint32_t n = p->n_instr, nb = p->n_blocks;
  c->n_succ = p->succ_ptr[nb];
  c->block_of = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  for (uint32_t b = 0; b < nb; ++b)
    for (uint32_t i = p->block_begin[b]; i < p->block_begin[b + 1]; ++i) c->block_of[i] = b;
  c->func_of_block = (uint32_t *)xmalloc(sizeof(uint32_t) * (nb + 1));
  for (uint32_t f = 0; f < p->n_funcs; ++f)
    for (uint32_t b = p->func_block_begin[f]; b < p->func_block_begin[f + 1]; ++b)
      c->func_of_block[b] = f;
  /* predecessor lists */
  c->pred_ptr = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
  c->pred = (uint32_t *)xmalloc(sizeof(uint32_t) * (c->n_succ + 1));
  for (uint32_t e = 0; e < c->n_succ; ++e) c->pred_ptr[p->succ[e] + 1] += 1;
  for (uint32_t b = 0; b < nb; ++b) c->pred_ptr[b + 1] += c->pred_ptr[b];
  uint32_t *fill = (uint32_t *)xmalloc(sizeof(uint32_t) * (nb + 1));
  memcpy(fill, c->pred_ptr, sizeof(uint32_t) * nb);
  for (uint32_t b = 0; b < nb; ++b)
    for (uint32_t e = p->succ_ptr[b]; e < p->succ_ptr[b + 1]; ++e) c->pred[fill[p->succ[e]]++] = b;
  free(fill);
  c->retreat = (uint8_t *)calloc(c->n_succ + 1, 1);
  c->tpos = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  c->topo = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  for (uint32_t f = 0; f < p->n_funcs; ++f) dfs_function(c, f);
  c->stamp = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
  c->cur = 0;
  c->stack_cap = 2 * n + c->n_succ + 16;
  c->stack = (uint32_t *)xmalloc(sizeof(uint32_t) * c->stack_cap);
  c->len = (int32_t *)xmalloc(sizeof(int32_t) * (n + 1));
  c->queue = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  c->qd = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  return c;
}

void orc_ctx_free(orc_ctx *c) {
  if (!c) return;
  free(c->block_of);
  free(c->func_of_block);
  free(c->pred_ptr);
  free(c->pred);
  free(c->retreat);
  free(c->tpos);
  free(c->topo);
  free(c->stamp);
  free(c->stack);
  free(c->len);
  free(c->queue);
  free(c->qd);
  free(c);
}

static uint32_t next_stamp(orc_ctx *c) {
  if (++c->cur == 0) {
    memset(c->stamp, 0, sizeof(uint32_t) * (c->p.n_instr + 1));
    c->cur = 1;
  }
  return c->cur;
}

/* ------------------------------------------------------------- sources */
/* index of the def of location x in instruction k, or -1 */
static int64_t def_of(const orc_prog *p, uint32_t k, uint32_t x) {
  for (uint32_t d = p->def_ptr[k]; d < p->def_ptr[k + 1]; ++d)
    if (p->def_loc[d] == x) return d;
  return -1;
}

static int uses_loc(const orc_prog *p, uint32_t k, uint32_t x) {
  for (uint32_t u = p->use_ptr[k]; u < p->use_ptr[k + 1]; ++u)
    if (p->use_loc[u] == x) return 1;
  return 0;
}

/* A def with guard g covers the use condition c iff g is `_` or g == c:
 * the set of predicates met on the path "contains" the use's predicate
 * (Sec. 4, predicated instructions).  Guards are compared syntactically. */
static int covers(uint8_t g, uint8_t c) { return g == 0 || g == c; }

static uint8_t complement(uint8_t g) { return (g & 1) ? (uint8_t)(g + 1) : (uint8_t)(g - 1); }

/* Pair rule ({Pi} together with {!Pi} covers `_`): a guarded def k of x whose
 * previous def of x in the same block carries the complementary literal of
 * the same predicate completes a pair; returns that partner or -1. */
static int64_t partner_of(const orc_ctx *c, uint32_t k, uint32_t x) {
  const orc_prog *p = &c->p;
  uint8_t g = p->guard[k];
  if (g == 0) return -1;
  uint32_t start = first_of(c, c->block_of[k]);
  for (uint32_t q = k; q-- > start;) {
    if (def_of(p, q, x) >= 0) return p->guard[q] == complement(g) ? (int64_t)q : -1;
  }
  return -1;
}

static void push(orc_ctx *c, uint32_t *sp, uint32_t v) {
  if (*sp >= c->stack_cap) {
    c->stack_cap *= 2;
    c->stack = (uint32_t *)realloc(c->stack, sizeof(uint32_t) * c->stack_cap);
    if (!c->stack) abort();
  }
  c->stack[(*sp)++] = v;
}

/* the positions executed right before instruction k */
static void push_preds(orc_ctx *c, uint32_t *sp, uint32_t k) {
  uint32_t b = c->block_of[k];
  if (k > first_of(c, b)) {
    push(c, sp, k - 1);
    return;
  }
  for (uint32_t e = c->pred_ptr[b]; e < c->pred_ptr[b + 1]; ++e) push(c, sp, last_of(c, c->pred[e]));
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

typedef struct {
  uint32_t *v;
  uint32_t n, cap;
} vec32;

static void vpush(vec32 *a, uint32_t x) {
  if (a->n == a->cap) {
    a->cap = a->cap ? 2 * a->cap : 16;
    a->v = (uint32_t *)realloc(a->v, sizeof(uint32_t) * a->cap);
    if (!a->v) abort();
  }
  a->v[a->n++] = x;
}

/* Backward search for the use site u = (j, x, c), c = guard of j for an
 * operand use and `_` for a guard or wait use.  From the point right before
 * j, every path is followed backwards; a def of x met on the way is a
 * source; the path stops there if the def's guard covers c, or continues
 * only as far as the partner def if the def completes a complementary pair.
 * With `blocked`, a path also stops (without adding anything) at an
 * unpredicated instruction that uses x: a stall caused by an earlier def
 * would have been observed there first (dominator pruning).  Within one
 * instruction the def is looked at before the use, because the use reads
 * its operands before the def writes. */
static void search(orc_ctx *c, uint32_t u, int blocked, vec32 *out) {
  const orc_prog *p = &c->p;
  out->n = 0;
  /* instruction of the use site */
  uint32_t lo = 0, hi = p->n_instr;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (p->use_ptr[mid] <= u) lo = mid; else hi = mid;
  }
  uint32_t j = lo;
  uint32_t x = p->use_loc[u];
  uint8_t cond = p->use_kind[u] == ORC_USE_OPND ? p->guard[j] : 0;
  uint32_t st = next_stamp(c);
  uint32_t sp = 0;
  push_preds(c, &sp, j);
  while (sp) {
    uint32_t k = c->stack[--sp];
    if (c->stamp[k] == st) continue;
    c->stamp[k] = st;
    if (def_of(p, k, x) >= 0) {
      vpush(out, k);
      if (covers(p->guard[k], cond)) continue;
      int64_t partner = partner_of(c, k, x);
      if (partner >= 0) {
        for (uint32_t q = k - 1;; --q) {
          if (q == (uint32_t)partner) {
            vpush(out, q);
            break;
          }
          if (blocked && p->guard[q] == 0 && uses_loc(p, q, x)) break;
        }
        continue;
      }
    }
    if (blocked && p->guard[k] == 0 && uses_loc(p, k, x)) continue;
    push_preds(c, &sp, k);
  }
  qsort(out->v, out->n, sizeof(uint32_t), cmp_u32);
  uint32_t m = 0;
  for (uint32_t t = 0; t < out->n; ++t)
    if (m == 0 || out->v[m - 1] != out->v[t]) out->v[m++] = out->v[t];
  out->n = m;
}

uint32_t orc_sources(orc_ctx *c, uint32_t use_idx, int blocked, uint32_t *out, uint32_t cap) {
  vec32 v = {0, 0, 0};
  search(c, use_idx, blocked, &v);
  for (uint32_t t = 0; t < v.n && t < cap; ++t) out[t] = v.v[t];
  uint32_t n = v.n;
  free(v.v);
  return n;
}

/* ----------------------------------------------------------- distances */
/* Walk graph over instructions: k -> k+1 inside a block, last(b) -> first(s)
 * for every CFG successor s of b.  G' drops the retreating block edges. */

/* dmin for every target: breadth-first search from i over walks of at least
 * one edge; a walk of m edges has m-1 instructions strictly between.
 * dmax: longest walk in G', by dynamic programming over G' in topological
 * order; a target with no G' walk from i keeps dmax = dmin. */
static void dist_from(orc_ctx *c, uint32_t i, const uint32_t *tg, uint32_t nt, uint32_t *dmin,
                      uint32_t *dmax) {
  const orc_prog *p = &c->p;
  uint32_t st = next_stamp(c);
  /* mark targets */
  uint32_t left = 0;
  for (uint32_t t = 0; t < nt; ++t) {
    dmin[t] = ORC_NONE;
    dmax[t] = ORC_NONE;
  }
  /* BFS; qd holds walk lengths */
  uint32_t qh = 0, qt = 0;
  left = nt;
#define VISIT(w, dd)                         \
  do {                                       \
    if (c->stamp[(w)] != st) {               \
      c->stamp[(w)] = st;                    \
      c->queue[qt] = (w);                    \
      c->qd[qt] = (dd);                      \
      ++qt;                                  \
    }                                        \
  } while (0)
  {
    uint32_t b = c->block_of[i];
    if (i < last_of(c, b)) VISIT(i + 1, 1u);
    else
      for (uint32_t e = p->succ_ptr[b]; e < p->succ_ptr[b + 1]; ++e) VISIT(first_of(c, p->succ[e]), 1u);
  }
  while (qh < qt && left) {
    uint32_t v = c->queue[qh], d = c->qd[qh];
    ++qh;
    for (uint32_t t = 0; t < nt; ++t)
      if (tg[t] == v && dmin[t] == ORC_NONE) {
        dmin[t] = d - 1;
        --left;
      }
    uint32_t b = c->block_of[v];
    if (v < last_of(c, b)) VISIT(v + 1, d + 1);
    else
      for (uint32_t e = p->succ_ptr[b]; e < p->succ_ptr[b + 1]; ++e)
        VISIT(first_of(c, p->succ[e]), d + 1);
  }
#undef VISIT
  /* longest walk in G' */
  uint32_t maxpos = c->tpos[i];
  for (uint32_t t = 0; t < nt; ++t)
    if (c->tpos[tg[t]] > maxpos) maxpos = c->tpos[tg[t]];
  for (uint32_t pos = c->tpos[i]; pos <= maxpos; ++pos) c->len[c->topo[pos]] = -1;
  c->len[i] = 0;
  for (uint32_t pos = c->tpos[i]; pos < maxpos; ++pos) {
    uint32_t v = c->topo[pos];
    int32_t lv = c->len[v];
    if (lv < 0) continue;
    uint32_t b = c->block_of[v];
    if (v < last_of(c, b)) {
      if (c->len[v + 1] < lv + 1) c->len[v + 1] = lv + 1;
    } else {
      for (uint32_t e = p->succ_ptr[b]; e < p->succ_ptr[b + 1]; ++e) {
        if (c->retreat[e]) continue;
        uint32_t w = first_of(c, p->succ[e]);
        if (c->tpos[w] <= maxpos && c->len[w] < lv + 1) c->len[w] = lv + 1;
      }
    }
  }
  for (uint32_t t = 0; t < nt; ++t) {
    uint32_t j = tg[t];
    if (c->tpos[j] > c->tpos[i] && c->len[j] >= 1) dmax[t] = (uint32_t)(c->len[j] - 1);
    else dmax[t] = dmin[t];
  }
}

int orc_dist(orc_ctx *c, uint32_t i, uint32_t j, uint32_t *dmin, uint32_t *dmax) {
  dist_from(c, i, &j, 1, dmin, dmax);
  return *dmin != ORC_NONE;
}

/* ------------------------------------------------------------ analysis */
struct orc_analysis {
  orc_ctx *c;
  uint64_t n_rd, n_edges;
  uint32_t *rd_ptr, *rd_src;
  uint8_t *rd_blk;
  uint32_t *e_src, *e_dst, *e_dmin, *e_dmax;
  uint8_t *e_flags;
  uint32_t *in_ptr; /* edges into j: [in_ptr[j], in_ptr[j+1]) */
};

typedef struct {
  uint32_t src;
  uint8_t blk, nonrbar;
} cand_t;

static int cmp_cand(const void *a, const void *b) {
  uint32_t x = ((const cand_t *)a)->src, y = ((const cand_t *)b)->src;
  return (x > y) - (x < y);
}

orc_analysis *orc_analyze(orc_ctx *c) {
  const orc_prog *p = &c->p;
  orc_analysis *a = (orc_analysis *)calloc(1, sizeof(orc_analysis));
  a->c = c;
  uint32_t n = p->n_instr;
  uint32_t n_uses = p->use_ptr[n];
  vec32 full = {0, 0, 0}, blk = {0, 0, 0};
  /* per-use source lists */
  a->rd_ptr = (uint32_t *)xmalloc(sizeof(uint32_t) * (n_uses + 1));
  vec32 all = {0, 0, 0};
  vec32 allb = {0, 0, 0};
  a->rd_ptr[0] = 0;
  /* edges: gather per destination */
  cand_t *cands = NULL;
  size_t ncand = 0, capc = 0;
  vec32 esrc = {0, 0, 0}, edst = {0, 0, 0}, eflag = {0, 0, 0};
  a->in_ptr = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  for (uint32_t j = 0; j < n; ++j) {
    ncand = 0;
    a->in_ptr[j] = esrc.n;
    for (uint32_t u = p->use_ptr[j]; u < p->use_ptr[j + 1]; ++u) {
      uint32_t x = p->use_loc[u];
      search(c, u, 0, &full);
      search(c, u, 1, &blk);
      uint32_t bi = 0;
      for (uint32_t t = 0; t < full.n; ++t) {
        uint32_t i = full.v[t];
        while (bi < blk.n && blk.v[bi] < i) ++bi;
        uint8_t inb = (uint8_t)(bi < blk.n && blk.v[bi] == i);
        vpush(&all, i);
        vpush(&allb, inb);
        int64_t d = def_of(p, i, x);
        if (ncand == capc) {
          capc = capc ? 2 * capc : 64;
          cands = (cand_t *)realloc(cands, sizeof(cand_t) * capc);
          if (!cands) abort();
        }
        cands[ncand].src = i;
        cands[ncand].blk = inb;
        cands[ncand].nonrbar = (uint8_t)(p->def_kind[d] != ORC_DEF_RBAR);
        ++ncand;
      }
      a->rd_ptr[u + 1] = all.n;
    }
    /* one edge per (i, j): kept by dominance if any carrying location keeps
     * it; write-after-read only if every carrying location is a read
     * barrier of i */
    if (ncand) qsort(cands, ncand, sizeof(cand_t), cmp_cand);
    for (size_t t = 0; t < ncand;) {
      size_t s = t;
      uint8_t bk = 0, nr = 0;
      while (t < ncand && cands[t].src == cands[s].src) {
        bk |= cands[t].blk;
        nr |= cands[t].nonrbar;
        ++t;
      }
      vpush(&esrc, cands[s].src);
      vpush(&edst, j);
      vpush(&eflag, (uint32_t)((bk ? ORC_E_DOM_KEEP : 0) | (nr ? 0 : ORC_E_WAR)));
    }
  }
  a->in_ptr[n] = esrc.n;
  free(cands);
  free(full.v);
  free(blk.v);
  a->n_rd = all.n;
  a->rd_src = all.v;
  a->rd_blk = (uint8_t *)xmalloc(all.n + 1);
  for (uint32_t t = 0; t < all.n; ++t) a->rd_blk[t] = (uint8_t)allb.v[t];
  free(allb.v);
  a->n_edges = esrc.n;
  a->e_src = esrc.v;
  a->e_dst = edst.v;
  a->e_flags = (uint8_t *)xmalloc(esrc.n + 1);
  for (uint32_t t = 0; t < esrc.n; ++t) a->e_flags[t] = (uint8_t)eflag.v[t];
  free(eflag.v);
  /* distances, grouped by source instruction */
  uint64_t ne = a->n_edges;
  a->e_dmin = (uint32_t *)xmalloc(sizeof(uint32_t) * (ne + 1));
  a->e_dmax = (uint32_t *)xmalloc(sizeof(uint32_t) * (ne + 1));
  uint32_t *cnt = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
  for (uint64_t e = 0; e < ne; ++e) cnt[a->e_src[e] + 1] += 1;
  for (uint32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  uint32_t *by_src = (uint32_t *)xmalloc(sizeof(uint32_t) * (ne + 1));
  uint32_t *pos = (uint32_t *)xmalloc(sizeof(uint32_t) * (n + 1));
  memcpy(pos, cnt, sizeof(uint32_t) * (n + 1));
  for (uint64_t e = 0; e < ne; ++e) by_src[pos[a->e_src[e]]++] = (uint32_t)e;
  uint32_t *tg = (uint32_t *)xmalloc(sizeof(uint32_t) * (ne + 1));
  uint32_t *d0 = (uint32_t *)xmalloc(sizeof(uint32_t) * (ne + 1));
  uint32_t *d1 = (uint32_t *)xmalloc(sizeof(uint32_t) * (ne + 1));
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t k0 = cnt[i], k1 = cnt[i + 1];
    if (k0 == k1) continue;
    for (uint32_t k = k0; k < k1; ++k) tg[k - k0] = a->e_dst[by_src[k]];
    dist_from(c, i, tg, k1 - k0, d0, d1);
    for (uint32_t k = k0; k < k1; ++k) {
      uint32_t e = by_src[k];
      a->e_dmin[e] = d0[k - k0];
      a->e_dmax[e] = d1[k - k0];
      /* latency pruning: keep iff some CFG path from i to j holds at most
       * lat[class(i)] instructions */
      if (d0[k - k0] <= p->lat[p->op_class[i]]) a->e_flags[e] |= ORC_E_LAT_KEEP;
    }
  }
  free(cnt);
  free(by_src);
  free(pos);
  free(tg);
  free(d0);
  free(d1);
  return a;
}

void orc_analysis_free(orc_analysis *a) {
  if (!a) return;
  free(a->rd_ptr);
  free(a->rd_src);
  free(a->rd_blk);
  free(a->e_src);
  free(a->e_dst);
  free(a->e_flags);
  free(a->e_dmin);
  free(a->e_dmax);
  free(a->in_ptr);
  free(a);
}

void orc_analysis_sizes(const orc_analysis *a, uint64_t *n_rd, uint64_t *n_edges) {
  *n_rd = a->n_rd;
  *n_edges = a->n_edges;
}

void orc_analysis_rd(const orc_analysis *a, uint32_t *rd_ptr, uint32_t *rd_src, uint8_t *rd_blk) {
  uint32_t n_uses = a->c->p.use_ptr[a->c->p.n_instr];
  memcpy(rd_ptr, a->rd_ptr, sizeof(uint32_t) * (n_uses + 1));
  if (a->n_rd) {
    memcpy(rd_src, a->rd_src, sizeof(uint32_t) * a->n_rd);
    memcpy(rd_blk, a->rd_blk, a->n_rd);
  }
}

void orc_analysis_edges(const orc_analysis *a, uint32_t *src, uint32_t *dst, uint8_t *flags,
                        uint32_t *dmin, uint32_t *dmax) {
  size_t ne = a->n_edges;
  if (!ne) return;
  memcpy(src, a->e_src, 4 * ne);
  memcpy(dst, a->e_dst, 4 * ne);
  memcpy(flags, a->e_flags, ne);
  memcpy(dmin, a->e_dmin, 4 * ne);
  memcpy(dmax, a->e_dmax, 4 * ne);
}

/* --------------------------------------------------------------- blame */
static uint32_t popcount32(uint32_t v) {
  uint32_t n = 0;
  while (v) {
    n += v & 1u;
    v >>= 1;
  }
  return n;
}

/* share slot of a blamable reason r: its rank among the blamable reasons */
static int reason_slot(uint32_t blamable, uint32_t r) {
  if (!((blamable >> r) & 1u)) return -1;
  return (int)popcount32(blamable & ((1u << r) - 1u));
}

static int fine_class(uint32_t r, uint8_t cls, int war) {
  if (r == ORC_MEM_DEP) {
    if (cls == ORC_LOCAL_LOAD || cls == ORC_LOCAL_STORE) return ORC_F_MEM_LOCAL;
    if (cls == ORC_CONST_LOAD) return ORC_F_MEM_CONST;
    return ORC_F_MEM_GLOBAL;
  }
  if (r == ORC_EXEC_DEP) {
    if (war) return ORC_F_EXEC_WAR;
    if (cls == ORC_SHARED_LOAD) return ORC_F_EXEC_SHARED;
    return ORC_F_EXEC_ARITH;
  }
  if (r == ORC_SYNC) return ORC_F_SYNC;
  return ORC_F_OTHER;
}

/* For every sampled instruction j, blamable reason r and latency bit l with
 * S = C[j][r][l] > 0: the incoming edges that survive dominator and latency
 * pruning and whose source opcode class may cause r (opcode pruning) are
 * the candidates.  Eq. (1): S_i = S * R_path(i) R_issue(i) / sum_k (...),
 * with R_issue(i) proportional to the issued samples of i and R_path(i) to
 * 1/(dmax+1) (the longer the longest path, the less blame); when no
 * candidate has issued samples only R_path is used.  No candidate: the
 * stalls stay on j.  Non-blamable reasons stay on j. */
void orc_blame(const orc_analysis *a, const uint32_t *C, double *share, double *blamed,
               double *self_, double *fine) {
  const orc_prog *p = &a->c->p;
  uint32_t n = p->n_instr;
  uint32_t nbl = popcount32(p->blamable & 0xFFFu);
  memset(share, 0, sizeof(double) * a->n_edges * nbl * 2);
  memset(blamed, 0, sizeof(double) * (size_t)n * 24);
  memset(self_, 0, sizeof(double) * (size_t)n * 24);
  memset(fine, 0, sizeof(double) * (size_t)n * ORC_N_FINE * 2);
  for (uint32_t j = 0; j < n; ++j) {
    uint32_t e0 = a->in_ptr[j], e1 = a->in_ptr[j + 1];
    for (uint32_t r = 0; r < 12; ++r) {
      for (uint32_t l = 0; l < 2; ++l) {
        uint32_t S = C[((size_t)j * 12 + r) * 2 + l];
        if (S == 0) continue;
        int slot = reason_slot(p->blamable, r);
        if (slot < 0) {
          self_[((size_t)j * 12 + r) * 2 + l] += S;
          continue;
        }
        /* candidates and their weights */
        double W = 0.0;
        uint32_t ncand = 0;
        for (uint32_t e = e0; e < e1; ++e) {
          uint32_t i = a->e_src[e];
          if (!(a->e_flags[e] & ORC_E_DOM_KEEP) || !(a->e_flags[e] & ORC_E_LAT_KEEP)) continue;
          if (!((p->allowed[r] >> p->op_class[i]) & 1u)) continue;
          ++ncand;
          double issued = (double)C[((size_t)i * 12 + ORC_SELECTED) * 2 + 0] +
                          (double)C[((size_t)i * 12 + ORC_SELECTED) * 2 + 1];
          W += issued / ((double)a->e_dmax[e] + 1.0);
        }
        if (ncand == 0) {
          self_[((size_t)j * 12 + r) * 2 + l] += S;
          continue;
        }
        int by_path_only = (W == 0.0);
        if (by_path_only) {
          for (uint32_t e = e0; e < e1; ++e) {
            uint32_t i = a->e_src[e];
            if (!(a->e_flags[e] & ORC_E_DOM_KEEP) || !(a->e_flags[e] & ORC_E_LAT_KEEP)) continue;
            if (!((p->allowed[r] >> p->op_class[i]) & 1u)) continue;
            W += 1.0 / ((double)a->e_dmax[e] + 1.0);
          }
        }
        for (uint32_t e = e0; e < e1; ++e) {
          uint32_t i = a->e_src[e];
          if (!(a->e_flags[e] & ORC_E_DOM_KEEP) || !(a->e_flags[e] & ORC_E_LAT_KEEP)) continue;
          if (!((p->allowed[r] >> p->op_class[i]) & 1u)) continue;
          double issued = (double)C[((size_t)i * 12 + ORC_SELECTED) * 2 + 0] +
                          (double)C[((size_t)i * 12 + ORC_SELECTED) * 2 + 1];
          double w = by_path_only ? 1.0 / ((double)a->e_dmax[e] + 1.0)
                                  : issued / ((double)a->e_dmax[e] + 1.0);
          double s = (double)S * w / W;
          share[((size_t)e * nbl + (uint32_t)slot) * 2 + l] = s;
          blamed[((size_t)i * 12 + r) * 2 + l] += s;
          int fc = fine_class(r, p->op_class[i], (a->e_flags[e] & ORC_E_WAR) != 0);
          fine[((size_t)i * ORC_N_FINE + (uint32_t)fc) * 2 + l] += s;
        }
      }
    }
  }
}

/* ------------------------------------------------------------ estimates */
static uint32_t root_of_scope(const orc_prog *p, uint32_t s) {
  while (p->scope_parent[s] != ORC_NONE) s = p->scope_parent[s];
  return s;
}

static int is_anc(const orc_prog *p, uint32_t anc, uint32_t s) {
  for (;;) {
    if (s == anc) return 1;
    if (p->scope_parent[s] == ORC_NONE) return 0;
    s = p->scope_parent[s];
  }
}

static uint32_t lca(const orc_prog *p, uint32_t s, uint32_t t) {
  for (uint32_t a = s;; a = p->scope_parent[a]) {
    if (is_anc(p, a, t)) return a;
    if (p->scope_parent[a] == ORC_NONE) return ORC_NONE;
  }
}

/* innermost LOOP scope enclosing both, not looking above the scope of the
 * CFG function the two instructions belong to */
static uint32_t common_loop(const orc_prog *p, uint32_t s, uint32_t t, uint32_t fscope) {
  uint32_t a = lca(p, s, t);
  while (a != ORC_NONE) {
    if (p->scope_kind[a] == ORC_SCOPE_LOOP) return a;
    if (a == fscope) return ORC_NONE;
    a = p->scope_parent[a];
  }
  return ORC_NONE;
}

/* some FUNCTION scope above s carries the flag(s) in mask (all of them) */
static int in_function_with(const orc_prog *p, uint32_t s, uint8_t mask) {
  for (;;) {
    if (p->scope_kind[s] == ORC_SCOPE_FUNCTION && (p->scope_flags[s] & mask) == mask) return 1;
    if (p->scope_parent[s] == ORC_NONE) return 0;
    s = p->scope_parent[s];
  }
}

/* add v to scope s and every scope above it: afterwards m[l] is the sum over
 * the subtree of l, the nested(l) of Eq. (5) */
static void add_up(const orc_prog *p, double *m, uint32_t stride, uint32_t off, uint32_t s,
                   double v) {
  for (;;) {
    m[(size_t)s * stride + off] += v;
    if (p->scope_parent[s] == ORC_NONE) return;
    s = p->scope_parent[s];
  }
}

typedef struct {
  double sp;
  uint32_t opt, scope;
} rank_t;

static int cmp_rank(const void *a, const void *b) {
  const rank_t *x = (const rank_t *)a, *y = (const rank_t *)b;
  if (x->sp != y->sp) return x->sp > y->sp ? -1 : 1;
  if (x->opt != y->opt) return x->opt < y->opt ? -1 : 1;
  return (x->scope > y->scope) - (x->scope < y->scope);
}

void orc_estimate(const orc_analysis *a, const uint32_t *C, const double *share,
                  const double *blamed, const double *self_, double *active, double *matched,
                  double *speedup, uint32_t *root_of, double *kernel_T, double *kernel_L,
                  double *eq3, uint32_t k, uint32_t *top_opt, uint32_t *top_scope,
                  double *top_speed) {
  const orc_prog *p = &a->c->p;
  const orc_ctx *c = a->c;
  uint32_t n = p->n_instr, ns = p->n_scopes;
  uint32_t nbl = popcount32(p->blamable & 0xFFFu);
  int s_mem = reason_slot(p->blamable, ORC_MEM_DEP);
  int s_exec = reason_slot(p->blamable, ORC_EXEC_DEP);
  memset(active, 0, sizeof(double) * ns);
  memset(matched, 0, sizeof(double) * ns * ORC_N_OPT);
  memset(kernel_T, 0, sizeof(double) * ns);
  memset(kernel_L, 0, sizeof(double) * ns);
  memset(eq3, 0, sizeof(double) * ns * 3);
  for (uint32_t s = 0; s < ns; ++s) root_of[s] = root_of_scope(p, s);
#define CNT(j, r, l) ((double)C[((size_t)(j) * 12 + (r)) * 2 + (l)])
  /* T, L per kernel (Sec. 2.1: T = A + L) and A per scope subtree */
  for (uint32_t j = 0; j < n; ++j) {
    uint32_t s = p->instr_scope[j];
    double tot = 0.0, lat = 0.0, act = 0.0;
    for (uint32_t r = 0; r < 12; ++r) {
      act += CNT(j, r, 0);
      lat += CNT(j, r, 1);
    }
    tot = act + lat;
    kernel_T[root_of[s]] += tot;
    kernel_L[root_of[s]] += lat;
    add_up(p, active, 1, 0, s, act);
  }
  /* matched samples of the code optimizers (Table 2) */
  for (uint32_t j = 0; j < n; ++j) {
    uint32_t s = p->instr_scope[j];
    uint8_t cls = p->op_class[j];
    /* Register Reuse: memory dependency stalls blamed on local memory instructions */
    if (cls == ORC_LOCAL_LOAD || cls == ORC_LOCAL_STORE)
      add_up(p, matched, ORC_N_OPT, ORC_O_REG_REUSE, s,
             blamed[((size_t)j * 12 + ORC_MEM_DEP) * 2] + blamed[((size_t)j * 12 + ORC_MEM_DEP) * 2 + 1]);
    /* Strength Reduction: execution dependency stalls blamed on long-latency arithmetic */
    if (cls == ORC_FP64 || cls == ORC_LONG_ALU)
      add_up(p, matched, ORC_N_OPT, ORC_O_STRENGTH, s,
             blamed[((size_t)j * 12 + ORC_EXEC_DEP) * 2] + blamed[((size_t)j * 12 + ORC_EXEC_DEP) * 2 + 1]);
    /* Function Split: instruction fetch stalls */
    add_up(p, matched, ORC_N_OPT, ORC_O_FUNC_SPLIT, s, CNT(j, ORC_INST_FETCH, 0) + CNT(j, ORC_INST_FETCH, 1));
    /* Fast Math: stall samples inside math functions */
    if (in_function_with(p, s, ORC_SF_MATH)) {
      double v = 0.0;
      for (uint32_t r = 0; r < 12; ++r)
        if (r != ORC_SELECTED) v += CNT(j, r, 0) + CNT(j, r, 1);
      add_up(p, matched, ORC_N_OPT, ORC_O_FAST_MATH, s, v);
    }
    /* Warp Balance: synchronization stalls, blamed on sources or kept */
    add_up(p, matched, ORC_N_OPT, ORC_O_WARP_BAL, s,
           blamed[((size_t)j * 12 + ORC_SYNC) * 2] + blamed[((size_t)j * 12 + ORC_SYNC) * 2 + 1] +
               self_[((size_t)j * 12 + ORC_SYNC) * 2] + self_[((size_t)j * 12 + ORC_SYNC) * 2 + 1]);
    /* Memory Transaction Reduction: throttling stalls on global memory instructions */
    if (cls == ORC_GLOBAL_LOAD || cls == ORC_GLOBAL_STORE)
      add_up(p, matched, ORC_N_OPT, ORC_O_MEM_TRANS, s, CNT(j, ORC_MEM_THROTTLE, 0) + CNT(j, ORC_MEM_THROTTLE, 1));
    /* Function Inlining: latency samples inside (non-inlined) device functions or at calls */
    if (cls == ORC_CALL || in_function_with(p, s, ORC_SF_DEVICE | ORC_SF_CFG)) {
      double v = 0.0;
      for (uint32_t r = 0; r < 12; ++r) v += CNT(j, r, 1);
      add_up(p, matched, ORC_N_OPT, ORC_O_INLINE, s, v);
    }
  }
  /* Loop Unrolling and Code Reordering: latency samples of global memory and
   * execution dependency stalls attributed along an edge i -> j; unrolling
   * needs a loop holding both ends */
  for (uint64_t e = 0; e < a->n_edges; ++e) {
    uint32_t i = a->e_src[e], j = a->e_dst[e];
    double v = 0.0;
    if (s_mem >= 0 && p->op_class[i] == ORC_GLOBAL_LOAD) v += share[((size_t)e * nbl + (uint32_t)s_mem) * 2 + 1];
    if (s_exec >= 0) v += share[((size_t)e * nbl + (uint32_t)s_exec) * 2 + 1];
    uint32_t si = p->instr_scope[i], sj = p->instr_scope[j];
    uint32_t fscope = p->func_scope[c->func_of_block[c->block_of[i]]];
    uint32_t loop = common_loop(p, si, sj, fscope);
    if (loop != ORC_NONE) add_up(p, matched, ORC_N_OPT, ORC_O_LOOP_UNROLL, loop, v);
    add_up(p, matched, ORC_N_OPT, ORC_O_REORDER, lca(p, si, sj), v);
  }
  /* Eq. (2) for stall elimination, Eq. (5) (Eq. (4) at the kernel scope)
   * for latency hiding; T is the kernel's total.  Removing x >= T of the
   * kernel's T samples gives +inf (the formula would divide by zero, or by
   * a negative number when rounding in the share sums puts x above T). */
  for (uint32_t s = 0; s < ns; ++s) {
    double T = kernel_T[root_of[s]];
    for (uint32_t o = 0; o < ORC_N_OPT; ++o) {
      double M = matched[(size_t)s * ORC_N_OPT + o];
      double x = (o >= ORC_O_LOOP_UNROLL) ? (active[s] < M ? active[s] : M) : M;
      double sp = (T == 0.0) ? 1.0 : (x >= T ? INFINITY : T / (T - x));
      speedup[(size_t)s * ORC_N_OPT + o] = sp;
    }
    if (p->scope_parent[s] == ORC_NONE) {
      for (uint32_t h = 0; h < 3; ++h) {
        double M = matched[(size_t)s * ORC_N_OPT + ORC_O_LOOP_UNROLL + h];
        eq3[(size_t)s * 3 + h] = (T == 0.0) ? 1.0 : (M >= T ? INFINITY : T / (T - M));
      }
    }
  }
  /* top-k per kernel: speedup descending, optimizer ascending, scope ascending */
  rank_t *buf = (rank_t *)xmalloc(sizeof(rank_t) * ((size_t)ns * ORC_N_OPT + 1));
  for (size_t t = 0; t < (size_t)ns * k; ++t) {
    top_opt[t] = ORC_NONE;
    top_scope[t] = ORC_NONE;
    top_speed[t] = 0.0;
  }
  for (uint32_t r = 0; r < ns; ++r) {
    if (p->scope_parent[r] != ORC_NONE) continue;
    size_t m = 0;
    for (uint32_t s = 0; s < ns; ++s) {
      if (root_of[s] != r) continue;
      for (uint32_t o = 0; o < ORC_N_OPT; ++o) {
        buf[m].sp = speedup[(size_t)s * ORC_N_OPT + o];
        buf[m].opt = o;
        buf[m].scope = s;
        ++m;
      }
    }
    qsort(buf, m, sizeof(rank_t), cmp_rank);
    for (uint32_t t = 0; t < k && t < m; ++t) {
      top_opt[(size_t)r * k + t] = buf[t].opt;
      top_scope[(size_t)r * k + t] = buf[t].scope;
      top_speed[(size_t)r * k + t] = buf[t].sp;
    }
  }
  free(buf);
#undef CNT
}

/* ------------------------------------------------- parallel optimizers */
/* Sec. 5.2, Eqs. (6)-(10), with the readings the library documents for
 * the new configurations and the factor f (the paper leaves them open).
 * launch = {blocks, threads per block, registers per thread (0: none),
 * shared bytes per block (0: none)}; device = {SMs, schedulers per SM,
 * warp size, max warps per SM, max blocks per SM, max threads per block,
 * registers per SM, shared bytes per SM}.  out[11*o + k] for o = 0 (Block
 * Increase), 1 (Thread Increase): k = 0 matched, 1 W, 2 W_new, 3 R_I, 4 I,
 * 5 I_new, 6 C_W, 7 C_I, 8 f, 9 speedup, 10 unused. */
static double orc_issue(double r, double w) { return 1.0 - pow(1.0 - r, w); }

void orc_parallel(const orc_analysis *a, const uint32_t *C, uint32_t root, const uint32_t *launch,
                  const uint32_t *device, double *out) {
  const orc_prog *p = &a->c->p;
  double T = 0.0, issued = 0.0, contention = 0.0;
  for (uint32_t j = 0; j < p->n_instr; ++j) {
    if (root_of_scope(p, p->instr_scope[j]) != root) continue;
    for (uint32_t r = 0; r < 12; ++r) {
      double v = (double)C[((size_t)j * 12 + r) * 2] + (double)C[((size_t)j * 12 + r) * 2 + 1];
      T += v;
      if (r == ORC_SELECTED) issued += v;
      if (r == ORC_PIPE_BUSY || r == ORC_MEM_THROTTLE || r == ORC_NOT_SELECTED) contention += v;
    }
  }
  uint32_t blocks = launch[0], threads = launch[1], regs = launch[2], shared = launch[3];
  uint32_t sms = device[0], sched = device[1], warp = device[2], max_warps = device[3];
  uint32_t max_blocks = device[4], regs_sm = device[6], shared_sm = device[7];
  /* occupancy: the smallest of the per-SM limits, and of the grid's share */
  uint32_t wpb = (threads + warp - 1) / warp;
  uint64_t lim_blocks = max_blocks;
  uint64_t lim_warps = max_warps / wpb;
  uint64_t lim_regs = regs ? regs_sm / ((uint64_t)regs * warp * wpb) : UINT64_MAX;
  uint64_t lim_shared = shared ? shared_sm / shared : UINT64_MAX;
  uint64_t per_sm = lim_blocks;
  if (lim_warps < per_sm) per_sm = lim_warps;
  if (lim_regs < per_sm) per_sm = lim_regs;
  if (lim_shared < per_sm) per_sm = lim_shared;
  uint64_t grid_share = ((uint64_t)blocks + sms - 1) / sms;
  uint64_t resident = per_sm < grid_share ? per_sm : grid_share;
  double W = (double)resident * wpb / sched;
  double R = T > 0.0 ? issued / T : 0.0;
  for (int o = 0; o < 2; ++o) {
    double *e = out + 11 * o;
    int matched;
    double W_new, f;
    if (o == 0) {
      /* Block Increase: fewer blocks than SMs; spread over one per SM */
      matched = blocks < sms;
      W_new = matched ? W * (double)blocks / sms : W;
      f = (matched && W_new < 1.0 && T > contention) ? T / (T - contention) : 1.0;
    } else {
      /* Thread Increase: the block cap is the binding limit and leaves warps */
      uint64_t other = lim_warps;
      if (lim_regs < other) other = lim_regs;
      if (lim_shared < other) other = lim_shared;
      uint64_t warps_now = resident * wpb;
      matched = lim_blocks < other && resident == lim_blocks && warps_now < max_warps;
      W_new = W;
      if (matched) {
        uint64_t hold = max_warps;
        if (regs && regs_sm / ((uint64_t)regs * warp) < hold) hold = regs_sm / ((uint64_t)regs * warp);
        if (shared && (uint64_t)shared_sm * wpb / shared < hold) hold = (uint64_t)shared_sm * wpb / shared;
        uint64_t grid_warps = ((uint64_t)blocks * wpb + sms - 1) / sms;
        if (grid_warps < hold) hold = grid_warps;
        if (hold < warps_now) hold = warps_now;
        W_new = (double)hold / sched;
      }
      f = W > 0.0 ? W_new / W : 1.0;
    }
    double I = orc_issue(R, W), I_new = orc_issue(R, W_new);
    double C_W = W > 0.0 ? W_new / W : 1.0;      /* Eq. (6) */
    double C_I = I > 0.0 ? I_new / I : 1.0;      /* Eq. (7) */
    e[0] = matched;
    e[1] = W;
    e[2] = W_new;
    e[3] = R;
    e[4] = I;
    e[5] = I_new;
    e[6] = C_W;
    e[7] = C_I;
    e[8] = f;
    e[9] = (matched && T > 0.0 && I > 0.0 && C_W > 0.0) ? (1.0 / C_W) * C_I * f : 1.0;  /* Eq. (10) */
    e[10] = 0.0;
  }
}

/* -------------------------------------------------------------- report */
/* Single dependency coverage (Sec. 6): an instruction is a single
 * dependency node when no use site of it has two or more sources; before
 * pruning all its reaching definitions count, after pruning only those that
 * survive the dominator rule for that use and the latency rule for their
 * edge (the opcode rule depends on the stall reason and is left out). */
void orc_coverage(const orc_analysis *a, uint64_t *before, uint64_t *after) {
  const orc_prog *p = &a->c->p;
  uint64_t nb = 0, na = 0;
  for (uint32_t j = 0; j < p->n_instr; ++j) {
    int single_before = 1, single_after = 1;
    for (uint32_t u = p->use_ptr[j]; u < p->use_ptr[j + 1]; ++u) {
      uint32_t all = a->rd_ptr[u + 1] - a->rd_ptr[u], kept = 0;
      for (uint32_t q = a->rd_ptr[u]; q < a->rd_ptr[u + 1]; ++q) {
        if (!a->rd_blk[q]) continue;
        for (uint32_t e = a->in_ptr[j]; e < a->in_ptr[j + 1]; ++e)
          if (a->e_src[e] == a->rd_src[q] && (a->e_flags[e] & ORC_E_LAT_KEEP)) ++kept;
      }
      if (all > 1) single_before = 0;
      if (kept > 1) single_after = 0;
    }
    nb += (uint64_t)single_before;
    na += (uint64_t)single_after;
  }
  *before = nb;
  *after = na;
}

typedef struct {
  uint32_t src, dst, dmin, dmax;
  double v;
} orc_spot;

static int cmp_spot(const void *x, const void *y) {
  const orc_spot *a = (const orc_spot *)x, *b = (const orc_spot *)y;
  if (a->v != b->v) return a->v > b->v ? -1 : 1;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  return (a->dst > b->dst) - (a->dst < b->dst);
}

/* Hotspots of optimizer `opt` in the kernel rooted at scope `root`: the
 * edges (src, dst) or instructions (src = ORC_NONE) carrying its matched
 * samples, Table 2's matching as in orc_estimate, largest first (ties by
 * src, then dst).  Writes up to k rows of out[5] = {src, dst, dmin, dmax,
 * samples} and returns how many. */
uint32_t orc_hotspots(const orc_analysis *a, const uint32_t *C, const double *share,
                      const double *self_, uint32_t root, uint32_t opt, uint32_t k, double *out) {
  const orc_prog *p = &a->c->p;
  uint32_t nbl = popcount32(p->blamable & 0xFFFu);
  int s_mem = reason_slot(p->blamable, ORC_MEM_DEP);
  int s_exec = reason_slot(p->blamable, ORC_EXEC_DEP);
  int s_sync = reason_slot(p->blamable, ORC_SYNC);
  orc_spot *all = (orc_spot *)xmalloc(sizeof(orc_spot) * ((size_t)a->n_edges + p->n_instr + 1));
  size_t m = 0;
#define SH(e, slot, l) ((slot) < 0 ? 0.0 : share[((size_t)(e) * nbl + (uint32_t)(slot)) * 2 + (l)])
  for (uint64_t e = 0; e < a->n_edges; ++e) {
    uint32_t i = a->e_src[e], j = a->e_dst[e];
    if (root_of_scope(p, p->instr_scope[j]) != root) continue;
    uint8_t ci = p->op_class[i];
    double v = 0.0;
    if (opt == ORC_O_REG_REUSE && (ci == ORC_LOCAL_LOAD || ci == ORC_LOCAL_STORE))
      v = SH(e, s_mem, 0) + SH(e, s_mem, 1);
    if (opt == ORC_O_STRENGTH && (ci == ORC_FP64 || ci == ORC_LONG_ALU))
      v = SH(e, s_exec, 0) + SH(e, s_exec, 1);
    if (opt == ORC_O_WARP_BAL) v = SH(e, s_sync, 0) + SH(e, s_sync, 1);
    if (opt == ORC_O_LOOP_UNROLL || opt == ORC_O_REORDER) {
      v = (ci == ORC_GLOBAL_LOAD ? SH(e, s_mem, 1) : 0.0) + SH(e, s_exec, 1);
      if (opt == ORC_O_LOOP_UNROLL) {
        uint32_t fscope = p->func_scope[a->c->func_of_block[a->c->block_of[i]]];
        if (common_loop(p, p->instr_scope[i], p->instr_scope[j], fscope) == ORC_NONE) v = 0.0;
      }
    }
    if (v > 0.0) {
      all[m].src = i;
      all[m].dst = j;
      all[m].dmin = a->e_dmin[e];
      all[m].dmax = a->e_dmax[e];
      all[m].v = v;
      ++m;
    }
  }
#undef SH
  for (uint32_t j = 0; j < p->n_instr; ++j) {
    uint32_t s = p->instr_scope[j];
    if (root_of_scope(p, s) != root) continue;
    uint8_t cj = p->op_class[j];
    double v = 0.0;
    if (opt == ORC_O_FUNC_SPLIT) v = (double)C[((size_t)j * 12 + ORC_INST_FETCH) * 2] +
                                     (double)C[((size_t)j * 12 + ORC_INST_FETCH) * 2 + 1];
    if (opt == ORC_O_FAST_MATH && in_function_with(p, s, ORC_SF_MATH))
      for (uint32_t r = 0; r < 12; ++r)
        if (r != ORC_SELECTED)
          v += (double)C[((size_t)j * 12 + r) * 2] + (double)C[((size_t)j * 12 + r) * 2 + 1];
    if (opt == ORC_O_WARP_BAL)
      v = self_[((size_t)j * 12 + ORC_SYNC) * 2] + self_[((size_t)j * 12 + ORC_SYNC) * 2 + 1];
    if (opt == ORC_O_MEM_TRANS && (cj == ORC_GLOBAL_LOAD || cj == ORC_GLOBAL_STORE))
      v = (double)C[((size_t)j * 12 + ORC_MEM_THROTTLE) * 2] +
          (double)C[((size_t)j * 12 + ORC_MEM_THROTTLE) * 2 + 1];
    if (opt == ORC_O_INLINE && (cj == ORC_CALL || in_function_with(p, s, ORC_SF_DEVICE | ORC_SF_CFG)))
      for (uint32_t r = 0; r < 12; ++r) v += (double)C[((size_t)j * 12 + r) * 2 + 1];
    if (v > 0.0) {
      all[m].src = ORC_NONE;
      all[m].dst = j;
      all[m].dmin = 0;
      all[m].dmax = 0;
      all[m].v = v;
      ++m;
    }
  }
  qsort(all, m, sizeof(orc_spot), cmp_spot);
  uint32_t n = (uint32_t)(m < k ? m : k);
  for (uint32_t t = 0; t < n; ++t) {
    out[5 * t] = all[t].src;
    out[5 * t + 1] = all[t].dst;
    out[5 * t + 2] = all[t].dmin;
    out[5 * t + 3] = all[t].dmax;
    out[5 * t + 4] = all[t].v;
  }
  free(all);
  return n;
}
