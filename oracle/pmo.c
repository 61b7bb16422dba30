/*
 * pmo.c -- CPU oracle for hierarchical process mapping (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, single-threaded C written from the
 * paper "GPU-Accelerated Algorithms for Process Mapping" (arXiv 2510.12196).
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Every parallel loop of the paper is executed here as a synchronous round:
 * it reads the state as it was when the loop started and its writes become
 * visible only after the loop.  Every list filled through an atomic index in
 * the paper is a set here (a flag per vertex), and every running sum that the
 * paper accumulates through atomics is an exclusive prefix in vertex-id order.
 * The readings taken where the paper is silent or ambiguous are listed at
 * each function.
 *
 * Parity unpinned (fixed only by this file; no closed form or printed value
 * reaches them): the breadth-first split used as initial partitioner (beyond
 * its closed-form cases: a path, a star, two interleaved components), and the
 * coarsening stop on stalls (the 8k threshold itself is pinned).
 */
#include "pmo.h"

#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <math.h>

#define NOT_IN_X INT64_MIN

static void *xmalloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) abort();
  return p;
}
static void *xcalloc(size_t count, size_t size) {
  void *p = calloc(count ? count : 1, size ? size : 1);
  if (!p) abort();
  return p;
}

static double now_seconds(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ======================================================================
 * Hierarchy and objective (Section 2, "hierarchical process mapping")
 * ====================================================================== */

int64_t pmo_num_pes(int32_t levels, const int32_t *a) {
  int64_t k = 1;
  for (int32_t i = 0; i < levels; ++i) k *= a[i];
  return k;
}

/* D(x,y): the hierarchy a_1:...:a_l groups a_1 PEs into a processor, a_2
 * processors into a node, and so on; PEs that first share a component at
 * level j communicate at cost d_j.  PEs are numbered so that a_1 is the least
 * significant mixed-radix digit, i.e. x and y share their level-j component
 * iff floor(x/P_j) == floor(y/P_j) with P_j = a_1*...*a_j.  A PE with itself
 * costs 0 (co-located tasks do not communicate over the machine). */
int32_t pmo_distance(int32_t levels, const int32_t *a, const int32_t *d,
                     int32_t x, int32_t y) {
  if (x == y) return 0;
  int64_t p = 1;
  for (int32_t i = 0; i < levels; ++i) {
    p *= a[i];
    if ((int64_t)x / p == (int64_t)y / p) return d[i];
  }
  return d[levels - 1];
}

/* J(C, D, Pi) = sum over ordered pairs (i,j) of C_ij * D(Pi(i), Pi(j))
 * (Section 2, definition of GPMP).  With both directions of every edge
 * stored, this is the sum over all CSR arcs; it counts each undirected edge
 * twice. */
int64_t pmo_comm_cost(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                      const int32_t *adjwgt, const int32_t *part,
                      int32_t levels, const int32_t *a, const int32_t *d) {
  int64_t j = 0;
  for (int32_t v = 0; v < n; ++v)
    for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e)
      j += (int64_t)adjwgt[e] *
           pmo_distance(levels, a, d, part[v], part[adjncy[e]]);
  return j;
}

/* c(V_b) for every block b (Section 2). */
void pmo_block_weights(int32_t n, const int32_t *vwgt, const int32_t *part,
                       int64_t k, int64_t *w_out) {
  for (int64_t b = 0; b < k; ++b) w_out[b] = 0;
  for (int32_t v = 0; v < n; ++v) w_out[part[v]] += vwgt[v];
}

/* L_max = ceil((1 + eps) * c(V) / k) (Section 2), with eps given in parts
 * per million so that the ceiling is exact in integers. */
int64_t pmo_lmax(int64_t total_weight, int64_t k, int64_t eps_ppm) {
  int64_t num = (1000000 + eps_ppm) * total_weight;
  int64_t den = 1000000 * k;
  return (num + den - 1) / den;
}

/* Gain of moving v from its block to block b, equation (1):
 * G_b(v) = sum over neighbours u of C_vu * (D(Pi(v),Pi(u)) - D(b,Pi(u))). */
int64_t pmo_gain(const int64_t *xadj, const int32_t *adjncy,
                 const int32_t *adjwgt, const int32_t *part,
                 int32_t levels, const int32_t *a, const int32_t *d,
                 int32_t v, int32_t b) {
  int64_t g = 0;
  for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
    int32_t pu = part[adjncy[e]];
    g += (int64_t)adjwgt[e] * (pmo_distance(levels, a, d, part[v], pu) -
                               pmo_distance(levels, a, d, b, pu));
  }
  return g;
}

/* ======================================================================
 * Counter-based hash: the output function of splitmix64 (Steele, Lea and
 * Flood, OOPSLA 2014), applied to the state seed + (word+1)*golden, i.e.
 * the (word+1)-th output of a splitmix64 stream started at `seed`.
 * ====================================================================== */
uint64_t pmo_hash(uint64_t seed, uint64_t word) {
  uint64_t z = seed + (word + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

#define TAG_HEM 0x48454D31ULL
#define TAG_REB 0x5245424CULL

/* ======================================================================
 * Unconstrained label propagation (Section 4.2, Algorithm 4)
 * ====================================================================== */

static int cmp_i32(const void *x, const void *y) {
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

static int64_t max_degree(int32_t n, const int64_t *xadj) {
  int64_t m = 0;
  for (int32_t v = 0; v < n; ++v)
    if (xadj[v + 1] - xadj[v] > m) m = xadj[v + 1] - xadj[v];
  return m;
}

/* One round of unconstrained label propagation.
 *
 * Phase 1: for every vertex that is not locked, the candidate blocks are the
 * blocks of its neighbours other than its own (a vertex with no such
 * neighbour is skipped).  The best candidate maximises the gain of equation
 * (1); ties go to the smaller block id.  If that gain is >= 0 the vertex
 * enters the first-filter set X with its target and gain.  Equation (1) is
 * evaluated with the neighbours grouped by block, i.e. from the connectivity
 * conn(v,x) = sum of C_vu over neighbours u in block x (the per-vertex
 * structure the paper keeps for gains):
 *   G_b(v) = sum_x conn(v,x) * (D(Pi(v),x) - D(b,x)).
 *
 * Phase 2: X is ordered implicitly -- u precedes v iff g(u) > g(v), or
 * g(u) == g(v) and u < v.  Each v in X re-evaluates the gain of its move
 * with every neighbour u in X that precedes it counted at u's target and
 * every other neighbour at its current block.  v moves iff this re-evaluated
 * gain is >= 0.
 *
 * Afterwards the moves are applied and exactly the moved vertices are locked
 * for the next round of label propagation.
 *
 * Outputs: target_out[v] (= part[v] if v not in X), gain_out[v] (INT64_MIN if
 * v not in X), moved_out[v]; part and lock are updated in place. */
typedef struct {
  int32_t b;
  int32_t w;
} blk_w;

static int cmp_blkw(const void *x, const void *y) {
  const blk_w *a = (const blk_w *)x, *b = (const blk_w *)y;
  return (a->b > b->b) - (a->b < b->b);
}

/* conn(v,.) as a list of (block, summed weight), ascending block id.
 * `row` receives the raw (block, weight) pairs; the aggregated list is
 * written to blocks/conns.  Returns its length. */
static int64_t connectivity(const int64_t *xadj, const int32_t *adjncy,
                            const int32_t *adjwgt, const int32_t *part,
                            int32_t v, blk_w *row, int32_t *blocks,
                            int64_t *conns) {
  int64_t cnt = 0;
  for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
    row[cnt].b = part[adjncy[e]];
    row[cnt].w = adjwgt[e];
    ++cnt;
  }
  qsort(row, (size_t)cnt, sizeof(blk_w), cmp_blkw);
  int64_t r = 0;
  for (int64_t i = 0; i < cnt;) {
    int32_t b = row[i].b;
    int64_t c = 0;
    while (i < cnt && row[i].b == b) c += row[i++].w;
    blocks[r] = b;
    conns[r] = c;
    ++r;
  }
  return r;
}

void pmo_lp_round(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                  const int32_t *adjwgt, int32_t levels, const int32_t *a,
                  const int32_t *d, int32_t *part, uint8_t *lock,
                  int32_t *target_out, int64_t *gain_out, uint8_t *moved_out) {
  pmo_lp_round_v(n, xadj, adjncy, adjwgt, levels, a, d, part, lock, target_out,
                 gain_out, moved_out, NULL);
}

/* Label propagation round (Algorithm 4).  With the relaxed first filter of
 * Jet (variants->jet_c_num > 0, Section 4.2 after Algorithm 4), a vertex also
 * enters X when its best gain is negative but -G < floor(c * conn(v,Pi(v))),
 * c = jet_c_num / jet_c_den; the second filter is unchanged. */
void pmo_lp_round_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                    const int32_t *adjwgt, int32_t levels, const int32_t *a,
                    const int32_t *d, int32_t *part, uint8_t *lock,
                    int32_t *target_out, int64_t *gain_out, uint8_t *moved_out,
                    const pmo_variants *var) {
  const int64_t jet_num = var ? var->jet_c_num : 0;
  const int64_t jet_den = (var && var->jet_c_den > 0) ? var->jet_c_den : 1;
  int64_t maxdeg = max_degree(n, xadj);
  blk_w *row = (blk_w *)xmalloc(sizeof(blk_w) * (size_t)maxdeg);
  int32_t *blocks = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)maxdeg);
  int64_t *conns = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)maxdeg);

  /* phase 1 (first filter) */
  for (int32_t v = 0; v < n; ++v) {
    target_out[v] = part[v];
    gain_out[v] = NOT_IN_X;
    if (lock[v]) continue;
    int32_t p = part[v];
    int64_t r = connectivity(xadj, adjncy, adjwgt, part, v, row, blocks, conns);
    int64_t best_g = 0, conn_own = 0;
    int32_t best_b = -1;
    for (int64_t i = 0; i < r; ++i) {
      int32_t b = blocks[i];
      if (b == p) {
        conn_own = conns[i];
        continue;
      }
      int64_t g = 0;
      for (int64_t j = 0; j < r; ++j)
        g += conns[j] * (pmo_distance(levels, a, d, p, blocks[j]) -
                         pmo_distance(levels, a, d, b, blocks[j]));
      if (best_b < 0 || g > best_g) {
        best_g = g;
        best_b = b;
      }
    }
    const int passes = best_g >= 0 || (jet_num > 0 && -best_g < (jet_num * conn_own) / jet_den);
    if (best_b >= 0 && passes) {
      target_out[v] = best_b;
      gain_out[v] = best_g;
    }
  }

  /* phase 2 (re-evaluation under the approximate future state) */
  for (int32_t v = 0; v < n; ++v) {
    moved_out[v] = 0;
    if (gain_out[v] == NOT_IN_X) continue;
    int64_t gv = gain_out[v];
    int64_t g2 = 0;
    for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
      int32_t u = adjncy[e];
      int32_t pu = part[u];
      int64_t gu = gain_out[u];
      if (gu != NOT_IN_X && (gu > gv || (gu == gv && u < v))) pu = target_out[u];
      g2 += (int64_t)adjwgt[e] * (pmo_distance(levels, a, d, part[v], pu) -
                                  pmo_distance(levels, a, d, target_out[v], pu));
    }
    moved_out[v] = (uint8_t)(g2 >= 0);
  }

  /* apply the moves; lock exactly the moved vertices */
  for (int32_t v = 0; v < n; ++v) {
    if (moved_out[v]) part[v] = target_out[v];
    lock[v] = moved_out[v];
  }
  free(row);
  free(blocks);
  free(conns);
}

/* ======================================================================
 * Rebalancing (Section 4.2, "Rebalancing", Algorithm 5)
 * ====================================================================== */

/* sigma = L_max - 100 as in the paper, but never below the average block
 * weight ceil(c(V)/k): otherwise, on small graphs, no block could ever be a
 * destination. */
int64_t pmo_sigma(int64_t lmax, int64_t total_weight, int64_t k) {
  int64_t avg = (total_weight + k - 1) / k;
  int64_t s = lmax - 100;
  return s > avg ? s : avg;
}

typedef struct {
  int32_t key1;  /* source block (selection) or destination (acceptance) */
  int32_t bucket;
  int32_t v;
} reb_item;

static int cmp_reb(const void *x, const void *y) {
  const reb_item *a = (const reb_item *)x, *b = (const reb_item *)y;
  if (a->key1 != b->key1) return (a->key1 > b->key1) - (a->key1 < b->key1);
  if (a->bucket != b->bucket) return (a->bucket > b->bucket) - (a->bucket < b->bucket);
  return (a->v > b->v) - (a->v < b->v);
}

static int32_t floor_log2_u64(uint64_t x) { return 63 - __builtin_clzll(x); }

/* smallest q with c <= 2^q (c >= 1) */
static int32_t weight_class(int64_t c) {
  return c <= 1 ? 0 : 1 + floor_log2_u64((uint64_t)(c - 1));
}

/* One rebalancing round, weak (strong = 0) or strong (strong = 1).
 *
 * Sources: vertices of overloaded blocks (c(block) > L_max) that are not
 * heavy; v is heavy when c(v) > 1.5 * (c(block) - c(V)/k), tested exactly as
 * 2k*c(v) > 3*(k*c(block) - c(V)).
 *
 * Destination of a source: among the blocks of its neighbours whose weight is
 * at most the cap (sigma for weak, L_max for strong), the one with the
 * largest connection conn(v,b) (smaller id on ties) -- the rebalancing uses
 * the edge-cut loss, as the paper reports.  Without such a neighbour block,
 * a seeded pseudo-random block among all blocks within the cap (ascending id
 * list, index = hash mod size).  A source with no block within the cap does
 * not take part.
 *
 * Loss g = conn(v,t) - conn(v,Pi(v)); bucket 0 for g > 0, 1 for g == 0 and
 * 2 + floor(log2(-g)) for g < 0 (log2-spaced buckets).
 *
 * Selection: the sources of every overloaded block A, ordered by (bucket,
 * vertex id), move while the weight of the sources before them is smaller
 * than c(A) - L_max.
 *
 * Weak: all selected sources move to their destination.
 * Strong: the selected movers of every destination b, ordered by (bucket,
 * id), are accepted while c(b) + (weight before them) + c(v) <= L_max.  The
 * rejected ones are reassigned to blocks with residual capacity
 * r_b = L_max - c(b) - accepted_b > 0 without overloading any of them, by
 * weight class, heaviest first (the rule is spelled out where it is done);
 * the ones that find no room stay.
 *
 * moved_out[v] = 1 for every vertex that changed block; part is updated. */
void pmo_rebalance(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                   const int32_t *adjwgt, const int32_t *vwgt, int64_t k,
                   int32_t strong, int64_t lmax, int64_t sigma, uint64_t seed,
                   int32_t level, int32_t iter, int32_t *part,
                   uint8_t *moved_out) {
  pmo_rebalance_v(n, xadj, adjncy, adjwgt, vwgt, 0, NULL, NULL, k, strong, lmax,
                  sigma, seed, level, iter, part, moved_out, NULL);
}

/* J-objective rebalancing (variants->j_rebalance, the variant of Section 4.2
 * that the authors tried): the loss of a move to block b is the J gain of
 * eq. 1, G_b(v) = sum_x conn(v,x) (D(Pi(v),x) - D(b,x)); the destination is
 * the neighbour block within the cap with the largest J gain (smaller id on
 * ties), else the pseudo-random block, whose loss is its J gain as well.
 * Everything else is as in pmo_rebalance.  levels/a/d are only read by the
 * variant. */
void pmo_rebalance_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                     const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                     const int32_t *a, const int32_t *d, int64_t k,
                     int32_t strong, int64_t lmax, int64_t sigma, uint64_t seed,
                     int32_t level, int32_t iter, int32_t *part,
                     uint8_t *moved_out, const pmo_variants *var) {
  const int jobj = var && var->j_rebalance;
  int64_t *w = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  pmo_block_weights(n, vwgt, part, k, w);
  int64_t total = 0;
  for (int64_t b = 0; b < k; ++b) total += w[b];
  int64_t cap = strong ? lmax : sigma;

  int32_t *elig = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)k);
  int64_t nelig = 0;
  for (int64_t b = 0; b < k; ++b)
    if (w[b] <= cap) elig[nelig++] = (int32_t)b;

  uint64_t hseed = pmo_hash(pmo_hash(seed ^ TAG_REB, (uint64_t)level),
                            (uint64_t)iter);
  int64_t maxdeg = max_degree(n, xadj);
  blk_w *row = (blk_w *)xmalloc(sizeof(blk_w) * (size_t)maxdeg);
  int32_t *dest = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  reb_item *items = (reb_item *)xmalloc(sizeof(reb_item) * (size_t)n);
  int64_t nitems = 0;

  for (int32_t v = 0; v < n; ++v) {
    dest[v] = -1;
    moved_out[v] = 0;
    int32_t p = part[v];
    if (w[p] <= lmax) continue;
    if (2 * k * (int64_t)vwgt[v] > 3 * (k * w[p] - total)) continue; /* heavy */
    /* connection of v to each neighbour block */
    int64_t cnt = 0;
    for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
      row[cnt].b = part[adjncy[e]];
      row[cnt].w = adjwgt[e];
      ++cnt;
    }
    qsort(row, (size_t)cnt, sizeof(blk_w), cmp_blkw);
    /* merge to (block, conn) pairs, ascending block (a row's sum stays
     * below 2^31: all edge weights together do) */
    int64_t r = 0;
    for (int64_t i = 0; i < cnt;) {
      int32_t b = row[i].b;
      int64_t c = 0;
      while (i < cnt && row[i].b == b) c += row[i++].w;
      row[r].b = b;
      row[r].w = c;
      ++r;
    }
    int64_t conn_own = 0, best_val = 0;
    int32_t t = -1;
    for (int64_t i = 0; i < r; ++i) {
      int32_t b = row[i].b;
      int64_t c = row[i].w;
      if (b == p) {
        conn_own = c;
        continue;
      }
      if (w[b] > cap) continue;
      int64_t val = c;
      if (jobj) {
        val = 0;
        for (int64_t j = 0; j < r; ++j)
          val += (int64_t)row[j].w * (pmo_distance(levels, a, d, p, row[j].b) -
                                      pmo_distance(levels, a, d, b, row[j].b));
      }
      if (t < 0 || val > best_val) {
        best_val = val;
        t = b;
      }
    }
    int64_t g;
    if (t < 0) {
      if (nelig == 0) continue;
      t = elig[pmo_hash(hseed, (uint64_t)v) % (uint64_t)nelig];
      if (jobj) {
        g = 0;
        for (int64_t j = 0; j < r; ++j)
          g += (int64_t)row[j].w * (pmo_distance(levels, a, d, p, row[j].b) -
                                    pmo_distance(levels, a, d, t, row[j].b));
      } else {
        g = -conn_own; /* not a neighbour block: conn(v,t) = 0 */
      }
    } else {
      g = jobj ? best_val : best_val - conn_own;
    }
    int32_t bucket = g > 0 ? 0 : (g == 0 ? 1 : 2 + floor_log2_u64((uint64_t)(-g)));
    dest[v] = t;
    items[nitems].key1 = p;
    items[nitems].bucket = bucket;
    items[nitems].v = v;
    ++nitems;
  }

  /* per overloaded block: prefix in (bucket, id) order covering the excess */
  qsort(items, (size_t)nitems, sizeof(reb_item), cmp_reb);
  uint8_t *sel = (uint8_t *)xcalloc((size_t)n, 1);
  for (int64_t i = 0; i < nitems;) {
    int32_t blk = items[i].key1;
    int64_t excess = w[blk] - lmax, before = 0;
    for (; i < nitems && items[i].key1 == blk; ++i) {
      int32_t v = items[i].v;
      if (before < excess) sel[v] = 1;
      before += vwgt[v];
    }
  }

  if (!strong) {
    for (int32_t v = 0; v < n; ++v)
      if (sel[v]) {
        part[v] = dest[v];
        moved_out[v] = 1;
      }
  } else {
    /* acceptance per destination, in (bucket, id) order */
    int64_t nsel = 0;
    int32_t *bucket_of = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < nitems; ++i) bucket_of[items[i].v] = items[i].bucket;
    for (int32_t v = 0; v < n; ++v)
      if (sel[v]) {
        items[nsel].key1 = dest[v];
        items[nsel].bucket = bucket_of[v];
        items[nsel].v = v;
        ++nsel;
      }
    qsort(items, (size_t)nsel, sizeof(reb_item), cmp_reb);
    int64_t *acc = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    uint8_t *accepted = (uint8_t *)xcalloc((size_t)n, 1);
    for (int64_t i = 0; i < nsel;) {
      int32_t b = items[i].key1;
      int64_t before = 0;
      for (; i < nsel && items[i].key1 == b; ++i) {
        int32_t v = items[i].v;
        if (w[b] + before + vwgt[v] <= lmax) {
          accepted[v] = 1;
          acc[b] += vwgt[v];
        }
        before += vwgt[v];
      }
    }
    /* residual capacity of every block after the accepted moves */
    int64_t *resid = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
    int64_t *got = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    for (int64_t b = 0; b < k; ++b) resid[b] = lmax - w[b] - acc[b];
    /* the accepted movers go to their destinations */
    int32_t qmax = -1;
    for (int32_t v = 0; v < n; ++v) {
      if (!sel[v]) continue;
      if (accepted[v]) {
        part[v] = dest[v];
        moved_out[v] = 1;
      } else if (weight_class(vwgt[v]) > qmax) {
        qmax = weight_class(vwgt[v]);
      }
    }
    /* The rejected movers are reassigned without overloading any block, by
     * weight class q(v) = ceil(log2 c(v)) (the smallest q with c(v) <= 2^q),
     * heaviest class first.  For class q, every block b with residual
     * r_b >= 2^q offers the interval of length s_b = r_b - 2^q + 1 (blocks
     * in ascending id, exclusive prefix C_b); the movers of the class, in
     * id order with exclusive weight prefix R, go to the block with
     * C_b <= R < C_b + s_b, and stay where they are when R >= sum s_b.  The
     * movers a block receives in one class occupy consecutive positions that
     * start inside its interval, so together they weigh at most
     * (s_b - 1) + 2^q = r_b; the block's residual then shrinks by what it
     * received before the next class. */
    int64_t *slot_start = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
    for (int32_t q = qmax; q >= 0; --q) {
      int64_t unit = (int64_t)1 << q, csum = 0;
      for (int64_t b = 0; b < k; ++b) {
        slot_start[b] = csum;
        if (resid[b] >= unit) csum += resid[b] - unit + 1;
      }
      int64_t R = 0, b = 0;
      for (int32_t v = 0; v < n; ++v) {
        if (!sel[v] || accepted[v] || weight_class(vwgt[v]) != q) continue;
        if (R < csum) {
          /* the block whose interval holds R */
          while (!(resid[b] >= unit && slot_start[b] <= R &&
                   R < slot_start[b] + resid[b] - unit + 1))
            ++b;
          part[v] = (int32_t)b;
          moved_out[v] = 1;
          got[b] += vwgt[v];
        }
        R += vwgt[v];
      }
      for (int64_t x = 0; x < k; ++x) {
        resid[x] -= got[x];
        got[x] = 0;
      }
    }
    free(slot_start);
    free(resid);
    free(got);
    free(acc);
    free(accepted);
    free(bucket_of);
  }
  free(sel);
  free(items);
  free(dest);
  free(row);
  free(elig);
  free(w);
}

/* ======================================================================
 * Overall refinement (Section 4.2, Algorithm 6)
 * ====================================================================== */

#define REFINE_PATIENCE 12
#define REFINE_WEAK_ROUNDS 2
#define REFINE_MAX_BODIES 4096 /* safety bound on loop bodies per call */

static int64_t max_block(int32_t n, const int32_t *vwgt, const int32_t *part,
                         int64_t k, int64_t *scratch) {
  pmo_block_weights(n, vwgt, part, k, scratch);
  int64_t m = 0;
  for (int64_t b = 0; b < k; ++b)
    if (scratch[b] > m) m = scratch[b];
  return m;
}

/* Alternates label propagation (when the current mapping is balanced) with
 * weak rebalancing (at most twice in a row) and strong rebalancing, and keeps
 * the best mapping seen.  Readings:
 *  - a balanced candidate replaces the best if the best is unbalanced or the
 *    candidate's J is strictly smaller; the counter restarts if the best was
 *    unbalanced or J' < 0.999 * J_best (tested as 1000 J' < 999 J_best),
 *    both judged against the best as it was before the update;
 *  - an unbalanced candidate replaces the best (and restarts the counter) iff
 *    its heaviest block is strictly lighter than the best's;
 *  - the lock set is that of the latest label-propagation round; it starts
 *    empty and rebalancing neither reads nor changes it;
 *  - the pseudo-random choices of rebalancing draw with (seed, level, loop
 *    body number starting at 1).
 * Returns 0 if the returned mapping is balanced, 1 otherwise. */
int32_t pmo_refine(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                   const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                   const int32_t *a, const int32_t *d, int64_t eps_ppm,
                   uint64_t seed, int32_t level, int32_t *part,
                   pmo_refine_stats *stats) {
  return pmo_refine_v(n, xadj, adjncy, adjwgt, vwgt, levels, a, d, eps_ppm, seed,
                      level, part, stats, NULL);
}

int32_t pmo_refine_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                     const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                     const int32_t *a, const int32_t *d, int64_t eps_ppm,
                     uint64_t seed, int32_t level, int32_t *part,
                     pmo_refine_stats *stats, const pmo_variants *var) {
  return pmo_refine_trace(n, xadj, adjncy, adjwgt, vwgt, levels, a, d, eps_ppm,
                          seed, level, part, stats, var, 0, NULL, NULL, NULL,
                          NULL);
}

/* pmo_refine_v with a record of the loop bodies: for body t < trace_cap,
 * kind[t] is 'L' (label propagation), 'w' (weak) or 'S' (strong
 * rebalancing); j_after[t] and imb_after[t] are J and the heaviest block of
 * the current mapping after the body, and counter[t] is Algorithm 6's
 * counter i after the body's best-mapping update.  Any of the four arrays
 * may be NULL. */
int32_t pmo_refine_trace(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                         const int32_t *adjwgt, const int32_t *vwgt,
                         int32_t levels, const int32_t *a, const int32_t *d,
                         int64_t eps_ppm, uint64_t seed, int32_t level,
                         int32_t *part, pmo_refine_stats *stats,
                         const pmo_variants *var, int32_t trace_cap,
                         char *kind, int64_t *j_after, int64_t *imb_after,
                         int32_t *counter) {
  int64_t k = pmo_num_pes(levels, a);
  int64_t total = 0;
  for (int32_t v = 0; v < n; ++v) total += vwgt[v];
  int64_t lmax = pmo_lmax(total, k, eps_ppm);
  int64_t sigma = pmo_sigma(lmax, total, k);

  int64_t *wscratch = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  int32_t *cur = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  uint8_t *lock = (uint8_t *)xcalloc((size_t)n, 1);
  int32_t *target = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  int64_t *gain = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  uint8_t *moved = (uint8_t *)xmalloc((size_t)n);
  memcpy(cur, part, sizeof(int32_t) * (size_t)n);

  int64_t j_best = pmo_comm_cost(n, xadj, adjncy, adjwgt, part, levels, a, d);
  int64_t imb_best = max_block(n, vwgt, part, k, wscratch);
  int32_t feas_best = imb_best <= lmax;
  int64_t imb_cur = imb_best;
  pmo_refine_stats st;
  memset(&st, 0, sizeof(st));
  st.j_initial = j_best;
  st.maxw_initial = imb_best;

  int32_t i = 0, iw = 0, bodies = 0;
  while (i < REFINE_PATIENCE && bodies < REFINE_MAX_BODIES) {
    ++i;
    ++bodies;
    char what;
    if (imb_cur <= lmax) {
      pmo_lp_round_v(n, xadj, adjncy, adjwgt, levels, a, d, cur, lock, target,
                     gain, moved, var);
      iw = 0;
      ++st.lp_iterations;
      what = 'L';
    } else if (iw < REFINE_WEAK_ROUNDS) {
      pmo_rebalance_v(n, xadj, adjncy, adjwgt, vwgt, levels, a, d, k, 0, lmax,
                      sigma, seed, level, bodies, cur, moved, var);
      ++iw;
      ++st.weak_iterations;
      what = 'w';
    } else {
      pmo_rebalance_v(n, xadj, adjncy, adjwgt, vwgt, levels, a, d, k, 1, lmax,
                      sigma, seed, level, bodies, cur, moved, var);
      iw = 0;
      ++st.strong_iterations;
      what = 'S';
    }
    int64_t j_cur = pmo_comm_cost(n, xadj, adjncy, adjwgt, cur, levels, a, d);
    imb_cur = max_block(n, vwgt, cur, k, wscratch);
    if (imb_cur <= lmax) {
      int32_t improve = !feas_best || j_cur < j_best;
      int32_t reset = !feas_best || 1000 * j_cur < 999 * j_best;
      if (improve) {
        memcpy(part, cur, sizeof(int32_t) * (size_t)n);
        j_best = j_cur;
        imb_best = imb_cur;
        feas_best = 1;
      }
      if (reset) i = 0;
    } else if (imb_cur < imb_best) {
      memcpy(part, cur, sizeof(int32_t) * (size_t)n);
      j_best = j_cur;
      imb_best = imb_cur;
      i = 0;
    }
    if (bodies <= trace_cap) {
      if (kind) kind[bodies - 1] = what;
      if (j_after) j_after[bodies - 1] = j_cur;
      if (imb_after) imb_after[bodies - 1] = imb_cur;
      if (counter) counter[bodies - 1] = i;
    }
  }
  st.iterations = bodies;
  st.j_final = j_best;
  st.maxw_final = imb_best;
  st.feasible = feas_best;
  if (stats) *stats = st;
  free(wscratch);
  free(cur);
  free(lock);
  free(target);
  free(gain);
  free(moved);
  return feas_best ? 0 : 1;
}

/* ======================================================================
 * Heavy-edge matching (Section 4.2, "Matching")
 * ====================================================================== */

/* Is edge (v,u1,w1) rated above edge (v,u2,w2)?  The rating is
 * w^2 / (c(u) c(v)); c(v) is common to both, so the comparison is
 * w1^2 * c(u2) > w2^2 * c(u1), exactly, in 128 bits.  Equal ratings are
 * separated by deterministic noise: the smaller hash of the unordered pair,
 * then the smaller lower endpoint, then the smaller upper endpoint. */
static int hem_better(int64_t w1, int64_t c1, uint64_t h1, int32_t lo1,
                      int32_t hi1, int64_t w2, int64_t c2, uint64_t h2,
                      int32_t lo2, int32_t hi2) {
  unsigned __int128 l = (unsigned __int128)(uint64_t)(w1 * w1) * (uint64_t)c2;
  unsigned __int128 r = (unsigned __int128)(uint64_t)(w2 * w2) * (uint64_t)c1;
  if (l != r) return l > r;
  if (h1 != h2) return h1 < h2;
  if (lo1 != lo2) return lo1 < lo2;
  return hi1 < hi2;
}

typedef struct {
  uint64_t key;
  int32_t v;
} keyed_vertex;

static int cmp_keyed(const void *x, const void *y) {
  const keyed_vertex *a = (const keyed_vertex *)x, *b = (const keyed_vertex *)y;
  if (a->key != b->key) return (a->key > b->key) - (a->key < b->key);
  return (a->v > b->v) - (a->v < b->v);
}

/* Pairs the members of every group of equal keys, in id order: the 1st with
 * the 2nd, the 3rd with the 4th, ..., a pair only when its weight fits
 * L_max (otherwise both stay unmatched).  Returns the vertices matched. */
static int64_t pair_groups(keyed_vertex *items, int64_t cnt, const int32_t *vwgt,
                           int64_t lmax, int32_t *match) {
  qsort(items, (size_t)cnt, sizeof(keyed_vertex), cmp_keyed);
  int64_t added = 0;
  for (int64_t i = 0; i < cnt;) {
    int64_t j = i;
    while (j < cnt && items[j].key == items[i].key) ++j;
    for (int64_t p = i; p + 1 < j; p += 2) {
      int32_t a = items[p].v, b = items[p + 1].v;
      if ((int64_t)vwgt[a] + vwgt[b] <= lmax) {
        match[a] = b;
        match[b] = a;
        added += 2;
      }
    }
    i = j;
  }
  return added;
}

#define TAG_TWIN 0x5457494EULL

/* Heavy-edge matching in synchronous rounds, followed by two-hop matching.
 *
 * Heavy-edge rounds: every unmatched vertex v prefers the unmatched
 * neighbour u with c(u)+c(v) <= L_max whose edge rates highest (see
 * hem_better); v and u are matched iff they prefer each other.  Rounds repeat
 * until one adds no match (at most 64).
 *
 * Two-hop matching (the leaf, twin and relative categories), each step only
 * while 75 % or fewer of the vertices are matched:
 *  - leaves: unmatched vertices of degree one, grouped by their neighbour;
 *  - twins: unmatched vertices with the same neighbourhood, recognised by an
 *    order-independent neighbourhood hash (sum of the splitmix64 hashes of
 *    the neighbour ids) together with the degree; all isolated vertices
 *    share the empty neighbourhood;
 *  - relatives: unmatched vertices with a neighbour, grouped by their
 *    matchmaker -- the neighbour of smallest (degree, id).
 * In every group the members are paired in id order (see pair_groups).
 * match_out[v] = partner, or v itself if unmatched.  Returns the number of
 * heavy-edge rounds executed. */
int32_t pmo_hem(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                const int32_t *adjwgt, const int32_t *vwgt, int64_t lmax,
                uint64_t seed, int32_t level, int32_t *match_out) {
  uint64_t hseed = pmo_hash(seed ^ TAG_HEM, (uint64_t)level);
  int32_t *match = match_out;
  int32_t *pref = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; ++v) match[v] = -1;
  int32_t rounds = 0;
  int64_t matched = 0;
  while (rounds < 64) {
    ++rounds;
    for (int32_t v = 0; v < n; ++v) {
      pref[v] = -1;
      if (match[v] >= 0) continue;
      int64_t bw = 0, bc = 0;
      uint64_t bh = 0;
      int32_t blo = 0, bhi = 0;
      for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
        int32_t u = adjncy[e];
        if (match[u] >= 0) continue;
        if ((int64_t)vwgt[u] + vwgt[v] > lmax) continue;
        int32_t lo = u < v ? u : v, hi = u < v ? v : u;
        uint64_t h = pmo_hash(hseed, ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi);
        if (pref[v] < 0 || hem_better(adjwgt[e], vwgt[u], h, lo, hi, bw, bc, bh, blo, bhi)) {
          pref[v] = u;
          bw = adjwgt[e];
          bc = vwgt[u];
          bh = h;
          blo = lo;
          bhi = hi;
        }
      }
    }
    int64_t added = 0;
    for (int32_t v = 0; v < n; ++v) {
      int32_t u = pref[v];
      if (u >= 0 && pref[u] == v) {
        match[v] = u;
        ++added;
      }
    }
    matched += added;
    if (added == 0) break;
  }
  free(pref);

  keyed_vertex *items = (keyed_vertex *)xmalloc(sizeof(keyed_vertex) * (size_t)n);
  /* leaves, grouped by their only neighbour */
  if (4 * matched <= 3 * (int64_t)n) {
    int64_t cnt = 0;
    for (int32_t v = 0; v < n; ++v)
      if (match[v] < 0 && xadj[v + 1] - xadj[v] == 1) {
        items[cnt].key = (uint64_t)(uint32_t)adjncy[xadj[v]];
        items[cnt].v = v;
        ++cnt;
      }
    matched += pair_groups(items, cnt, vwgt, lmax, match);
  }
  /* twins, grouped by neighbourhood hash and degree */
  if (4 * matched <= 3 * (int64_t)n) {
    uint64_t tseed = pmo_hash(seed ^ TAG_TWIN, (uint64_t)level);
    int64_t cnt = 0;
    for (int32_t v = 0; v < n; ++v) {
      if (match[v] >= 0) continue;
      uint64_t h = 0;
      for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e)
        h += pmo_hash(tseed, (uint64_t)(uint32_t)adjncy[e]);
      items[cnt].key = pmo_hash(h, (uint64_t)(xadj[v + 1] - xadj[v]));
      items[cnt].v = v;
      ++cnt;
    }
    matched += pair_groups(items, cnt, vwgt, lmax, match);
  }
  /* relatives, grouped by their matchmaker */
  if (4 * matched <= 3 * (int64_t)n) {
    int64_t cnt = 0;
    for (int32_t v = 0; v < n; ++v) {
      if (match[v] >= 0 || xadj[v + 1] == xadj[v]) continue;
      int32_t mm = -1;
      int64_t mdeg = 0;
      for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
        int32_t u = adjncy[e];
        int64_t du = xadj[u + 1] - xadj[u];
        if (mm < 0 || du < mdeg || (du == mdeg && u < mm)) {
          mm = u;
          mdeg = du;
        }
      }
      items[cnt].key = (uint64_t)(uint32_t)mm;
      items[cnt].v = v;
      ++cnt;
    }
    matched += pair_groups(items, cnt, vwgt, lmax, match);
  }
  free(items);
  for (int32_t v = 0; v < n; ++v)
    if (match[v] < 0) match[v] = v;
  return rounds;
}

/* Coarse vertex ids: every matched pair (or single vertex) is represented by
 * its smaller id; the coarse id is the rank of that representative in
 * ascending order.  Returns the number of coarse vertices. */
int32_t pmo_coarse_map(int32_t n, const int32_t *match, int32_t *cmap_out) {
  int32_t nc = 0;
  for (int32_t v = 0; v < n; ++v)
    if (match[v] >= v) cmap_out[v] = nc++;
  for (int32_t v = 0; v < n; ++v)
    if (match[v] < v) cmap_out[v] = cmap_out[match[v]];
  return nc;
}

typedef struct {
  int32_t cu, cv, w;
} carc;

static int cmp_carc(const void *x, const void *y) {
  const carc *a = (const carc *)x, *b = (const carc *)y;
  if (a->cu != b->cu) return (a->cu > b->cu) - (a->cu < b->cu);
  return (a->cv > b->cv) - (a->cv < b->cv);
}

/* Contraction (Section 2 "Multilevel Graph Partitioning" and Section 4.2
 * "Contraction"): a coarse vertex weighs the sum of its members; every arc
 * (u,v,w) becomes (M(u),M(v),w); arcs with M(u) == M(v) are dropped and
 * parallel arcs are fused with their weights summed.  Rows come out sorted.
 * Output arrays must hold nc+1 / nnz / nnz / nc entries.  Returns the coarse
 * number of arcs. */
int64_t pmo_contract(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                     const int32_t *adjwgt, const int32_t *vwgt,
                     const int32_t *cmap, int32_t nc, int64_t *cxadj,
                     int32_t *cadjncy, int32_t *cadjwgt, int32_t *cvwgt) {
  for (int32_t c = 0; c < nc; ++c) cvwgt[c] = 0;
  for (int32_t v = 0; v < n; ++v) cvwgt[cmap[v]] += vwgt[v];
  int64_t nnz = xadj[n], cnt = 0;
  carc *arcs = (carc *)xmalloc(sizeof(carc) * (size_t)nnz);
  for (int32_t v = 0; v < n; ++v)
    for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
      int32_t cu = cmap[v], cv = cmap[adjncy[e]];
      if (cu == cv) continue;
      arcs[cnt].cu = cu;
      arcs[cnt].cv = cv;
      arcs[cnt].w = adjwgt[e];
      ++cnt;
    }
  qsort(arcs, (size_t)cnt, sizeof(carc), cmp_carc);
  for (int32_t c = 0; c <= nc; ++c) cxadj[c] = 0;
  int64_t out = 0;
  for (int64_t i = 0; i < cnt;) {
    int32_t cu = arcs[i].cu, cv = arcs[i].cv;
    int64_t w = 0;
    while (i < cnt && arcs[i].cu == cu && arcs[i].cv == cv) w += arcs[i++].w;
    cadjncy[out] = cv;
    cadjwgt[out] = (int32_t)w;
    ++out;
    cxadj[cu + 1] += 1;
  }
  for (int32_t c = 0; c < nc; ++c) cxadj[c + 1] += cxadj[c];
  free(arcs);
  return out;
}

/* ======================================================================
 * Initial partitioning (Section 4.2): hierarchical multisection (Section
 * 3.1, Algorithm 2) run on the host with a simple k-way partitioner.
 * ====================================================================== */

typedef struct {
  const int64_t *xadj;
  const int32_t *sorted_adj; /* every row sorted ascending */
  const int32_t *vwgt;
  const int32_t *a;
  int32_t *part;
  int32_t *stamp;  /* membership marker per vertex */
  uint8_t *seen;
  int32_t *queue;
  int32_t next_stamp;
} ip_ctx;

/* The simple a_i-way partitioner: breadth-first order over the subgraph
 * (start at the smallest unvisited id, neighbours in ascending id, restart at
 * the smallest unvisited id when the queue runs dry), cut into a_i
 * consecutive pieces where the running weight first reaches
 * ceil(j * c(V') / a_i), j = 1..a_i-1.  A vertex whose exclusive running
 * weight is w goes to piece #{j >= 1 : w >= ceil(j c(V')/a_i)}.  Pieces are
 * then split recursively one level down (Algorithm 2); the piece index at
 * level i is the level-i mixed-radix digit of the PE id. */
static void ip_recurse(ip_ctx *c, const int32_t *verts, int32_t cnt,
                       int32_t level, int64_t base) {
  if (cnt == 0) return;
  int32_t ai = c->a[level - 1];
  int64_t pstride = 1;
  for (int32_t i = 0; i < level - 1; ++i) pstride *= c->a[i];

  int32_t mark = ++c->next_stamp;
  int64_t wsum = 0;
  for (int32_t i = 0; i < cnt; ++i) {
    c->stamp[verts[i]] = mark;
    c->seen[verts[i]] = 0;
    wsum += c->vwgt[verts[i]];
  }
  int32_t *order = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)cnt);
  int32_t no = 0;
  for (int32_t s = 0; s < cnt; ++s) {
    int32_t root = verts[s];
    if (c->seen[root]) continue;
    int32_t qh = 0, qt = 0;
    c->queue[qt++] = root;
    c->seen[root] = 1;
    while (qh < qt) {
      int32_t x = c->queue[qh++];
      order[no++] = x;
      for (int64_t e = c->xadj[x]; e < c->xadj[x + 1]; ++e) {
        int32_t y = c->sorted_adj[e];
        if (c->stamp[y] == mark && !c->seen[y]) {
          c->seen[y] = 1;
          c->queue[qt++] = y;
        }
      }
    }
  }
  int32_t *piece = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)cnt);
  int64_t run = 0;
  for (int32_t i = 0; i < cnt; ++i) {
    int32_t j = 0;
    for (int32_t t = 1; t < ai; ++t)
      if (run >= ((int64_t)t * wsum + ai - 1) / ai) j = t;
    piece[i] = j;
    run += c->vwgt[order[i]];
  }
  int32_t *sub = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)cnt);
  for (int32_t j = 0; j < ai; ++j) {
    int32_t ns = 0;
    for (int32_t i = 0; i < cnt; ++i)
      if (piece[i] == j) sub[ns++] = order[i];
    qsort(sub, (size_t)ns, sizeof(int32_t), cmp_i32);
    if (level == 1) {
      for (int32_t i = 0; i < ns; ++i) c->part[sub[i]] = (int32_t)(base + j);
    } else {
      /* the recursion reuses stamp/seen; copy the piece first */
      int32_t *copy = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(ns ? ns : 1));
      memcpy(copy, sub, sizeof(int32_t) * (size_t)ns);
      ip_recurse(c, copy, ns, level - 1, base + (int64_t)j * pstride);
      free(copy);
    }
  }
  free(sub);
  free(piece);
  free(order);
}

void pmo_initial_partition(int32_t n, const int64_t *xadj,
                           const int32_t *adjncy, const int32_t *vwgt,
                           int32_t levels, const int32_t *a, int32_t *part_out) {
  int64_t nnz = xadj[n];
  int32_t *sorted_adj = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)nnz);
  memcpy(sorted_adj, adjncy, sizeof(int32_t) * (size_t)nnz);
  for (int32_t v = 0; v < n; ++v)
    qsort(sorted_adj + xadj[v], (size_t)(xadj[v + 1] - xadj[v]), sizeof(int32_t),
          cmp_i32);
  ip_ctx c;
  c.xadj = xadj;
  c.sorted_adj = sorted_adj;
  c.vwgt = vwgt;
  c.a = a;
  c.part = part_out;
  c.stamp = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
  c.seen = (uint8_t *)xcalloc((size_t)n, 1);
  c.queue = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  c.next_stamp = 0;
  int32_t *all = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; ++v) all[v] = v;
  ip_recurse(&c, all, n, levels, 0);
  free(all);
  free(c.queue);
  free(c.seen);
  free(c.stamp);
  free(sorted_adj);
}

/* ======================================================================
 * Multilevel integrated mapping (Section 4.2)
 * ====================================================================== */

typedef struct {
  int32_t n;
  int64_t *xadj;
  int32_t *adjncy, *adjwgt, *vwgt;
  int32_t *cmap; /* map to the next coarser level */
} level_graph;

/* Coarsen while the graph has at least 8k vertices (the initial partitioning
 * threshold), at most 64 graphs in total, and stop early when a level would
 * keep more than 95 % of the vertices (the matching has stalled; that level
 * is not built).  Then partition the coarsest graph with hierarchical
 * multisection, refine it, and for every finer level project the mapping
 * (Pi_fine(v) = Pi_coarse(M(v))) and refine again.  Refinement uses the
 * level index (0 = input graph) in its pseudo-random choices; the matching
 * of level t uses t as well.  Returns the status of the last refinement. */
int32_t pmo_map(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                const int32_t *a, const int32_t *d, int64_t eps_ppm,
                uint64_t seed, int32_t *part_out, pmo_map_stats *stats) {
  return pmo_map_v(n, xadj, adjncy, adjwgt, vwgt, levels, a, d, eps_ppm, seed,
                   part_out, stats, NULL);
}

int32_t pmo_map_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                  const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                  const int32_t *a, const int32_t *d, int64_t eps_ppm,
                  uint64_t seed, int32_t *part_out, pmo_map_stats *stats,
                  const pmo_variants *var) {
  double t0 = now_seconds();
  int64_t k = pmo_num_pes(levels, a);
  int64_t total = 0;
  for (int32_t v = 0; v < n; ++v) total += vwgt[v];
  int64_t lmax = pmo_lmax(total, k, eps_ppm);
  pmo_map_stats st;
  memset(&st, 0, sizeof(st));
  st.lmax = lmax;

  level_graph lv[PMO_MAX_LEVELS];
  memset(lv, 0, sizeof(lv));
  lv[0].n = n;
  lv[0].xadj = (int64_t *)xadj;
  lv[0].adjncy = (int32_t *)adjncy;
  lv[0].adjwgt = (int32_t *)adjwgt;
  lv[0].vwgt = (int32_t *)vwgt;
  int32_t t = 0;
  while ((int64_t)lv[t].n >= 8 * k && t + 1 < PMO_MAX_LEVELS) {
    level_graph *g = &lv[t];
    int32_t *match = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)g->n);
    st.level_hem_rounds[t] = pmo_hem(g->n, g->xadj, g->adjncy, g->adjwgt,
                                     g->vwgt, lmax, seed, t, match);
    g->cmap = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)g->n);
    int32_t nc = pmo_coarse_map(g->n, match, g->cmap);
    free(match);
    if (20 * (int64_t)nc > 19 * (int64_t)g->n) {
      free(g->cmap);
      g->cmap = NULL;
      st.level_hem_rounds[t] = 0;
      break;
    }
    level_graph *cg = &lv[t + 1];
    int64_t nnz = g->xadj[g->n];
    cg->n = nc;
    cg->xadj = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(nc + 1));
    cg->adjncy = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    cg->adjwgt = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    cg->vwgt = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)nc);
    pmo_contract(g->n, g->xadj, g->adjncy, g->adjwgt, g->vwgt, g->cmap, nc,
                 cg->xadj, cg->adjncy, cg->adjwgt, cg->vwgt);
    ++t;
  }
  st.levels = t + 1;
  for (int32_t s = 0; s <= t; ++s) {
    st.level_n[s] = lv[s].n;
    st.level_nnz[s] = lv[s].xadj[lv[s].n];
  }

  int32_t *part = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)lv[t].n);
  pmo_initial_partition(lv[t].n, lv[t].xadj, lv[t].adjncy, lv[t].vwgt, levels,
                        a, part);
  int32_t status = 0;
  double tr = 0.0;
  /* "ultra": the complete refinement runs `repeats` times at every level,
   * run r from the result of run r - 1 (empty lock set), with seed + r for
   * its pseudo-random choices */
  const int32_t repeats = (var && var->refine_repeats > 1) ? var->refine_repeats : 1;
  for (int32_t s = t;; --s) {
    level_graph *g = &lv[s];
    st.level_iterations[s] = 0;
    for (int32_t r = 0; r < repeats; ++r) {
      pmo_refine_stats rs;
      double r0 = now_seconds();
      status = pmo_refine_v(g->n, g->xadj, g->adjncy, g->adjwgt, g->vwgt, levels,
                            a, d, eps_ppm, seed + (uint64_t)r, s, part, &rs, var);
      tr += now_seconds() - r0;
      st.level_iterations[s] += rs.iterations;
      st.j_final = rs.j_final;
      st.feasible = rs.feasible;
    }
    if (s == 0) break;
    level_graph *f = &lv[s - 1];
    int32_t *fine = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)f->n);
    for (int32_t v = 0; v < f->n; ++v) fine[v] = part[f->cmap[v]];
    free(part);
    part = fine;
  }
  memcpy(part_out, part, sizeof(int32_t) * (size_t)n);
  free(part);
  for (int32_t s = 0; s <= t; ++s) {
    if (lv[s].cmap) free(lv[s].cmap);
    if (s > 0) {
      free(lv[s].xadj);
      free(lv[s].adjncy);
      free(lv[s].adjwgt);
      free(lv[s].vwgt);
    }
  }
  st.refine_seconds = tr;
  st.total_seconds = now_seconds() - t0;
  if (stats) *stats = st;
  return status;
}

/* ======================================================================
 * Hierarchical multisection (Section 4.1, Algorithms 1 and 2)
 * ====================================================================== */

/* The induced subgraphs of a partition into `parts` blocks (Algorithm 1, all
 * blocks at once).  Block b's vertices are the vertices v with part[v] = b in
 * ascending id order; its local id of v is v's rank among them.  Outputs, all
 * blocks concatenated in block order:
 *   vstart[parts+1]  first position of each block in order[]
 *   estart[parts+1]  first arc of each block
 *   order[n]         original id at every position
 *   xadj_out[n+parts] block b's row offsets (relative to estart[b]) at
 *                    xadj_out[vstart[b] + b .. vstart[b+1] + b]
 *   adjncy_out, adjwgt_out: each row keeps the neighbours of the same block
 *                    in the original row order, as local ids
 *   vwgt_out[n]      vertex weights by position
 * Returns the number of arcs kept. */
int64_t pmo_subgraphs(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                      const int32_t *adjwgt, const int32_t *vwgt, const int32_t *part,
                      int32_t parts, int32_t *vstart, int64_t *estart, int32_t *order,
                      int64_t *xadj_out, int32_t *adjncy_out, int32_t *adjwgt_out,
                      int32_t *vwgt_out) {
  int32_t *local = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t b = 0; b <= parts; ++b) vstart[b] = 0;
  for (int32_t v = 0; v < n; ++v) ++vstart[part[v] + 1];
  for (int32_t b = 0; b < parts; ++b) vstart[b + 1] += vstart[b];
  int32_t *fill = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(parts > 0 ? parts : 1));
  for (int32_t b = 0; b < parts; ++b) fill[b] = vstart[b];
  for (int32_t v = 0; v < n; ++v) {
    int32_t b = part[v];
    local[v] = fill[b] - vstart[b];
    order[fill[b]++] = v;
  }
  int64_t arcs = 0;
  for (int32_t b = 0; b < parts; ++b) {
    estart[b] = arcs;
    int64_t rel = 0;
    for (int32_t j = vstart[b]; j < vstart[b + 1]; ++j) {
      int32_t v = order[j];
      xadj_out[j + b] = rel;
      vwgt_out[j] = vwgt[v];
      for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
        int32_t u = adjncy[e];
        if (part[u] != b) continue;
        adjncy_out[arcs] = local[u];
        adjwgt_out[arcs] = adjwgt[e];
        ++arcs;
        ++rel;
      }
    }
    xadj_out[vstart[b + 1] + b] = rel;
  }
  estart[parts] = arcs;
  free(fill);
  free(local);
  return arcs;
}

/* Adaptive imbalance for a subgraph of weight cvp that will end up in kp of
 * the k blocks, d hierarchy levels from the bottom (equation (2)):
 * eps' = ((1 + eps) kp c(V) / (k c(V')))^(1/d) - 1, in parts per million,
 * rounded, never negative. */
int64_t pmo_adaptive_eps_ppm(int64_t eps_ppm, int64_t kp, int64_t k, int64_t cv,
                             int64_t cvp, int32_t d) {
  if (cvp <= 0 || d <= 0) return eps_ppm;
  double eps = (double)eps_ppm / 1e6;
  double base = ((1.0 + eps) * (double)kp) * (double)cv / ((double)k * (double)cvp);
  double e = pow(base, 1.0 / (double)d) - 1.0;
  int64_t ppm = llround(e * 1e6);
  return ppm > 0 ? ppm : 0;
}

typedef struct {
  int32_t levels;
  const int32_t *a;
  int64_t k, cv, eps_ppm;
  uint64_t seed;
  int32_t *part_out;
  int32_t status;
  const pmo_variants *var;
} hm_ctx;

static void hm_rec(hm_ctx *c, int32_t n, const int64_t *xadj, const int32_t *adjncy,
                   const int32_t *adjwgt, const int32_t *vwgt, const int32_t *orig,
                   int32_t i, int64_t base) {
  int64_t kp = 1;
  for (int32_t j = 0; j < i; ++j) kp *= c->a[j];
  int64_t cvp = 0;
  for (int32_t v = 0; v < n; ++v) cvp += vwgt[v];
  int64_t ppm = pmo_adaptive_eps_ppm(c->eps_ppm, kp, c->k, c->cv, cvp, i);
  int32_t ai = c->a[i - 1], one = 1;
  int32_t *part = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t st = pmo_map_v(n, xadj, adjncy, adjwgt, vwgt, 1, &ai, &one, ppm, c->seed, part, NULL,
                         c->var);
  if (st > c->status) c->status = st;
  int64_t pstride = kp / ai; /* P_{i-1} */
  if (i == 1) {
    for (int32_t v = 0; v < n; ++v) c->part_out[orig[v]] = (int32_t)(base + part[v]);
    free(part);
    return;
  }
  int64_t nnz = xadj[n];
  int32_t *vstart = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(ai > 0 ? ai + 1 : 1));
  int64_t *estart = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(ai > 0 ? ai + 1 : 1));
  int32_t *order = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t *sx = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n > 0 ? n + ai : ai));
  int32_t *sa = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int32_t *sw = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int32_t *sv = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *so = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  pmo_subgraphs(n, xadj, adjncy, adjwgt, vwgt, part, ai, vstart, estart, order, sx, sa, sw, sv);
  for (int32_t j = 0; j < n; ++j) so[j] = orig[order[j]];
  for (int32_t b = 0; b < ai; ++b)
    hm_rec(c, vstart[b + 1] - vstart[b], sx + vstart[b] + b, sa + estart[b], sw + estart[b],
           sv + vstart[b], so + vstart[b], i - 1, base + (int64_t)b * pstride);
  free(vstart);
  free(estart);
  free(order);
  free(sx);
  free(sa);
  free(sw);
  free(sv);
  free(so);
  free(part);
}

/* Recursive hierarchical multisection (Algorithm 2): partition the graph into
 * a_l blocks with the adaptive imbalance of equation (2), build the induced
 * subgraphs, partition each into a_{l-1} blocks, and so on down to a_1.  The
 * graph partitioner is pmo_map with the one-level hierarchy (a_i) and d = 1,
 * where J is twice the edge cut.  A vertex's block is the mixed-radix number
 * of its digits, a_1 least significant.  Returns 1 if any partitioning call
 * ended imbalanced, else 0. */
int32_t pmo_hm(int32_t n, const int64_t *xadj, const int32_t *adjncy,
               const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
               const int32_t *a, int64_t eps_ppm, uint64_t seed, int32_t *part_out) {
  return pmo_hm_v(n, xadj, adjncy, adjwgt, vwgt, levels, a, eps_ppm, seed, part_out, NULL);
}

/* pmo_hm with refinement variants for every partitioning call (e.g. the
 * "ultra" repetition, which the paper's GPU-HM-ultra uses). */
int32_t pmo_hm_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                 const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                 const int32_t *a, int64_t eps_ppm, uint64_t seed, int32_t *part_out,
                 const pmo_variants *var) {
  hm_ctx c;
  c.var = var;
  c.levels = levels;
  c.a = a;
  c.k = pmo_num_pes(levels, a);
  c.cv = 0;
  for (int32_t v = 0; v < n; ++v) c.cv += vwgt[v];
  c.eps_ppm = eps_ppm;
  c.seed = seed;
  c.part_out = part_out;
  c.status = 0;
  int32_t *orig = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t v = 0; v < n; ++v) orig[v] = v;
  hm_rec(&c, n, xadj, adjncy, adjwgt, vwgt, orig, levels, 0);
  free(orig);
  return c.status;
}
