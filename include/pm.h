/*
 * pm.h -- C ABI of the MI355X (gfx950) hierarchical process-mapping library.
 *
 * The library computes, on one GPU, the data-parallel hot path of the
 * integrated multilevel process-mapping method of "GPU-Accelerated Algorithms
 * for Process Mapping" (arXiv 2510.12196, Section 4.2): refinement of a
 * mapping Pi of a task graph onto the PEs of a hierarchical machine under the
 * communication cost J (Section 2), heavy-edge-matching coarsening, CSR
 * contraction, initial partitioning of the coarsest graph, and projection of
 * Pi through the levels.
 *
 * Common conventions
 * ------------------
 * Graph (pm_graph): undirected, both directions of every edge stored (CSR as
 *   in Section 3.4 "CSR Graph Format").  All arrays live in DEVICE memory owned
 *   by the caller and are only read:
 *     xadj   int64[n+1], xadj[0] = 0, non-decreasing, xadj[n] = nnz
 *     adjncy int32[nnz]  neighbour ids in [0,n), no self-loops, no duplicate
 *                        neighbour within a row, symmetric
 *     adjwgt int32[nnz]  edge weights > 0, w(u,v) = w(v,u)
 *     vwgt   int32[n]    vertex weights > 0
 *   Row order inside xadj ranges is irrelevant: every result is identical
 *   for any order of the entries of a row.
 *   Limits: n < 2^31, nnz < 2^31, sum(vwgt) < 2^31, sum(adjwgt) < 2^31.
 * Hierarchy (pm_hierarchy): a[0] = a_1 (PEs per processor, innermost level)
 *   ... a[levels-1] = a_l; d[i] = distance d_{i+1} of level i+1.  k = prod a.
 *   PE ids are mixed-radix numbers with a_1 the least significant digit;
 *   PEs x != y first share a component at level j (the smallest j with
 *   floor(x/P_j) == floor(y/P_j), P_j = a_1*...*a_j) and are at distance d_j;
 *   D(x,x) = 0.  Limits: 1 <= levels <= 8, a_i >= 1, 0 <= d_i < 2^30,
 *   sum over i of ceil(log2 a_i) <= 13 (k <= 8192 when all a_i are powers of
 *   two).
 * Mapping: int32[n] PE ids in [0,k), device memory.
 * eps: imbalance; L_max = ceil((1+eps) c(V) / k) evaluated exactly with eps
 *   rounded to parts per million.
 * stream: a hipStream_t passed as void*; NULL is the default stream.  Every
 *   function enqueues its work on that stream and returns after the results
 *   are complete (it synchronises the stream).
 * Scratch memory is allocated by the library (hipMalloc, cached per device and
 *   reused across calls, released by pm_release).  Calls may come from
 *   several host threads; each call uses its own scratch.
 * Return codes: PM_OK (0), PM_WARN_IMBALANCED (1, result written but not
 *   within L_max), negative on error (nothing written to outputs):
 *   PM_EINVAL (bad argument), PM_EGRAPH (graph fails validation, only checked
 *   when PM_FLAG_VALIDATE is given), PM_EOVERFLOW (a limit above is
 *   exceeded), PM_ENOMEM, PM_EHIP (HIP runtime error), PM_ENODEVICE.
 */
#ifndef PM_H
#define PM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM_OK 0
#define PM_WARN_IMBALANCED 1
#define PM_EINVAL (-1)
#define PM_EGRAPH (-2)
#define PM_EOVERFLOW (-3)
#define PM_ENOMEM (-4)
#define PM_EHIP (-5)
#define PM_ENODEVICE (-6)

#define PM_FLAG_VALIDATE 1u
/* pm_map: time every launch of the kernels listed under pm_map_stats with
 * start/stop events (adds a little host work per launch) */
#define PM_FLAG_KERNEL_TIMES 2u
/* pm_map: count the units of work of every launch of those kernels (extra
 * counting launches beside them; results unchanged, the map takes longer) */
#define PM_FLAG_KERNEL_COUNTS 4u
#define PM_TIMED_KERNELS 5

#define PM_MAX_LEVELS 8
#define PM_MAX_GRAPH_LEVELS 64

typedef struct pm_graph {
  int32_t n;
  int64_t nnz;
  const int64_t *xadj;
  const int32_t *adjncy;
  const int32_t *adjwgt;
  const int32_t *vwgt;
} pm_graph;

typedef struct pm_hierarchy {
  int32_t levels;
  int32_t a[PM_MAX_LEVELS];
  int32_t d[PM_MAX_LEVELS];
} pm_hierarchy;

/* Refinement variants (Section 4.2, the alternatives the paper discusses).
 *   PM_VARIANT_JET_FILTER: Jet's relaxed first filter of label propagation --
 *     a vertex whose best gain G is negative still enters the first-filter
 *     set when -G < floor(c * conn(v, own block)), c = jet_c_num / jet_c_den
 *     (1 <= jet_c_num <= 2^15, jet_c_den >= 1); the second filter is
 *     unchanged.
 *   PM_VARIANT_J_REBALANCE: rebalancing ranks moves by the gain of equation
 *     (1) instead of the edge-cut loss: the destination is the neighbour block
 *     within the cap with the largest gain (smaller block on ties), and the
 *     bucket of every source comes from that gain (for the pseudo-random
 *     destination too).
 * refine_repeats: the "ultra" repetition (Section 5: Jet's ultra
 *   configuration runs the complete refinement 18 times): in pm_map, pm_map_ex
 *   and the partitioning calls of pm_map_hm_ex, Algorithm 6 runs this many
 *   times at every level, run r from the result of run r - 1 (empty lock
 *   set) with seed + r for its pseudo-random choices; 0 or 1: once, at most
 *   64.  pm_refine_ex ignores it.
 * A NULL pm_options pointer, or variants = 0 and refine_repeats <= 1, is the
 * method as evaluated.  Invalid bits or constants: PM_EINVAL.  Host struct. */
#define PM_VARIANT_JET_FILTER 1u
#define PM_VARIANT_J_REBALANCE 2u
typedef struct pm_options {
  uint32_t variants;
  int32_t jet_c_num;
  int32_t jet_c_den;
  int32_t refine_repeats;  /* 0 or 1: once; "ultra": 18 */
} pm_options;

/* Statistics of one refinement run (Algorithm 6).  Host struct. */
typedef struct pm_refine_stats {
  int64_t j_initial;         /* J of the input mapping                    */
  int64_t j_final;           /* J of the returned mapping                 */
  int64_t maxw_initial;      /* heaviest block of the input mapping       */
  int64_t maxw_final;        /* heaviest block of the returned mapping    */
  int32_t iterations;        /* loop bodies executed                      */
  int32_t lp_iterations;
  int32_t weak_iterations;
  int32_t strong_iterations;
  int32_t feasible;          /* returned mapping within L_max             */
  int32_t pad_;
  double refine_ms;          /* device time of the refinement kernels     */
  int64_t arcs_processed;    /* iterations x nnz (logical arcs)           */
} pm_refine_stats;

/* Statistics of one multilevel run.  Host struct. */
typedef struct pm_map_stats {
  int32_t levels;                               /* graphs incl. the input */
  int32_t feasible;
  int64_t j_final;
  int64_t lmax;
  int32_t level_n[PM_MAX_GRAPH_LEVELS];
  int64_t level_nnz[PM_MAX_GRAPH_LEVELS];
  int32_t level_iterations[PM_MAX_GRAPH_LEVELS];
  int32_t level_hem_rounds[PM_MAX_GRAPH_LEVELS];
  double coarsen_ms;       /* matching rounds                             */
  double contract_ms;      /* coarse numbering + contraction              */
  double initial_ms;       /* coarsest graph to host, partition, back     */
  double uncoarsen_ms;     /* projections                                 */
  double refine_ms;        /* refinement incl. rebalancing, all levels    */
  double total_ms;         /* whole call, host wall clock                 */
  int64_t refine_arcs;     /* sum over levels of iterations x nnz         */
  /* Per timed kernel -- [0] label propagation phase 1, [1] phase 2,
   * [2] move accounting, [3] matching preference, [4] rebalancing
   * selection: with PM_FLAG_KERNEL_TIMES the launches and their summed
   * device time (start/stop events of each launch); with
   * PM_FLAG_KERNEL_COUNTS, summed over the launches, the vertices tiled
   * ([i][0]), the vertices that did the kernel's work ([i][1]: unlocked,
   * members of X, movers, vertices looking for a partner, sources) and
   * their arcs ([i][2]), and the algorithmic bytes those imply:
   *   [0] 12 per active arc (neighbour id, edge weight, neighbour block)
   *       + 25 per tiled vertex (row offsets, block, lock, target, gain)
   *   [1] 24 per active arc (neighbour id, weight, block, target, gain)
   *       + 16 per active vertex (row offsets, block, target) + 9 per tiled
   *       vertex (gain, moved flag)
   *   [2] 16 per active arc (neighbour id, weight, and the neighbour's
   *       block and target-or-none) + 24 per mover (row offsets, block,
   *       target, weight, and its new block written)
   *   [3] 12 per active arc (neighbour id, weight, and its weight-or-
   *       matched word) + 12 per tiled vertex (look-again flag, match
   *       word and weight, rounded up; the row offsets and preference
   *       of the vertices that look are left out)
   *   [4] 12 per active arc + 24 per source (row offsets, block, weight,
   *       key, destination) */
  int64_t kernel_launches[PM_TIMED_KERNELS];
  double kernel_ms[PM_TIMED_KERNELS];
  double kernel_bytes[PM_TIMED_KERNELS];
  int64_t kernel_units[PM_TIMED_KERNELS][3];
} pm_map_stats;

/* Library version string. */
const char *pm_version(void);
/* Message for a return code. */
const char *pm_strerror(int code);
/* Frees cached scratch memory of every device.  Not to be called while any
 * other pm_* call is running. */
void pm_release(void);

/* Launch parameters (process-wide).  They decide how vertices are mapped to
 * lanes and which vertices a launch tiles, never a result: every mapping,
 * J and status is the same under any valid setting.  The initial values come
 * from the environment variables of the same names in upper case with a PM_
 * prefix (PM_GROUP_V, ...), else the defaults below.
 *   group_v            vertices per lane group in a tile of the degree
 *                      classes up to 64 arcs: 1 or 2 (default 1)
 *   wave_min_count     a level uses the one-wave-per-vertex class (65..512
 *                      arcs) once it has this many such vertices, else they
 *                      take a workgroup each (default 8192; >= 1)
 *   hem_compact_min_n  from this level size on, matching rounds tile only the
 *                      vertices that must look again (default 2^18; >= 1)
 *   reb_compact_min_n  from this level size on, rebalancing tiles only the
 *                      vertices of overloaded blocks (default 2^19; >= 1)
 *   contract_rows_min_nnz  from this many arcs on, a level may be contracted
 *                      row by row (rows of at most 512 arcs merged in
 *                      registers, of at most 2048 in LDS, one radix sort over
 *                      the longer rows' arcs only) instead of by one radix
 *                      sort over all arcs (default 2^20; >= 1)
 *   contract_rows_long_pct  ... provided that coarse rows above 64 arcs hold
 *                      at most this percentage of the level's arcs
 *                      (default 100; 0..100)
 *   lp_cache           1: label propagation keeps the first filter's result
 *                      of a vertex while neither it nor a neighbour has moved
 *                      (Section 4.2, "Refinement": results are cached and
 *                      reused while the neighbourhood is unchanged); 0:
 *                      every round evaluates every unlocked vertex (default
 *                      0: the marking of moved neighbourhoods costs more
 *                      than the skipped evaluations save on the R-MAT
 *                      workload)
 *   graph_bodies       1: on levels whose loop bodies read nothing back, the
 *                      label-propagation and weak-rebalancing bodies of a
 *                      level are captured in HIP graphs the first time and
 *                      replayed (calls on a stream other than the null
 *                      stream); 0: every kernel is launched (default 0)
 * pm_set_tuning returns PM_EINVAL (nothing changed) for values outside these
 * ranges.  Calls already running may see either setting. */
typedef struct pm_tuning {
  int32_t group_v;
  int32_t wave_min_count;
  int32_t hem_compact_min_n;
  int32_t reb_compact_min_n;
  int32_t contract_rows_min_nnz;
  int32_t contract_rows_long_pct;
  int32_t lp_cache;
  int32_t graph_bodies;
} pm_tuning;
int pm_get_tuning(pm_tuning *out);
int pm_set_tuning(const pm_tuning *t);

/* J(Pi) = sum over all arcs (u,v) of w(u,v) * D(Pi(u),Pi(v)) (Section 2,
 * GPMP objective; both directions of each edge count, so J is twice the sum
 * over undirected edges).  part: device int32[n].  j_out: HOST int64. */
int pm_comm_cost(const pm_graph *g, const pm_hierarchy *h, const int32_t *part,
                 int64_t *j_out, uint32_t flags, void *stream);

/* pm_comm_cost without any allocation, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).
 * Same J and the same mapping check (a block id outside [0,k) returns
 * PM_EINVAL, *j_out = 0); the CSR structure and weights are trusted as
 * pm_comm_cost without PM_FLAG_VALIDATE trusts the structure.  Arguments as
 * for pm_comm_cost; more than INT32_MAX arcs returns PM_EOVERFLOW.  Its work
 * space is a fixed device array of the library (4096 partial sums, 33 280
 * bytes per device, kept until the process ends): any graph size fits it, as
 * a grid of at most 4096 workgroups walks the vertices.  Every call on
 * one device shares that array, so calls that overlap on a device (several
 * streams or threads at once) race and must be serialised by the caller.
 * Returns after the result is on the host (the stream is synchronised). */
int pm_comm_cost_noalloc(const pm_graph *g, const pm_hierarchy *h, const int32_t *part,
                         int64_t *j_out, void *stream);

/* Block weights c(V_b) for b in [0,k) (Section 2).  w_out: device int64[k]. */
int pm_block_weights(const pm_graph *g, const pm_hierarchy *h,
                     const int32_t *part, int64_t *w_out, void *stream);

/* One round of unconstrained label propagation (Section 4.2, Algorithm 4,
 * equation (1), implicit order by (gain desc, id asc), second filter under
 * the approximate future state, moved vertices locked).
 * part: device int32[n], in/out.  lock: device uint8[n], in/out (nonzero =
 * locked; on return exactly the moved vertices are locked).  target_out:
 * device int32[n] (best block, or own block when not in the first-filter
 * set).  gain_out: device int64[n] (INT64_MIN when not in that set).
 * moved_out: device uint8[n]. */
int pm_lp_round(const pm_graph *g, const pm_hierarchy *h, int32_t *part,
                uint8_t *lock, int32_t *target_out, int64_t *gain_out,
                uint8_t *moved_out, void *stream);
/* pm_lp_round with refinement variants (opts may be NULL). */
int pm_lp_round_ex(const pm_graph *g, const pm_hierarchy *h, int32_t *part,
                   uint8_t *lock, int32_t *target_out, int64_t *gain_out,
                   uint8_t *moved_out, const pm_options *opts, void *stream);

/* One weak (strong = 0) or strong (strong = 1) rebalancing round (Section
 * 3.2, Rebalancing, Algorithm 5) with the edge-cut loss; lmax and sigma as
 * host integers; (seed, level, iter) select the pseudo-random fallback
 * destinations.  part: device int32[n], in/out.  moved_out: device uint8[n]. */
int pm_rebalance(const pm_graph *g, const pm_hierarchy *h, int32_t strong,
                 int64_t lmax, int64_t sigma, uint64_t seed, int32_t level,
                 int32_t iter, int32_t *part, uint8_t *moved_out, void *stream);
/* pm_rebalance with refinement variants (opts may be NULL). */
int pm_rebalance_ex(const pm_graph *g, const pm_hierarchy *h, int32_t strong,
                    int64_t lmax, int64_t sigma, uint64_t seed, int32_t level,
                    int32_t iter, int32_t *part, uint8_t *moved_out,
                    const pm_options *opts, void *stream);

/* Refinement (Section 4.2, Algorithm 6): label propagation while balanced,
 * otherwise up to two weak then one strong rebalancing; keeps the best
 * mapping; stops after 12 loop bodies without sufficient improvement.
 * part: device int32[n], in/out (input mapping, returned best mapping).
 * level: tag mixed into the pseudo-random choices (0 for a single graph).
 * stats: host, may be NULL.  Returns PM_OK or PM_WARN_IMBALANCED. */
int pm_refine(const pm_graph *g, const pm_hierarchy *h, double eps,
              uint64_t seed, int32_t level, int32_t *part,
              pm_refine_stats *stats, void *stream);
/* pm_refine with refinement variants (opts may be NULL). */
int pm_refine_ex(const pm_graph *g, const pm_hierarchy *h, double eps,
                 uint64_t seed, int32_t level, int32_t *part,
                 pm_refine_stats *stats, const pm_options *opts, void *stream);

/* Heavy-edge matching rounds (Section 4.2, Matching): rating w^2/(c(u)c(v)),
 * exact comparison with a hash tie-break, mutual preference, rounds until no
 * new match; then two-hop matching, each step only while at most 75 % of the
 * vertices are matched: leaves (degree 1) sharing their neighbour, twins
 * (equal neighbourhood key; all isolated vertices form one group), relatives
 * sharing their matchmaker, paired in id order inside a group when the pair
 * fits L_max.  match_out: device int32[n] (partner, or the vertex itself).
 * rounds_out: host int32, may be NULL. */
int pm_hem(const pm_graph *g, int64_t lmax, uint64_t seed, int32_t level,
           int32_t *match_out, int32_t *rounds_out, void *stream);

/* Coarse numbering and contraction (Section 4.2, Contraction): coarse id =
 * rank of the smaller member; coarse vertex weight = sum; arcs mapped, self
 * loops dropped, parallel arcs fused with summed weights.  Outputs (device,
 * caller-allocated at the fine sizes): cmap int32[n], cxadj int64[n+1],
 * cadjncy int32[nnz], cadjwgt int32[nnz], cvwgt int32[n]; nc_out and
 * nnz_out are host.  Coarse rows come out sorted by neighbour id.
 * match: device int32[n], the partner of every vertex, the vertex itself or
 * -1 when unmatched; PM_EINVAL unless every partner points back. */
int pm_contract(const pm_graph *g, const int32_t *match, int32_t *cmap,
                int64_t *cxadj, int32_t *cadjncy, int32_t *cadjwgt,
                int32_t *cvwgt, int32_t *nc_out, int64_t *nnz_out,
                void *stream);

/* Initial partitioning (Section 4.2): hierarchical multisection (Section
 * 3.1, Algorithm 2) with a breadth-first split as the simple partitioner,
 * run on the host on a copy of the graph.  part_out: device int32[n]. */
int pm_initial_partition(const pm_graph *g, const pm_hierarchy *h,
                         int32_t *part_out, void *stream);

/* The whole multilevel mapping (Section 4.2): coarsen while n >= 8k (stop
 * when a level would keep more than 95 % of the vertices, at most 64
 * graphs), initial partitioning, then project and refine level by level.
 * part_out: device int32[n].  stats: host, may be NULL. */
int pm_map(const pm_graph *g, const pm_hierarchy *h, double eps,
           uint64_t seed, int32_t *part_out, pm_map_stats *stats,
           uint32_t flags, void *stream);
/* pm_map with refinement variants at every level (opts may be NULL). */
int pm_map_ex(const pm_graph *g, const pm_hierarchy *h, double eps,
              uint64_t seed, int32_t *part_out, pm_map_stats *stats,
              uint32_t flags, const pm_options *opts, void *stream);

/* Induced subgraphs of a partition (Section 4.1, Algorithm 1), all blocks at
 * once.  Block b's vertices are numbered in ascending input id order; its
 * subgraph keeps every arc whose two ends lie in b, in the input row order,
 * with the local ids and the arc weights.  part: device int32[n], every id in
 * [0, parts) (else PM_EINVAL, nothing defined written).  Outputs (device,
 * caller-allocated): vstart int32[parts+1] first position of each block in
 * order; estart int64[parts+1] first arc of each block; order int32[n] input
 * id per position; xadj_out int64[n+parts], block b's row offsets (relative to
 * its first arc) at [vstart[b]+b, vstart[b+1]+b]; adjncy_out and adjwgt_out
 * int32[nnz] (estart[parts] arcs used); vwgt_out int32[n] by position.
 * arcs_out: host, may be NULL, total arcs kept. */
int pm_subgraphs(const pm_graph *g, const int32_t *part, int32_t parts,
                 int32_t *vstart, int64_t *estart, int32_t *order,
                 int64_t *xadj_out, int32_t *adjncy_out, int32_t *adjwgt_out,
                 int32_t *vwgt_out, int64_t *arcs_out, void *stream);

/* Hierarchical multisection (Section 4.1, Algorithm 2, the GPU-HM variant):
 * partition into a_l blocks, then every block's induced subgraph into
 * a_{l-1} blocks, down to a_1; the partitioner is pm_map with the one-level
 * hierarchy (a_i) and d = 1.  A subgraph of weight c(V') that ends up in k'
 * = a_1 ... a_i of the k blocks, i levels from the bottom, gets the adaptive
 * imbalance of equation (2), eps' = ((1 + eps) k' c(V) / (k c(V')))^(1/i) - 1,
 * taken in whole parts per million (rounded, at least 0).  A vertex's block
 * is the mixed-radix number of its digits, a_1 least significant.  h is
 * checked as for pm_map; the partitioning reads only h->levels and h->a, and
 * j_out (host, may be NULL) receives J of the result under all of h.  The subgraphs of one level run
 * concurrently on `workers` threads (<= 0: 8), each with a stream of its
 * own; the result does not depend on the count.  part_out: device int32[n].
 * calls_out: host, may be NULL, number of partitioning calls.  Returns PM_OK
 * or PM_WARN_IMBALANCED if any partitioning call ended above its L_max. */
int pm_map_hm(const pm_graph *g, const pm_hierarchy *h, double eps,
              uint64_t seed, int32_t workers, int32_t *part_out,
              int64_t *j_out, int32_t *calls_out, void *stream);
/* pm_map_hm with refinement variants for every partitioning call (opts may
 * be NULL); refine_repeats = 18 is the paper's GPU-HM-ultra. */
int pm_map_hm_ex(const pm_graph *g, const pm_hierarchy *h, double eps,
                 uint64_t seed, int32_t workers, int32_t *part_out,
                 int64_t *j_out, int32_t *calls_out, const pm_options *opts,
                 void *stream);

/* ---------------------------------------------------------------------------
 * Many instances.  A job is one independent mapping instance: a device graph,
 * its own hierarchy, eps and seed, and a device output array.  Every job is
 * computed by exactly the code path of pm_map, so its mapping and status are
 * the ones pm_map returns for it, whatever else runs beside it.
 * ------------------------------------------------------------------------- */
typedef struct pm_map_job {
  pm_graph graph;          /* device arrays, owned by the caller, complete   */
  pm_hierarchy hierarchy;
  double eps;
  uint64_t seed;
  int32_t *part_out;       /* device int32[n]                               */
  int32_t status;          /* out: the instance's return code               */
  int32_t levels;          /* out: graphs in its hierarchy                  */
  int64_t j_final;         /* out: J of the returned mapping                */
  double ms;               /* out: wall time of the instance                */
} pm_map_job;

/* Batched mapping (many uneven task graphs at once): the jobs are
 * spread over `workers` host threads (0: 8), each with its own HIP stream and
 * scratch, so that the small kernels and host round trips of many instances
 * overlap on the device.  Jobs are started largest first.  `stream` is
 * synchronised before any job starts.  Returns PM_OK if every job has a
 * non-negative status, otherwise the first negative status. */
int pm_map_batch(pm_map_job *jobs, int32_t count, int32_t workers,
                 void *stream);

/* Estimated device scratch of one pm_map call on this graph and hierarchy
 * (bytes); the server admits jobs against its budget with it. */
int64_t pm_job_footprint(const pm_graph *g, const pm_hierarchy *h);

/* Serving with continuous batching: a server owns `workers` host threads with
 * their own streams.  Submitted jobs wait in a FIFO queue and are admitted in
 * order as soon as the summed footprint of the admitted, unfinished jobs
 * plus theirs fits `hbm_budget_bytes` and a worker is free; jobs that
 * arrive while others run overlap with them on the device.  The job's device
 * arrays must be complete when it is submitted and stay valid until it is
 * done. */
typedef struct pm_server pm_server;
pm_server *pm_server_create(int64_t hbm_budget_bytes, int32_t workers);
/* Returns a ticket >= 0, or PM_EINVAL / PM_ENOMEM (footprint above the
 * budget).  The job struct is copied. */
int64_t pm_server_submit(pm_server *srv, const pm_map_job *job);
/* 1 if the ticket is done, 0 if queued or running, PM_EINVAL if unknown. */
int pm_server_poll(pm_server *srv, int64_t ticket);
/* Blocks until the ticket is done; copies the finished job (status, levels,
 * j_final, ms) into *out (may be NULL) and the latency from submission to
 * completion into *latency_ms (may be NULL), then releases the ticket.
 * Returns the job's status (PM_EINVAL for an unknown ticket).  Two threads
 * must not wait on the same ticket. */
int pm_server_wait(pm_server *srv, int64_t ticket, pm_map_job *out,
                   double *latency_ms);
/* Waits for every submitted job, then stops the workers. */
void pm_server_destroy(pm_server *srv);

#ifdef __cplusplus
}
#endif
#endif
