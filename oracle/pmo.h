/*
 * pmo.h -- CPU oracle for hierarchical process mapping (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of what the GPU path computes, written from the paper
 * "GPU-Accelerated Algorithms for Process Mapping" (arXiv 2510.12196).  It is
 * used by tests/, by the smoke check and by the benchmark's CPU-baseline leg,
 * and by nothing else.  It shares no code with the GPU library.
 *
 * Conventions (the same for every function):
 *   graph   : CSR with both directions of every undirected edge stored
 *             (Section 3.4, "CSR Graph Format"): xadj int64[n+1], adjncy
 *             int32[nnz], adjwgt int32[nnz] (> 0, symmetric), vwgt int32[n]
 *             (> 0).  All pointers are host pointers.
 *   hierarchy: levels l in [1,8], a[0] = a_1 (PEs per processor, innermost)
 *             ... a[l-1] = a_l; d[i] = d_{i+1}.  k = a_1 * ... * a_l.
 *   part    : int32[n] block (PE) ids in [0,k).
 *   eps_ppm : imbalance in parts per million (eps = 0.03 -> 30000).
 * All arithmetic is integer: int64 for costs, gains and block weights.
 */
#ifndef PMO_H
#define PMO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* statistics of one refinement run (Algorithm 6) */
typedef struct {
  int64_t j_initial;        /* J of the input mapping                      */
  int64_t j_final;          /* J of the returned mapping                   */
  int64_t maxw_initial;     /* heaviest block of the input mapping         */
  int64_t maxw_final;       /* heaviest block of the returned mapping      */
  int32_t iterations;       /* loop bodies executed                        */
  int32_t lp_iterations;
  int32_t weak_iterations;
  int32_t strong_iterations;
  int32_t feasible;         /* returned mapping satisfies L_max            */
  int32_t pad_;
} pmo_refine_stats;

#define PMO_MAX_LEVELS 64
/* statistics of one multilevel run */
typedef struct {
  int32_t levels;                         /* graphs in the hierarchy (>= 1) */
  int32_t feasible;
  int64_t j_final;
  int64_t lmax;
  int32_t level_n[PMO_MAX_LEVELS];
  int64_t level_nnz[PMO_MAX_LEVELS];
  int32_t level_iterations[PMO_MAX_LEVELS];  /* refinement loop bodies      */
  int32_t level_hem_rounds[PMO_MAX_LEVELS];  /* rounds that built level t+1 */
  double refine_seconds;                     /* time inside refinement      */
  double total_seconds;
} pmo_map_stats;

/* Refinement variants (Section 4.2): all zero = the method as evaluated.
 *   jet_c_num / jet_c_den: with jet_c_num > 0, Jet's relaxed first filter of
 *     label propagation, c = jet_c_num / jet_c_den (jet_c_den > 0);
 *   j_rebalance: rebalancing by the J gain instead of the edge-cut loss;
 *   refine_repeats: the "ultra" repetition of Section 5 -- the complete
 *     refinement (Algorithm 6) runs this many times at every level of a
 *     multilevel map (0 or 1: once). */
typedef struct {
  int32_t jet_c_num;
  int32_t jet_c_den;
  int32_t j_rebalance;
  int32_t refine_repeats;
} pmo_variants;

/* ---- hierarchy and objective (Section 2) ---- */
int64_t pmo_num_pes(int32_t levels, const int32_t *a);
int32_t pmo_distance(int32_t levels, const int32_t *a, const int32_t *d,
                     int32_t x, int32_t y);
int64_t pmo_comm_cost(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                      const int32_t *adjwgt, const int32_t *part,
                      int32_t levels, const int32_t *a, const int32_t *d);
void pmo_block_weights(int32_t n, const int32_t *vwgt, const int32_t *part,
                       int64_t k, int64_t *w_out);
int64_t pmo_lmax(int64_t total_weight, int64_t k, int64_t eps_ppm);
int64_t pmo_gain(const int64_t *xadj, const int32_t *adjncy,
                 const int32_t *adjwgt, const int32_t *part,
                 int32_t levels, const int32_t *a, const int32_t *d,
                 int32_t v, int32_t b);

/* ---- counter-based hash (splitmix64 output function) ---- */
uint64_t pmo_hash(uint64_t seed, uint64_t word);

/* ---- refinement (Section 4.2, Algorithms 4, 5 and 6) ---- */
void pmo_lp_round(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                  const int32_t *adjwgt, int32_t levels, const int32_t *a,
                  const int32_t *d, int32_t *part, uint8_t *lock,
                  int32_t *target_out, int64_t *gain_out, uint8_t *moved_out);
void pmo_rebalance(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                   const int32_t *adjwgt, const int32_t *vwgt, int64_t k,
                   int32_t strong, int64_t lmax, int64_t sigma, uint64_t seed,
                   int32_t level, int32_t iter, int32_t *part,
                   uint8_t *moved_out);
int64_t pmo_sigma(int64_t lmax, int64_t total_weight, int64_t k);
void pmo_lp_round_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                    const int32_t *adjwgt, int32_t levels, const int32_t *a,
                    const int32_t *d, int32_t *part, uint8_t *lock,
                    int32_t *target_out, int64_t *gain_out, uint8_t *moved_out,
                    const pmo_variants *var);
void pmo_rebalance_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                     const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                     const int32_t *a, const int32_t *d, int64_t k,
                     int32_t strong, int64_t lmax, int64_t sigma, uint64_t seed,
                     int32_t level, int32_t iter, int32_t *part,
                     uint8_t *moved_out, const pmo_variants *var);
int32_t pmo_refine_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                     const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                     const int32_t *a, const int32_t *d, int64_t eps_ppm,
                     uint64_t seed, int32_t level, int32_t *part,
                     pmo_refine_stats *stats, const pmo_variants *var);
int32_t pmo_refine_trace(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                         const int32_t *adjwgt, const int32_t *vwgt,
                         int32_t levels, const int32_t *a, const int32_t *d,
                         int64_t eps_ppm, uint64_t seed, int32_t level,
                         int32_t *part, pmo_refine_stats *stats,
                         const pmo_variants *var, int32_t trace_cap,
                         char *kind, int64_t *j_after, int64_t *imb_after,
                         int32_t *counter);
int32_t pmo_refine(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                   const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                   const int32_t *a, const int32_t *d, int64_t eps_ppm,
                   uint64_t seed, int32_t level, int32_t *part,
                   pmo_refine_stats *stats);

/* ---- coarsening (Section 4.2: matching, contraction) ---- */
int32_t pmo_hem(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                const int32_t *adjwgt, const int32_t *vwgt, int64_t lmax,
                uint64_t seed, int32_t level, int32_t *match_out);
int32_t pmo_coarse_map(int32_t n, const int32_t *match, int32_t *cmap_out);
int64_t pmo_contract(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                     const int32_t *adjwgt, const int32_t *vwgt,
                     const int32_t *cmap, int32_t nc, int64_t *cxadj,
                     int32_t *cadjncy, int32_t *cadjwgt, int32_t *cvwgt);

/* ---- initial partitioning and the multilevel driver ---- */
void pmo_initial_partition(int32_t n, const int64_t *xadj,
                           const int32_t *adjncy, const int32_t *vwgt,
                           int32_t levels, const int32_t *a, int32_t *part_out);
int32_t pmo_map(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                const int32_t *a, const int32_t *d, int64_t eps_ppm,
                uint64_t seed, int32_t *part_out, pmo_map_stats *stats);
int32_t pmo_map_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                  const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                  const int32_t *a, const int32_t *d, int64_t eps_ppm,
                  uint64_t seed, int32_t *part_out, pmo_map_stats *stats,
                  const pmo_variants *var);

/* ---- hierarchical multisection (Section 4.1, Algorithms 1 and 2) ---- */
int64_t pmo_subgraphs(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                      const int32_t *adjwgt, const int32_t *vwgt, const int32_t *part,
                      int32_t parts, int32_t *vstart, int64_t *estart, int32_t *order,
                      int64_t *xadj_out, int32_t *adjncy_out, int32_t *adjwgt_out,
                      int32_t *vwgt_out);
int64_t pmo_adaptive_eps_ppm(int64_t eps_ppm, int64_t kp, int64_t k, int64_t cv,
                             int64_t cvp, int32_t d);
int32_t pmo_hm(int32_t n, const int64_t *xadj, const int32_t *adjncy,
               const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
               const int32_t *a, int64_t eps_ppm, uint64_t seed, int32_t *part_out);
int32_t pmo_hm_v(int32_t n, const int64_t *xadj, const int32_t *adjncy,
                 const int32_t *adjwgt, const int32_t *vwgt, int32_t levels,
                 const int32_t *a, int64_t eps_ppm, uint64_t seed, int32_t *part_out,
                 const pmo_variants *var);

#ifdef __cplusplus
}
#endif
#endif
