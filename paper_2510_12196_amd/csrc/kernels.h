// kernels.h -- host-side launchers of the gfx950 kernels.
#pragma once

#include "pm_internal.h"

namespace pm {

// Small device-side status block for read-backs (one per call).
struct Status {
  int64_t dj;          // J change accumulated by apply_moves
  int64_t maxw;        // heaviest block (max_block)
  int64_t j;           // full J (comm_cost)
  int32_t count;       // generic counter (matches, sources, ...)
  int32_t n_elig_weak;   // blocks within the weak rebalancing cap (sigma)
  int32_t n_elig_strong; // blocks within L_max
  int64_t aux;         // generic 64-bit result
};

// Label propagation's per-vertex result: block, target and gain (one 16-byte
// record, so that phase 2 gathers a neighbour's in one load).
struct __align__(16) LpRec {
  int32_t p;
  int32_t t;
  int64_t g;
};

// A status publication: the kernel that ends a step copies the Status into
// mapped host memory (host, device view) and then stores seq into seq_slot;
// the host polls seq_slot.  host == nullptr: no publication.
struct Pub {
  Status *host;
  int64_t *seq_slot;
  int64_t seq;
  // with a device counter the sequence number is the counter, incremented
  // (a publication captured in a graph then releases a new number on every
  // replay); the host expects the same numbers in the same order
  int64_t *seq_ctr = nullptr;
};

// End of a refinement step, run by one workgroup of the commit: the heaviest
// block, the J change and the blocks eligible as rebalancing destinations
// for the next step, into the device status.
struct StepEnd {
  Hier h;
  int64_t *w;            // block weights (final when the epilogue runs)
  int64_t *dj_stripes;   // folded into st->dj (nullptr: st->dj untouched)
  int64_t sigma, lmax;   // caps of weak and strong rebalancing
  int32_t *elig_weak;    // blocks with w <= sigma, ascending
  int32_t *elig_strong;  // blocks with w <= L_max, ascending
  Status *st;
  int64_t *body_ctr = nullptr;  // loop bodies done (incremented by each step end)
  Pub pub{};  // publication of the status at the end (host == nullptr: none)
};
// StepEnd alone, as one workgroup (the start of a level).
void step_status(const StepEnd &E, hipStream_t s);

// ---- device helpers for the epilogues ----------------------------------------
// load through the device-coherent level (skips a possibly stale CU cache)
__device__ __forceinline__ int64_t agent_load(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t agent_load(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Thread 0 copies the status words to the host mirror, then releases seq.
// The caller orders the status stores before (fence + barrier).
__device__ __forceinline__ void publish_dev(const Status *st, const Pub &p) {
  if (!p.host || threadIdx.x != 0) return;
  const int64_t *src = reinterpret_cast<const int64_t *>(st);
  int64_t *dst = reinterpret_cast<int64_t *>(p.host);
  for (size_t i = 0; i < sizeof(Status) / sizeof(int64_t); ++i) dst[i] = agent_load(src + i);
  int64_t seq = p.seq;
  if (p.seq_ctr) {
    seq = *p.seq_ctr + 1;
    *p.seq_ctr = seq;
  }
  __threadfence_system();
  __hip_atomic_store(p.seq_slot, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Striped accumulator buffers of one call (kStripes x 16 int64 each, zeroed
// at creation and by every fold).
struct Stripes {
  int64_t *a;   // sums of J / J changes
  int64_t *b;   // counts
};
// Copies *dev into the mapped host mirror (device view host_dev), then stores
// seq into *seq_dev, all with system-scope visibility.
void publish_status(const Status *dev, Status *host_dev, int64_t *seq_dev, int64_t seq,
                    hipStream_t s, int64_t *seq_ctr = nullptr);
// Adds up the stripes into *out64 (if non-null) or *out32, clears them;
// publishes if pub.host.
void fold_stripes(int64_t *stripes, int64_t *out64, int32_t *out32, hipStream_t s,
                  const Pub &pub = Pub{nullptr, nullptr, 0}, const Status *st = nullptr);
int stripe_words();
unsigned classed_grid(const Classes &cl);   // one tile per workgroup
unsigned capped_grid(const Classes &cl);    // at most kMaxGrid workgroups

// ---- optional per-launch kernel timing --------------------------------------
enum { KT_LP1 = 0, KT_LP2, KT_APPLY, KT_HEM, KT_REB, NKT };
// What a counting launch counts as active (see count_units).
enum { CU_UNLOCKED = 0, CU_IN_X, CU_MOVED, CU_HEM_ACTIVE, CU_SOURCE };
constexpr int kCountStripes = 32;
struct KernelTimer {
  bool timing = false;    // start/stop events around every timed launch
  bool counting = false;  // counting launches beside the timed ones
  std::vector<hipEvent_t> start[NKT], stop[NKT];
  int64_t *dcount = nullptr;  // device [NKT][3][kCountStripes][kStripeStride]
  // event pair for one launch of kernel id (nullptrs when not timing)
  void pair(int id, hipEvent_t &a, hipEvent_t &b);
  // the counters of kernel id (nullptr when not counting)
  int64_t *counters(int id);
  // sums the elapsed times and reads the counters; call after the stream has
  // been synchronised
  void finish(int64_t *launches, double *ms, double *bytes_out, int64_t (*units)[3]);
  ~KernelTimer();
};
// Counting launch: over the tiled vertices of cl, the number of vertices,
// of those active by `what`, and of their arcs, into out (nullptr: none).
struct CountArgs {
  const uint8_t *flag8;  // lock (CU_UNLOCKED) or moved (CU_MOVED)
  const uint8_t *dirty;  // CU_UNLOCKED with result caching: only dirty vertices
  const LpRec *rec;      // CU_IN_X
  const int32_t *key;    // CU_SOURCE
  const int32_t *match;  // CU_HEM_ACTIVE
  const int32_t *pref;
};
void count_units(const Classes &cl, const int64_t *xadj, int what, const CountArgs &a,
                 int64_t *out, hipStream_t s);
// timer of the call running on this host thread (nullptr: no timing)
extern thread_local KernelTimer *tl_timer;

// ---- per-level setup ------------------------------------------------------
// Classifies every vertex by degree and builds the class lists.  `list` must
// hold n entries.  Synchronises the stream (reads the class sizes).
Classes build_classes(Arena &ar, const DGraph &g, int32_t *list, Status *st_dev,
                      Status *st_host, hipStream_t s);
int32_t classes_workgroups(const Classes &cl);
// The same classes laid out as tiles of V vertices per lane group (ISO: V
// per thread); BIG keeps one vertex per workgroup.
// w_as_big: W vertices one per tile (the block path), for kernels without
// the per-wave histogram
Classes tiled(const Classes &cl, int V, bool w_as_big = false);
// Vertices per lane group of the staged kernels: 1 (PM_GROUP_V=2 selects
// 2).
int group_v();

// ---- mapping conversion ---------------------------------------------------
void ids_to_codes(const Hier &h, const int32_t *ids, int32_t *codes, int32_t n, hipStream_t s);
void codes_to_ids(const Hier &h, const int32_t *codes, int32_t *ids, int32_t n, hipStream_t s);
// flags any id outside [0,k) into st->count
void check_ids(const Hier &h, const int32_t *ids, int32_t n, int64_t *stripes, Status *st,
               hipStream_t s);

// ---- objective and balance ------------------------------------------------
void comm_cost(const DGraph &g, const Classes &cl, const Hier &h, const int32_t *part,
               int64_t *stripes, Status *st, hipStream_t s);   // st->j = J
void block_weights(const DGraph &g, const Hier &h, const int32_t *part, int64_t *w,
                   hipStream_t s);                     // w[0..2^bits)

// ---- refinement variants (Section 4.2) ----------------------------------------
// jet_num > 0: Jet's relaxed first filter, c = jet_num / jet_den;
// j_rebalance: rebalancing by the J gain instead of the edge-cut loss.
struct Variants {
  int64_t jet_num = 0;
  int64_t jet_den = 1;
  bool j_rebalance = false;
  int32_t repeats = 1;  // runs of Algorithm 6 per level of a multilevel map
};

// ---- label propagation (Algorithm 4) --------------------------------------
// Phase 1 writes rec[v] = {block, target, gain} for every vertex (gain
// kNotInX outside X).  dirty != nullptr: result caching (unlocked vertices
// that are not dirty keep their last record; see apply_moves)
void lp_phase1(const DGraph &g, const Classes &cl, const Hier &h, const int32_t *part,
               const uint8_t *lock, LpRec *rec, hipStream_t s,
               const Variants &var = Variants{}, uint8_t *dirty = nullptr);
// target[v], gain[v] <- rec[v] (the per-phase entry point's outputs)
void unpack_lp(const LpRec *rec, int32_t *target, int64_t *gain, int64_t n, hipStream_t s);
// Phase 2 writes moved[v] and pn[v] = {block, moved ? target : -1} (every
// vertex with a neighbour), the records apply_moves gathers.
void lp_phase2(const DGraph &g, const Classes &cl, const Hier &h, const LpRec *rec,
               uint8_t *moved, int2 *pn, hipStream_t s);
// Applies moved[v] -> part[v] = target[v]; accumulates the exact J change into
// dj_stripes and the block weight changes into w (through the weight-delta
// stripes wst, zero on entry and on return); sets lock = moved if lock != 0.
// With end != nullptr the commit's last workgroup runs the StepEnd epilogue
// (end->w must be w, end->dj_stripes dj_stripes).
constexpr int kWeightStripes = 32;
int weight_stripes(const Hier &h, int64_t n);   // stripes in use (power of two)
int64_t *alloc_weight_stripes(Arena &ar, const Hier &h, hipStream_t s);
// dirty != nullptr: marks every mover and every neighbour of a mover (the
// result caching of label propagation)
// pn: g.n records {block, moved ? target : -1} gathered for the neighbours of
// movers (written by label propagation's phase 2, or by the rebalancing
// round); every mover must be in cl, and its target goes to part[] where it
// is handled (no tile reads part[] meanwhile).
void apply_moves(const DGraph &g, const Classes &cl, const Hier &h, int32_t *part,
                 const uint8_t *moved, uint8_t *lock, int64_t *w, int64_t *wst,
                 int64_t *dj_stripes, const StepEnd *end, const int2 *pn, hipStream_t s,
                 uint8_t *dirty = nullptr);

// ---- rebalancing (Algorithm 5) --------------------------------------------
// Rebalancing loss buckets per block, and the stripes of the bucket-weight
// and accepted-weight accumulators (a stripe per workgroup index modulo the
// count: their atomics are bound by contention on hot counters).
constexpr int kBuckets = 64;
constexpr int kBucketStripes = 32;
struct RebalanceBuffers {
  int32_t *key;        // n: (block << 6 | bucket) for sources, -1 otherwise
  int32_t *dest;       // n: chosen destination
  uint8_t *reject;     // n: strong rounds, movers refused by their destination
  int32_t *rlist;      // n: strong rounds, the refused movers in id order
  int32_t *rcount;     // 1: their number
  int64_t *resid;      // 2^bits: residual capacity per code
  int32_t *elig_weak;  // 2^bits: blocks within sigma, ascending
  int32_t *elig_strong;// 2^bits: blocks within L_max, ascending
  int64_t *bw;         // 32 x 2^bits x 64 bucket weights (kept zero between rounds)
  int64_t *acc;        // 32 x 2^bits accepted weights (kept zero between rounds)
  int32_t *crit;       // 2^bits
  int64_t *need;       // 2^bits
  int32_t *tcrit;      // 2^bits
  int64_t *tneed;      // 2^bits
  int32_t *tsum;       // 2^bits x ntiles
  int64_t *rstart;     // 2^bits: first position of a code in a weight class
  int32_t *rweight;    // n: weights of the refused movers, in list order
  int32_t tile;        // ids per tile
  int32_t ntiles;
};
RebalanceBuffers alloc_rebalance(Arena &ar, int64_t n, const Hier &h, hipStream_t s);
// One weak/strong rebalancing round: writes moved/target for every vertex,
// and pn (apply's records), ready for apply_moves.  The eligible destinations (rb.elig_*, counts in
// *st_dev) must be those of the current weights (StepEnd / step_status).  No
// host synchronisation.
// Rebalancing sources on large levels: the vertices of blocks heavier than
// lmax, compacted in class order (list_out, off_out as for compact_bounds);
// every other vertex gets key -1 (not a source) here.
void reb_sources(Arena &ar, const Classes &cl, int32_t n, const int32_t *part, const int64_t *w,
                 int64_t lmax, int32_t *key, int32_t *list_out, int32_t *off_out, hipStream_t s);
// body_ctr != nullptr: the pseudo-random destinations use
// mix_hash(hseed, *body_ctr + 1) read on the device (a round captured in a
// graph then draws for the body it runs in) instead of hseed itself.
void rebalance_round(Arena &ar, const DGraph &g, const Classes &cl, const Hier &h, bool strong,
                     int64_t lmax, int64_t sigma, int64_t total, uint64_t hseed,
                     const int32_t *part, const int64_t *w, int32_t *target, uint8_t *moved,
                     int2 *pn, const RebalanceBuffers &rb, Status *st_dev, hipStream_t s,
                     const Variants &var = Variants{}, const int64_t *body_ctr = nullptr);

// ---- induced subgraphs (Section 4.1, Algorithm 1) ----------------------------
// Layout of all blocks' subgraphs, concatenated in block order (device
// arrays): vstart[parts+1] first position of each block, estart[parts+1]
// first arc, order[n] original id per position, xadj[n+parts] block b's
// relative row offsets at [vstart[b]+b, vstart[b+1]+b], adjncy/adjwgt
// (local ids, original row order), vwgt[n] by position, wsum[parts] block
// weights (may be nullptr).
struct SubgraphOut {
  int32_t *vstart;
  int64_t *estart;
  int32_t *order;
  int64_t *xadj;
  int32_t *adjncy;
  int32_t *adjwgt;
  int32_t *vwgt;
  int64_t *wsum;
};
// part: device int32[n] in [0, parts) (checked by the caller).
void subgraphs(Arena &ar, const DGraph &g, const int32_t *part, int32_t parts,
               const SubgraphOut &o, hipStream_t s);
// flags into *bad (device int32, cleared here) whether any part[v] is
// outside [0, parts)
void check_parts(const int32_t *part, int32_t n, int32_t parts, int32_t *bad, hipStream_t s);
void compose_ids(int32_t n, const int32_t *orig, const int32_t *order, int32_t *out,
                 hipStream_t s);
void scatter_blocks(int32_t n, const int32_t *orig, const int32_t *part, int32_t base,
                    int32_t *part_out, hipStream_t s);

// Hierarchical multisection (Section 4.1, Algorithm 2) with the multilevel
// mapper as partitioner; part_out: device ids in [0, k).  Returns PM_OK or
// PM_WARN_IMBALANCED (some partitioning call ended above its L_max).
int hm_impl(const DGraph &dg, const int32_t *a, int32_t levels, double eps, uint64_t seed,
            int32_t *part_out, int32_t workers, int32_t *calls_out, hipStream_t s,
            const Variants &var = Variants{});
// equation (2) in parts per million, rounded, never negative
int64_t adaptive_eps_ppm(int64_t eps_ppm, int64_t kp, int64_t k, int64_t cv, int64_t cvp,
                         int32_t d);
// Structure and overflow validation (validate.hip); *total_vwgt = c(V).
void validate_graph(Arena &ar, const DGraph &g, bool full, int64_t *total_vwgt, hipStream_t s);

// ---- matching and contraction ---------------------------------------------
// cm: per vertex its weight while unmatched, -1 once matched (kept by
// hem_commit), so that a neighbour costs one gather
// hact: per vertex 1 if it looks for a partner this round (all at the
// first round of a level; then written by hem_commit).
void hem_prefer(const DGraph &g, const Classes &cl, int64_t lmax, uint64_t hseed,
                const int32_t *match, int32_t *pref, const int32_t *cm, const uint8_t *hact,
                hipStream_t s);
// The same over the compacted class list (list, with its NCLS + 1 class
// offsets dev_off on the device) of a level whose full class list is cl
// (whose tiles bound the grid); nothing is read back.
void hem_prefer_dev(const DGraph &g, const Classes &cl, const int32_t *list,
                    const int32_t *dev_off, int64_t lmax, uint64_t hseed, const int32_t *match,
                    int32_t *pref, const int32_t *cm, const uint8_t *hact, hipStream_t s);
// st->count = new matches.  counter: 65 64-bit completion counters, zero
// between launches.
// Given the positions pos[0..*count) (ascending) of selected entries of the
// class list, writes their vertex ids (list_out) and the class offsets into
// that compacted list (off_out, NCLS + 1 entries).
void compact_bounds(int32_t n, const Classes &cl, const int32_t *pos, const int32_t *count,
                    int32_t *list_out, int32_t *off_out, hipStream_t s);
// Compacts the vertices that must recompute their preference: list_out
// (device int32[n]) gets their ids in class order, off_out (device
// int32[NCLS + 1]) the class offsets into it.
void hem_compact(Arena &ar, const Classes &cl, int32_t n, const uint8_t *hact,
                 int32_t *list_out, int32_t *off_out, hipStream_t s);
// One matching commit; the number of new pairs goes to st->count and, if
// count_out is not null, to *count_out (device).
void hem_commit(int32_t n, const int32_t *pref, int32_t *match, int32_t *cm, uint8_t *hact,
                uint64_t *counter, Status *st, int32_t *count_out, hipStream_t s);
// Two-hop matching step (TWOHOP_LEAF / _TWIN / _RELATIVE): groups unmatched
// vertices and pairs each group in id order.  Returns the vertices matched.
// Synchronises the stream.
enum { TWOHOP_LEAF = 0, TWOHOP_TWIN = 1, TWOHOP_RELATIVE = 2 };
int64_t two_hop_step(Arena &ar, const DGraph &g, const Classes &cl, int mode, uint64_t tseed,
                     int64_t lmax, int32_t *match, int64_t *stripes, Status *st_dev,
                     Status *st_host, hipStream_t s);
void hem_finish(int32_t n, int32_t *match, int32_t *leader, hipStream_t s);
void coarse_ids(int32_t n, const int32_t *match, const int32_t *rank, int32_t *cmap,
                hipStream_t s);
void coarse_vwgt(int32_t n, const int32_t *match, const int32_t *cmap, const int32_t *vwgt,
                 int32_t *cvwgt, hipStream_t s);
void contract_keys(const DGraph &g, const Classes &cl, const int32_t *cmap, int bits,
                   uint64_t *key, int32_t *val, int64_t *stripes, Status *st,
                   hipStream_t s);   // st->count = arcs inside coarse vertices
// Over the nnz sorted keys, of which the last *self (device) are the
// self-loop sentinels.
// *bad = 1 unless match is an involution with -1 for unmatched vertices
void check_match(int32_t n, const int32_t *match, int32_t *bad, hipStream_t s);
// Row-local contraction: ub / ubig (ub when above 2048, else 0) per coarse row;
// *above64 = sum of ub over rows above 64
void contract_rowub(const DGraph &g, const int32_t *match, const int32_t *cmap, int32_t *ub,
                    int32_t *ubig, int64_t *above64, hipStream_t s);
void contract_stage(const DGraph &g, const Classes &cl, const int32_t *match, const int32_t *cmap,
                    const int64_t *uxadj, uint32_t *scu, int32_t *sw, hipStream_t s);
void contract_rows(const Classes &rc, const int64_t *uxadj, uint32_t *scu, int32_t *sw,
                   int32_t *rowcnt, hipStream_t s);
void contract_mid_rows(const int32_t *list, int32_t nl, const int64_t *uxadj, uint32_t *scu,
                       int32_t *sw, int32_t *rowcnt, hipStream_t s);
void contract_long_rows(Arena &ar, const int32_t *list, int32_t nl, int64_t m, int32_t nc,
                        const int64_t *uxadj, const int64_t *rstart, uint32_t *scu, int32_t *sw,
                        int32_t *rowcnt, hipStream_t s);
void contract_copy(const Classes &rc, const int64_t *uxadj, const int64_t *cxadj,
                   const uint32_t *scu, const int32_t *sw, int32_t *cadj, int32_t *cw,
                   hipStream_t s);
void contract_heads(int64_t nnz, const int32_t *self, const uint64_t *key, int32_t *head,
                    hipStream_t s);
void contract_emit(int64_t nnz, const int32_t *self, const uint64_t *key, const int32_t *val,
                   const int32_t *head, const int32_t *pos, int bits, int32_t *cadj, int32_t *cw,
                   int32_t *rowcnt, hipStream_t s);
void project(int32_t n, const int32_t *cmap, const int32_t *coarse, int32_t *fine,
             hipStream_t s);

// ---- whole mapping ------------------------------------------------------------
// The multilevel mapping of one instance on `stream` (throws Error).
int map_impl(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed,
             int32_t *part_out, pm_map_stats *stats, uint32_t flags, hipStream_t stream,
             const Variants &var = Variants{});

// ---- misc -----------------------------------------------------------------
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);

}  // namespace pm
