// driver.cpp -- host orchestration and the C ABI of the process-mapping library.
#include <chrono>
#include <cmath>
#include <functional>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_ip.h"
#include "kernels.h"
#include "prim.h"

namespace pm {

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------
Hier make_hier(const pm_hierarchy *ph) {
  if (!ph) throw Error(PM_EINVAL, "hierarchy is NULL");
  if (ph->levels < 1 || ph->levels > PM_MAX_LEVELS)
    throw Error(PM_EINVAL, "hierarchy levels must be in [1,8]");
  Hier h{};
  h.levels = ph->levels;
  h.P[0] = 1;
  h.shift[0] = 0;
  h.pow2 = 1;
  for (int i = 0; i < h.levels; ++i) {
    const int32_t a = ph->a[i], d = ph->d[i];
    if (a < 1) throw Error(PM_EINVAL, "a_i must be >= 1");
    if (d < 0 || d >= (1 << 30)) throw Error(PM_EINVAL, "d_i must be in [0, 2^30)");
    int width = 0;
    while ((1 << width) < a) ++width;
    h.a[i] = a;
    h.d[i] = d;
    h.shift[i + 1] = h.shift[i] + width;
    h.P[i + 1] = h.P[i] * a;
    if (h.P[i + 1] > INT32_MAX) throw Error(PM_EOVERFLOW, "k exceeds 2^31");
    if (a & (a - 1)) h.pow2 = 0;
  }
  h.bits = h.shift[h.levels];
  if (h.bits > kMaxCodeBits)
    throw Error(PM_EOVERFLOW, "hierarchy needs more than 13 code bits");
  h.k = h.P[h.levels];
  return h;
}

namespace {

int64_t lmax_of(int64_t total, int64_t k, double eps) {
  if (!(eps >= 0.0) || eps > 1e6) throw Error(PM_EINVAL, "eps must be >= 0");
  const int64_t ppm = (int64_t)std::llround(eps * 1e6);
  const int64_t num = (1000000 + ppm) * total;
  const int64_t den = 1000000 * k;
  return (num + den - 1) / den;
}

int64_t sigma_of(int64_t lmax, int64_t total, int64_t k) {
  const int64_t avg = (total + k - 1) / k;
  return lmax - 100 > avg ? lmax - 100 : avg;
}

Variants variants_of(const pm_options *o) {
  Variants v;
  if (!o) return v;
  if (o->variants & ~(PM_VARIANT_JET_FILTER | PM_VARIANT_J_REBALANCE))
    throw Error(PM_EINVAL, "unknown variant bits");
  if (o->variants & PM_VARIANT_JET_FILTER) {
    if (o->jet_c_num < 1 || o->jet_c_num > (1 << 15) || o->jet_c_den < 1)
      throw Error(PM_EINVAL, "jet filter needs 1 <= c_num <= 2^15 and c_den >= 1");
    v.jet_num = o->jet_c_num;
    v.jet_den = o->jet_c_den;
  }
  v.j_rebalance = (o->variants & PM_VARIANT_J_REBALANCE) != 0;
  if (o->refine_repeats < 0 || o->refine_repeats > 64)
    throw Error(PM_EINVAL, "refine_repeats must be in [0, 64]");
  v.repeats = o->refine_repeats > 1 ? o->refine_repeats : 1;
  return v;
}

DGraph view(const pm_graph *g) {
  if (!g) throw Error(PM_EINVAL, "graph is NULL");
  if (g->n < 0 || g->nnz < 0) throw Error(PM_EINVAL, "negative graph size");
  if (g->nnz > INT32_MAX) throw Error(PM_EOVERFLOW, "nnz exceeds 2^31 - 1");
  if (!g->xadj || (g->n > 0 && !g->vwgt) || (g->nnz > 0 && (!g->adjncy || !g->adjwgt)))
    throw Error(PM_EINVAL, "graph array is NULL");
  DGraph d{g->n, g->nnz, g->xadj, g->adjncy, g->adjwgt, g->vwgt};
  return d;
}

// Device-side status block + host mirror for one call.
struct Ctx {
  Arena &ar;
  hipStream_t s;
  Status *dev;
  Status *host;
  Stripes sp;
  // mapped mirror: [0, sizeof(Status)) status words, then the sequence slot
  Status *mirror = nullptr;
  Status *mirror_dev = nullptr;
  int64_t *seq_dev = nullptr;
  const volatile int64_t *seq_host = nullptr;
  uint64_t *counter = nullptr;  // completion counter of the matching commit
  int64_t *seq_ctr = nullptr;   // device copy of the publication sequence
  explicit Ctx(Arena &a, hipStream_t st) : ar(a), s(st) {
    dev = ar.alloc_n<Status>(1);
    seq_ctr = ar.alloc_n<int64_t>(1);
    fill_i64(seq_ctr, ar.publish_seq(), 1, s);
    counter = ar.alloc_n<uint64_t>(65);
    PM_HIP(hipMemsetAsync(counter, 0, sizeof(uint64_t) * 65, s));
    host = static_cast<Status *>(ar.host_stage(sizeof(Status) + 4096));
    void *mdev = nullptr;
    char *m = static_cast<char *>(ar.host_mapped(&mdev));
    mirror = reinterpret_cast<Status *>(m);
    mirror_dev = static_cast<Status *>(mdev);
    seq_host = reinterpret_cast<const volatile int64_t *>(m + 256);
    seq_dev = reinterpret_cast<int64_t *>(static_cast<char *>(mdev) + 256);
    sp.a = ar.alloc_n<int64_t>(2 * (size_t)stripe_words());
    sp.b = sp.a + stripe_words();
    PM_HIP(hipMemsetAsync(dev, 0, sizeof(Status), s));
    PM_HIP(hipMemsetAsync(sp.a, 0, sizeof(int64_t) * 2 * (size_t)stripe_words(), s));
  }
  // pinned host words after the status copy (the staging buffer holds
  // sizeof(Status) + 4096 bytes), for small copies that a pull() orders
  int32_t *aux() {
    static_assert(sizeof(Status) <= 512, "status block grew");
    return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(host) + 512);
  }
  // Status read-back: a kernel publishes the status into mapped host memory
  // and the host polls its sequence number, which returns sooner than a copy
  // plus a stream synchronisation.  next_pub() names a publication for a
  // kernel that ends a step; wait() blocks until it has happened.  A stream
  // that fails or goes idle without publishing raises PM_EHIP.
  Pub next_pub() { return Pub{mirror_dev, seq_dev, ar.next_publish(), seq_ctr}; }
  // enqueues a publication (the device counts the sequence) and returns the
  // number the host then waits for
  Pub publish() {
    const Pub p = next_pub();
    publish_status(dev, mirror_dev, seq_dev, p.seq, s, seq_ctr);
    return p;
  }
  void pull() { wait(publish()); }
  void wait(const Pub &p) {
    const int64_t seq = p.seq;
    for (uint64_t it = 1;; ++it) {
      if (__atomic_load_n(seq_host, __ATOMIC_ACQUIRE) == seq) break;
      __builtin_ia32_pause();
      if ((it & 1023) == 0) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) {
          (void)hipGetLastError();
          throw Error(PM_EHIP, hipGetErrorString(e));
        }
        // idle stream: the release store is visible by now
        bool seen = false;
        for (int r = 0; r < 4096 && !seen; ++r)
          seen = __atomic_load_n(seq_host, __ATOMIC_ACQUIRE) == seq;
        if (!seen) throw Error(PM_EHIP, "status publish not observed");
        break;
      }
    }
    std::memcpy(host, mirror, sizeof(Status));
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Refinement (Algorithm 6)
// ---------------------------------------------------------------------------
struct RefineResult {
  int32_t status;
  pm_refine_stats st;
};

static RefineResult refine_level(Ctx &cx, const DGraph &g, const Classes &cl, const Hier &h,
                                 int64_t lmax, int64_t sigma, int64_t total, uint64_t seed,
                                 int32_t level, int32_t *best, const Variants &var) {
  Arena &ar = cx.ar;
  hipStream_t s = cx.s;
  const size_t mark = ar.mark();
  const int64_t n = g.n;
  const int32_t ncodes = 1 << h.bits;
  int32_t *cur = ar.alloc_n<int32_t>(n);
  LpRec *rec = ar.alloc_n<LpRec>(n);          // label propagation (kept between its rounds)
  int32_t *rtarget = ar.alloc_n<int32_t>(n);  // rebalancing
  int2 *pn = ar.alloc_n<int2>(n);             // apply's neighbour records
  uint8_t *moved = ar.alloc_n<uint8_t>(n);
  uint8_t *lock = ar.alloc_n<uint8_t>(n);
  int64_t *w = ar.alloc_n<int64_t>(ncodes);
  int64_t *wst = alloc_weight_stripes(ar, h, s);
  RebalanceBuffers rb = alloc_rebalance(ar, n, h, s);
  // (the size threshold is a launch parameter: pm_set_tuning)
  const int64_t rmin = tuning().reb_compact_min_n;
  int32_t *slist = n >= rmin && n > 0 ? ar.alloc_n<int32_t>(n) : nullptr;
  int32_t *soff = slist ? ar.alloc_n<int32_t>(NCLS + 1) : nullptr;

  EventSet evs;
  hipEvent_t ev0 = evs.make(), ev1 = evs.make();
  PM_HIP(hipEventRecord(ev0, s));

  if (n > 0) PM_HIP(hipMemcpyAsync(cur, best, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  fill_u8(lock, 0, n, s);
  // result caching of label propagation (a launch parameter: pm_set_tuning)
  uint8_t *dirty = nullptr;
  if (tuning().lp_cache && n > 0) {
    dirty = ar.alloc_n<uint8_t>(n);
    fill_u8(dirty, 1, n, s);
  }
  block_weights(g, h, cur, w, s);
  comm_cost(g, cl, h, cur, cx.sp.a, cx.dev, s);
  // step epilogue: heaviest block, J change, eligible destinations, publication
  StepEnd E{h, w, cx.sp.a, sigma, lmax, rb.elig_weak, rb.elig_strong, cx.dev};
  {
    StepEnd E0 = E;
    E0.dj_stripes = nullptr;
    step_status(E0, s);
    cx.pull();
  }
  int64_t j_cur = cx.host->j, imb_cur = cx.host->maxw;
  if (n == 0) imb_cur = 0;
  int64_t j_best = j_cur, imb_best = imb_cur;
  bool feas_best = imb_best <= lmax;

  RefineResult R{};
  R.st.j_initial = j_cur;
  R.st.maxw_initial = imb_cur;
  const uint64_t reb_seed = mix_hash(seed ^ kTagRebalance, (uint64_t)(int64_t)level);

  // Loop bodies replayed from HIP graphs (launch parameter graph_bodies):
  // the label-propagation body and the weak-rebalancing body of this level
  // are captured the first time they run and replayed afterwards.  Every
  // argument of their kernels is the same in every body of the level; the
  // body number of the pseudo-random destinations and the publication's
  // sequence number are read from device counters.  Levels that read sizes
  // back inside a body (compacted rebalancing), strong rounds (a library
  // selection inside) and calls on the null stream (which cannot be
  // captured) are launched as usual.
  struct BodyGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~BodyGraph() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  } bgs[2];
  const bool use_graphs = tuning().graph_bodies && !tl_timer && !slist && n > 0 && s != nullptr;
  int64_t *body_ctr = nullptr;
  if (use_graphs) {
    body_ctr = ar.alloc_n<int64_t>(1);
    fill_i64(body_ctr, 0, 1, s);
    E.body_ctr = body_ctr;
  }
  auto replay = [&](BodyGraph &bg, const std::function<void()> &body) -> Pub {
    if (!bg.x) {
      PM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        // the commit publishes; its sequence number comes from the device
        // counter (the host's count advances per launch, below)
        E.pub = Pub{cx.mirror_dev, cx.seq_dev, 0, cx.seq_ctr};
        body();
        E.pub = Pub{};
      } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(s, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
      }
      PM_HIP(hipStreamEndCapture(s, &bg.g));
      PM_HIP(hipGraphInstantiate(&bg.x, bg.g, nullptr, nullptr, 0));
    }
    const Pub p = cx.next_pub();
    PM_HIP(hipGraphLaunch(bg.x, s));
    return p;
  };

  int32_t i = 0, iw = 0, bodies = 0;
  while (i < 12 && bodies < 4096) {
    ++i;
    ++bodies;
    Pub pub{};
    if (imb_cur <= lmax) {
      auto body = [&] {
        lp_phase1(g, cl, h, cur, lock, rec, s, var, dirty);
        lp_phase2(g, cl, h, rec, moved, pn, s);
        apply_moves(g, cl, h, cur, moved, lock, w, wst, cx.sp.a, &E, pn, s, dirty);
      };
      if (use_graphs) {
        pub = replay(bgs[0], body);
      } else {
        E.pub = pub = cx.next_pub();  // published by the commit's step end
        body();
        E.pub = Pub{};
      }
      iw = 0;
      ++R.st.lp_iterations;
    } else {
      const bool strong = iw >= 2;
      const uint64_t hseed = mix_hash(reb_seed, (uint64_t)bodies);
      // large levels: only the vertices of overloaded blocks are tiled for
      // the selection and the moves (movers are sources)
      Classes rcl = cl;
      if (slist) {
        const size_t m2 = ar.mark();
        reb_sources(ar, cl, (int32_t)n, cur, w, lmax, rb.key, slist, soff, s);
        PM_HIP(hipMemcpyAsync(cx.aux(), soff, sizeof(int32_t) * (NCLS + 1), hipMemcpyDeviceToHost,
                              s));
        cx.pull();
        ar.rewind(m2);
        rcl.list = slist;
        for (int c = 0; c <= NCLS; ++c) rcl.off[c] = cx.aux()[c];
      }
      if (use_graphs && !strong) {
        pub = replay(bgs[1], [&] {
          rebalance_round(ar, g, rcl, h, false, lmax, sigma, total, reb_seed, cur, w, rtarget,
                          moved, pn, rb, cx.dev, s, var, body_ctr);
          apply_moves(g, rcl, h, cur, moved, nullptr, w, wst, cx.sp.a, &E, pn, s, dirty);
        });
      } else {
        E.pub = pub = cx.next_pub();  // published by the commit's step end
        rebalance_round(ar, g, rcl, h, strong, lmax, sigma, total, hseed, cur, w, rtarget, moved,
                        pn, rb, cx.dev, s, var);
        apply_moves(g, rcl, h, cur, moved, nullptr, w, wst, cx.sp.a, &E, pn, s, dirty);
        E.pub = Pub{};
      }
      if (strong) {
        iw = 0;
        ++R.st.strong_iterations;
      } else {
        ++iw;
        ++R.st.weak_iterations;
      }
    }
    cx.wait(pub);
    j_cur += cx.host->dj;
    imb_cur = cx.host->maxw;
    if (imb_cur <= lmax) {
      const bool improve = !feas_best || j_cur < j_best;
      const bool reset = !feas_best || 1000 * j_cur < 999 * j_best;
      if (improve) {
        PM_HIP(hipMemcpyAsync(best, cur, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        j_best = j_cur;
        imb_best = imb_cur;
        feas_best = true;
      }
      if (reset) i = 0;
    } else if (imb_cur < imb_best) {
      PM_HIP(hipMemcpyAsync(best, cur, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
      j_best = j_cur;
      imb_best = imb_cur;
      i = 0;
    }
  }
  PM_HIP(hipEventRecord(ev1, s));
  PM_HIP(hipEventSynchronize(ev1));
  float ms = 0.f;
  PM_HIP(hipEventElapsedTime(&ms, ev0, ev1));

  R.st.iterations = bodies;
  R.st.j_final = j_best;
  R.st.maxw_final = imb_best;
  R.st.feasible = feas_best ? 1 : 0;
  R.st.refine_ms = ms;
  R.st.arcs_processed = (int64_t)bodies * g.nnz;
  R.status = feas_best ? PM_OK : PM_WARN_IMBALANCED;
  ar.rewind(mark);
  return R;
}

// ---------------------------------------------------------------------------
// Coarsening: one level of matching + contraction
// ---------------------------------------------------------------------------
struct Level {
  DGraph g;
  int32_t *list = nullptr;
  Classes cl{};
  int32_t *cmap = nullptr;  // to the next coarser level
  int32_t hem_rounds = 0;
};

static int32_t bitlen(uint64_t x) {
  int32_t b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

// HEM on level L; returns rounds, fills match (device, n).
static int32_t run_hem(Ctx &cx, const Level &L, int64_t lmax, uint64_t seed, int32_t level,
                       int32_t *match, int32_t *pref) {
  const DGraph &g = L.g;
  hipStream_t s = cx.s;
  fill_i32(match, -1, g.n, s);
  fill_i32(pref, -2, g.n, s);  // no preference computed yet
  const uint64_t hseed = mix_hash(seed ^ kTagMatch, (uint64_t)(int64_t)level);
  int32_t rounds = 0;
  int64_t matched = 0;
  // large levels: after each round only the vertices that must look again
  // are tiled for the next one
  // (the size threshold is a launch parameter: pm_set_tuning)
  const int64_t cmin = tuning().hem_compact_min_n;
  const bool compact = g.n >= cmin;
  const size_t mark = cx.ar.mark();
  int32_t *cm = cx.ar.alloc_n<int32_t>(g.n);  // weights; -1 marks a matched vertex
  if (g.n > 0) PM_HIP(hipMemcpyAsync(cm, g.c, sizeof(int32_t) * g.n, hipMemcpyDeviceToDevice, s));
  uint8_t *hact = cx.ar.alloc_n<uint8_t>(g.n);  // looks for a partner this round
  fill_u8(hact, 1, g.n, s);
  int32_t *clist = compact ? cx.ar.alloc_n<int32_t>(g.n) : nullptr;
  int32_t *coff = compact ? cx.ar.alloc_n<int32_t>(NCLS + 1) : nullptr;
  int32_t *hoff = cx.aux();
  Classes cur = L.cl;
  if (compact && tl_timer) {
    // (counted and timed runs: the compacted sizes are read back each round,
    // for the host-side unit counts)
    while (rounds < 64) {
      ++rounds;
      hem_prefer(g, cur, lmax, hseed, match, pref, cm, hact, s);
      hem_commit(g.n, pref, match, cm, hact, cx.counter, cx.dev, nullptr, s);
      const size_t round_mark = cx.ar.mark();
      hem_compact(cx.ar, L.cl, g.n, hact, clist, coff, s);
      PM_HIP(hipMemcpyAsync(hoff, coff, sizeof(int32_t) * (NCLS + 1), hipMemcpyDeviceToHost, s));
      cx.pull();  // the round's work is done: its scratch can go
      cx.ar.rewind(round_mark);
      const int32_t added = cx.host->count;
      matched += added;
      if (added == 0) break;
      cur.list = clist;
      for (int c = 0; c <= NCLS; ++c) cur.off[c] = hoff[c];
    }
  } else if (compact) {
    // After each commit the vertices that look again are compacted on the
    // device (list and class offsets), and the next round's launch reads the
    // offsets there: rounds go in groups of kHemRoundsPerRead between
    // read-backs of their match counts, as on small levels (a round after
    // one that added no pair is a no-op).  The compaction's scratch is
    // stream-ordered, so the arena is rewound after each group.
    int32_t *counts = cx.ar.alloc_n<int32_t>(64);
    bool done = false;
    while (!done && rounds < 64) {
      const int k = 64 - rounds < kHemRoundsPerRead ? 64 - rounds : kHemRoundsPerRead;
      const size_t group_mark = cx.ar.mark();
      for (int j = 0; j < k; ++j) {
        if (rounds + j == 0) hem_prefer(g, L.cl, lmax, hseed, match, pref, cm, hact, s);
        else hem_prefer_dev(g, L.cl, clist, coff, lmax, hseed, match, pref, cm, hact, s);
        hem_commit(g.n, pref, match, cm, hact, cx.counter, cx.dev, counts + rounds + j, s);
        if (j + 1 < k || rounds + k < 64) hem_compact(cx.ar, L.cl, g.n, hact, clist, coff, s);
      }
      PM_HIP(hipMemcpyAsync(hoff, counts + rounds, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
      cx.pull();
      cx.ar.rewind(group_mark);
      for (int j = 0; j < k && !done; ++j) {
        ++rounds;
        matched += hoff[j];
        done = hoff[j] == 0;
      }
    }
  } else {
    // Rounds go in groups of kHemRoundsPerRead between status read-backs:
    // once a round adds no pair, every later round is a no-op (no vertex is
    // active and no mutual preference exists), so running a few past the
    // last one changes nothing; the per-round counts say where it stopped.
    int32_t *counts = cx.ar.alloc_n<int32_t>(64);
    bool done = false;
    while (!done && rounds < 64) {
      const int k = 64 - rounds < kHemRoundsPerRead ? 64 - rounds : kHemRoundsPerRead;
      for (int j = 0; j < k; ++j) {
        hem_prefer(g, cur, lmax, hseed, match, pref, cm, hact, s);
        hem_commit(g.n, pref, match, cm, hact, cx.counter, cx.dev, counts + rounds + j, s);
      }
      PM_HIP(hipMemcpyAsync(hoff, counts + rounds, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
      cx.pull();
      for (int j = 0; j < k && !done; ++j) {
        ++rounds;
        matched += hoff[j];
        done = hoff[j] == 0;
      }
    }
  }
  cx.ar.rewind(mark);
  // two-hop matching while 75 % or fewer of the vertices are matched
  const int64_t lim = 3 * (int64_t)g.n;
  const uint64_t tseed = mix_hash(seed ^ kTagTwin, (uint64_t)(int64_t)level);
  for (int mode : {TWOHOP_LEAF, TWOHOP_TWIN, TWOHOP_RELATIVE})
    if (4 * matched <= lim)
      matched += two_hop_step(cx.ar, g, L.cl, mode, tseed, lmax, match, cx.sp.b, cx.dev, cx.host, s);
  return rounds;
}

// Coarse numbering + contraction into pre-allocated coarse arrays.
// Contraction by one radix sort of all arcs keyed by (coarse row, coarse
// neighbour): runs of equal keys merge, self loops (keyed all-ones) drop out.
static void run_contract_sorted(Ctx &cx, const Level &L, int32_t *cmap, int32_t nc,
                                int64_t *cxadj, int32_t *cadj, int32_t *cw, int64_t *nnz_out) {
  const DGraph &g = L.g;
  hipStream_t s = cx.s;
  Arena &ar = cx.ar;
  const size_t m = ar.mark();
  const int64_t nnz = g.nnz;
  const int bits = bitlen((uint64_t)(nc > 1 ? nc - 1 : 1));
  uint64_t *key = ar.alloc_n<uint64_t>(nnz);
  uint64_t *key2 = ar.alloc_n<uint64_t>(nnz);
  int32_t *val = ar.alloc_n<int32_t>(nnz);
  int32_t *val2 = ar.alloc_n<int32_t>(nnz);
  contract_keys(g, L.cl, cmap, bits, key, val, cx.sp.b, cx.dev, s);  // cx.dev->count: self loops
  sort_pairs(ar, key, key2, val, val2, nnz, 2 * bits, s);
  int32_t *head = ar.alloc_n<int32_t>(nnz + 1);
  int32_t *pos = ar.alloc_n<int32_t>(nnz + 1);
  int32_t *rowcnt = ar.alloc_n<int32_t>((size_t)nc + 1);
  fill_i32(rowcnt, 0, (int64_t)nc + 1, s);
  contract_heads(nnz, &cx.dev->count, key2, head, s);
  scan_excl(ar, head, pos, nnz, s);
  contract_emit(nnz, &cx.dev->count, key2, val2, head, pos, bits, cadj, cw, rowcnt, s);
  scan_excl_widen(ar, rowcnt, cxadj, (int64_t)nc + 1, s);
  PM_HIP(hipMemcpyAsync(&cx.host->j, cxadj + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  *nnz_out = cx.host->j;
  ar.rewind(m);
}

static void run_contract(Ctx &cx, const Level &L, int32_t *match, int32_t *cmap, int32_t nc,
                         int64_t *cxadj, int32_t *cadj, int32_t *cw, int32_t *cvwgt,
                         int64_t *nnz_out) {
  const DGraph &g = L.g;
  hipStream_t s = cx.s;
  Arena &ar = cx.ar;
  coarse_vwgt(g.n, match, cmap, g.c, cvwgt, s);
  const size_t m = ar.mark();
  const int64_t nnz = g.nnz;
  // A fine vertex above 64 arcs puts its coarse row above 64: with W formed
  // BIG means above 512, else above 64.  When these alone exceed the share,
  // the level takes the sort without the row pre-pass.
  const int64_t cnt_w = L.cl.off[CLS_W + 1] - L.cl.off[CLS_W];
  const int64_t cnt_big = L.cl.off[CLS_BIG + 1] - L.cl.off[CLS_BIG];
  const int64_t long_lb = 65 * cnt_w + (cnt_w > 0 ? kWaveMaxDeg + 1 : 65) * cnt_big;
  const int64_t pct = tuning().contract_rows_long_pct;
  if (nnz > 0 && nnz >= tuning().contract_rows_min_nnz && long_lb * 100 <= nnz * pct) {
    // row-local path: stage every coarse row at its upper-bound offset, merge
    // rows of up to 512 arcs in registers and up to 2048 in LDS, and sort
    // only the arcs of longer rows.  A share limit below 100 % sends levels
    // whose rows above 64 hold more of the arcs to the sort.
    int32_t *ub = ar.alloc_n<int32_t>((size_t)nc + 1);
    int32_t *ubig = ar.alloc_n<int32_t>((size_t)nc + 1);
    int64_t *uxadj = ar.alloc_n<int64_t>((size_t)nc + 1);
    int64_t *rstart = ar.alloc_n<int64_t>((size_t)nc + 1);
    int64_t *above64 = ar.alloc_n<int64_t>(1);
    fill_i32(ub + nc, 0, 1, s);
    fill_i32(ubig + nc, 0, 1, s);
    contract_rowub(g, match, cmap, ub, ubig, above64, s);
    int64_t *hb = reinterpret_cast<int64_t *>(cx.aux());
    if (pct < 100) {
      PM_HIP(hipMemcpyAsync(hb, above64, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      PM_HIP(hipStreamSynchronize(s));
    }
    if (pct < 100 && hb[0] * 100 > nnz * pct) {
      ar.rewind(m);
      run_contract_sorted(cx, L, cmap, nc, cxadj, cadj, cw, nnz_out);
      return;
    }
    scan_excl_widen(ar, ub, uxadj, (int64_t)nc + 1, s);
    scan_excl_widen(ar, ubig, rstart, (int64_t)nc + 1, s);
    int64_t *long_arcs = hb + 1;
    PM_HIP(hipMemcpyAsync(long_arcs, rstart + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    uint32_t *scu = ar.alloc_n<uint32_t>(nnz);
    int32_t *sw = ar.alloc_n<int32_t>(nnz);
    contract_stage(g, L.cl, match, cmap, uxadj, scu, sw, s);
    int32_t *rlist = ar.alloc_n<int32_t>((size_t)nc);
    DGraph rg{};
    rg.n = nc;
    rg.xadj = uxadj;
    const Classes rc = build_classes(ar, rg, rlist, cx.dev, cx.host, s);  // synchronises
    const int64_t lm = *long_arcs;
    int32_t *rowcnt = ar.alloc_n<int32_t>((size_t)nc + 1);
    fill_i32(rowcnt + nc, 0, 1, s);
    contract_rows(rc, uxadj, scu, sw, rowcnt, s);
    const int32_t *llist = rc.list + rc.off[CLS_BIG];  // rows above 64 (BIG, then W)
    const int32_t nl = rc.off[CLS_W + 1] - rc.off[CLS_BIG];
    contract_mid_rows(llist, nl, uxadj, scu, sw, rowcnt, s);
    contract_long_rows(ar, llist, nl, lm, nc, uxadj, rstart, scu, sw, rowcnt, s);
    scan_excl_widen(ar, rowcnt, cxadj, (int64_t)nc + 1, s);
    contract_copy(rc, uxadj, cxadj, scu, sw, cadj, cw, s);
    PM_HIP(hipMemcpyAsync(&cx.host->j, cxadj + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    *nnz_out = cx.host->j;
    ar.rewind(m);
    return;
  }
  run_contract_sorted(cx, L, cmap, nc, cxadj, cadj, cw, nnz_out);
  ar.rewind(m);
}

// number of coarse vertices from the leader flags; fills cmap
static int32_t run_coarse_ids(Ctx &cx, int32_t n, int32_t *match, int32_t *cmap) {
  Arena &ar = cx.ar;
  hipStream_t s = cx.s;
  const size_t m = ar.mark();
  int32_t *leader = ar.alloc_n<int32_t>((size_t)n + 1);
  int32_t *rank = ar.alloc_n<int32_t>((size_t)n + 1);
  hem_finish(n, match, leader, s);
  fill_i32(leader + n, 0, 1, s);
  scan_excl(ar, leader, rank, (int64_t)n + 1, s);
  coarse_ids(n, match, rank, cmap, s);
  PM_HIP(hipMemcpyAsync(&cx.host->count, rank + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  const int32_t nc = cx.host->count;
  ar.rewind(m);
  return nc;
}

// Initial partition of level L on the host; writes codes into part (device).
static void run_initial(Ctx &cx, const DGraph &g, const Hier &h, int32_t *part) {
  hipStream_t s = cx.s;
  std::vector<int64_t> xadj(g.n + 1);
  std::vector<int32_t> adj(g.nnz), vw(g.n), ids(g.n);
  PM_HIP(hipMemcpyAsync(xadj.data(), g.xadj, sizeof(int64_t) * (g.n + 1), hipMemcpyDeviceToHost, s));
  if (g.nnz)
    PM_HIP(hipMemcpyAsync(adj.data(), g.adj, sizeof(int32_t) * g.nnz, hipMemcpyDeviceToHost, s));
  if (g.n) PM_HIP(hipMemcpyAsync(vw.data(), g.c, sizeof(int32_t) * g.n, hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  host_initial_partition(g.n, xadj.data(), adj.data(), vw.data(), h, ids.data());
  for (int32_t v = 0; v < g.n; ++v) ids[v] = (int32_t)id_to_code(h, ids[v]);
  if (g.n) {
    PM_HIP(hipMemcpyAsync(part, ids.data(), sizeof(int32_t) * g.n, hipMemcpyHostToDevice, s));
    PM_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace pm

// ===========================================================================
// C ABI
// ===========================================================================
using namespace pm;

namespace {

template <class F>
int guarded(F f) {
  try {
    return f();
  } catch (const Error &e) {
    (void)hipGetLastError();
    return e.code;
  } catch (const std::bad_alloc &) {
    return PM_ENOMEM;
  } catch (...) {
    return PM_EHIP;
  }
}

void check_device() {
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0) {
    (void)hipGetLastError();
    throw Error(PM_ENODEVICE, "no HIP device");
  }
}

// Rejects mappings with ids outside [0,k): block ids index device arrays.
void require_ids(Ctx &cx, const Hier &h, const int32_t *part, int32_t n) {
  check_ids(h, part, n, cx.sp.b, cx.dev, cx.s);
  cx.pull();
  if (cx.host->count) throw Error(PM_EINVAL, "mapping holds ids outside [0,k)");
}

}  // namespace

extern "C" {

const char *pm_version(void) { return "pm 0.1.0 (gfx950)"; }

const char *pm_strerror(int code) {
  switch (code) {
    case PM_OK: return "ok";
    case PM_WARN_IMBALANCED: return "mapping written but exceeds L_max";
    case PM_EINVAL: return "invalid argument";
    case PM_EGRAPH: return "graph failed validation";
    case PM_EOVERFLOW: return "size or weight limit exceeded";
    case PM_ENOMEM: return "out of device memory";
    case PM_EHIP: return "HIP runtime error";
    case PM_ENODEVICE: return "no HIP device";
    default: return "unknown error";
  }
}

void pm_release(void) { release_all_arenas(); }

int pm_comm_cost(const pm_graph *g, const pm_hierarchy *h, const int32_t *part, int64_t *j_out,
                 uint32_t flags, void *stream) {
  return guarded([&] {
    check_device();
    if (!j_out || (!part && g && g->n > 0)) throw Error(PM_EINVAL, "NULL output or mapping");
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    ArenaLease lease(as_stream(stream));
    hipStream_t s = as_stream(stream);
    Ctx cx(*lease, s);
    int64_t total = 0;
    validate_graph(*lease, dg, (flags & PM_FLAG_VALIDATE) != 0, &total, s);
    require_ids(cx, hh, part, dg.n);
    int32_t *codes = const_cast<int32_t *>(part);
    if (!hh.pow2) {
      codes = lease->alloc_n<int32_t>(dg.n);
      ids_to_codes(hh, part, codes, dg.n, s);
    }
    int32_t *list = lease->alloc_n<int32_t>(dg.n);
    Classes cl = build_classes(*lease, dg, list, cx.dev, cx.host, s);
    comm_cost(dg, cl, hh, codes, cx.sp.a, cx.dev, s);
    cx.pull();
    *j_out = cx.host->j;
    return PM_OK;
  });
}

int pm_block_weights(const pm_graph *g, const pm_hierarchy *h, const int32_t *part,
                     int64_t *w_out, void *stream) {
  return guarded([&] {
    check_device();
    if (!w_out || (!part && g && g->n > 0)) throw Error(PM_EINVAL, "NULL output or mapping");
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    ArenaLease lease(as_stream(stream));
    hipStream_t s = as_stream(stream);
    Ctx cx(*lease, s);
    require_ids(cx, hh, part, dg.n);
    int32_t *codes = lease->alloc_n<int32_t>(dg.n);
    ids_to_codes(hh, part, codes, dg.n, s);
    int64_t *w = lease->alloc_n<int64_t>((size_t)1 << hh.bits);
    block_weights(dg, hh, codes, w, s);
    // codes -> ids order: gather on the host (k is small)
    std::vector<int64_t> wc((size_t)1 << hh.bits), wi(hh.k);
    PM_HIP(hipMemcpyAsync(wc.data(), w, sizeof(int64_t) * wc.size(), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    for (int64_t b = 0; b < hh.k; ++b) wi[b] = wc[id_to_code(hh, b)];
    PM_HIP(hipMemcpyAsync(w_out, wi.data(), sizeof(int64_t) * hh.k, hipMemcpyHostToDevice, s));
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
  });
}

int pm_lp_round(const pm_graph *g, const pm_hierarchy *h, int32_t *part, uint8_t *lock,
                int32_t *target_out, int64_t *gain_out, uint8_t *moved_out, void *stream) {
  return pm_lp_round_ex(g, h, part, lock, target_out, gain_out, moved_out, nullptr, stream);
}

int pm_lp_round_ex(const pm_graph *g, const pm_hierarchy *h, int32_t *part, uint8_t *lock,
                   int32_t *target_out, int64_t *gain_out, uint8_t *moved_out,
                   const pm_options *opts, void *stream) {
  return guarded([&] {
    const Variants var = variants_of(opts);
    check_device();
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    if (dg.n > 0 && (!part || !lock || !target_out || !gain_out || !moved_out))
      throw Error(PM_EINVAL, "NULL array");
    ArenaLease lease(as_stream(stream));
    hipStream_t s = as_stream(stream);
    Ctx cx(*lease, s);
    int64_t total = 0;
    validate_graph(*lease, dg, false, &total, s);
    require_ids(cx, hh, part, dg.n);
    int32_t *codes = lease->alloc_n<int32_t>(dg.n);
    ids_to_codes(hh, part, codes, dg.n, s);
    int32_t *list = lease->alloc_n<int32_t>(dg.n);
    Classes cl = build_classes(*lease, dg, list, cx.dev, cx.host, s);
    int64_t *w = lease->alloc_n<int64_t>((size_t)1 << hh.bits);
    block_weights(dg, hh, codes, w, s);
    LpRec *rec = lease->alloc_n<LpRec>(dg.n);
    int2 *pn = lease->alloc_n<int2>(dg.n);
    lp_phase1(dg, cl, hh, codes, lock, rec, s, var);
    unpack_lp(rec, target_out, gain_out, dg.n, s);
    lp_phase2(dg, cl, hh, rec, moved_out, pn, s);
    apply_moves(dg, cl, hh, codes, moved_out, lock, w, alloc_weight_stripes(*lease, hh, s),
                cx.sp.a, nullptr, pn, s);
    codes_to_ids(hh, codes, part, dg.n, s);
    codes_to_ids(hh, target_out, target_out, dg.n, s);
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
  });
}

int pm_rebalance(const pm_graph *g, const pm_hierarchy *h, int32_t strong, int64_t lmax,
                 int64_t sigma, uint64_t seed, int32_t level, int32_t iter, int32_t *part,
                 uint8_t *moved_out, void *stream) {
  return pm_rebalance_ex(g, h, strong, lmax, sigma, seed, level, iter, part, moved_out, nullptr,
                         stream);
}

int pm_rebalance_ex(const pm_graph *g, const pm_hierarchy *h, int32_t strong, int64_t lmax,
                    int64_t sigma, uint64_t seed, int32_t level, int32_t iter, int32_t *part,
                    uint8_t *moved_out, const pm_options *opts, void *stream) {
  return guarded([&] {
    const Variants var = variants_of(opts);
    check_device();
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    if (dg.n > 0 && (!part || !moved_out)) throw Error(PM_EINVAL, "NULL array");
    ArenaLease lease(as_stream(stream));
    Arena &ar = *lease;
    hipStream_t s = as_stream(stream);
    Ctx cx(ar, s);
    int64_t total = 0;
    validate_graph(ar, dg, false, &total, s);
    require_ids(cx, hh, part, dg.n);
    const int64_t n = dg.n;
    const int32_t ncodes = 1 << hh.bits;
    int32_t *codes = ar.alloc_n<int32_t>(n);
    ids_to_codes(hh, part, codes, dg.n, s);
    int32_t *list = ar.alloc_n<int32_t>(n);
    Classes cl = build_classes(ar, dg, list, cx.dev, cx.host, s);
    int64_t *w = ar.alloc_n<int64_t>(ncodes);
    int32_t *target = ar.alloc_n<int32_t>(n);
    RebalanceBuffers rb = alloc_rebalance(ar, n, hh, s);
    block_weights(dg, hh, codes, w, s);
    step_status(StepEnd{hh, w, nullptr, sigma, lmax, rb.elig_weak, rb.elig_strong, cx.dev}, s);
    const uint64_t hseed =
        mix_hash(mix_hash(seed ^ kTagRebalance, (uint64_t)(int64_t)level), (uint64_t)(int64_t)iter);
    int2 *pn = ar.alloc_n<int2>(n);
    rebalance_round(ar, dg, cl, hh, strong != 0, lmax, sigma, total, hseed, codes, w, target,
                    moved_out, pn, rb, cx.dev, s, var);
    apply_moves(dg, cl, hh, codes, moved_out, nullptr, w, alloc_weight_stripes(ar, hh, s), cx.sp.a,
                nullptr, pn, s);
    codes_to_ids(hh, codes, part, dg.n, s);
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
  });
}

int pm_refine(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed, int32_t level,
              int32_t *part, pm_refine_stats *stats, void *stream) {
  return pm_refine_ex(g, h, eps, seed, level, part, stats, nullptr, stream);
}

int pm_refine_ex(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed,
                 int32_t level, int32_t *part, pm_refine_stats *stats, const pm_options *opts,
                 void *stream) {
  return guarded([&] {
    const Variants var = variants_of(opts);
    check_device();
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    if (dg.n > 0 && !part) throw Error(PM_EINVAL, "NULL mapping");
    ArenaLease lease(as_stream(stream));
    Arena &ar = *lease;
    hipStream_t s = as_stream(stream);
    Ctx cx(ar, s);
    int64_t total = 0;
    validate_graph(ar, dg, false, &total, s);
    require_ids(cx, hh, part, dg.n);
    const int64_t lmax = lmax_of(total, hh.k, eps);
    const int64_t sigma = sigma_of(lmax, total, hh.k);
    int32_t *best = ar.alloc_n<int32_t>(dg.n);
    ids_to_codes(hh, part, best, dg.n, s);
    int32_t *list = ar.alloc_n<int32_t>(dg.n);
    Classes cl = build_classes(ar, dg, list, cx.dev, cx.host, s);
    RefineResult R = refine_level(cx, dg, cl, hh, lmax, sigma, total, seed, level, best, var);
    codes_to_ids(hh, best, part, dg.n, s);
    PM_HIP(hipStreamSynchronize(s));
    if (stats) *stats = R.st;
    return R.status;
  });
}

int pm_hem(const pm_graph *g, int64_t lmax, uint64_t seed, int32_t level, int32_t *match_out,
           int32_t *rounds_out, void *stream) {
  return guarded([&] {
    check_device();
    const DGraph dg = view(g);
    if (dg.n > 0 && !match_out) throw Error(PM_EINVAL, "NULL output");
    ArenaLease lease(as_stream(stream));
    Arena &ar = *lease;
    hipStream_t s = as_stream(stream);
    Ctx cx(ar, s);
    int64_t total = 0;
    validate_graph(ar, dg, false, &total, s);
    Level L;
    L.g = dg;
    L.list = ar.alloc_n<int32_t>(dg.n);
    L.cl = build_classes(ar, dg, L.list, cx.dev, cx.host, s);
    int32_t *pref = ar.alloc_n<int32_t>(dg.n);
    const int32_t r = run_hem(cx, L, lmax, seed, level, match_out, pref);
    int32_t *leader = ar.alloc_n<int32_t>(dg.n);
    hem_finish(dg.n, match_out, leader, s);
    PM_HIP(hipStreamSynchronize(s));
    if (rounds_out) *rounds_out = r;
    return PM_OK;
  });
}

int pm_contract(const pm_graph *g, const int32_t *match, int32_t *cmap, int64_t *cxadj,
                int32_t *cadjncy, int32_t *cadjwgt, int32_t *cvwgt, int32_t *nc_out,
                int64_t *nnz_out, void *stream) {
  return guarded([&] {
    check_device();
    const DGraph dg = view(g);
    if (dg.n > 0 && (!match || !cmap || !cxadj || !cvwgt || !nc_out || !nnz_out))
      throw Error(PM_EINVAL, "NULL array");
    ArenaLease lease(as_stream(stream));
    Arena &ar = *lease;
    hipStream_t s = as_stream(stream);
    Ctx cx(ar, s);
    Level L;
    L.g = dg;
    L.list = ar.alloc_n<int32_t>(dg.n);
    L.cl = build_classes(ar, dg, L.list, cx.dev, cx.host, s);
    check_match(dg.n, match, &cx.dev->count, s);
    cx.pull();
    if (cx.host->count) throw Error(PM_EINVAL, "match is not a matching of the vertices");
    int32_t *m = ar.alloc_n<int32_t>(dg.n);
    if (dg.n) PM_HIP(hipMemcpyAsync(m, match, sizeof(int32_t) * dg.n, hipMemcpyDeviceToDevice, s));
    const int32_t nc = run_coarse_ids(cx, dg.n, m, cmap);
    int64_t nnz = 0;
    run_contract(cx, L, m, cmap, nc, cxadj, cadjncy, cadjwgt, cvwgt, &nnz);
    *nc_out = nc;
    *nnz_out = nnz;
    return PM_OK;
  });
}

int pm_initial_partition(const pm_graph *g, const pm_hierarchy *h, int32_t *part_out,
                         void *stream) {
  return guarded([&] {
    check_device();
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    if (dg.n > 0 && !part_out) throw Error(PM_EINVAL, "NULL output");
    ArenaLease lease(as_stream(stream));
    hipStream_t s = as_stream(stream);
    Ctx cx(*lease, s);
    run_initial(cx, dg, hh, part_out);
    codes_to_ids(hh, part_out, part_out, dg.n, s);
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
  });
}

int pm_subgraphs(const pm_graph *g, const int32_t *part, int32_t parts, int32_t *vstart,
                 int64_t *estart, int32_t *order, int64_t *xadj_out, int32_t *adjncy_out,
                 int32_t *adjwgt_out, int32_t *vwgt_out, int64_t *arcs_out, void *stream) {
  return guarded([&] {
    check_device();
    const DGraph dg = view(g);
    if (parts < 1 || parts == INT32_MAX) throw Error(PM_EINVAL, "parts out of range");
    if (!vstart || !estart || !xadj_out) throw Error(PM_EINVAL, "NULL output");
    if (dg.n > 0 && (!part || !order || !vwgt_out)) throw Error(PM_EINVAL, "NULL array");
    if (dg.nnz > 0 && (!adjncy_out || !adjwgt_out)) throw Error(PM_EINVAL, "NULL array");
    ArenaLease lease(as_stream(stream));
    hipStream_t s = as_stream(stream);
    Ctx cx(*lease, s);
    check_parts(part, dg.n, parts, &cx.dev->count, s);
    cx.pull();
    if (cx.host->count) throw Error(PM_EINVAL, "partition holds ids outside [0,parts)");
    SubgraphOut o{vstart, estart, order, xadj_out, adjncy_out, adjwgt_out, vwgt_out, nullptr};
    subgraphs(*lease, dg, part, parts, o, s);
    int64_t arcs = 0;
    PM_HIP(hipMemcpyAsync(&arcs, estart + parts, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (arcs_out) *arcs_out = arcs;
    return PM_OK;
  });
}

int pm_map_hm(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed,
              int32_t workers, int32_t *part_out, int64_t *j_out, int32_t *calls_out,
              void *stream) {
  return pm_map_hm_ex(g, h, eps, seed, workers, part_out, j_out, calls_out, nullptr, stream);
}

int pm_map_hm_ex(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed,
                 int32_t workers, int32_t *part_out, int64_t *j_out, int32_t *calls_out,
                 const pm_options *opts, void *stream) {
  return guarded([&] {
    const Variants var = variants_of(opts);
    check_device();
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    hipStream_t s = as_stream(stream);
    PM_HIP(hipStreamSynchronize(s));
    const int rc = hm_impl(dg, h->a, h->levels, eps, seed, part_out, workers, calls_out, s, var);
    if (j_out) {
      *j_out = 0;
      if (dg.n > 0) {
        ArenaLease lease(s);
        Ctx cx(*lease, s);
        int32_t *codes = part_out;
        if (!hh.pow2) {
          codes = lease->alloc_n<int32_t>(dg.n);
          ids_to_codes(hh, part_out, codes, dg.n, s);
        }
        int32_t *list = lease->alloc_n<int32_t>(dg.n);
        Classes cl = build_classes(*lease, dg, list, cx.dev, cx.host, s);
        comm_cost(dg, cl, hh, codes, cx.sp.a, cx.dev, s);
        cx.pull();
        *j_out = cx.host->j;
      }
    }
    return rc;
  });
}

int pm_map(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed, int32_t *part_out,
           pm_map_stats *stats, uint32_t flags, void *stream) {
  return pm_map_ex(g, h, eps, seed, part_out, stats, flags, nullptr, stream);
}

int pm_map_ex(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed,
              int32_t *part_out, pm_map_stats *stats, uint32_t flags, const pm_options *opts,
              void *stream) {
  return guarded([&] {
    const Variants var = variants_of(opts);
    check_device();
    return map_impl(g, h, eps, seed, part_out, stats, flags, as_stream(stream), var);
  });
}

}  // extern "C"

namespace pm {
// The whole multilevel mapping on stream `stream` (throws Error).
int map_impl(const pm_graph *g, const pm_hierarchy *h, double eps, uint64_t seed,
             int32_t *part_out, pm_map_stats *stats, uint32_t flags, hipStream_t stream,
             const Variants &var) {
  {
    const auto t_start = std::chrono::steady_clock::now();
    const DGraph dg = view(g);
    const Hier hh = make_hier(h);
    if (dg.n > 0 && !part_out) throw Error(PM_EINVAL, "NULL output");
    ArenaLease lease(stream);
    Arena &ar = *lease;
    hipStream_t s = stream;
    Ctx cx(ar, s);
    int64_t total = 0;
    validate_graph(ar, dg, (flags & PM_FLAG_VALIDATE) != 0, &total, s);
    const int64_t lmax = lmax_of(total, hh.k, eps);
    const int64_t sigma = sigma_of(lmax, total, hh.k);
    pm_map_stats st;
    std::memset(&st, 0, sizeof(st));
    st.lmax = lmax;
    KernelTimer timer;
    timer.timing = (flags & PM_FLAG_KERNEL_TIMES) != 0;
    timer.counting = (flags & PM_FLAG_KERNEL_COUNTS) != 0;
    struct TimerScope {
      explicit TimerScope(KernelTimer *t) { tl_timer = t; }
      ~TimerScope() { tl_timer = nullptr; }
    } timer_scope((timer.timing || timer.counting) ? &timer : nullptr);

    EventSet evs;
    auto mark_event = [&]() {
      hipEvent_t e = evs.make();
      PM_HIP(hipEventRecord(e, s));
      return e;
    };
    struct Span { hipEvent_t a, b; double *acc; };
    std::vector<Span> spans;

    std::vector<Level> levels;
    levels.reserve(PM_MAX_GRAPH_LEVELS);
    Level L0;
    L0.g = dg;
    L0.list = ar.alloc_n<int32_t>(dg.n);
    L0.cl = build_classes(ar, dg, L0.list, cx.dev, cx.host, s);
    levels.push_back(L0);

    // ---- coarsening ----
    while ((int64_t)levels.back().g.n >= 8 * hh.k && (int)levels.size() < PM_MAX_GRAPH_LEVELS) {
      Level &L = levels.back();
      const int32_t n = L.g.n;
      const size_t mark0 = ar.mark();
      int32_t *cmap = ar.alloc_n<int32_t>(n);
      int64_t *cxadj = ar.alloc_n<int64_t>((size_t)n + 1);
      int32_t *cadj = ar.alloc_n<int32_t>(L.g.nnz);
      int32_t *cw = ar.alloc_n<int32_t>(L.g.nnz);
      int32_t *cvw = ar.alloc_n<int32_t>(n);
      int32_t *clist = ar.alloc_n<int32_t>(n);
      const size_t mark1 = ar.mark();
      int32_t *match = ar.alloc_n<int32_t>(n);
      int32_t *pref = ar.alloc_n<int32_t>(n);
      hipEvent_t e0 = mark_event();
      const int32_t rounds = run_hem(cx, L, lmax, seed, (int32_t)levels.size() - 1, match, pref);
      hipEvent_t e1 = mark_event();
      spans.push_back({e0, e1, &st.coarsen_ms});
      const int32_t nc = run_coarse_ids(cx, n, match, cmap);
      if (20 * (int64_t)nc > 19 * (int64_t)n) {
        ar.rewind(mark0);
        break;
      }
      int64_t cnnz = 0;
      run_contract(cx, L, match, cmap, nc, cxadj, cadj, cw, cvw, &cnnz);
      ar.rewind(mark1);
      Level C;
      C.g = DGraph{nc, cnnz, cxadj, cadj, cw, cvw};
      C.list = clist;
      C.cl = build_classes(ar, C.g, C.list, cx.dev, cx.host, s);
      hipEvent_t e2 = mark_event();
      spans.push_back({e1, e2, &st.contract_ms});
      L.cmap = cmap;
      L.hem_rounds = rounds;
      levels.push_back(C);
    }
    const int t = (int)levels.size() - 1;
    st.levels = t + 1;
    for (int i = 0; i <= t; ++i) {
      st.level_n[i] = levels[i].g.n;
      st.level_nnz[i] = levels[i].g.nnz;
      st.level_hem_rounds[i] = levels[i].hem_rounds;
    }

    // ---- initial partitioning ----
    int32_t *part = ar.alloc_n<int32_t>(levels[t].g.n);
    {
      hipEvent_t e0 = mark_event();
      run_initial(cx, levels[t].g, hh, part);
      hipEvent_t e1 = mark_event();
      spans.push_back({e0, e1, &st.initial_ms});
    }
    // ---- uncoarsening with refinement ----
    int32_t status = PM_OK;
    for (int lv = t;; --lv) {
      const Level &L = levels[lv];
      // "ultra": run r of Algorithm 6 starts from run r - 1's result
      for (int32_t r = 0; r < var.repeats; ++r) {
        RefineResult R = refine_level(cx, L.g, L.cl, hh, lmax, sigma, total,
                                      seed + (uint64_t)r, lv, part, var);
        st.refine_ms += R.st.refine_ms;
        st.refine_arcs += R.st.arcs_processed;
        st.level_iterations[lv] += R.st.iterations;
        st.j_final = R.st.j_final;
        st.feasible = R.st.feasible;
        status = R.status;
      }
      if (lv == 0) break;
      const Level &F = levels[lv - 1];
      int32_t *fine = ar.alloc_n<int32_t>(F.g.n);
      hipEvent_t e0 = mark_event();
      project(F.g.n, F.cmap, part, fine, s);
      hipEvent_t e1 = mark_event();
      spans.push_back({e0, e1, &st.uncoarsen_ms});
      part = fine;
    }
    codes_to_ids(hh, part, part_out, dg.n, s);
    PM_HIP(hipStreamSynchronize(s));
    for (auto &sp : spans) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) *sp.acc += ms;
    }
    if (timer.timing || timer.counting)
      timer.finish(st.kernel_launches, st.kernel_ms, st.kernel_bytes, st.kernel_units);
    st.total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
            .count();
    if (stats) *stats = st;
    return status;
  }
}
}  // namespace pm

