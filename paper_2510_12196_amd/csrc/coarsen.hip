// coarsen.hip -- heavy-edge matching, coarse numbering, contraction and
// projection for gfx950 (Section 4.2: Matching, Contraction, Uncontraction).
#include <hip/hip_ext.h>

#include "device_util.h"
#include "kernels.h"
#include "prim.h"

namespace pm {

static inline unsigned grid_for(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

// ===========================================================================
// Heavy-edge matching.  Edge rating w^2 / (c(u) c(v)); within v's row c(v)
// cancels, so candidate a beats b iff w_a^2 c_b > w_b^2 c_a (exact, 128-bit).
// Equal ratings: smaller hash of the unordered pair, then smaller lower
// endpoint, then smaller upper endpoint.  This is a total order on edges, so
// the best remaining edge is always mutually preferred.
// ===========================================================================
struct Cand {
  int32_t u;   // -1: none
  int32_t w;
  int32_t cu;
  uint64_t h;
};

__device__ __forceinline__ bool cand_better(const Cand &a, const Cand &b, int32_t v) {
  if (b.u < 0) return a.u >= 0;
  if (a.u < 0) return false;
  const unsigned __int128 l = (unsigned __int128)((uint64_t)a.w * (uint64_t)a.w) * (uint64_t)b.cu;
  const unsigned __int128 r = (unsigned __int128)((uint64_t)b.w * (uint64_t)b.w) * (uint64_t)a.cu;
  if (l != r) return l > r;
  if (a.h != b.h) return a.h < b.h;
  const int32_t alo = a.u < v ? a.u : v, blo = b.u < v ? b.u : v;
  if (alo != blo) return alo < blo;
  const int32_t ahi = a.u < v ? v : a.u, bhi = b.u < v ? v : b.u;
  return ahi < bhi;
}

// The best candidate of the group (a total order, so the pairing of the
// reduction steps does not matter); every lane gets it.
template <int G>
__device__ __forceinline__ void cand_reduce(Cand &c, int32_t v) {
  xsteps<G>([&](auto st) {
    Cand o;
    o.u = st(c.u);
    o.w = st(c.w);
    o.cu = st(c.cu);
    o.h = st(c.h);
    if (cand_better(o, c, v)) c = o;
  });
}

struct HemArgs {
  DGraph g;
  Classes cl;
  int64_t lmax;
  uint64_t hseed;
  const int32_t *match;
  int32_t *pref;
  const int32_t *cm;  // per vertex: its weight while unmatched, -1 once matched
  const uint8_t *hact;  // per vertex: looks for a partner this round (written by the commit)
};

// one gather per arc: the neighbour's weight-or-matched word
struct HemN {
  int32_t u, cmu, w;
};

// Whether v must (re)compute its preference this round.  Candidates only
// leave (neighbours get matched, weights are fixed), so the best candidate
// of the previous round stays the best while it is unmatched, and a vertex
// without candidates keeps none: only an unmatched vertex whose preferred
// partner was matched since, or that has none yet (kPrefUnknown), looks
// again.  The commit of the previous round decides this (hact), so that a
// tile does not wait for the match word of every preferred partner.  A
// matched vertex gets -1 (its stale preference must not pair it again).
constexpr int32_t kPrefUnknown = -2;
struct HemV {
  int32_t cv;
  bool matched;
};
__device__ __forceinline__ HemV hem_vertex(const HemArgs &A, int32_t v, bool &act) {
  act = A.hact[v] != 0;
  return HemV{A.g.c[v], A.match[v] >= 0};
}

template <int G, int V, class CL>
__device__ __forceinline__ void hem_group(const HemArgs &A, const CL &cl, int cls, int local) {
  group_tiles<G, V>(
      A.g.xadj, A.g.adj, cl, cls, local,
      [&](int32_t v, bool &act) { return hem_vertex(A, v, act); },
      [&](int32_t u, int64_t e) { return HemN{u, A.cm[u], A.g.w[e]}; },
      [&](int, bool ok, int32_t v, const HemV &hv, bool act, int, bool valid, const HemN &a) {
        if (!ok) return;
        const int lane = threadIdx.x % G;
        const int32_t cv = hv.cv;
        if (!act) {
          if (lane == 0 && hv.matched) A.pref[v] = -1;
          return;
        }
        Cand c{-1, 0, 1, 0};
        if (valid && a.cmu >= 0 && (int64_t)a.cmu + cv <= A.lmax) {
          const uint32_t lo = (uint32_t)(a.u < v ? a.u : v), hi = (uint32_t)(a.u < v ? v : a.u);
          c = Cand{a.u, a.w, a.cmu, mix_hash(A.hseed, ((uint64_t)lo << 32) | hi)};
        }
        cand_reduce<G>(c, v);
        if (lane == 0) A.pref[v] = c.u;
      });
}

struct CandScratch {
  Cand c[kThreads / 64];
};

// One class tile (blk) of the class list cl.
template <int V, class CL>
__device__ __forceinline__ void hem_tile(const HemArgs &A, const CL &cl, CandScratch &sc,
                                         int blk) {
  {
    const int cls = find_class(cl, blk);
    const int local = blk - cl.wg[cls];
    switch (cls) {
      case CLS_ISO:
        iso_tiles<V>(cl, local, [&](int32_t v) { A.pref[v] = -1; });
        break;
      case CLS_G8: hem_group<8, V>(A, cl, cls, local); break;
      case CLS_G16: hem_group<16, V>(A, cl, cls, local); break;
      case CLS_G32: hem_group<32, V>(A, cl, cls, local); break;
      case CLS_G64: hem_group<64, V>(A, cl, cls, local); break;
      case CLS_W: {
        int32_t v;
        if (!w_vertex(cl, local, v)) break;
        bool act;
        const HemV hv = hem_vertex(A, v, act);
        if (!act) {
          if ((threadIdx.x & 63) == 0 && hv.matched) A.pref[v] = -1;
          break;
        }
        const int32_t cv = hv.cv;
        Cand best{-1, 0, 1, 0};
        wave_arcs<4>(
            A.g.xadj[v], A.g.xadj[v + 1],
            [&](int64_t e) {
              const int32_t u = A.g.adj[e];
              return make_int3(u, A.cm[u], A.g.w[e]);
            },
            [&](int64_t, int3 a) {
              if (a.y < 0 || (int64_t)a.y + cv > A.lmax) return;
              const uint32_t lo = (uint32_t)(a.x < v ? a.x : v), hi = (uint32_t)(a.x < v ? v : a.x);
              const Cand c{a.x, a.z, a.y, mix_hash(A.hseed, ((uint64_t)lo << 32) | hi)};
              if (cand_better(c, best, v)) best = c;
            });
        cand_reduce<64>(best, v);
        if ((threadIdx.x & 63) == 0) A.pref[v] = best.u;
        break;
      }
      default: {
        const int32_t v = cl.list[cl.off[CLS_BIG] + local];
        bool act;
        const HemV hv = hem_vertex(A, v, act);
        if (!act) {
          if (threadIdx.x == 0 && hv.matched) A.pref[v] = -1;
          break;
        }
        const int32_t cv = hv.cv;
        Cand best{-1, 0, 1, 0};
        big_arcs(
            A.g.xadj[v], A.g.xadj[v + 1],
            [&](int64_t e) {
              const int32_t u = A.g.adj[e];
              return make_int3(u, A.cm[u], A.g.w[e]);
            },
            [&](int64_t, int3 a) {
              if (a.y < 0 || (int64_t)a.y + cv > A.lmax) return;
              const uint32_t lo = (uint32_t)(a.x < v ? a.x : v), hi = (uint32_t)(a.x < v ? v : a.x);
              const Cand c{a.x, a.z, a.y, mix_hash(A.hseed, ((uint64_t)lo << 32) | hi)};
              if (cand_better(c, best, v)) best = c;
            });
        cand_reduce<64>(best, v);
        const int wave = threadIdx.x >> 6;
        __syncthreads();  // the previous tile's reads of sc are done
        if ((threadIdx.x & 63) == 0) sc.c[wave] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
          Cand bb = sc.c[0];
          for (int i = 1; i < kThreads / 64; ++i)
            if (cand_better(sc.c[i], bb, v)) bb = sc.c[i];
          A.pref[v] = bb.u;
        }
        break;
      }
    }
  }
}

template <int V>
__global__ __launch_bounds__(kThreads) void k_hem_prefer(HemArgs A) {
  __shared__ CandScratch sc;
  hem_tile<V>(A, A.cl, sc, blockIdx.x);  // one class tile per workgroup
}

// The same over a class list whose offsets are on the device (dev_off,
// NCLS + 1 entries, written by the active-set compaction of the previous
// round): every workgroup loads them (uniform loads) and derives the tile
// bounds, then walks the tiles blockIdx.x, blockIdx.x + gridDim.x, ...  No
// read-back of the compacted sizes is needed between rounds.
// Class view of the device-offset launch: the offsets in LDS, the list
// pointer the kernel argument's (read back from LDS it would lose its
// address space, and a per-thread copy of the offsets would be indexed
// dynamically).
struct ClassesView {
  const int32_t *list;
  const int32_t *off;
  const int32_t *wg;
};

template <int V>
__global__ __launch_bounds__(kThreads) void k_hem_prefer_dev(HemArgs A, const int32_t *dev_off) {
  __shared__ CandScratch sc;
  __shared__ int32_t soff[NCLS + 1], swg[NCLS + 1];
  if (threadIdx.x == 0) {
    swg[0] = 0;
    for (int c = 0; c <= NCLS; ++c) soff[c] = dev_off[c];
    for (int c = 0; c < NCLS; ++c) {
      const int per = class_per_wg(c) * (c == CLS_BIG || c == CLS_W ? 1 : V);
      swg[c + 1] = swg[c] + (soff[c + 1] - soff[c] + per - 1) / per;
    }
  }
  __syncthreads();
  const ClassesView cl{A.cl.list, soff, swg};
  const int ntiles = swg[NCLS];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) hem_tile<V>(A, cl, sc, t);
}

// Grid of the device-offset launch: at most this many workgroups, which
// walk the tiles (at most those of the full class list).
constexpr unsigned kHemDevGrid = 4096;

void hem_prefer_dev(const DGraph &g, const Classes &cl, const int32_t *list,
                    const int32_t *dev_off, int64_t lmax, uint64_t hseed, const int32_t *match,
                    int32_t *pref, const int32_t *cm, const uint8_t *hact, hipStream_t s) {
  const int V = group_v();
  const Classes tc = tiled(cl, V);  // upper bound of the tiles
  unsigned nwg = classed_grid(tc);
  if (nwg == 0) return;
  if (nwg > kHemDevGrid) nwg = kHemDevGrid;
  Classes dc{};
  dc.list = list;
  HemArgs A{g, dc, lmax, hseed, match, pref, cm, hact};
  auto kern = V == 2 ? k_hem_prefer_dev<2> : k_hem_prefer_dev<1>;
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, A, dev_off);
  PM_LAUNCH_CHECK();
}

void hem_prefer(const DGraph &g, const Classes &cl, int64_t lmax, uint64_t hseed,
                const int32_t *match, int32_t *pref, const int32_t *cm, const uint8_t *hact,
                hipStream_t s) {
  const int V = group_v();
  const Classes tc = tiled(cl, V);
  const unsigned nwg = classed_grid(tc);
  if (nwg == 0) return;
  HemArgs A{g, tc, lmax, hseed, match, pref, cm, hact};
  auto kern = V == 2 ? k_hem_prefer<2> : k_hem_prefer<1>;
  if (tl_timer) count_units(cl, g.xadj, CU_HEM_ACTIVE, CountArgs{nullptr, nullptr, nullptr, nullptr, match,
                                                                 pref},
                            tl_timer->counters(KT_HEM), s);
  hipEvent_t a = nullptr, b = nullptr;
  if (tl_timer) tl_timer->pair(KT_HEM, a, b);
  if (a) {
    hipExtLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, a, b, 0, A);
  } else {
    hipLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, A);
  }
  PM_LAUNCH_CHECK();
}

// ---- active-set compaction between matching rounds ---------------------------
// After the first rounds few vertices must look again (those whose preferred
// partner was matched), but a launch over all class tiles still visits every
// vertex.  On large levels the active ones are therefore compacted: a stable
// selection of the class-list positions whose vertex has its look-again flag
// (read through the list; class order kept), then the new class offsets and
// the list of vertex ids.
// off_out[c] = first compacted position of class c (classes by the offsets
// off[] of the full list); list_out[j] = list[pos[j]].
__global__ void k_compact_bounds(int32_t n, Classes cl, const int32_t *pos, const int32_t *count,
                                 int32_t *list_out, int32_t *off_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t m = *count;
  if (j > m) return;
  auto cls_of = [&](int32_t p) {
    int c = 0;
    while (c < NCLS - 1 && p >= cl.off[c + 1]) ++c;
    return c;
  };
  const int prev = j > 0 ? cls_of(pos[j - 1]) : -1;
  const int cur = j < m ? cls_of(pos[j]) : NCLS;
  for (int c = prev + 1; c <= cur; ++c) off_out[c] = (int32_t)j;
  if (j < m) list_out[j] = cl.list[pos[j]];
}

void compact_bounds(int32_t n, const Classes &cl, const int32_t *pos, const int32_t *count,
                    int32_t *list_out, int32_t *off_out, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_bounds, dim3(grid_for((int64_t)n + 1)), dim3(kThreads), 0, s, n,
                     cl, pos, count, list_out, off_out);
  PM_LAUNCH_CHECK();
}

void hem_compact(Arena &ar, const Classes &cl, int32_t n, const uint8_t *hact,
                 int32_t *list_out, int32_t *off_out, hipStream_t s) {
  int32_t *pos = ar.alloc_n<int32_t>((size_t)n + 1);
  int32_t *count = ar.alloc_n<int32_t>(1);
  select_list_flagged(ar, hact, cl.list, pos, count, n, s);  // positions whose vertex looks again
  compact_bounds(n, cl, pos, count, list_out, off_out, s);
}

// v and pref[v] are matched iff they prefer each other.  The count goes up a
// two-level tree of 64-bit counters, each word (1 << 32) x workgroups done +
// matches: workgroup b adds to leaf b % 64; the workgroup that completes a
// leaf clears it and adds the leaf's total to the root; the one that
// completes the root stores st->count and clears the root.  Each step is one
// atomic that carries both the data and the completion, so no fence is
// needed, and no address sees more than 64 atomics.
constexpr int kHemLeaves = 64;
// It also decides which unmatched vertices look again in the next round
// (hact): those whose preferred partner u is matched after this commit,
// that is, matched before (its match word; read while u's own thread may
// write it, but then u is matched now and the second test holds too) or now
// (u and its preferred partner prefer each other).
__global__ __launch_bounds__(kThreads) void k_hem_commit(int32_t n, const int32_t *pref,
                                                         int32_t *match, int32_t *cm,
                                                         uint8_t *hact, uint64_t *counter,
                                                         Status *st, int32_t *count_out) {
  __shared__ BlockScratch sc;
  int64_t hits = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (match[v] >= 0) continue;  // (its flag went to 0 when it was matched)
    const int32_t u = pref[v];
    const int32_t pu = u >= 0 ? pref[u] : -1;
    if (u >= 0 && pu == (int32_t)v) {
      match[v] = u;
      cm[v] = -1;
      hact[v] = 0;
      ++hits;
      continue;
    }
    bool again = u == kPrefUnknown;
    if (u >= 0) again = match[u] >= 0 || (pu >= 0 && pref[pu] == u);
    hact[v] = again ? 1 : 0;
  }
  hits = block_sum64(hits, sc);
  if (threadIdx.x != 0) return;
  const unsigned G = gridDim.x;
  const unsigned leaf = blockIdx.x % kHemLeaves;
  const unsigned leaf_wgs = (G - leaf + kHemLeaves - 1) / kHemLeaves;
  const unsigned leaves = G < (unsigned)kHemLeaves ? G : (unsigned)kHemLeaves;
  unsigned long long *lp = (unsigned long long *)&counter[1 + leaf];
  const uint64_t add = (1ull << 32) + (uint64_t)hits;
  const uint64_t l = atomicAdd(lp, (unsigned long long)add) + add;
  if ((l >> 32) != leaf_wgs) return;
  atomicExch(lp, 0ull);
  unsigned long long *rp = (unsigned long long *)&counter[0];
  const uint64_t radd = (1ull << 32) + (l & 0xFFFFFFFFull);
  const uint64_t r = atomicAdd(rp, (unsigned long long)radd) + radd;
  if ((r >> 32) != leaves) return;
  atomicExch(rp, 0ull);
  st->count = (int32_t)(r & 0xFFFFFFFFull);
  if (count_out) *count_out = (int32_t)(r & 0xFFFFFFFFull);
}

void hem_commit(int32_t n, const int32_t *pref, int32_t *match, int32_t *cm, uint8_t *hact,
                uint64_t *counter, Status *st, int32_t *count_out, hipStream_t s) {
  unsigned g = grid_for(n > 0 ? n : 1);
  if (g > kMaxGrid) g = kMaxGrid;
  hipLaunchKernelGGL(k_hem_commit, dim3(g), dim3(kThreads), 0, s, n, pref, match, cm, hact,
                     counter, st, count_out);
  PM_LAUNCH_CHECK();
}

// unmatched -> self; leader flag (the smaller member of a pair, or a single)
__global__ void k_hem_finish(int32_t n, int32_t *match, int32_t *leader) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t m = match[v];
  if (m < 0) {
    m = (int32_t)v;
    match[v] = m;
  }
  leader[v] = m >= v ? 1 : 0;
}
void hem_finish(int32_t n, int32_t *match, int32_t *leader, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_hem_finish, dim3(grid_for(n)), dim3(kThreads), 0, s, n, match, leader);
  PM_LAUNCH_CHECK();
}

// A matching as the contraction takes it: every entry is -1 (unmatched), the
// vertex itself, or a partner that points back.
__global__ void k_check_match(int32_t n, const int32_t *match, int32_t *bad) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t m = match[v];
  const bool ok = m == -1 || m == v || (m >= 0 && m < n && match[m] == v);
  if (!ok) atomicOr(bad, 1);
}
void check_match(int32_t n, const int32_t *match, int32_t *bad, hipStream_t s) {
  PM_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_match, dim3(grid_for(n)), dim3(kThreads), 0, s, n, match, bad);
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Coarse numbering: coarse id = rank of the pair's smaller member.
// `rank` holds, for every leader, the number of leaders before it.
// ===========================================================================
__global__ void k_coarse_ids(int32_t n, const int32_t *match, const int32_t *rank,
                             int32_t *cmap) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t m = match[v];
  cmap[v] = rank[m < v ? m : (int32_t)v];
}
void coarse_ids(int32_t n, const int32_t *match, const int32_t *rank, int32_t *cmap,
                hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_coarse_ids, dim3(grid_for(n)), dim3(kThreads), 0, s, n, match, rank, cmap);
  PM_LAUNCH_CHECK();
}

__global__ void k_coarse_vwgt(int32_t n, const int32_t *match, const int32_t *cmap,
                              const int32_t *vwgt, int32_t *cvwgt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t m = match[v];
  if (m < v) return;
  cvwgt[cmap[v]] = vwgt[v] + (m != v ? vwgt[m] : 0);
}
void coarse_vwgt(int32_t n, const int32_t *match, const int32_t *cmap, const int32_t *vwgt,
                 int32_t *cvwgt, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_coarse_vwgt, dim3(grid_for(n)), dim3(kThreads), 0, s, n, match, cmap,
                     vwgt, cvwgt);
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Contraction: every arc e = (v, u, w) becomes the key (M(v) << B | M(u)),
// arcs inside one coarse vertex get the all-ones key and sort to the end.
// After a radix sort of the keys, runs of equal keys are fused with their
// weights summed; rows come out in ascending neighbour order.
// ===========================================================================
struct KeyArgs {
  DGraph g;
  Classes cl;
  const int32_t *cmap;
  int bits;
  uint64_t *key;
  int32_t *val;
  int64_t *stripes;
};

__device__ __forceinline__ int32_t key_arc(const KeyArgs &A, uint64_t cv, int64_t e) {
  const uint64_t cu = (uint64_t)A.cmap[A.g.adj[e]];
  A.val[e] = A.g.w[e];
  if (cu == cv) {
    A.key[e] = (A.bits >= 32) ? ~0ull : ((1ull << (2 * A.bits)) - 1ull);
    return 1;
  }
  A.key[e] = (cv << A.bits) | cu;
  return 0;
}

template <int G>
__device__ __forceinline__ int32_t key_group(const KeyArgs &A, int cls, int local) {
  int32_t v;
  if (!group_vertex<G>(A.cl, cls, local, v)) return 0;
  const int lane = threadIdx.x % G;
  const int64_t e = A.g.xadj[v] + lane;
  if (e >= A.g.xadj[v + 1]) return 0;
  return key_arc(A, (uint64_t)A.cmap[v], e);
}

__global__ __launch_bounds__(kThreads) void k_contract_keys(KeyArgs A) {
  __shared__ BlockScratch sc;
  int64_t self = 0;
  {  // one class tile per workgroup
    const int blk = blockIdx.x;
    const int cls = find_class(A.cl, blk);
    const int local = blk - A.cl.wg[cls];
    switch (cls) {
      case CLS_ISO: break;
      case CLS_G8: self += key_group<8>(A, cls, local); break;
      case CLS_G16: self += key_group<16>(A, cls, local); break;
      case CLS_G32: self += key_group<32>(A, cls, local); break;
      case CLS_G64: self += key_group<64>(A, cls, local); break;
      case CLS_W: {
        int32_t v;
        if (!w_vertex(A.cl, local, v)) break;
        const uint64_t cv = (uint64_t)A.cmap[v];
        const uint64_t sentinel = (A.bits >= 32) ? ~0ull : ((1ull << (2 * A.bits)) - 1ull);
        wave_arcs<4>(
            A.g.xadj[v], A.g.xadj[v + 1],
            [&](int64_t e) { return make_int2(A.cmap[A.g.adj[e]], A.g.w[e]); },
            [&](int64_t e, int2 a) {
              const uint64_t cu = (uint64_t)a.x;
              A.val[e] = a.y;
              A.key[e] = cu == cv ? sentinel : ((cv << A.bits) | cu);
              self += cu == cv ? 1 : 0;
            });
        break;
      }
      default: {
        const int32_t v = A.cl.list[A.cl.off[CLS_BIG] + local];
        const uint64_t cv = (uint64_t)A.cmap[v];
        const uint64_t sentinel = (A.bits >= 32) ? ~0ull : ((1ull << (2 * A.bits)) - 1ull);
        big_arcs(
            A.g.xadj[v], A.g.xadj[v + 1],
            [&](int64_t e) { return make_int2(A.cmap[A.g.adj[e]], A.g.w[e]); },
            [&](int64_t e, int2 a) {
              const uint64_t cu = (uint64_t)a.x;
              A.val[e] = a.y;
              A.key[e] = cu == cv ? sentinel : ((cv << A.bits) | cu);
              self += cu == cv ? 1 : 0;
            });
        break;
      }
    }
  }
  self = block_sum64(self, sc);
  if (threadIdx.x == 0) stripe_add(A.stripes, self);
}

void contract_keys(const DGraph &g, const Classes &cl, const int32_t *cmap, int bits,
                   uint64_t *key, int32_t *val, int64_t *stripes, Status *st, hipStream_t s) {
  const unsigned nwg = classed_grid(cl);
  if (nwg > 0) {
    KeyArgs A{g, cl, cmap, bits, key, val, stripes};
    hipLaunchKernelGGL(k_contract_keys, dim3(nwg), dim3(kThreads), 0, s, A);
    PM_LAUNCH_CHECK();
  }
  fold_stripes(stripes, nullptr, &st->count, s);
}

// The sorted keys end with the self-loop sentinels: m = nnz - *self arcs are
// real (the count is read on the device, so no host read-back is needed
// between the sort and the emission).
__global__ void k_contract_heads(int64_t nnz, const int32_t *self, const uint64_t *key,
                                 int32_t *head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = nnz - *self;
  if (i < nnz) head[i] = i < m && (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

void contract_heads(int64_t nnz, const int32_t *self, const uint64_t *key, int32_t *head,
                    hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_contract_heads, dim3(grid_for(nnz)), dim3(kThreads), 0, s, nnz, self, key,
                     head);
  PM_LAUNCH_CHECK();
}

// One thread per run head: fuse the run (at most 4 arcs: two members per
// side).  The runs of a coarse row are consecutive, so its length is
// (position of its last run + 1) - (position of its first run); only the
// threads of those two runs touch the row's counter (a hub row would
// otherwise take one atomic per run on a single address).
__global__ void k_contract_emit(int64_t nnz, const int32_t *self, const uint64_t *key,
                                const int32_t *val, const int32_t *head, const int32_t *pos,
                                int bits, int32_t *cadj, int32_t *cw, int32_t *rowcnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = nnz - *self;
  if (i >= m || !head[i]) return;
  const uint64_t k = key[i];
  int64_t sum = 0;
  int64_t j = i;
  for (; j < m && key[j] == k; ++j) sum += val[j];
  const int32_t o = pos[i];
  cadj[o] = (int32_t)(k & ((1ull << bits) - 1ull));
  cw[o] = (int32_t)sum;
  const uint64_t row = k >> bits;
  const bool first = i == 0 || (key[i - 1] >> bits) != row;
  const bool last = j == m || (key[j] >> bits) != row;
  if (first && last) rowcnt[row] = 1;
  else if (first) atomicAdd(&rowcnt[row], -o);
  else if (last) atomicAdd(&rowcnt[row], o + 1);
}

void contract_emit(int64_t nnz, const int32_t *self, const uint64_t *key, const int32_t *val,
                   const int32_t *head, const int32_t *pos, int bits, int32_t *cadj, int32_t *cw,
                   int32_t *rowcnt, hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_contract_emit, dim3(grid_for(nnz)), dim3(kThreads), 0, s, nnz, self, key,
                     val, head, pos, bits, cadj, cw, rowcnt);
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Row-local contraction (large levels).  Coarse row c = {v, M(v)} has at most
// ub(c) = deg(v) + deg(M(v)) arcs before merging.  The arcs of every row are
// first staged at that upper-bound offset, as (coarse neighbour, weight), with
// self loops marked.  A row with ub <= 64 is then sorted, merged and
// compacted in place by G lanes in registers (bitonic network, segmented sum
// of equal neighbours), a row with ub <= 512 by one wave holding up to eight
// arcs per lane, a row with ub <= 2048 by a workgroup in LDS; longer rows go
// through one global radix sort keyed by (row, neighbour) over their arcs
// only.  The merged lengths give the coarse offsets, and a last pass copies
// every row to its place.  The result is the same CSR as the global sort over
// all arcs: per row the distinct coarse neighbours other than itself,
// ascending, with summed weights.
// ===========================================================================
constexpr uint32_t kStageSelf = 0xFFFFFFFFu;
constexpr int kRowMaxG = 64;      // rows up to this bound: lane groups
constexpr int kRowMaxWave = 512;  // ... one wave, eight arcs per lane in registers
constexpr int kRowMaxLds = 2048;  // ... a workgroup in LDS

__global__ __launch_bounds__(kThreads) void k_contract_rowub(int32_t n, const int64_t *xadj,
                                                             const int32_t *match,
                                                             const int32_t *cmap, int32_t *ub,
                                                             int32_t *ubig, int64_t *above64) {
  __shared__ BlockScratch sc;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t a = 0;
  if (v < n) {
    const int32_t m = match[v];
    if (m >= v) {  // the row is written by its leader, the smaller member
      const int64_t d = (xadj[v + 1] - xadj[v]) + (m != v ? xadj[m + 1] - xadj[m] : 0);
      const int32_t c = cmap[v];
      ub[c] = (int32_t)d;
      ubig[c] = d > kRowMaxLds ? (int32_t)d : 0;
      a = d > kRowMaxG ? d : 0;
    }
  }
  a = block_sum64(a, sc);
  if (threadIdx.x == 0 && a) atomicAdd((unsigned long long *)above64, (unsigned long long)a);
}

void contract_rowub(const DGraph &g, const int32_t *match, const int32_t *cmap, int32_t *ub,
                    int32_t *ubig, int64_t *above64, hipStream_t s) {
  fill_i64(above64, 0, 1, s);
  if (g.n <= 0) return;
  hipLaunchKernelGGL(k_contract_rowub, dim3(grid_for(g.n)), dim3(kThreads), 0, s, g.n, g.xadj,
                     match, cmap, ub, ubig, above64);
  PM_LAUNCH_CHECK();
}

struct StageArgs {
  DGraph g;
  Classes cl;
  const int32_t *match;
  const int32_t *cmap;
  const int64_t *uxadj;
  uint32_t *scu;
  int32_t *sw;
};

// first staged slot of fine vertex v: the leader's arcs come first
__device__ __forceinline__ int64_t stage_base(const StageArgs &A, int32_t v) {
  const int32_t m = A.match[v];
  const int64_t b = A.uxadj[A.cmap[v]];
  return m < v ? b + (A.g.xadj[m + 1] - A.g.xadj[m]) : b;
}

__device__ __forceinline__ void stage_arc(const StageArgs &A, uint32_t cv, int64_t dst, int32_t cu,
                                          int32_t w) {
  A.scu[dst] = (uint32_t)cu == cv ? kStageSelf : (uint32_t)cu;
  A.sw[dst] = w;
}

__global__ __launch_bounds__(kThreads) void k_contract_stage(StageArgs A) {
  const int blk = blockIdx.x;
  const int cls = find_class(A.cl, blk);
  const int local = blk - A.cl.wg[cls];
  int32_t v;
  switch (cls) {
    case CLS_ISO: break;
    case CLS_G8:
    case CLS_G16:
    case CLS_G32:
    case CLS_G64: {
      const int G = class_group(cls);
      const int idx = local * (kThreads / G) + (int)threadIdx.x / G;
      if (idx >= A.cl.off[cls + 1] - A.cl.off[cls]) break;
      v = A.cl.list[A.cl.off[cls] + idx];
      const int lane = threadIdx.x % G;
      const int64_t beg = A.g.xadj[v];
      if (beg + lane >= A.g.xadj[v + 1]) break;
      const int64_t e = beg + lane;
      stage_arc(A, (uint32_t)A.cmap[v], stage_base(A, v) + lane, A.cmap[A.g.adj[e]], A.g.w[e]);
      break;
    }
    case CLS_W: {
      if (!w_vertex(A.cl, local, v)) break;
      const uint32_t cv = (uint32_t)A.cmap[v];
      const int64_t beg = A.g.xadj[v];
      const int64_t base = stage_base(A, v) - beg;
      wave_arcs<4>(
          beg, A.g.xadj[v + 1],
          [&](int64_t e) { return make_int2(A.cmap[A.g.adj[e]], A.g.w[e]); },
          [&](int64_t e, int2 a) { stage_arc(A, cv, base + e, a.x, a.y); });
      break;
    }
    default: {
      v = A.cl.list[A.cl.off[CLS_BIG] + local];
      const uint32_t cv = (uint32_t)A.cmap[v];
      const int64_t beg = A.g.xadj[v];
      const int64_t base = stage_base(A, v) - beg;
      big_arcs(
          beg, A.g.xadj[v + 1],
          [&](int64_t e) { return make_int2(A.cmap[A.g.adj[e]], A.g.w[e]); },
          [&](int64_t e, int2 a) { stage_arc(A, cv, base + e, a.x, a.y); });
      break;
    }
  }
}

void contract_stage(const DGraph &g, const Classes &cl, const int32_t *match, const int32_t *cmap,
                    const int64_t *uxadj, uint32_t *scu, int32_t *sw, hipStream_t s) {
  const unsigned nwg = classed_grid(cl);
  if (nwg == 0 || g.nnz <= 0) return;
  StageArgs A{g, cl, match, cmap, uxadj, scu, sw};
  hipLaunchKernelGGL(k_contract_stage, dim3(nwg), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
}

struct RowArgs {
  Classes rc;           // coarse rows classed by ub
  const int64_t *uxadj;
  uint32_t *scu;
  int32_t *sw;
  int32_t *rowcnt;
};

// One row of at most G staged arcs on G lanes: sort by neighbour, add the
// weights of equal neighbours, write the distinct ones back from the row's
// first slot, and its length to rowcnt.
template <int G>
__device__ __forceinline__ void merge_row(const RowArgs &A, int cls, int local) {
  int32_t c;
  if (!group_vertex<G>(A.rc, cls, local, c)) return;
  const int lane = threadIdx.x % G;
  const int64_t beg = A.uxadj[c];
  const int ub = (int)(A.uxadj[c + 1] - beg);
  uint32_t key = kStageSelf;
  int32_t w = 0;
  if (lane < ub) {
    key = A.scu[beg + lane];
    w = A.sw[beg + lane];
  }
#pragma unroll
  for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t pk = (uint32_t)xor_lane((int32_t)key, j);
      const int32_t pw = xor_lane(w, j);
      const bool up = (lane & k) == 0, low = (lane & j) == 0;
      if (low == up ? pk < key : pk > key) {
        key = pk;
        w = pw;
      }
    }
  }
  // suffix sums within runs of equal keys: the run's first lane gets its total
  int32_t sum = w;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const uint32_t nk = (uint32_t)__shfl_down((int32_t)key, d, G);
    const int32_t ns = __shfl_down(sum, d, G);
    if (lane + d < G && nk == key) sum += ns;
  }
  const uint32_t pk = (uint32_t)__shfl_up((int32_t)key, 1, G);
  const bool head = key != kStageSelf && (lane == 0 || pk != key);
  const int wl = threadIdx.x & 63;
  const uint64_t gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << (wl & ~(G - 1)));
  const uint64_t heads = __ballot(head) & gmask;
  if (head) {
    const int r = __popcll(heads & ((1ull << wl) - 1ull));
    A.scu[beg + r] = key;
    A.sw[beg + r] = sum;
  }
  if (lane == 0) A.rowcnt[c] = __popcll(heads);
}

__global__ __launch_bounds__(kThreads) void k_contract_rows(RowArgs A) {
  const int blk = blockIdx.x;
  const int cls = find_class(A.rc, blk);
  const int local = blk - A.rc.wg[cls];
  switch (cls) {
    case CLS_ISO:
      iso_tiles<1>(A.rc, local, [&](int32_t c) { A.rowcnt[c] = 0; });
      break;
    case CLS_G8: merge_row<8>(A, cls, local); break;
    case CLS_G16: merge_row<16>(A, cls, local); break;
    case CLS_G32: merge_row<32>(A, cls, local); break;
    case CLS_G64: merge_row<64>(A, cls, local); break;
    default: break;  // W and BIG rows: the sorted path
  }
}

void contract_rows(const Classes &rc, const int64_t *uxadj, uint32_t *scu, int32_t *sw,
                   int32_t *rowcnt, hipStream_t s) {
  const unsigned nwg = classed_grid(rc);
  if (nwg == 0) return;
  RowArgs A{rc, uxadj, scu, sw, rowcnt};
  hipLaunchKernelGGL(k_contract_rows, dim3(nwg), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
}

// Rows with 64 < ub <= 512: one wave, element i = lane * E + slot (E = 2, 4
// or 8 per lane, N = 64 E).  Bitonic network: partners within a lane are
// swapped in registers, partners in other lanes exchanged by shuffles.
// After the sort a run of equal neighbours may span lanes: each lane's
// leading run is summed, and a backward segmented scan over the lanes adds
// the continuation from the following lanes.
template <int E>
__device__ __forceinline__ void wave_merge_row(int32_t c, int64_t beg, int ub, uint32_t *scu,
                                               int32_t *sw, int32_t *rowcnt) {
  const int lane = threadIdx.x & 63;
  uint32_t k[E];
  int32_t w[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int i = lane * E + q;
    k[q] = i < ub ? scu[beg + i] : kStageSelf;
    w[q] = i < ub ? sw[beg + i] : 0;
  }
#pragma unroll
  for (int kk = 2; kk <= 64 * E; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= E) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int i = lane * E + q;
          const uint32_t pk = (uint32_t)xor_lane((int32_t)k[q], j / E);
          const int32_t pw = xor_lane(w[q], j / E);
          const bool up = (i & kk) == 0, low = (i & j) == 0;
          if (low == up ? pk < k[q] : pk > k[q]) {
            k[q] = pk;
            w[q] = pw;
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < E; ++q) {
          if (q & j) continue;
          const int p = q | j;
          const bool up = ((lane * E + q) & kk) == 0;
          if ((k[q] > k[p]) == up) {
            const uint32_t tk = k[q];
            k[q] = k[p];
            k[p] = tk;
            const int32_t tw = w[q];
            w[q] = w[p];
            w[p] = tw;
          }
        }
      }
    }
  }
  const uint32_t prev_last = (uint32_t)__shfl_up((int32_t)k[E - 1], 1, 64);
  const uint32_t next_first = (uint32_t)__shfl_down((int32_t)k[0], 1, 64);
  bool head[E];
  uint32_t cnt = 0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const uint32_t pv = q ? k[q - 1] : prev_last;
    head[q] = k[q] != kStageSelf && ((lane == 0 && q == 0) || pv != k[q]);
    cnt += head[q] ? 1u : 0u;
  }
  // the lane's leading run, and whether it fills the lane
  int64_t S = w[0];
  bool full = true;
#pragma unroll
  for (int q = 1; q < E; ++q) {
    full = full && k[q] == k[0];
    if (full) S += w[q];
  }
  // S(L) = lead(L) + S(L + 1) while lane L is one run continued by lane L + 1
  bool F = !(full && lane < 63 && next_first == k[0]);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t Sn = gshfl64<64>(S, lane + d < 64 ? lane + d : lane);
    const bool Fn = __shfl_down((int)F, d, 64) != 0;
    if (!F && lane + d < 64) {
      S += Sn;
      F = Fn;
    }
  }
  const int64_t s_next = gshfl64<64>(S, lane < 63 ? lane + 1 : lane);
  uint32_t r = cnt;  // exclusive scan of the head counts over the lanes
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int32_t)r, o, 64);
    if (lane >= o) r += y;
  }
  const uint32_t total = (uint32_t)__shfl((int32_t)r, 63, 64);
  r -= cnt;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    if (!head[q]) continue;
    int64_t sum = 0;
    bool open = true;
#pragma unroll
    for (int t = q; t < E; ++t) {
      open = open && k[t] == k[q];
      if (open) sum += w[t];
    }
    if (open && lane < 63 && next_first == k[q]) sum += s_next;
    scu[beg + r] = k[q];
    sw[beg + r] = (int32_t)sum;
    ++r;
  }
  if (lane == 0) rowcnt[c] = (int32_t)total;
}

// Rows with 512 < ub <= 2048: the whole workgroup sorts (neighbour, weight)
// in LDS with a bitonic network over the next power of two, then writes the
// distinct neighbours in order with their summed weights from the row's
// first slot.
struct LdsRow {
  uint32_t key[kRowMaxLds];
  int32_t w[kRowMaxLds];
};

__device__ __forceinline__ void lds_merge_row(LdsRow &R, BlockScratch &sc, int32_t c, int64_t beg,
                                              int ub, uint32_t *scu, int32_t *sw,
                                              int32_t *rowcnt) {
  int N = 1;
  while (N < ub) N <<= 1;
  __syncthreads();  // the previous row's readers are done
  for (int i = threadIdx.x; i < N; i += kThreads) {
    R.key[i] = i < ub ? scu[beg + i] : kStageSelf;
    R.w[i] = i < ub ? sw[beg + i] : 0;
  }
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < (N >> 1); t += kThreads) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int p = i + j;
        const uint32_t a = R.key[i], b = R.key[p];
        if ((a > b) == ((i & k) == 0)) {
          R.key[i] = b;
          R.key[p] = a;
          const int32_t x = R.w[i];
          R.w[i] = R.w[p];
          R.w[p] = x;
        }
      }
      __syncthreads();
    }
  }
  // each thread takes a contiguous chunk: count its run heads, scan, write
  const int per = (N + kThreads - 1) / kThreads;
  const int lo = threadIdx.x * per < N ? threadIdx.x * per : N;
  const int hi = lo + per < N ? lo + per : N;
  uint32_t cnt = 0;
  for (int i = lo; i < hi; ++i)
    cnt += R.key[i] != kStageSelf && (i == 0 || R.key[i] != R.key[i - 1]) ? 1u : 0u;
  uint32_t r = block_excl_scan(cnt, sc);
  const uint32_t total = sc.u[0] + sc.u[1] + sc.u[2] + sc.u[3];
  for (int i = lo; i < hi; ++i) {
    const uint32_t k = R.key[i];
    if (k == kStageSelf || (i > 0 && R.key[i - 1] == k)) continue;
    int64_t sum = 0;
    for (int j = i; j < N && R.key[j] == k; ++j) sum += R.w[j];
    scu[beg + r] = k;
    sw[beg + r] = (int32_t)sum;
    ++r;
  }
  if (threadIdx.x == 0) rowcnt[c] = (int32_t)total;
}

// Rows above 64 (the list of BIG and W rows), four per workgroup: first every
// wave merges its own row if it is at most 512, then the workgroup merges
// those of 513..2048 one after another.  Longer rows are left to the sort.
__global__ __launch_bounds__(kThreads) void k_contract_mid_rows(const int32_t *list, int32_t nl,
                                                                const int64_t *uxadj,
                                                                uint32_t *scu, int32_t *sw,
                                                                int32_t *rowcnt) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  LdsRow &R = *reinterpret_cast<LdsRow *>(lds_raw);
  __shared__ BlockScratch sc;
  const int64_t base = (int64_t)blockIdx.x * (kThreads / 64);
  {
    const int64_t idx = base + (threadIdx.x >> 6);
    if (idx < nl) {
      const int32_t c = list[idx];
      const int64_t beg = uxadj[c];
      const int ub = (int)(uxadj[c + 1] - beg);
      if (ub <= 128) wave_merge_row<2>(c, beg, ub, scu, sw, rowcnt);
      else if (ub <= 256) wave_merge_row<4>(c, beg, ub, scu, sw, rowcnt);
      else if (ub <= kRowMaxWave) wave_merge_row<8>(c, beg, ub, scu, sw, rowcnt);
    }
  }
  for (int q = 0; q < kThreads / 64 && base + q < nl; ++q) {
    const int32_t c = list[base + q];
    const int64_t beg = uxadj[c];
    const int ub = (int)(uxadj[c + 1] - beg);
    if (ub > kRowMaxWave && ub <= kRowMaxLds) lds_merge_row(R, sc, c, beg, ub, scu, sw, rowcnt);
  }
}

void contract_mid_rows(const int32_t *list, int32_t nl, const int64_t *uxadj, uint32_t *scu,
                       int32_t *sw, int32_t *rowcnt, hipStream_t s) {
  if (nl <= 0) return;
  const unsigned nwg = (unsigned)((nl + kThreads / 64 - 1) / (kThreads / 64));
  hipLaunchKernelGGL(k_contract_mid_rows, dim3(nwg), dim3(kThreads), sizeof(LdsRow), s, list, nl,
                     uxadj, scu, sw, rowcnt);
  PM_LAUNCH_CHECK();
}

// Rows above 2048: keys (row << bits | neighbour) at the row's place among
// those rows (rstart: exclusive prefix of their ub in row order; rows of the
// list with no place are skipped), self loops keyed with the all-ones
// neighbour so that they sort last in their row.  Four list entries per
// workgroup; a row with a place is copied by the whole workgroup, four
// elements per thread loaded before any store.
__global__ __launch_bounds__(kThreads) void k_long_keys(const int32_t *list, int32_t nl,
                                                        const int64_t *uxadj,
                                                        const int64_t *rstart,
                                                        const uint32_t *scu, const int32_t *sw,
                                                        int bits, uint64_t *key, int32_t *val) {
  const uint64_t mask = (1ull << bits) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * (kThreads / 64);
  for (int q = 0; q < kThreads / 64 && base + q < nl; ++q) {
    const int32_t c = list[base + q];
    const int64_t dst = rstart[c], ub = rstart[c + 1] - dst;  // 0: merged in place
    if (ub == 0) continue;
    const int64_t beg = uxadj[c];
    const uint64_t row = (uint64_t)c << bits;
    for (int64_t j0 = 0; j0 < ub; j0 += 4 * kThreads) {
      uint32_t x[4];
      int32_t y[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + r * kThreads + threadIdx.x;
        const int64_t jj = j < ub ? j : ub - 1;
        x[r] = scu[beg + jj];
        y[r] = sw[beg + jj];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + r * kThreads + threadIdx.x;
        if (j < ub) {
          key[dst + j] = row | (x[r] == kStageSelf ? mask : (uint64_t)x[r]);
          val[dst + j] = y[r];
        }
      }
    }
  }
}

__global__ void k_long_heads(int64_t m, const uint64_t *key, int bits, int32_t *head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  const uint64_t mask = (1ull << bits) - 1ull;
  head[i] = i < m && (key[i] & mask) != mask && (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// Every run head writes its merged arc at its rank within the row, from the
// row's first staged slot.
__global__ void k_long_emit(int64_t m, const uint64_t *key, const int32_t *val,
                            const int32_t *head, const int32_t *pos, const int64_t *rstart,
                            const int64_t *uxadj, int bits, uint32_t *scu, int32_t *sw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m || !head[i]) return;
  const uint64_t k = key[i];
  int64_t sum = 0;
  for (int64_t j = i; j < m && key[j] == k; ++j) sum += val[j];
  const int32_t c = (int32_t)(k >> bits);
  const int64_t o = uxadj[c] + (pos[i] - pos[rstart[c]]);
  scu[o] = (uint32_t)(k & ((1ull << bits) - 1ull));
  sw[o] = (int32_t)sum;
}

__global__ void k_long_count(int32_t nl, const int32_t *list, const int64_t *rstart,
                             const int32_t *pos, int32_t *rowcnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const int32_t c = list[i];
  if (rstart[c + 1] > rstart[c]) rowcnt[c] = pos[rstart[c + 1]] - pos[rstart[c]];
}

void contract_long_rows(Arena &ar, const int32_t *list, int32_t nl, int64_t m, int32_t nc,
                        const int64_t *uxadj, const int64_t *rstart, uint32_t *scu, int32_t *sw,
                        int32_t *rowcnt, hipStream_t s) {
  if (nl <= 0 || m <= 0) return;
  int bits = 1;
  while (bits < 31 && (int64_t(1) << bits) <= (int64_t)nc) ++bits;  // 2^bits - 1 >= nc
  const size_t mk = ar.mark();
  uint64_t *key = ar.alloc_n<uint64_t>(m);
  uint64_t *key2 = ar.alloc_n<uint64_t>(m);
  int32_t *val = ar.alloc_n<int32_t>(m);
  int32_t *val2 = ar.alloc_n<int32_t>(m);
  int32_t *head = ar.alloc_n<int32_t>(m + 1);
  int32_t *pos = ar.alloc_n<int32_t>(m + 1);
  hipLaunchKernelGGL(k_long_keys, dim3((unsigned)((nl + kThreads / 64 - 1) / (kThreads / 64))),
                     dim3(kThreads), 0, s, list, nl, uxadj, rstart, scu, sw, bits, key, val);
  PM_LAUNCH_CHECK();
  sort_pairs(ar, key, key2, val, val2, m, 2 * bits, s);
  hipLaunchKernelGGL(k_long_heads, dim3(grid_for(m + 1)), dim3(kThreads), 0, s, m, key2, bits,
                     head);
  PM_LAUNCH_CHECK();
  scan_excl(ar, head, pos, m + 1, s);
  hipLaunchKernelGGL(k_long_emit, dim3(grid_for(m)), dim3(kThreads), 0, s, m, key2, val2, head,
                     pos, rstart, uxadj, bits, scu, sw);
  PM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_long_count, dim3(grid_for(nl)), dim3(kThreads), 0, s, nl, list, rstart,
                     pos, rowcnt);
  PM_LAUNCH_CHECK();
  ar.rewind(mk);
}

struct CopyArgs {
  Classes rc;
  const int64_t *uxadj;
  const int64_t *cxadj;
  const uint32_t *scu;
  const int32_t *sw;
  int32_t *cadj;
  int32_t *cw;
};

// Four elements per thread are loaded before any is stored (long rows).
__device__ __forceinline__ void copy_row(const CopyArgs &A, int32_t c, int first, int step) {
  const int64_t src = A.uxadj[c], dst = A.cxadj[c];
  const int64_t len = A.cxadj[c + 1] - dst;
  for (int64_t j0 = first; j0 < len; j0 += 4 * (int64_t)step) {
    uint32_t x[4];
    int32_t y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = j0 + r * step;
      const int64_t jj = j < len ? j : len - 1;
      x[r] = A.scu[src + jj];
      y[r] = A.sw[src + jj];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = j0 + r * step;
      if (j < len) {
        A.cadj[dst + j] = (int32_t)x[r];
        A.cw[dst + j] = y[r];
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_contract_copy(CopyArgs A) {
  const int blk = blockIdx.x;
  const int cls = find_class(A.rc, blk);
  const int local = blk - A.rc.wg[cls];
  int32_t c;
  switch (cls) {
    case CLS_ISO: break;
    case CLS_G8:
    case CLS_G16:
    case CLS_G32:
    case CLS_G64: {
      const int G = class_group(cls);
      const int idx = local * (kThreads / G) + (int)threadIdx.x / G;
      if (idx >= A.rc.off[cls + 1] - A.rc.off[cls]) break;
      copy_row(A, A.rc.list[A.rc.off[cls] + idx], threadIdx.x % G, G);
      break;
    }
    case CLS_W:
      if (w_vertex(A.rc, local, c)) copy_row(A, c, threadIdx.x & 63, 64);
      break;
    default:
      copy_row(A, A.rc.list[A.rc.off[CLS_BIG] + local], threadIdx.x, kThreads);
      break;
  }
}

void contract_copy(const Classes &rc, const int64_t *uxadj, const int64_t *cxadj,
                   const uint32_t *scu, const int32_t *sw, int32_t *cadj, int32_t *cw,
                   hipStream_t s) {
  const unsigned nwg = classed_grid(rc);
  if (nwg == 0) return;
  CopyArgs A{rc, uxadj, cxadj, scu, sw, cadj, cw};
  hipLaunchKernelGGL(k_contract_copy, dim3(nwg), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Projection (uncontraction): Pi_fine(v) = Pi_coarse(M(v)).
// ===========================================================================
__global__ void k_project(int32_t n, const int32_t *cmap, const int32_t *coarse,
                          int32_t *fine) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) fine[v] = coarse[cmap[v]];
}
void project(int32_t n, const int32_t *cmap, const int32_t *coarse, int32_t *fine,
             hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_project, dim3(grid_for(n)), dim3(kThreads), 0, s, n, cmap, coarse, fine);
  PM_LAUNCH_CHECK();
}

}  // namespace pm
