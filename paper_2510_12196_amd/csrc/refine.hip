// refine.hip -- objective, balance, label propagation and rebalancing kernels
// for gfx950.
//
// Vertices are processed by degree class (see Classes): a vertex of degree
// <= G is owned by a group of G consecutive lanes of a wave64 holding one arc
// per lane, so a single load instruction of the wave streams the adjacent rows
// of 64/G vertices; vertices of degree > 64 get a whole workgroup that
// aggregates the neighbour-block connectivity in an LDS histogram over block
// codes (the per-vertex connectivity structure of Section 4.2, kept in LDS
// instead of a global hash table).  All arithmetic is integer; sums are
// order-independent, and every choice has a total-order tie-break, so results
// do not depend on thread scheduling or on the order of entries in a row.
#include <hip/hip_ext.h>

#include <cstdlib>

#include "device_util.h"
#include "kernels.h"
#include "prim.h"

namespace pm {

static inline unsigned grid_for(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

// ===========================================================================
// misc fills
// ===========================================================================
template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
template <class T>
static void fill(T *p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(kThreads), 0, s, p, v, n);
  PM_LAUNCH_CHECK();
}
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }

// ===========================================================================
// status read-back: one thread copies the status words into mapped host
// memory, then releases the sequence number the host is polling
// ===========================================================================
__global__ void k_publish(const Status *dev, Pub pub) { publish_dev(dev, pub); }

// Counting launch (PM_FLAG_KERNEL_COUNTS): per tiled vertex one unit, and
// for the active ones their arcs.
__global__ __launch_bounds__(kThreads) void k_count_units(Classes cl, const int64_t *xadj,
                                                          int what, CountArgs a, int64_t *out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int64_t nt = 0, na = 0, ar = 0;
  if (i < cl.off[NCLS]) {
    const int32_t v = cl.list[i];
    nt = 1;
    bool act = false;
    switch (what) {
      case CU_UNLOCKED: act = a.flag8[v] == 0 && (!a.dirty || a.dirty[v]); break;
      case CU_IN_X: act = a.rec[v].g != kNotInX; break;
      case CU_MOVED: act = a.flag8[v] != 0; break;
      case CU_SOURCE: act = a.key[v] >= 0; break;
      default: {  // a vertex that looks for a partner (matching preference)
        const int32_t m = a.match[v], p = a.pref[v];
        act = m < 0 && (p == -2 || (p >= 0 && a.match[p] >= 0));
      }
    }
    if (act) {
      na = 1;
      ar = xadj[v + 1] - xadj[v];
    }
  }
  nt = gsum64<64>(nt);
  na = gsum64<64>(na);
  ar = gsum64<64>(ar);
  if ((threadIdx.x & 63) == 0) {
    const size_t st = (size_t)(blockIdx.x & (kCountStripes - 1)) * kStripeStride;
    const int64_t x[3] = {nt, na, ar};
    for (int j = 0; j < 3; ++j)
      if (x[j]) atomicAdd((unsigned long long *)&out[(size_t)j * kCountStripes * kStripeStride + st],
                          (unsigned long long)x[j]);
  }
}

void count_units(const Classes &cl, const int64_t *xadj, int what, const CountArgs &a,
                 int64_t *out, hipStream_t s) {
  const int64_t m = cl.off[NCLS];
  if (!out || m <= 0) return;
  hipLaunchKernelGGL(k_count_units, dim3((unsigned)((m + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, cl, xadj, what, a, out);
  PM_LAUNCH_CHECK();
}
static_assert(sizeof(Status) % sizeof(int64_t) == 0, "Status is copied in 8-byte words");

void publish_status(const Status *dev, Status *host_dev, int64_t *seq_dev, int64_t seq,
                    hipStream_t s, int64_t *seq_ctr) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, dev,
                     Pub{host_dev, seq_dev, seq, seq_ctr});
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// degree classes
// ===========================================================================
// Also writes the workgroup's count of every class to blockcnt[class * nb +
// workgroup] (class-major: an exclusive scan of it gives each workgroup's
// first slot per class in the concatenated class lists).
__global__ void k_classify(DGraph g, int32_t wmax, uint8_t *cls, int32_t *counts,
                           int32_t *blockcnt, int32_t nb) {
  __shared__ int32_t c[NCLS];
  if (threadIdx.x < NCLS) c[threadIdx.x] = 0;
  __syncthreads();
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < g.n) {
    int64_t d = g.xadj[v + 1] - g.xadj[v];
    int k = d == 0 ? CLS_ISO : d <= 8 ? CLS_G8 : d <= 16 ? CLS_G16 : d <= 32 ? CLS_G32
          : d <= 64 ? CLS_G64 : d <= wmax ? CLS_W : CLS_BIG;
    cls[v] = (uint8_t)k;
    atomicAdd(&c[k], 1);
  }
  __syncthreads();
  if (threadIdx.x < NCLS) {
    blockcnt[threadIdx.x * nb + blockIdx.x] = c[threadIdx.x];
    if (c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], c[threadIdx.x]);
  }
}

// Stable scatter of every vertex id into its class list: the workgroup's
// first slot per class (blockoff) plus the ids of the same class before it
// in the workgroup (counted per wave by ballots).
__global__ __launch_bounds__(kThreads) void k_class_scatter(int32_t n, const uint8_t *cls,
                                                            const int32_t *blockoff, int32_t nb,
                                                            int32_t *list) {
  __shared__ int32_t wc[kThreads / 64][NCLS];
  const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = v < n ? (int)cls[v] : -1;
  uint64_t same = 0;
  for (int k = 0; k < NCLS; ++k) {
    const uint64_t m = __ballot(c == k);
    if (c == k) same = m;
    if (lane == 0) wc[wave][k] = __popcll(m);
  }
  __syncthreads();
  if (c < 0) return;
  int32_t off = blockoff[c * nb + blockIdx.x];
  for (int w = 0; w < wave; ++w) off += wc[w][c];
  off += __popcll(same & ((1ull << lane) - 1ull));
  list[off] = (int32_t)v;
}

Classes build_classes(Arena &ar, const DGraph &g, int32_t *list, Status *st_dev,
                      Status *st_host, hipStream_t s) {
  (void)st_dev;
  (void)st_host;
  Classes cl{};
  cl.list = list;
  size_t m = ar.mark();
  uint8_t *cls = ar.alloc_n<uint8_t>((size_t)g.n + 1);
  int32_t *counts = ar.alloc_n<int32_t>(NCLS);
  const int32_t nb = g.n > 0 ? (int32_t)grid_for(g.n) : 0;
  int32_t *blockcnt = ar.alloc_n<int32_t>((size_t)NCLS * nb + 1);
  int32_t *blockoff = ar.alloc_n<int32_t>((size_t)NCLS * nb + 1);
  int32_t *host = static_cast<int32_t *>(ar.host_stage(sizeof(int32_t) * NCLS));
  // W tiles (a wave per vertex) pay off once they fill the chip; with fewer
  // such vertices a workgroup per vertex finishes sooner, so degrees above 64
  // then all go to BIG (the two paths compute the same results).
  // (the threshold is a launch parameter: pm_set_tuning)
  const int64_t wmin = tuning().wave_min_count;
  for (int32_t wmax : {kWaveMaxDeg, 64}) {
    PM_HIP(hipMemsetAsync(counts, 0, sizeof(int32_t) * NCLS, s));
    if (g.n > 0) {
      hipLaunchKernelGGL(k_classify, dim3(nb), dim3(kThreads), 0, s, g, wmax, cls, counts,
                         blockcnt, nb);
      PM_LAUNCH_CHECK();
    }
    PM_HIP(hipMemcpyAsync(host, counts, sizeof(int32_t) * NCLS, hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (host[CLS_W] == 0 || host[CLS_W] >= wmin) break;
  }
  int32_t cnt[NCLS];
  for (int c = 0; c < NCLS; ++c) cnt[c] = host[c];
  cl.off[0] = 0;
  cl.wg[0] = 0;
  for (int c = 0; c < NCLS; ++c) {
    cl.off[c + 1] = cl.off[c] + cnt[c];
    int per = class_per_wg(c);
    cl.wg[c + 1] = cl.wg[c] + (cnt[c] + per - 1) / per;
  }
  if (nb > 0) {
    scan_excl(ar, blockcnt, blockoff, (int64_t)NCLS * nb, s);
    hipLaunchKernelGGL(k_class_scatter, dim3(nb), dim3(kThreads), 0, s, g.n, cls, blockoff, nb,
                       list);
    PM_LAUNCH_CHECK();
  }
  ar.rewind(m);
  return cl;
}

int32_t classes_workgroups(const Classes &cl) { return cl.wg[NCLS]; }

Classes tiled(const Classes &cl, int V, bool w_as_big) {
  Classes t = cl;
  t.wg[0] = 0;
  for (int c = 0; c < NCLS; ++c) {
    const int cnt = cl.off[c + 1] - cl.off[c];
    const int per = c == CLS_W && w_as_big ? 1 : class_per_wg(c) * (c == CLS_BIG || c == CLS_W ? 1 : V);
    t.wg[c + 1] = t.wg[c] + (cnt + per - 1) / per;
  }
  return t;
}

int group_v() { return tuning().group_v; }

// ===========================================================================
// id <-> code conversion
// ===========================================================================
__global__ void k_ids_to_codes(Hier h, const int32_t *ids, int32_t *codes, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) codes[i] = (int32_t)id_to_code(h, ids[i]);
}
__global__ void k_codes_to_ids(Hier h, const int32_t *codes, int32_t *ids, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ids[i] = code_to_id(h, (uint32_t)codes[i]);
}
__global__ void k_check_ids(int64_t k, const int32_t *ids, int32_t n, int64_t *stripes) {
  __shared__ BlockScratch sc;
  int64_t bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad += (ids[i] < 0 || (int64_t)ids[i] >= k) ? 1 : 0;
  bad = block_sum64(bad, sc);
  if (threadIdx.x == 0) stripe_add(stripes, bad);
}

void ids_to_codes(const Hier &h, const int32_t *ids, int32_t *codes, int32_t n, hipStream_t s) {
  if (n <= 0) return;
  if (h.pow2) {
    if (ids != codes)
      PM_HIP(hipMemcpyAsync(codes, ids, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    return;
  }
  hipLaunchKernelGGL(k_ids_to_codes, dim3(grid_for(n)), dim3(kThreads), 0, s, h, ids, codes, n);
  PM_LAUNCH_CHECK();
}
void codes_to_ids(const Hier &h, const int32_t *codes, int32_t *ids, int32_t n, hipStream_t s) {
  if (n <= 0) return;
  if (h.pow2) {
    if (ids != codes)
      PM_HIP(hipMemcpyAsync(ids, codes, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    return;
  }
  hipLaunchKernelGGL(k_codes_to_ids, dim3(grid_for(n)), dim3(kThreads), 0, s, h, codes, ids, n);
  PM_LAUNCH_CHECK();
}
void check_ids(const Hier &h, const int32_t *ids, int32_t n, int64_t *stripes, Status *st,
               hipStream_t s) {
  unsigned g = grid_for(n);
  if (g > kMaxGrid) g = kMaxGrid;
  if (n > 0) {
    hipLaunchKernelGGL(k_check_ids, dim3(g), dim3(kThreads), 0, s, h.k, ids, n, stripes);
    PM_LAUNCH_CHECK();
  }
  fold_stripes(stripes, nullptr, &st->count, s);
}

// ===========================================================================
// striped accumulators
// ===========================================================================
// One workgroup; used standalone (k_fold) and as the last workgroup of a
// producer kernel.
__device__ __forceinline__ void fold_block(int64_t *stripes, int64_t *out64, int32_t *out32,
                                           const Pub &pub, const Status *st) {
  __shared__ BlockScratch sc;
  int64_t x = agent_load(&stripes[threadIdx.x * kStripeStride]);
  stripes[threadIdx.x * kStripeStride] = 0;
  x = block_sum64(x, sc);
  if (threadIdx.x == 0) {
    if (out64) *out64 = x;
    else *out32 = (int32_t)x;
    __threadfence();
    if (st) publish_dev(st, pub);
  }
}
static_assert(kStripes == kThreads, "one stripe per thread in the folds");

__global__ __launch_bounds__(kThreads) void k_fold(int64_t *stripes, int64_t *out64,
                                                   int32_t *out32, Pub pub, const Status *st) {
  fold_block(stripes, out64, out32, pub, st);
}

void fold_stripes(int64_t *stripes, int64_t *out64, int32_t *out32, hipStream_t s,
                  const Pub &pub, const Status *st) {
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(kThreads), 0, s, stripes, out64, out32, pub, st);
  PM_LAUNCH_CHECK();
}
int stripe_words() { return kStripeWords; }
// One class tile per workgroup: the hardware dispatcher balances the
// tiles across the chip better than a fixed grid-stride assignment (the
// kernels still loop, so a capped grid stays correct).
unsigned classed_grid(const Classes &cl) { return (unsigned)cl.wg[NCLS]; }
unsigned capped_grid(const Classes &cl) {
  const int t = cl.wg[NCLS];
  return (unsigned)(t < kMaxGrid ? t : kMaxGrid);
}

// ===========================================================================
// J (Section 2): sum over arcs of w * D(Pi(u), Pi(v))
// ===========================================================================
struct CostArgs {
  DGraph g;
  Classes cl;
  Hier h;
  const int32_t *part;
  int64_t *stripes;
};

template <int G>
__device__ __forceinline__ int64_t cost_group(const CostArgs &A, int cls, int local) {
  int32_t v;
  if (!group_vertex<G>(A.cl, cls, local, v)) return 0;
  const int lane = threadIdx.x % G;
  const int64_t e = A.g.xadj[v] + lane;
  if (e >= A.g.xadj[v + 1]) return 0;
  return (int64_t)A.g.w[e] * dist(A.h, (uint32_t)A.part[v], (uint32_t)A.part[A.g.adj[e]]);
}

__global__ __launch_bounds__(kThreads) void k_comm_cost(CostArgs A) {
  __shared__ BlockScratch sc;
  int64_t x = 0;
  {  // one class tile per workgroup
    const int blk = blockIdx.x;
    const int cls = find_class(A.cl, blk);
    const int local = blk - A.cl.wg[cls];
    switch (cls) {
      case CLS_G8: x += cost_group<8>(A, cls, local); break;
      case CLS_G16: x += cost_group<16>(A, cls, local); break;
      case CLS_G32: x += cost_group<32>(A, cls, local); break;
      case CLS_G64: x += cost_group<64>(A, cls, local); break;
      case CLS_W: {
        int32_t v;
        if (!w_vertex(A.cl, local, v)) break;
        const uint32_t p = (uint32_t)A.part[v];
        wave_arcs<4>(
            A.g.xadj[v], A.g.xadj[v + 1],
            [&](int64_t e) { return make_uint2((uint32_t)A.part[A.g.adj[e]], (uint32_t)A.g.w[e]); },
            [&](int64_t, uint2 a) { x += (int64_t)a.y * dist(A.h, p, a.x); });
        break;
      }
      case CLS_BIG: {
        const int32_t v = A.cl.list[A.cl.off[CLS_BIG] + local];
        const uint32_t p = (uint32_t)A.part[v];
        big_arcs(
            A.g.xadj[v], A.g.xadj[v + 1],
            [&](int64_t e) { return make_uint2((uint32_t)A.part[A.g.adj[e]], (uint32_t)A.g.w[e]); },
            [&](int64_t, uint2 a) { x += (int64_t)a.y * dist(A.h, p, a.x); });
        break;
      }
      default: break;
    }
  }
  x = block_sum64(x, sc);
  if (threadIdx.x == 0) stripe_add(A.stripes, x);
}

void comm_cost(const DGraph &g, const Classes &cl, const Hier &h, const int32_t *part,
               int64_t *stripes, Status *st, hipStream_t s) {
  const unsigned grid = classed_grid(cl);
  if (grid > 0) {
    CostArgs A{g, cl, h, part, stripes};
    hipLaunchKernelGGL(k_comm_cost, dim3(grid), dim3(kThreads), 0, s, A);
    PM_LAUNCH_CHECK();
  }
  fold_stripes(stripes, &st->j, nullptr, s);
}

// ===========================================================================
// block weights and the heaviest block
// ===========================================================================
__global__ __launch_bounds__(kThreads) void k_block_weights(const int32_t *part,
                                                            const int32_t *vwgt, int32_t n,
                                                            int32_t ncodes, int64_t *w) {
  extern __shared__ uint32_t hist[];
  for (int c = threadIdx.x; c < ncodes; c += kThreads) hist[c] = 0;
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kThreads)
    atomicAdd(&hist[part[v]], (uint32_t)vwgt[v]);
  __syncthreads();
  for (int c = threadIdx.x; c < ncodes; c += kThreads)
    if (hist[c]) atomicAdd((unsigned long long *)&w[c], (unsigned long long)hist[c]);
}

void block_weights(const DGraph &g, const Hier &h, const int32_t *part, int64_t *w,
                   hipStream_t s) {
  const int32_t ncodes = 1 << h.bits;
  PM_HIP(hipMemsetAsync(w, 0, sizeof(int64_t) * ncodes, s));
  if (g.n <= 0) return;
  unsigned grid = grid_for(g.n, kThreads * 16);
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_block_weights, dim3(grid), dim3(kThreads), sizeof(uint32_t) * ncodes, s,
                     part, g.c, g.n, ncodes, w);
  PM_LAUNCH_CHECK();
}

template <int NS>
__device__ __forceinline__ int64_t stripe_sum(const int64_t *wst, int32_t ncodes, int c) {
  int64_t x[NS];
#pragma unroll
  for (int st = 0; st < NS; ++st) x[st] = wst[(size_t)st * ncodes + c];
  int64_t d = 0;
#pragma unroll
  for (int st = 0; st < NS; ++st) d += x[st];
  return d;
}

// The StepEnd epilogue, by one workgroup: one round of loads (the block
// weights and their pending stripes, the J-change stripes, the status words),
// reductions and scans in LDS only (wl: ncodes words), then every global
// store at the end, so that no barrier waits for a store.  wst:
// weight-delta stripes to fold into w first (nullptr: none).  full = false:
// only the fold.  (The host publication is a launch of its own: a
// system-scope fence here would write back the L2 this launch has dirtied.)
__device__ __forceinline__ void step_epilogue(const StepEnd &E, int64_t *wst, int nstripes,
                                              int64_t *wl, bool full) {
  __shared__ int64_t red_m[kThreads / 64], red_d[kThreads / 64];
  __shared__ uint32_t red_u[kThreads / 64];
  const int32_t ncodes = 1 << E.h.bits;
  const int per = (ncodes + kThreads - 1) / kThreads;
  const int lo = threadIdx.x * per;
  const int hi = lo + per < ncodes ? lo + per : ncodes;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // ---- loads
  Status S{};
  if (full && threadIdx.x == 0) S = *E.st;
  int64_t dj = (full && E.dj_stripes) ? E.dj_stripes[threadIdx.x * kStripeStride] : 0;
  uint32_t changed = 0;  // bit c - lo: weight changed
  int64_t m = INT64_MIN;
  for (int c = lo; c < hi; ++c) {
    int64_t a = E.w[c];
    if (wst) {
      int64_t d;
      switch (nstripes) {  // unrolled per count: all stripe loads in flight together
        case 32: d = stripe_sum<32>(wst, ncodes, c); break;
        case 16: d = stripe_sum<16>(wst, ncodes, c); break;
        case 8: d = stripe_sum<8>(wst, ncodes, c); break;
        case 4: d = stripe_sum<4>(wst, ncodes, c); break;
        case 2: d = stripe_sum<2>(wst, ncodes, c); break;
        default: d = stripe_sum<1>(wst, ncodes, c); break;
      }
      if (d) changed |= 1u << (c - lo);
      a += d;
    }
    wl[c] = a;
    m = a > m ? a : m;
  }
  if (full) {
    // ---- LDS only: heaviest block, J change, eligible counts (two packed
    // 16-bit counts; each list has at most 2^13 entries)
    uint32_t cnt = 0;
    for (int c = lo; c < hi; ++c) {
      if (!code_valid(E.h, (uint32_t)c)) continue;
      if (wl[c] <= E.sigma) cnt += 1u;
      if (wl[c] <= E.lmax) cnt += 1u << 16;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const int64_t om = gxor64<64>(m, o);
      m = om > m ? om : m;
    }
    dj = gsum64<64>(dj);
    uint32_t incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int32_t)incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) red_u[wave] = incl;
    if (lane == 0) {
      red_m[wave] = m;
      red_d[wave] = dj;
    }
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int i = 0; i < kThreads / 64; ++i) {
      if (i < wave) off += red_u[i];
      tot += red_u[i];
      m = red_m[i] > m ? red_m[i] : m;
    }
    dj = 0;
    for (int i = 0; i < kThreads / 64; ++i) dj += red_d[i];
    uint32_t pos = off + incl - cnt;
    // ---- stores
    uint32_t pw = pos & 0xFFFFu, ps = pos >> 16;
    for (int c = lo; c < hi; ++c) {
      if (!code_valid(E.h, (uint32_t)c)) continue;
      if (wl[c] <= E.sigma) E.elig_weak[pw++] = c;
      if (wl[c] <= E.lmax) E.elig_strong[ps++] = c;
    }
    if (E.dj_stripes) E.dj_stripes[threadIdx.x * kStripeStride] = 0;
    if (threadIdx.x == 0) {
      S.maxw = m;
      if (E.dj_stripes) S.dj = dj;
      S.n_elig_weak = (int32_t)(tot & 0xFFFFu);
      S.n_elig_strong = (int32_t)(tot >> 16);
      E.st->maxw = S.maxw;
      E.st->dj = S.dj;
      E.st->n_elig_weak = S.n_elig_weak;
      E.st->n_elig_strong = S.n_elig_strong;
      // the step's publication, without a launch of its own
      if (E.pub.host) publish_dev(E.st, E.pub);
    }
  }
  if (wst) {
    for (int c = lo; c < hi; ++c) {
      if (!(changed & (1u << (c - lo)))) continue;
      E.w[c] = wl[c];
#pragma unroll
      for (int st = 0; st < kWeightStripes; ++st)
        if (st < nstripes) wst[(size_t)st * ncodes + c] = 0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_step_status(StepEnd E) {
  extern __shared__ int64_t wl[];
  step_epilogue(E, nullptr, 0, wl, true);
}

void step_status(const StepEnd &E, hipStream_t s) {
  hipLaunchKernelGGL(k_step_status, dim3(1), dim3(kThreads), sizeof(int64_t) << E.h.bits, s, E);
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Label propagation, phase 1 (Algorithm 4, first filter)
//
// For vertex v in block p with neighbour-block connectivity conn(v,x):
//   cost(b) = sum_x conn(v,x) D(b,x),  G_b(v) = cost(p) - cost(b)   (eq. 1)
// The best candidate b != p among the neighbour blocks maximises G, ties to
// the smaller block.  v enters X iff that gain is >= 0.
// ===========================================================================
struct LP1Args {
  DGraph g;
  Classes cl;
  Hier h;
  const int32_t *part;
  const uint8_t *lock;
  LpRec *rec;       // per vertex {block, target, gain}
  int64_t jet_num;  // > 0: relaxed filter -G < floor(jet_num * conn(v,own) / jet_den)
  int64_t jet_den;
  int32_t whist;    // G64 vertices use a per-wave LDS histogram (LDS: 4 slices)
  uint8_t *dirty;   // result caching (nullptr: off): see lp1_state
};

// Result caching.  The first filter's result for an unlocked vertex depends
// only on its block and its neighbours' blocks; dirty[v] is set when v or a
// neighbour moves (by the move accounting) and cleared when v is evaluated
// here, so an unlocked vertex that is not dirty keeps the target and gain of
// its last evaluation (they stay in rec[], which only this kernel writes).  State of v: 0 locked (trivial result), 1 cached (nothing to
// write), 2 evaluated.
__device__ __forceinline__ int lp1_state(const LP1Args &A, int32_t v) {
  if (A.lock[v]) return 0;
  if (A.dirty && !A.dirty[v]) return 1;
  return 2;
}
__device__ __forceinline__ void lp1_evaluated(const LP1Args &A, int32_t v) {
  if (A.dirty) A.dirty[v] = 0;
}
// The result of v: one 16-byte record (block, target, gain); gain kNotInX
// (and target = block) for a vertex outside X.
__device__ __forceinline__ void lp1_put(const LP1Args &A, int32_t v, uint32_t p, uint32_t t,
                                        int64_t g) {
  A.rec[v] = LpRec{(int32_t)p, (int32_t)t, g};
}

// First filter: G >= 0, or with Jet's relaxed filter -G < floor(c conn_own).
__device__ __forceinline__ bool lp1_pass(const LP1Args &A, int64_t g, int64_t conn_own) {
  return g >= 0 || (A.jet_num > 0 && -g < (A.jet_num * conn_own) / A.jet_den);
}

struct Lp1V {
  uint32_t p;
  int state;
};
struct Lp1N {
  uint32_t bu;
  int32_t wu;
};

template <int G, int V>
__device__ __forceinline__ void lp1_group(const LP1Args &A, int cls, int local) {
  group_tiles<G, V>(
      A.g.xadj, A.g.adj, A.cl, cls, local,
      [&](int32_t v, bool &act) {
        const int st = lp1_state(A, v);
        act = st == 2;
        return Lp1V{(uint32_t)A.part[v], st};
      },
      [&](int32_t u, int64_t e) { return Lp1N{(uint32_t)A.part[u], A.g.w[e]}; },
      [&](int, bool ok, int32_t v, const Lp1V &vv, bool act, int deg, bool valid,
          const Lp1N &nv) {
        if (!ok || vv.state == 1) return;
        const int lane = threadIdx.x % G;
        const uint32_t p = vv.p;
        const uint32_t bu = valid ? nv.bu : p;
        const int32_t wu = valid ? nv.wu : 0;
        const bool cand = valid && bu != p;
        if (act && lane == 0) lp1_evaluated(A, v);
        if (!act || !gor<G>(cand ? 1 : 0)) {
          if (lane == 0) {
            lp1_put(A, v, p, p, kNotInX);
          }
          return;
        }
        const int64_t costp = gsum64<G>((int64_t)wu * dist(A.h, p, bu));
        int64_t cost = 0;
        for (int j = 0; j < deg; ++j) {
          const uint32_t bj = (uint32_t)gshfl<G>((int32_t)bu, j);
          const int32_t wj = gshfl<G>(wu, j);
          cost += (int64_t)wj * dist(A.h, bu, bj);
        }
        int64_t g = cand ? costp - cost : INT64_MIN;
        uint32_t b = cand ? bu : 0xFFFFFFFFu;
        gargmax<G>(g, b);
        const int64_t conn_own = A.jet_num > 0 ? gsum64<G>(valid && bu == p ? wu : 0) : 0;
        if (lane == 0) {
          if (lp1_pass(A, g, conn_own)) {
            lp1_put(A, v, p, b, g);
          } else {
            lp1_put(A, v, p, p, kNotInX);
          }
        }
      });
}

// cost(c) from the exclusive prefix X over the connectivity histogram:
// conn(c) = X[c+1] - X[c], S_i(c) = sum of conn over c's level-i group.
__device__ __forceinline__ int64_t level_cost(const Hier &h, const uint32_t *X, uint32_t c,
                                              int32_t ncodes) {
  int64_t prev = (int64_t)(X[c + 1] - X[c]);
  int64_t cost = 0;
  for (int i = 1; i <= h.levels; ++i) {
    const int sh = h.shift[i];
    const uint32_t lo = (c >> sh) << sh;
    uint32_t hi = lo + (1u << sh);
    if (hi > (uint32_t)ncodes) hi = (uint32_t)ncodes;
    const int64_t S = (int64_t)(X[hi] - X[lo]);
    cost += (int64_t)h.d[i - 1] * (S - prev);
    prev = S;
  }
  return cost;
}

// Builds X[0..ncodes] = exclusive prefix of conn(v, .) in LDS.
__device__ __forceinline__ void big_histogram(const DGraph &g, const int32_t *part, int32_t v,
                                              uint32_t *X, int32_t ncodes, BlockScratch &sc) {
  __syncthreads();  // every wave is done reading the previous vertex's histogram
  for (int c = threadIdx.x; c <= ncodes; c += kThreads) X[c] = 0;
  __syncthreads();
  big_arcs(
      g.xadj[v], g.xadj[v + 1],
      [&](int64_t e) { return make_uint2((uint32_t)part[g.adj[e]], (uint32_t)g.w[e]); },
      [&](int64_t, uint2 a) { atomicAdd(&X[a.x + 1], a.y); });
  __syncthreads();
  block_scan_lds(X, ncodes + 1, sc);
}

__device__ __forceinline__ void lp1_big(const LP1Args &A, int32_t v, uint32_t *X,
                                        BlockScratch &sc) {
  const uint32_t p = (uint32_t)A.part[v];
  const int st = lp1_state(A, v);
  if (st == 1) return;
  if (st == 0) {
    if (threadIdx.x == 0) {
      lp1_put(A, v, p, p, kNotInX);
    }
    return;
  }
  const int32_t ncodes = 1 << A.h.bits;
  big_histogram(A.g, A.part, v, X, ncodes, sc);
  // (cleared only now: every wave of the workgroup has read the flag before
  // the histogram's barriers)
  if (threadIdx.x == 0) lp1_evaluated(A, v);
  const uint32_t total = X[ncodes];
  const uint32_t connp = X[p + 1] - X[p];
  if (total == connp) {
    if (threadIdx.x == 0) {
      lp1_put(A, v, p, p, kNotInX);
    }
    return;
  }
  const int64_t costp = level_cost(A.h, X, p, ncodes);
  int64_t g = INT64_MIN;
  uint32_t b = 0xFFFFFFFFu;
  for (int c = threadIdx.x; c < ncodes; c += kThreads) {
    if ((uint32_t)c == p || X[c + 1] == X[c]) continue;
    const int64_t gc = costp - level_cost(A.h, X, (uint32_t)c, ncodes);
    if (gc > g || (gc == g && (uint32_t)c < b)) {
      g = gc;
      b = (uint32_t)c;
    }
  }
  block_argmax(g, b, sc);
  if (threadIdx.x == 0) {
    if (lp1_pass(A, g, (int64_t)connp)) {
      lp1_put(A, v, p, b, g);
    } else {
      lp1_put(A, v, p, p, kNotInX);
    }
  }
}

// Degree 33..64, one vertex per wave: instead of pairing every arc with
// every other one (deg^2 shuffles), the wave adds its arcs into a
// connectivity histogram in its own LDS slice, scans it, and reads the cost
// of each candidate from the level group sums (level_cost).
template <int V>
__device__ __forceinline__ void lp1_wave(const LP1Args &A, int local, uint32_t *X) {
  const int32_t ncodes = 1 << A.h.bits;
  uint32_t *Xw = X + (threadIdx.x >> 6) * (ncodes + 1);
  group_tiles<64, V>(
      A.g.xadj, A.g.adj, A.cl, CLS_G64, local,
      [&](int32_t v, bool &act) {
        const int st = lp1_state(A, v);
        act = st == 2;
        return Lp1V{(uint32_t)A.part[v], st};
      },
      [&](int32_t u, int64_t e) { return Lp1N{(uint32_t)A.part[u], A.g.w[e]}; },
      [&](int, bool ok, int32_t v, const Lp1V &vv, bool act, int, bool valid, const Lp1N &nv) {
        if (!ok || vv.state == 1) return;
        const int lane = threadIdx.x & 63;
        const uint32_t p = vv.p;
        const uint32_t bu = valid ? nv.bu : p;
        const bool cand = valid && bu != p;
        if (act && lane == 0) lp1_evaluated(A, v);
        if (!act || !gor<64>(cand ? 1 : 0)) {
          if (lane == 0) {
            lp1_put(A, v, p, p, kNotInX);
          }
          return;
        }
        for (int c = lane; c <= ncodes; c += 64) Xw[c] = 0;
        wave_lds_sync();
        if (valid) atomicAdd(&Xw[bu + 1], (uint32_t)nv.wu);
        wave_lds_sync();
        wave_scan_lds(Xw, ncodes + 1);
        wave_lds_sync();
        const int64_t costp = level_cost(A.h, Xw, p, ncodes);
        int64_t g = cand ? costp - level_cost(A.h, Xw, bu, ncodes) : INT64_MIN;
        uint32_t b = cand ? bu : 0xFFFFFFFFu;
        gargmax<64>(g, b);
        if (lane == 0) {
          if (lp1_pass(A, g, (int64_t)(Xw[p + 1] - Xw[p]))) {
            lp1_put(A, v, p, b, g);
          } else {
            lp1_put(A, v, p, p, kNotInX);
          }
        }
        wave_lds_sync();  // the slice is cleared again for the next vertex
      });
}

// Degree 65..kWaveMaxDeg, one vertex per wave: the block path's histogram
// in the wave's own LDS slice, without workgroup barriers.
__device__ __forceinline__ void lp1_w(const LP1Args &A, int local, uint32_t *X) {
  int32_t v;
  if (!w_vertex(A.cl, local, v)) return;
  const int lane = threadIdx.x & 63;
  const uint32_t p = (uint32_t)A.part[v];
  const int st = lp1_state(A, v);
  if (st == 1) return;
  if (st == 0) {
    if (lane == 0) {
      lp1_put(A, v, p, p, kNotInX);
    }
    return;
  }
  if (lane == 0) lp1_evaluated(A, v);
  const int32_t ncodes = 1 << A.h.bits;
  uint32_t *Xw = X + (threadIdx.x >> 6) * (ncodes + 1);
  for (int c = lane; c <= ncodes; c += 64) Xw[c] = 0;
  wave_lds_sync();
  wave_arcs<4>(
      A.g.xadj[v], A.g.xadj[v + 1],
      [&](int64_t e) { return make_uint2((uint32_t)A.part[A.g.adj[e]], (uint32_t)A.g.w[e]); },
      [&](int64_t, uint2 a) { atomicAdd(&Xw[a.x + 1], a.y); });
  wave_lds_sync();
  wave_scan_lds(Xw, ncodes + 1);
  wave_lds_sync();
  const uint32_t connp = Xw[p + 1] - Xw[p];
  if (Xw[ncodes] == connp) {
    if (lane == 0) {
      lp1_put(A, v, p, p, kNotInX);
    }
    return;
  }
  const int64_t costp = level_cost(A.h, Xw, p, ncodes);
  int64_t g = INT64_MIN;
  uint32_t b = 0xFFFFFFFFu;
  for (int c = lane; c < ncodes; c += 64) {
    if ((uint32_t)c == p || Xw[c + 1] == Xw[c]) continue;
    const int64_t gc = costp - level_cost(A.h, Xw, (uint32_t)c, ncodes);
    if (gc > g || (gc == g && (uint32_t)c < b)) {
      g = gc;
      b = (uint32_t)c;
    }
  }
  gargmax<64>(g, b);
  if (lane == 0) {
    if (lp1_pass(A, g, (int64_t)connp)) {
      lp1_put(A, v, p, b, g);
    } else {
      lp1_put(A, v, p, p, kNotInX);
    }
  }
}

template <int V>
__global__ __launch_bounds__(kThreads) void k_lp_phase1(LP1Args A) {
  extern __shared__ uint32_t X[];
  __shared__ BlockScratch sc;
  {  // one class tile per workgroup
    const int blk = blockIdx.x;
    const int cls = find_class(A.cl, blk);
    const int local = blk - A.cl.wg[cls];
    switch (cls) {
      case CLS_ISO:
        iso_tiles<V>(A.cl, local, [&](int32_t v) {
          const uint32_t p = (uint32_t)A.part[v];
          lp1_put(A, v, p, p, kNotInX);
        });
        break;
      case CLS_G8: lp1_group<8, V>(A, cls, local); break;
      case CLS_G16: lp1_group<16, V>(A, cls, local); break;
      case CLS_G32: lp1_group<32, V>(A, cls, local); break;
      case CLS_G64:
        if (A.whist) lp1_wave<V>(A, local, X);
        else lp1_group<64, V>(A, cls, local);
        break;
      default:
        // BIG, and W without the per-wave histogram (then tiled one vertex
        // per workgroup, like BIG)
        if (cls == CLS_W && A.whist) lp1_w(A, local, X);
        else lp1_big(A, A.cl.list[A.cl.off[cls] + local], X, sc);
        break;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_unpack_lp(const LpRec *rec, int32_t *target,
                                                        int64_t *gain, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  const LpRec r = rec[v];
  target[v] = r.t;
  gain[v] = r.g;
}

void unpack_lp(const LpRec *rec, int32_t *target, int64_t *gain, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_unpack_lp, dim3(grid_for(n)), dim3(kThreads), 0, s, rec, target, gain, n);
  PM_LAUNCH_CHECK();
}

static size_t big_lds(const Hier &h) { return sizeof(uint32_t) * ((size_t(1) << h.bits) + 1); }

void lp_phase1(const DGraph &g, const Classes &cl, const Hier &h, const int32_t *part,
               const uint8_t *lock, LpRec *rec, hipStream_t s, const Variants &var,
               uint8_t *dirty) {
  const int V = group_v();
  // four per-wave histogram slices fit in 32 KiB up to 2^10 codes
  const int whist = h.bits <= 10;
  const Classes tc = tiled(cl, V, !whist);
  const unsigned nwg = classed_grid(tc);
  if (nwg == 0) return;
  LP1Args A{g, tc, h, part, lock, rec, var.jet_num, var.jet_den > 0 ? var.jet_den : 1, whist,
            dirty};
  const size_t lds = whist ? 4 * big_lds(h) : big_lds(h);
  auto kern = V == 2 ? k_lp_phase1<2> : k_lp_phase1<1>;
  if (tl_timer) count_units(cl, g.xadj, CU_UNLOCKED, CountArgs{lock, dirty, nullptr, nullptr,
                                                               nullptr, nullptr},
                            tl_timer->counters(KT_LP1), s);
  hipEvent_t a = nullptr, b = nullptr;
  if (tl_timer) tl_timer->pair(KT_LP1, a, b);
  if (a) {
    hipExtLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), lds, s, a, b, 0, A);
  } else {
    hipLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), lds, s, A);
  }
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Label propagation, phase 2 (Algorithm 4, second filter)
//
// For v in X the gain of its move is re-evaluated with every neighbour u in X
// that precedes v (g(u) > g(v), or equal gain and u < v) counted at u's
// target and every other neighbour at its current block; v moves iff >= 0.
// ===========================================================================
struct LP2Args {
  DGraph g;
  Classes cl;
  Hier h;
  const LpRec *rec;  // phase 1's {block, target, gain} per vertex
  uint8_t *moved;
  int2 *pn;          // out: {block, moved ? target : -1} per vertex (k_apply's records)
};

struct Lp2Arc {
  int32_t u, w, pu, tu;
  int64_t gu;
};

struct Lp2V {
  int64_t gv;
  uint32_t p, t;
};

// one 16-byte gather per arc: the neighbour's block, target and gain
__device__ __forceinline__ Lp2Arc lp2_arc(const LP2Args &A, int32_t u, int64_t e) {
  const LpRec r = A.rec[u];
  return Lp2Arc{u, A.g.w[e], r.p, r.t, r.g};
}
// v's outcome: moved flag and k_apply's record
__device__ __forceinline__ void lp2_put(const LP2Args &A, int32_t v, uint32_t p, uint32_t t,
                                        bool m) {
  A.moved[v] = m ? 1 : 0;
  A.pn[v] = make_int2((int32_t)p, m ? (int32_t)t : -1);
}

template <int G, int V>
__device__ __forceinline__ void lp2_group(const LP2Args &A, int cls, int local) {
  group_tiles<G, V>(
      A.g.xadj, A.g.adj, A.cl, cls, local,
      [&](int32_t v, bool &act) {
        const LpRec r = A.rec[v];
        act = r.g != kNotInX;
        return Lp2V{r.g, (uint32_t)r.p, (uint32_t)r.t};
      },
      [&](int32_t u, int64_t e) { return lp2_arc(A, u, e); },
      [&](int, bool ok, int32_t v, const Lp2V &vv, bool act, int, bool valid, const Lp2Arc &a) {
        if (!ok) return;
        const int lane = threadIdx.x % G;
        if (!act) {
          if (lane == 0) lp2_put(A, v, vv.p, vv.t, false);
          return;
        }
        int64_t x = 0;
        if (valid) {
          uint32_t pu = (uint32_t)a.pu;
          if (a.gu != kNotInX && (a.gu > vv.gv || (a.gu == vv.gv && a.u < v))) pu = (uint32_t)a.tu;
          x = (int64_t)a.w * (dist(A.h, vv.p, pu) - dist(A.h, vv.t, pu));
        }
        x = gsum64<G>(x);
        if (lane == 0) lp2_put(A, v, vv.p, vv.t, x >= 0);
      });
}

template <int V>
__global__ __launch_bounds__(kThreads) void k_lp_phase2(LP2Args A) {
  __shared__ BlockScratch sc;
  {  // one class tile per workgroup
    const int blk = blockIdx.x;
    const int cls = find_class(A.cl, blk);
    const int local = blk - A.cl.wg[cls];
    switch (cls) {
      case CLS_ISO:
        // (an isolated vertex is nobody's neighbour and never moves: its
        // record is never read)
        iso_tiles<V>(A.cl, local, [&](int32_t v) { A.moved[v] = 0; });
        break;
      case CLS_G8: lp2_group<8, V>(A, cls, local); break;
      case CLS_G16: lp2_group<16, V>(A, cls, local); break;
      case CLS_G32: lp2_group<32, V>(A, cls, local); break;
      case CLS_G64: lp2_group<64, V>(A, cls, local); break;
      case CLS_W: {
        int32_t v;
        if (!w_vertex(A.cl, local, v)) break;
        const LpRec r = A.rec[v];
        const int64_t gv = r.g;
        const uint32_t p = (uint32_t)r.p, t = (uint32_t)r.t;
        if (gv == kNotInX) {
          if ((threadIdx.x & 63) == 0) lp2_put(A, v, p, t, false);
          break;
        }
        int64_t x = 0;
        wave_arcs<2>(
            A.g.xadj[v], A.g.xadj[v + 1], [&](int64_t e) { return lp2_arc(A, A.g.adj[e], e); },
            [&](int64_t, const Lp2Arc &a) {
              uint32_t pu = (uint32_t)a.pu;
              if (a.gu != kNotInX && (a.gu > gv || (a.gu == gv && a.u < v))) pu = (uint32_t)a.tu;
              x += (int64_t)a.w * (dist(A.h, p, pu) - dist(A.h, t, pu));
            });
        x = gsum64<64>(x);
        if ((threadIdx.x & 63) == 0) lp2_put(A, v, p, t, x >= 0);
        break;
      }
      default: {
        const int32_t v = A.cl.list[A.cl.off[CLS_BIG] + local];
        const LpRec r = A.rec[v];
        const int64_t gv = r.g;
        const uint32_t p = (uint32_t)r.p, t = (uint32_t)r.t;
        if (gv == kNotInX) {
          if (threadIdx.x == 0) lp2_put(A, v, p, t, false);
          break;
        }
        int64_t x = 0;
        big_arcs(
            A.g.xadj[v], A.g.xadj[v + 1], [&](int64_t e) { return lp2_arc(A, A.g.adj[e], e); },
            [&](int64_t, const Lp2Arc &a) {
              uint32_t pu = (uint32_t)a.pu;
              if (a.gu != kNotInX && (a.gu > gv || (a.gu == gv && a.u < v))) pu = (uint32_t)a.tu;
              x += (int64_t)a.w * (dist(A.h, p, pu) - dist(A.h, t, pu));
            });
        x = block_sum64(x, sc);
        if (threadIdx.x == 0) lp2_put(A, v, p, t, x >= 0);
        break;
      }
    }
  }
}

void lp_phase2(const DGraph &g, const Classes &cl, const Hier &h, const LpRec *rec,
               uint8_t *moved, int2 *pn, hipStream_t s) {
  const int V = group_v();
  const Classes tc = tiled(cl, V);
  const unsigned nwg = classed_grid(tc);
  if (nwg == 0) return;
  LP2Args A{g, tc, h, rec, moved, pn};
  auto kern = V == 2 ? k_lp_phase2<2> : k_lp_phase2<1>;
  if (tl_timer) count_units(cl, g.xadj, CU_IN_X, CountArgs{nullptr, nullptr, rec, nullptr,
                                                           nullptr, nullptr},
                            tl_timer->counters(KT_LP2), s);
  hipEvent_t a = nullptr, b = nullptr;
  if (tl_timer) tl_timer->pair(KT_LP2, a, b);
  if (a) {
    hipExtLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, a, b, 0, A);
  } else {
    hipLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, A);
  }
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Applying a set of moves.
//
// apply_moves first accounts for the moves -- exact change of J and of the
// block weights -- reading the old mapping only, then commits
// part[v] <- target[v] in a second launch.  In the accounting, an arc with
// exactly one moved endpoint is seen once, from the moved side, and stands
// for both of its directions (weight 2); an arc with both endpoints moved is
// seen from each side (weight 1 each).
// ===========================================================================
struct ApplyArgs {
  DGraph g;
  Classes cl;
  Hier h;
  const uint8_t *moved;
  uint8_t *lock;
  int64_t *wst;  // weight-delta stripes [nstripes][ncodes]
  int32_t nstripes;
  int64_t *dj;
  uint8_t *dirty;  // label-propagation result caching (nullptr: off)
  const int2 *pn;  // per vertex {block, moved ? target : -1}
  int32_t *part;   // written for the movers only (read by no tile of this launch)
};

// Block-weight deltas of one mover (+c to its target, -c to its block): added
// into the weight-delta stripe of the workgroup, one atomic per distinct
// block per wave.
struct WMove {
  bool has = false;
  uint32_t p = 0, t = 0;
  int32_t c = 0;
};
__device__ __forceinline__ void wmove_flush(const ApplyArgs &A, const WMove &m) {
  int64_t *w = A.wst + (size_t)(blockIdx.x & (A.nstripes - 1)) * ((size_t)1 << A.h.bits);
  wave_keyed_add(m.has, m.t, (int64_t)m.c, [=](uint32_t k) { return &w[k]; });
  wave_keyed_add(m.has, m.p, -(int64_t)m.c, [=](uint32_t k) { return &w[k]; });
}

struct ApV {
  uint32_t p, t;
};

// One arc of a mover (u its other end): weight, u's block, target and moved
// flag, from one 8-byte gather of u's packed record.  With result caching u
// is marked here, where it is known.
__device__ __forceinline__ int4 ap_arc(const ApplyArgs &A, int32_t u, int64_t e) {
  if (A.dirty) A.dirty[u] = 1;
  const int2 q = A.pn[u];
  return make_int4(A.g.w[e], q.x, q.y, q.y >= 0 ? 1 : 0);
}
__device__ __forceinline__ int4 ap_arc(const ApplyArgs &A, int64_t e) {
  return ap_arc(A, A.g.adj[e], e);
}
// J change of one arc of a mover p -> t: an arc whose other end moved too is
// seen from both sides (once each), else from the mover only (twice).
__device__ __forceinline__ int64_t ap_delta(const ApplyArgs &A, uint32_t p, uint32_t t,
                                            const int4 &a) {
  const uint32_t old_u = (uint32_t)a.y;
  if (a.w) return (int64_t)a.x * (dist(A.h, t, (uint32_t)a.z) - dist(A.h, p, old_u));
  return 2 * (int64_t)a.x * (dist(A.h, t, old_u) - dist(A.h, p, old_u));
}
// The mover's own record: its new block, block-weight deltas, and its mark.
// (Every tile reads the blocks from the packed records, never from part[],
// so the move is committed here.)
__device__ __forceinline__ void ap_mover(const ApplyArgs &A, int32_t v, uint32_t p, uint32_t t,
                                         WMove &mv) {
  A.part[v] = (int32_t)t;
  mv.has = true;
  mv.p = p;
  mv.t = t;
  mv.c = A.g.c[v];
  if (A.dirty) A.dirty[v] = 1;
}

template <int G, int V>
__device__ __forceinline__ int64_t apply_group(const ApplyArgs &A, int cls, int local) {
  int64_t x = 0;
  WMove mv[V];
  group_tiles<G, V>(
      A.g.xadj, A.g.adj, A.cl, cls, local,
      [&](int32_t v, bool &act) {
        const int2 q = A.pn[v];
        act = q.y >= 0;
        return ApV{(uint32_t)q.x, (uint32_t)q.y};
      },
      [&](int32_t u, int64_t e) { return ap_arc(A, u, e); },
      [&](int r, bool ok, int32_t v, const ApV &vv, bool act, int, bool valid, const int4 &a) {
        if (!ok) return;
        const int lane = threadIdx.x % G;
        if (A.lock && lane == 0) A.lock[v] = act ? 1 : 0;
        if (!act) return;
        if (lane == 0) ap_mover(A, v, vv.p, vv.t, mv[r]);
        if (valid) x += ap_delta(A, vv.p, vv.t, a);
      });
#pragma unroll
  for (int r = 0; r < V; ++r) wmove_flush(A, mv[r]);
  return x;
}

// One class tile per workgroup; no LDS and no workgroup barrier, so that a
// tile without movers costs only its loads of moved[] and stores of lock[].
template <int V>
__global__ __launch_bounds__(kThreads) void k_apply(ApplyArgs A) {
  int64_t x = 0;
  const int blk = blockIdx.x;
  const int cls = find_class(A.cl, blk);
  const int local = blk - A.cl.wg[cls];
  switch (cls) {
    case CLS_ISO: {
      const int cnt = A.cl.off[CLS_ISO + 1] - A.cl.off[CLS_ISO];
      WMove mv[V];
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int idx = (local * V + r) * kThreads + threadIdx.x;
        if (idx < cnt) {
          const int32_t v = A.cl.list[A.cl.off[CLS_ISO] + idx];
          const uint8_t m = A.moved[v];
          if (A.lock) A.lock[v] = m;
          if (m) {
            const int2 q = A.pn[v];
            ap_mover(A, v, (uint32_t)q.x, (uint32_t)q.y, mv[r]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < V; ++r) wmove_flush(A, mv[r]);
      break;
    }
    case CLS_G8: x += apply_group<8, V>(A, cls, local); break;
    case CLS_G16: x += apply_group<16, V>(A, cls, local); break;
    case CLS_G32: x += apply_group<32, V>(A, cls, local); break;
    case CLS_G64: x += apply_group<64, V>(A, cls, local); break;
    case CLS_W: {
      int32_t v;
      WMove mv;
      if (w_vertex(A.cl, local, v)) {
        const int2 q = A.pn[v];
        const bool m = q.y >= 0;
        if (A.lock && (threadIdx.x & 63) == 0) A.lock[v] = m ? 1 : 0;
        if (m) {
          const uint32_t p = (uint32_t)q.x, t = (uint32_t)q.y;
          if ((threadIdx.x & 63) == 0) ap_mover(A, v, p, t, mv);
          wave_arcs<4>(
              A.g.xadj[v], A.g.xadj[v + 1], [&](int64_t e) { return ap_arc(A, e); },
              [&](int64_t, const int4 &a) { x += ap_delta(A, p, t, a); });
        }
      }
      wmove_flush(A, mv);
      break;
    }
    default: {
      const int32_t v = A.cl.list[A.cl.off[CLS_BIG] + local];
      const int2 q = A.pn[v];
      const bool m = q.y >= 0;
      if (A.lock && threadIdx.x == 0) A.lock[v] = m ? 1 : 0;
      if (m) {
        const uint32_t p = (uint32_t)q.x, t = (uint32_t)q.y;
        WMove mv;
        if (threadIdx.x == 0) ap_mover(A, v, p, t, mv);
        wmove_flush(A, mv);
        big_arcs(
            A.g.xadj[v], A.g.xadj[v + 1], [&](int64_t e) { return ap_arc(A, e); },
            [&](int64_t, const int4 &a) { x += ap_delta(A, p, t, a); });
      }
      break;
    }
  }
  x = gsum64<64>(x);
  if ((threadIdx.x & 63) == 0) stripe_add(A.dj, x);
}

// The step's end, one workgroup after k_apply (which has written the movers'
// blocks): folds the weight-delta stripes into w and, with has_end, runs the
// StepEnd epilogue.
__global__ __launch_bounds__(kThreads) void k_commit(int32_t nstripes, int64_t *wst, int has_end,
                                                     StepEnd E) {
  extern __shared__ int64_t wl[];
  step_epilogue(E, wst, nstripes, wl, has_end != 0);
  if (has_end && E.body_ctr && threadIdx.x == 0) *E.body_ctr += 1;
}

// Weight-delta stripes: at most kWeightStripes, and at most 16384 words in all
// so that one workgroup folds them quickly.
int weight_stripes(const Hier &h, int64_t n) {
  // one stripe per 2048 vertices (the adds of a small graph's few
  // workgroups hardly collide, and the step epilogue folds every stripe)
  int sc = kWeightStripes;
  while (sc > 1 && ((int64_t)sc << h.bits) > 16384) sc >>= 1;
  while (sc > 1 && (int64_t)sc * 2048 > n) sc >>= 1;
  return sc;
}

int64_t *alloc_weight_stripes(Arena &ar, const Hier &h, hipStream_t s) {
  const int64_t words = (int64_t)kWeightStripes << h.bits;
  int64_t *p = ar.alloc_n<int64_t>((size_t)words);
  fill_i64(p, 0, words, s);
  return p;
}

void apply_moves(const DGraph &g, const Classes &cl, const Hier &h, int32_t *part,
                 const uint8_t *moved, uint8_t *lock, int64_t *w, int64_t *wst,
                 int64_t *dj_stripes, const StepEnd *end, const int2 *pn, hipStream_t s,
                 uint8_t *dirty) {
  const int V = group_v();
  const Classes tc = tiled(cl, V);
  const unsigned nwg = classed_grid(tc);
  const int nstripes = weight_stripes(h, g.n);
  ApplyArgs A{g, tc, h, moved, lock, wst, nstripes, dj_stripes, dirty, pn, part};
  auto kern = V == 2 ? k_apply<2> : k_apply<1>;
  if (nwg > 0) {
    hipEvent_t ta = nullptr, tb = nullptr;
    if (tl_timer) {
      count_units(cl, g.xadj, CU_MOVED, CountArgs{moved, nullptr, nullptr, nullptr, nullptr,
                                                  nullptr},
                  tl_timer->counters(KT_APPLY), s);
      tl_timer->pair(KT_APPLY, ta, tb);
    }
    if (ta) hipExtLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, ta, tb, 0, A);
    else hipLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), 0, s, A);
    PM_LAUNCH_CHECK();
  }
  StepEnd E{};
  if (end) E = *end;
  E.h = h;
  E.w = w;
  hipLaunchKernelGGL(k_commit, dim3(1), dim3(kThreads), sizeof(int64_t) << h.bits, s, nstripes,
                     wst, end ? 1 : 0, E);
  PM_LAUNCH_CHECK();
}

// ===========================================================================
// Rebalancing (Algorithm 5 and the text around it)
//
// Sources: vertices of blocks heavier than L_max that are not heavy
// (2k c(v) > 3 (k c(block) - c(V))).  Destination: the neighbour block with
// the largest connection among blocks with weight <= cap (cap = sigma for
// weak, L_max for strong; ties to the smaller block), else a pseudo-random
// block within the cap.  Loss g = conn(v,t) - conn(v,own) (edge-cut loss),
// bucket 0 ("+"), 1 ("0") or 2 + floor(log2(-g)).  Per source block the
// sources ordered by (bucket, id) move while the weight before them is
// below the block's excess.  Strong rebalancing then accepts movers per
// destination while the destination stays within L_max, and spreads the
// rejected ones over the residual capacities.
//
// The ordered prefixes are computed without sorting ("keyed prefix"): with
// per-(key, bucket) weight sums the critical bucket of every key is found;
// only members of that bucket need an id-ordered prefix, which is split
// into per-tile sums (tiles of consecutive ids), a critical tile per key,
// and an in-tile scan.  Every size stays on the device.
// ===========================================================================

struct RebArgs {
  DGraph g;
  Classes cl;
  Hier h;
  const int32_t *part;
  const int64_t *w;
  int64_t lmax;
  int64_t cap;
  int64_t total;
  uint64_t hseed;
  const int32_t *elig;
  const int32_t *n_elig;
  const int64_t *body_ctr;  // non-null: hseed is the base, mixed with the body number
  const Status *st;
  int32_t *key;
  int32_t *dest;
  int64_t *bw;   // bucket weight stripes [stripe][code][bucket]
  int32_t jrb;   // loss = J gain of eq. 1 (variant) instead of the edge-cut loss
  int32_t whist; // W vertices use a per-wave LDS histogram (LDS: 4 slices)
};

__device__ __forceinline__ int32_t bucket_of(int64_t g) {
  if (g > 0) return 0;
  if (g == 0) return 1;
  return 2 + (63 - __builtin_clzll((unsigned long long)(-g)));
}

__device__ __forceinline__ bool is_source(const RebArgs &A, int32_t v, uint32_t p) {
  const int64_t wp = A.w[p];
  if (wp <= A.lmax) return false;
  return !(2 * A.h.k * (int64_t)A.g.c[v] > 3 * (A.h.k * wp - A.total));
}

// Source contributions to the bucket weights: key (block << 6 | bucket).
struct BwAdd {
  bool has = false;
  uint32_t key = 0;
  int64_t c = 0;
};
__device__ __forceinline__ void bw_flush(const RebArgs &A, const BwAdd &x) {
  int64_t *bw = A.bw + (size_t)(blockIdx.x & (kBucketStripes - 1)) * ((size_t)kBuckets << A.h.bits);
  wave_keyed_add(x.has, x.key, x.c, [=](uint32_t k) { return &bw[k]; });
}

// Final decision for a source v with best neighbour block (b, conn_b) or none
// (b == 0xFFFFFFFF), conn to own block connp.
// Source v of block p goes to b with loss g (bucket, key, destination).
__device__ __forceinline__ void reb_finish(const RebArgs &A, int32_t v, uint32_t p, uint32_t b,
                                           int64_t g, BwAdd &add) {
  const int32_t bucket = bucket_of(g);
  A.key[v] = (int32_t)((p << 6) | (uint32_t)bucket);
  A.dest[v] = (int32_t)b;
  add.has = true;
  add.key = (p << 6) | (uint32_t)bucket;
  add.c = A.g.c[v];
}

// The pseudo-random destination among the blocks within the cap (false:
// there is none).
__device__ __forceinline__ bool reb_random(const RebArgs &A, int32_t v, uint32_t &b) {
  const int32_t ne = *A.n_elig;
  if (ne <= 0) return false;
  // (the arguments stay unmodified: a written kernel argument is copied to
  // private memory, with the tables indexed from it)
  const uint64_t hs = A.body_ctr ? mix_hash(A.hseed, (uint64_t)(*A.body_ctr + 1)) : A.hseed;
  b = (uint32_t)A.elig[mix_hash(hs, (uint64_t)v) % (uint64_t)ne];
  return true;
}

// Edge-cut loss: destination b with connection conn_b, or none (b ==
// 0xFFFFFFFF: the random block, connection 0); connp = conn(v, p).
__device__ __forceinline__ void reb_decide(const RebArgs &A, int32_t v, uint32_t p, uint32_t b,
                                           int64_t conn_b, int64_t connp, BwAdd &add) {
  if (b == 0xFFFFFFFFu) {
    if (!reb_random(A, v, b)) {
      A.key[v] = -1;
      return;
    }
    conn_b = 0;
  }
  reb_finish(A, v, p, b, conn_b - connp, add);
}

__device__ __forceinline__ void reb_not_source(const RebArgs &A, int32_t v) { A.key[v] = -1; }

// V sources per lane group; every lane of the wave reaches the bucket flush.
struct RbN {
  uint32_t bu;
  int32_t wu;
  bool capok;
};

template <int G, int V>
__device__ __forceinline__ void reb_group(const RebArgs &A, int cls, int local) {
  BwAdd add[V];
  group_tiles<G, V>(
      A.g.xadj, A.g.adj, A.cl, cls, local,
      [&](int32_t v, bool &act) {
        const uint32_t p = (uint32_t)A.part[v];
        act = is_source(A, v, p);
        return p;
      },
      [&](int32_t u, int64_t e) {
        const uint32_t bu = (uint32_t)A.part[u];
        return RbN{bu, A.g.w[e], A.w[bu] <= A.cap};
      },
      [&](int r, bool ok, int32_t v, uint32_t p, bool act, int deg, bool valid, const RbN &nv) {
        if (!ok) return;
        const int lane = threadIdx.x % G;
        if (!act) {
          if (lane == 0) reb_not_source(A, v);
          return;
        }
        const uint32_t bu = valid ? nv.bu : p;
        const int32_t wu = valid ? nv.wu : 0;
        const bool cand = valid && bu != p && nv.capok;
        if (A.jrb) {
          // J gain of eq. 1: cost(p) - cost(b), cost(x) = sum_j w_j D(x, b_j)
          const int64_t costp = gsum64<G>((int64_t)wu * dist(A.h, p, bu));
          int64_t cost = 0;
          for (int j = 0; j < deg; ++j) {
            const uint32_t bj = (uint32_t)gshfl<G>((int32_t)bu, j);
            const int32_t wj = gshfl<G>(wu, j);
            cost += (int64_t)wj * dist(A.h, bu, bj);
          }
          int64_t val = cand ? costp - cost : INT64_MIN;
          uint32_t b = cand ? bu : 0xFFFFFFFFu;
          gargmax<G>(val, b);
          if (b == 0xFFFFFFFFu) {  // group-uniform
            uint32_t br;
            if (!reb_random(A, v, br)) {
              if (lane == 0) reb_not_source(A, v);
              return;
            }
            val = costp - gsum64<G>((int64_t)wu * dist(A.h, br, bu));
            b = br;
          }
          if (lane == 0) reb_finish(A, v, p, b, val, add[r]);
          return;
        }
        const int64_t connp = gsum64<G>(bu == p ? (int64_t)wu : 0);
        int64_t conn = 0;
        for (int j = 0; j < deg; ++j) {
          const uint32_t bj = (uint32_t)gshfl<G>((int32_t)bu, j);
          const int32_t wj = gshfl<G>(wu, j);
          conn += bj == bu ? wj : 0;
        }
        int64_t val = cand ? conn : INT64_MIN;
        uint32_t b = cand ? bu : 0xFFFFFFFFu;
        gargmax<G>(val, b);
        if (lane == 0) reb_decide(A, v, p, b, val, connp, add[r]);
      });
#pragma unroll
  for (int r = 0; r < V; ++r) bw_flush(A, add[r]);
}

__device__ __forceinline__ void reb_big(const RebArgs &A, int32_t v, uint32_t *X,
                                        BlockScratch &sc) {
  const uint32_t p = (uint32_t)A.part[v];
  if (!is_source(A, v, p)) {
    if (threadIdx.x == 0) reb_not_source(A, v);
    return;
  }
  const int32_t ncodes = 1 << A.h.bits;
  big_histogram(A.g, A.part, v, X, ncodes, sc);
  const int64_t costp = A.jrb ? level_cost(A.h, X, p, ncodes) : 0;
  int64_t val = INT64_MIN;
  uint32_t b = 0xFFFFFFFFu;
  for (int c = threadIdx.x; c < ncodes; c += kThreads) {
    const uint32_t conn = X[c + 1] - X[c];
    if ((uint32_t)c == p || conn == 0 || A.w[c] > A.cap) continue;
    const int64_t x = A.jrb ? costp - level_cost(A.h, X, (uint32_t)c, ncodes) : (int64_t)conn;
    if (x > val) {
      val = x;
      b = (uint32_t)c;
    }
  }
  block_argmax(val, b, sc);
  if (threadIdx.x == 0) {
    BwAdd add;
    if (!A.jrb) {
      reb_decide(A, v, p, b, val, (int64_t)(X[p + 1] - X[p]), add);
    } else if (b != 0xFFFFFFFFu) {
      reb_finish(A, v, p, b, val, add);
    } else if (reb_random(A, v, b)) {
      reb_finish(A, v, p, b, costp - level_cost(A.h, X, b, ncodes), add);
    } else {
      reb_not_source(A, v);
    }
    if (add.has)
      atomic_add_any(&A.bw[((size_t)(blockIdx.x & (kBucketStripes - 1)) << A.h.bits) * kBuckets +
                           add.key],
                     add.c);
  }
}

// Degree 65..kWaveMaxDeg, one vertex per wave, histogram in the wave's LDS
// slice (the block path without workgroup barriers).
// Selection from the scanned connectivity histogram Xw of source v (block
// p) in this wave's LDS slice; lane 0 gets the bucket addition.
__device__ __forceinline__ BwAdd reb_from_hist(const RebArgs &A, int32_t v, uint32_t p,
                                               const uint32_t *Xw) {
  const int lane = threadIdx.x & 63;
  const int32_t ncodes = 1 << A.h.bits;
  const int64_t costp = A.jrb ? level_cost(A.h, Xw, p, ncodes) : 0;
  int64_t val = INT64_MIN;
  uint32_t b = 0xFFFFFFFFu;
  for (int c = lane; c < ncodes; c += 64) {
    const uint32_t conn = Xw[c + 1] - Xw[c];
    if ((uint32_t)c == p || conn == 0 || A.w[c] > A.cap) continue;
    const int64_t x = A.jrb ? costp - level_cost(A.h, Xw, (uint32_t)c, ncodes) : (int64_t)conn;
    if (x > val) {
      val = x;
      b = (uint32_t)c;
    }
  }
  gargmax<64>(val, b);
  BwAdd add;
  if (lane == 0) {
    if (!A.jrb) {
      reb_decide(A, v, p, b, val, (int64_t)(Xw[p + 1] - Xw[p]), add);
    } else if (b != 0xFFFFFFFFu) {
      reb_finish(A, v, p, b, val, add);
    } else if (reb_random(A, v, b)) {
      reb_finish(A, v, p, b, costp - level_cost(A.h, Xw, b, ncodes), add);
    } else {
      reb_not_source(A, v);
    }
  }
  return add;
}

// Degree 65..kWaveMaxDeg, one vertex per wave, histogram in the wave's LDS
// slice (the block path without workgroup barriers).
__device__ __forceinline__ void reb_w(const RebArgs &A, int local, uint32_t *X) {
  int32_t v;
  if (!w_vertex(A.cl, local, v)) return;
  const int lane = threadIdx.x & 63;
  const uint32_t p = (uint32_t)A.part[v];
  if (!is_source(A, v, p)) {
    if (lane == 0) reb_not_source(A, v);
    return;
  }
  const int32_t ncodes = 1 << A.h.bits;
  uint32_t *Xw = X + (threadIdx.x >> 6) * (ncodes + 1);
  for (int c = lane; c <= ncodes; c += 64) Xw[c] = 0;
  wave_lds_sync();
  wave_arcs<4>(
      A.g.xadj[v], A.g.xadj[v + 1],
      [&](int64_t e) { return make_uint2((uint32_t)A.part[A.g.adj[e]], (uint32_t)A.g.w[e]); },
      [&](int64_t, uint2 a) { atomicAdd(&Xw[a.x + 1], a.y); });
  wave_lds_sync();
  wave_scan_lds(Xw, ncodes + 1);
  wave_lds_sync();
  const BwAdd add = reb_from_hist(A, v, p, Xw);
  bw_flush(A, add);
}

// Degree 33..64, one vertex per wave: the histogram instead of pairing every
// arc with every other one (as lp1_wave).
template <int V>
__device__ __forceinline__ void reb_wave(const RebArgs &A, int local, uint32_t *X) {
  const int32_t ncodes = 1 << A.h.bits;
  uint32_t *Xw = X + (threadIdx.x >> 6) * (ncodes + 1);
  BwAdd add[V];
  group_tiles<64, V>(
      A.g.xadj, A.g.adj, A.cl, CLS_G64, local,
      [&](int32_t v, bool &act) {
        const uint32_t p = (uint32_t)A.part[v];
        act = is_source(A, v, p);
        return p;
      },
      [&](int32_t u, int64_t e) { return make_uint2((uint32_t)A.part[u], (uint32_t)A.g.w[e]); },
      [&](int r, bool ok, int32_t v, uint32_t p, bool act, int, bool valid, uint2 a) {
        if (!ok) return;
        const int lane = threadIdx.x & 63;
        if (!act) {
          if (lane == 0) reb_not_source(A, v);
          return;
        }
        for (int c = lane; c <= ncodes; c += 64) Xw[c] = 0;
        wave_lds_sync();
        if (valid) atomicAdd(&Xw[a.x + 1], a.y);
        wave_lds_sync();
        wave_scan_lds(Xw, ncodes + 1);
        wave_lds_sync();
        add[r] = reb_from_hist(A, v, p, Xw);
        wave_lds_sync();  // the slice is cleared again for the next vertex
      });
#pragma unroll
  for (int r = 0; r < V; ++r) bw_flush(A, add[r]);
}

template <int V>
__global__ __launch_bounds__(kThreads) void k_reb_select(RebArgs A) {
  extern __shared__ uint32_t X[];
  __shared__ BlockScratch sc;
  const int blk = blockIdx.x;
  const int cls = find_class(A.cl, blk);
  const int local = blk - A.cl.wg[cls];
  switch (cls) {
    case CLS_ISO: {
      const int cnt = A.cl.off[CLS_ISO + 1] - A.cl.off[CLS_ISO];
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int idx = (local * V + r) * kThreads + threadIdx.x;
        BwAdd add;
        if (idx < cnt) {
          const int32_t v = A.cl.list[A.cl.off[CLS_ISO] + idx];
          const uint32_t p = (uint32_t)A.part[v];
          if (is_source(A, v, p)) reb_decide(A, v, p, 0xFFFFFFFFu, 0, 0, add);
          else reb_not_source(A, v);
        }
        bw_flush(A, add);
      }
      break;
    }
    case CLS_G8: reb_group<8, V>(A, cls, local); break;
    case CLS_G16: reb_group<16, V>(A, cls, local); break;
    case CLS_G32: reb_group<32, V>(A, cls, local); break;
    case CLS_G64:
      if (A.whist) reb_wave<V>(A, local, X);
      else reb_group<64, V>(A, cls, local);
      break;
    default:  // as in k_lp_phase1
      if (cls == CLS_W && A.whist) reb_w(A, local, X);
      else reb_big(A, A.cl.list[A.cl.off[cls] + local], X, sc);
      break;
  }
}

// ---------------------------------------------------------------------------
// Keyed prefix: an element v (key K, bucket b, weight c) passes iff
//   prefix(v) + delta * c < budget'(K),
// prefix(v) = weight of the elements of key K before v in (bucket, id) order.
// Selection of sources (key = source block): delta = 0, budget' = c(A) - L_max.
// Acceptance per destination (key = destination): delta = 1,
// budget' = L_max - c(t) + 1, i.e. prefix + c <= L_max - c(t).
// ---------------------------------------------------------------------------
enum { KP_SELECT = 0, KP_ACCEPT = 1 };

struct KPArgs {
  int32_t n;
  int32_t ncodes;
  int32_t tile;
  int32_t ntiles;
  int32_t pass;       // KP_SELECT or KP_ACCEPT
  int32_t strong;     // selection of a strong round: feed the acceptance sums
  int64_t lmax;
  const int64_t *w;   // block weights
  const int32_t *vwgt;
  const int32_t *key; // source block << 6 | bucket, or -1
  const int32_t *dest;
  int64_t *bw;        // bucket weight stripes
  int64_t *acc;       // accepted weight stripes [stripe][code]
  int32_t *crit;      // critical bucket per key (-1: key without elements)
  int64_t *need;      // budget left inside the critical bucket
  int32_t *tsum;      // [code][tile] weight of critical members per tile
  int32_t *tcrit;     // critical tile per key
  int64_t *tneed;     // budget left inside the critical tile
  uint8_t *moved;
  int32_t *target;
  uint8_t *reject;
  const int32_t *part;
  int2 *pn;           // apply's records {block, moved ? target : -1}
};

// element of the current pass?  (key K, bucket b)
__device__ __forceinline__ bool kp_element(const KPArgs &A, int32_t v, uint32_t &K, int32_t &b) {
  const int32_t k = A.key[v];
  if (A.pass == KP_SELECT) {
    if (k < 0) return false;
    K = (uint32_t)k >> 6;
  } else {
    if (!A.moved[v]) return false;
    K = (uint32_t)A.dest[v];
  }
  b = k & 63;
  return true;
}

// one wave per key: fold the bucket stripes, find the critical bucket
__global__ __launch_bounds__(kThreads) void k_kp_crit(KPArgs A) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t K = blockIdx.x * (kThreads / 64) + wave;
  if (K >= A.ncodes) return;
  int64_t budget;
  if (A.pass == KP_SELECT) {
    if (A.w[K] <= A.lmax) {
      if (lane == 0) A.crit[K] = -1;
      return;
    }
    budget = A.w[K] - A.lmax;
  } else {
    budget = A.lmax - A.w[K] + 1;
  }
  // eight stripes' loads in flight before their clears (a clear may not
  // pass a load of another stripe the compiler cannot tell apart)
  int64_t x = 0;
  for (int s0 = 0; s0 < kBucketStripes; s0 += 8) {
    int64_t sv[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) sv[s] = A.bw[((size_t)(s0 + s) * A.ncodes + K) * kBuckets + lane];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      x += sv[s];
      A.bw[((size_t)(s0 + s) * A.ncodes + K) * kBuckets + lane] = 0;
    }
  }
  // inclusive scan over the 64 buckets
  int64_t incl = x;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = gshfl64<64>(incl, lane >= o ? lane - o : lane);
    if (lane >= o) incl += y;
  }
  const unsigned long long reach = __ballot(incl >= budget);
  if (lane == 0) {
    if (!reach) {
      A.crit[K] = kBuckets;  // every element passes
      A.need[K] = 0;
    }
  }
  if (reach) {
    const int first = __ffsll((long long)reach) - 1;
    if (lane == first) {
      A.crit[K] = first;
      A.need[K] = budget - (incl - x);
    }
  }
}

// Per-vertex pass: weight of the critical members per (key, tile), one
// atomic per distinct key in a wave (a wave's 64 ids lie in one tile).
__global__ __launch_bounds__(kThreads) void k_kp_tilesum(KPArgs A) {
  const int64_t v0 = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63);
  const int64_t v = v0 + (threadIdx.x & 63);
  bool has = false;
  uint32_t K = 0;
  int64_t c = 0;
  if (v < A.n) {
    int32_t b;
    if (kp_element(A, (int32_t)v, K, b) && A.crit[K] == b) {
      has = true;
      c = A.vwgt[v];
    }
  }
  const int32_t t = (int32_t)(v0 / A.tile);
  int32_t *tsum = A.tsum;
  const int32_t ntiles = A.ntiles;
  wave_keyed_add(has, K, c, [=](uint32_t k) { return &tsum[(size_t)k * ntiles + t]; });
}

// one wave per key: the critical tile and the budget left inside it; clears
// the key's row of tile sums for the next round
__global__ __launch_bounds__(kThreads) void k_kp_tilecrit(KPArgs A) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t K = blockIdx.x * (kThreads / 64) + wave;
  if (K >= A.ncodes) return;
  const int32_t cb = A.crit[K];
  if (cb < 0 || cb >= kBuckets) return;
  const int64_t need = A.need[K];
  int64_t base = 0;
  bool found = false;
  int32_t *row = A.tsum + (size_t)K * A.ntiles;
  for (int32_t t0 = 0; t0 < A.ntiles; t0 += 64) {
    const int32_t t = t0 + lane;
    const int64_t x = t < A.ntiles ? row[t] : 0;
    if (x) row[t] = 0;
    if (found) continue;
    int64_t incl = x;
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = gshfl64<64>(incl, lane >= o ? lane - o : lane);
      if (lane >= o) incl += y;
    }
    const unsigned long long reach = __ballot(t < A.ntiles && base + incl >= need);
    if (reach) {
      const int first = __ffsll((long long)reach) - 1;
      if (lane == first) {
        A.tcrit[K] = t;
        A.tneed[K] = need - (base + incl - x);
      }
      found = true;
      continue;
    }
    base += gshfl64<64>(incl, 63);
  }
  if (!found && lane == 0) A.tcrit[K] = A.ntiles;  // every critical member passes
}

// Outcome of element v (key K, bucket b).  Returns in (has, akey, aval) the
// weight the outcome adds to a keyed accumulator: in a strong selection the
// bucket weights of the destination, in an acceptance the accepted weight.
__device__ __forceinline__ void kp_outcome(const KPArgs &A, int32_t v, uint32_t K, int32_t b,
                                           bool pass, bool &has, uint32_t &akey, int64_t &aval) {
  if (A.pass == KP_SELECT) {  // (K is v's block)
    if (pass) {
      const int32_t d = A.dest[v];
      A.moved[v] = 1;
      A.target[v] = d;
      A.pn[v] = make_int2((int32_t)K, d);
      if (A.strong) {
        has = true;
        akey = ((uint32_t)d << 6) | (uint32_t)b;
        aval = A.vwgt[v];
      }
    } else {
      A.moved[v] = 0;
      A.pn[v] = make_int2((int32_t)K, -1);
    }
  } else {
    if (pass) {
      A.reject[v] = 0;
      has = true;
      akey = K;
      aval = A.vwgt[v];
    } else {
      A.moved[v] = 0;
      A.pn[v].y = -1;
      A.reject[v] = 1;
    }
  }
}

// The keyed adds of a wave (every lane of the wave calls it).
__device__ __forceinline__ void kp_flush(const KPArgs &A, bool has, uint32_t akey, int64_t aval) {
  const size_t stripe = blockIdx.x & (kBucketStripes - 1);
  if (A.pass == KP_SELECT) {
    int64_t *bw = A.bw + stripe * (size_t)A.ncodes * kBuckets;
    wave_keyed_add(has, akey, aval, [=](uint32_t k) { return &bw[k]; });
  } else {
    int64_t *acc = A.acc + stripe * (size_t)A.ncodes;
    wave_keyed_add(has, akey, aval, [=](uint32_t k) { return &acc[k]; });
  }
}

// Per-vertex pass: the outcome of every element except the members of a key
// inside that key's critical tile (those are left to k_kp_walk).
__device__ __forceinline__ void kp_decide(const KPArgs &A, int blk) {
  const int64_t v = (int64_t)blk * kThreads + threadIdx.x;
  bool has = false;
  uint32_t akey = 0;
  int64_t aval = 0;
  if (v < A.n) {
    uint32_t K;
    int32_t b;
    // The selection clears every reject flag; the acceptance writes flags of
    // elements only.  (In the acceptance, the walk workgroups of the same
    // launch clear moved[] of refused members, so a vertex may look like a
    // non-element here; it must then be left alone.)
    if (A.pass == KP_SELECT) A.reject[v] = 0;
    if (!kp_element(A, (int32_t)v, K, b)) {
      if (A.pass == KP_SELECT) {
        A.moved[v] = 0;
        A.pn[v] = make_int2(A.part[v], -1);
      }
    } else {
      const int32_t cb = A.crit[K];
      if (b != cb) {
        kp_outcome(A, (int32_t)v, K, b, b < cb, has, akey, aval);
      } else {
        const int32_t t = (int32_t)(v / A.tile);
        const int32_t tc = A.tcrit[K];
        if (tc != t) kp_outcome(A, (int32_t)v, K, b, tc > t, has, akey, aval);
      }
    }
  }
  kp_flush(A, has, akey, aval);
}

// One workgroup per key with a critical tile: the members of the key's
// critical bucket inside that tile, in id order.  The tile is taken in
// chunks of 4096 ids, 16 consecutive ids per thread: member weights into
// registers, a workgroup exclusive scan, then every thread decides its
// members in order.
constexpr int kWalkPer = 16;
constexpr int kWalkChunk = kWalkPer * kThreads;
__device__ __forceinline__ void kp_walk(const KPArgs &A, int32_t K) {
  __shared__ BlockScratch sc;
  __shared__ uint32_t chunk_total;
  const int32_t cb = A.crit[K];
  if (cb < 0 || cb >= kBuckets) return;
  const int32_t tc = A.tcrit[K];
  if (tc >= A.ntiles) return;
  const int64_t lo = (int64_t)tc * A.tile;
  const int64_t hi = lo + A.tile < A.n ? lo + A.tile : A.n;
  const int64_t need = A.tneed[K];
  const int64_t delta = A.pass == KP_SELECT ? 0 : 1;
  int64_t base = 0;  // member weight of the earlier chunks
  for (int64_t c0 = lo; c0 < hi; c0 += kWalkChunk) {
    const int64_t v0 = c0 + (int64_t)threadIdx.x * kWalkPer;
    int32_t cw[kWalkPer];
    uint32_t mem = 0;  // bit i: id v0 + i is a member
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kWalkPer; ++i) {
      const int64_t v = v0 + i;
      uint32_t Kv;
      int32_t b;
      cw[i] = 0;
      if (v < hi && kp_element(A, (int32_t)v, Kv, b) && Kv == (uint32_t)K && b == cb) {
        cw[i] = A.vwgt[v];
        mem |= 1u << i;
      }
      sum += (uint32_t)cw[i];
    }
    const uint32_t excl = block_excl_scan(sum, sc);
    if (threadIdx.x == kThreads - 1) chunk_total = excl + sum;
    int64_t run = base + excl;
#pragma unroll
    for (int i = 0; i < kWalkPer; ++i) {
      bool has = false;
      uint32_t akey = 0;
      int64_t aval = 0;
      if (mem & (1u << i)) {
        kp_outcome(A, (int32_t)(v0 + i), (uint32_t)K, cb, run + delta * cw[i] < need, has, akey,
                   aval);
        run += cw[i];
      }
      kp_flush(A, has, akey, aval);
    }
    __syncthreads();
    base += chunk_total;
    __syncthreads();  // chunk_total is rewritten by the next chunk
  }
}

// The first `flat` workgroups decide per vertex, the next ncodes walk one key
// each (the two sets of elements are disjoint).
__global__ __launch_bounds__(kThreads) void k_kp_final(KPArgs A, int flat) {
  if ((int)blockIdx.x < flat) kp_decide(A, blockIdx.x);
  else kp_walk(A, (int32_t)blockIdx.x - flat);
}

// smallest q with c <= 2^q (c >= 1): the weight class of a refused mover
__device__ __forceinline__ int32_t weight_class(int32_t c) {
  return c <= 1 ? 0 : 32 - __clz((uint32_t)(c - 1));
}

// Strong rebalancing, the movers refused by their destination (list[0..
// *count), ascending ids), placed by one workgroup of kPlaceThreads.  First
// the accepted-weight stripes are folded (and cleared) into the residual
// capacity of every code, resid[c] = L_max - c(b) - accepted_b (0 for codes
// of no block), and the movers' weights are gathered once into rw[].  Then
// the movers are placed by weight class q = ceil(log2 c(v)), heaviest class
// first: in class q a block with residual r >= 2^q offers the r - 2^q + 1
// positions [C_b, C_b + r - 2^q + 1) of a prefix over ascending codes, and a
// mover of the class whose exclusive weight prefix R (over the class's movers
// in id order) falls into them goes there; R beyond the last position leaves
// it where it is.  The movers a block receives in one class start inside its
// positions, so they weigh at most r: no block ends above L_max.  The
// residuals shrink by what each block received before the next class.
//
// The position starts C (one per code, codes without positions repeat the
// next start) are searched for the last C <= R, which is always a code with
// positions.  With at most kPlaceLdsCodes codes, residuals and starts live
// in LDS; beyond, in the global arrays gresid / gstart.  A chunk of
// kPlaceChunk movers is read per step; a per-chunk mask of the classes it
// holds lets a class skip the chunks without members.
constexpr int kPlaceThreads = 1024;
constexpr int kPlacePer = 16;
constexpr int kPlaceChunk = kPlaceThreads * kPlacePer;
constexpr int kPlaceLdsCodes = 2048;
constexpr int kPlaceMaxChunks = 1024;  // chunks with a class mask; beyond: every class visits

__device__ __forceinline__ uint32_t place_excl_scan(uint32_t x, uint32_t *wsum) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int32_t)incl, o, 64);
    if (lane >= o) incl += y;
  }
  __syncthreads();
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int i = 0; i < wave; ++i) off += wsum[i];
  return off + incl - x;
}

__device__ __forceinline__ int64_t place_excl_scan64(int64_t x, int64_t *wsum, int64_t *total) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = gshfl64<64>(incl, lane >= o ? lane - o : lane);
    if (lane >= o) incl += y;
  }
  __syncthreads();
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int i = 0; i < kPlaceThreads / 64; ++i) {
    if (i < wave) off += wsum[i];
    tot += wsum[i];
  }
  *total = tot;
  return off + incl - x;
}

__global__ __launch_bounds__(kPlaceThreads) void k_place_rejects(
    Hier h, const int64_t *w, int64_t *acc, int64_t lmax, const int32_t *list,
    const int32_t *count, const int32_t *vwgt, int32_t *rw, int64_t *gresid, int64_t *gstart,
    int32_t *target, uint8_t *moved, int2 *pn) {
  extern __shared__ int64_t place_lds[];
  __shared__ uint32_t wsum[kPlaceThreads / 64];
  __shared__ int64_t wsum64[kPlaceThreads / 64];
  __shared__ uint32_t cmask[kPlaceMaxChunks];
  __shared__ uint32_t chunk_total;
  const int32_t ncodes = 1 << h.bits;
  const bool in_lds = ncodes <= kPlaceLdsCodes;
  int64_t *resid = in_lds ? place_lds : gresid;
  int64_t *start = in_lds ? place_lds + ncodes : gstart;
  uint32_t *got = reinterpret_cast<uint32_t *>(in_lds ? place_lds + 2 * ncodes : place_lds);
  const int per = (ncodes + kPlaceThreads - 1) / kPlaceThreads;
  const int lo = threadIdx.x * per;
  const int hi = lo + per < ncodes ? lo + per : ncodes;
  for (int c = lo; c < hi; ++c) {
    int64_t a = 0;
    for (int s0 = 0; s0 < kBucketStripes; s0 += 8) {
      int64_t sv[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) sv[s] = acc[(size_t)(s0 + s) * ncodes + c];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        a += sv[s];
        acc[(size_t)(s0 + s) * ncodes + c] = 0;
      }
    }
    resid[c] = code_valid(h, (uint32_t)c) ? lmax - w[c] - a : 0;
    got[c] = 0;
  }
  for (int i = threadIdx.x; i < kPlaceMaxChunks; i += kPlaceThreads) cmask[i] = 0;
  __syncthreads();
  const int32_t L = *count;
  const int32_t nchunks = (L + kPlaceChunk - 1) / kPlaceChunk;
  // weights of the movers, and the classes of every chunk
  uint32_t all = 0;
  for (int32_t c0 = 0; c0 < L; c0 += kPlaceChunk) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kPlacePer; ++i) {
      const int32_t j = c0 + i * kPlaceThreads + (int32_t)threadIdx.x;  // coalesced
      if (j < L) {
        const int32_t c = vwgt[list[j]];
        rw[j] = c;
        m |= 1u << weight_class(c);
      }
    }
    m = (uint32_t)gor<64>((int32_t)m);
    all |= m;
    const int32_t ch = c0 / kPlaceChunk;
    if ((threadIdx.x & 63) == 0 && m && ch < kPlaceMaxChunks) atomicOr(&cmask[ch], m);
  }
  __syncthreads();
  // the union of the classes over all waves
  uint32_t mask = 0;
  for (int32_t ch = 0; ch < nchunks && ch < kPlaceMaxChunks; ++ch) mask |= cmask[ch];
  if (nchunks > kPlaceMaxChunks) {
    all = (uint32_t)gor<64>((int32_t)all);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = all;
    __syncthreads();
    for (int i = 0; i < kPlaceThreads / 64; ++i) mask |= wsum[i];
    __syncthreads();
  }
  for (int q = 31; q >= 0; --q) {
    if (!((mask >> q) & 1u)) continue;
    const int64_t unit = int64_t(1) << q;
    // position starts of the class over ascending codes
    int64_t sum = 0;
    for (int c = lo; c < hi; ++c) {
      const int64_t r = resid[c];
      if (r >= unit) sum += r - unit + 1;
    }
    int64_t total = 0;
    int64_t run = place_excl_scan64(sum, wsum64, &total);
    for (int c = lo; c < hi; ++c) {
      start[c] = run;
      const int64_t r = resid[c];
      if (r >= unit) run += r - unit + 1;
    }
    __syncthreads();
    // the class's movers in id order, 16 consecutive entries per thread
    int64_t base = 0;
    for (int32_t c0 = 0; c0 < L && base < total; c0 += kPlaceChunk) {
      const int32_t ch = c0 / kPlaceChunk;
      if (ch < kPlaceMaxChunks && !((cmask[ch] >> q) & 1u)) continue;
      const int32_t i0 = c0 + (int32_t)threadIdx.x * kPlacePer;
      uint32_t cw[kPlacePer];
      uint32_t mem = 0, s = 0;
#pragma unroll
      for (int i = 0; i < kPlacePer; ++i) {
        cw[i] = 0;
        if (i0 + i < L) {
          const int32_t c = rw[i0 + i];
          if (weight_class(c) == q) {
            cw[i] = (uint32_t)c;
            mem |= 1u << i;
          }
        }
        s += cw[i];
      }
      const uint32_t excl = place_excl_scan(s, wsum);
      if (threadIdx.x == kPlaceThreads - 1) chunk_total = excl + s;
      int64_t R = base + excl;
#pragma unroll
      for (int i = 0; i < kPlacePer; ++i) {
        if (!(mem & (1u << i))) continue;
        if (R < total) {
          int32_t a = 0, b = ncodes - 1;  // last code with start <= R
          while (a < b) {
            const int32_t mid = (a + b + 1) >> 1;
            if (start[mid] <= R) a = mid;
            else b = mid - 1;
          }
          const int32_t v = list[i0 + i];
          target[v] = a;
          moved[v] = 1;
          pn[v].y = a;
          atomicAdd(&got[a], cw[i]);
        }
        R += cw[i];
      }
      __syncthreads();
      base += chunk_total;
    }
    __syncthreads();
    for (int c = lo; c < hi; ++c) {
      resid[c] -= got[c];
      got[c] = 0;
    }
    __syncthreads();
  }
}

RebalanceBuffers alloc_rebalance(Arena &ar, int64_t n, const Hier &h, hipStream_t s) {
  RebalanceBuffers rb{};
  const int32_t ncodes = 1 << h.bits;
  int64_t tile = 4096;
  while (((n + tile - 1) / tile) * (int64_t)ncodes > (int64_t(1) << 24)) tile *= 2;
  rb.tile = (int32_t)tile;
  rb.ntiles = (int32_t)((n + tile - 1) / tile);
  rb.key = ar.alloc_n<int32_t>(n);
  rb.dest = ar.alloc_n<int32_t>(n);
  rb.reject = ar.alloc_n<uint8_t>(n);
  rb.rlist = ar.alloc_n<int32_t>(n);
  rb.rcount = ar.alloc_n<int32_t>(1);
  rb.resid = ar.alloc_n<int64_t>(ncodes);
  rb.elig_weak = ar.alloc_n<int32_t>(ncodes);
  rb.elig_strong = ar.alloc_n<int32_t>(ncodes);
  rb.bw = ar.alloc_n<int64_t>((size_t)kBucketStripes * ncodes * kBuckets);
  rb.acc = ar.alloc_n<int64_t>((size_t)kBucketStripes * ncodes);
  rb.crit = ar.alloc_n<int32_t>(ncodes);
  rb.need = ar.alloc_n<int64_t>(ncodes);
  rb.tcrit = ar.alloc_n<int32_t>(ncodes);
  rb.tneed = ar.alloc_n<int64_t>(ncodes);
  rb.tsum = ar.alloc_n<int32_t>((size_t)ncodes * (rb.ntiles > 0 ? rb.ntiles : 1));
  rb.rstart = ar.alloc_n<int64_t>(ncodes);
  rb.rweight = ar.alloc_n<int32_t>(n);
  fill_i64(rb.bw, 0, (int64_t)kBucketStripes * ncodes * kBuckets, s);
  fill_i64(rb.acc, 0, (int64_t)kBucketStripes * ncodes, s);
  fill_i32(rb.tsum, 0, (int64_t)ncodes * (rb.ntiles > 0 ? rb.ntiles : 1), s);
  return rb;
}

static void keyed_prefix(KPArgs A, hipStream_t s) {
  const unsigned waves_grid = (unsigned)((A.ncodes + (kThreads / 64) - 1) / (kThreads / 64));
  hipLaunchKernelGGL(k_kp_crit, dim3(waves_grid), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
  if (A.n <= 0) return;
  const unsigned flat = grid_for(A.n);
  hipLaunchKernelGGL(k_kp_tilesum, dim3(flat), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_kp_tilecrit, dim3(waves_grid), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_kp_final, dim3(flat + A.ncodes), dim3(kThreads), 0, s, A, (int)flat);
  PM_LAUNCH_CHECK();
}

__global__ void k_reb_candidates(int32_t n, const int32_t *list, const int32_t *part,
                                 const int64_t *w, int64_t lmax, int32_t *key, uint8_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t v = list[i];
  const bool over = w[part[v]] > lmax;
  flag[i] = over ? 1 : 0;
  if (!over) key[v] = -1;
}

void reb_sources(Arena &ar, const Classes &cl, int32_t n, const int32_t *part, const int64_t *w,
                 int64_t lmax, int32_t *key, int32_t *list_out, int32_t *off_out, hipStream_t s) {
  uint8_t *flag = ar.alloc_n<uint8_t>((size_t)n + 1);
  int32_t *pos = ar.alloc_n<int32_t>((size_t)n + 1);
  int32_t *count = ar.alloc_n<int32_t>(1);
  if (n > 0) {
    hipLaunchKernelGGL(k_reb_candidates, dim3(grid_for(n)), dim3(kThreads), 0, s, n, cl.list, part,
                       w, lmax, key, flag);
    PM_LAUNCH_CHECK();
  }
  select_indices(ar, flag, pos, count, n, s);
  compact_bounds(n, cl, pos, count, list_out, off_out, s);
}

void rebalance_round(Arena &ar, const DGraph &g, const Classes &cl, const Hier &h, bool strong,
                     int64_t lmax, int64_t sigma, int64_t total, uint64_t hseed,
                     const int32_t *part, const int64_t *w, int32_t *target, uint8_t *moved,
                     int2 *pn, const RebalanceBuffers &rb, Status *st_dev, hipStream_t s,
                     const Variants &var, const int64_t *body_ctr) {
  const int V = group_v();
  const bool whist = h.bits <= 10;  // as in lp_phase1
  const Classes tc = tiled(cl, V, !whist);
  const unsigned nwg = classed_grid(tc);
  const int64_t n = g.n;
  if (n <= 0) return;
  const int32_t ncodes = 1 << h.bits;
  const int64_t cap = strong ? lmax : sigma;
  if (nwg > 0) {
    RebArgs A{g,
              tc,
              h,
              part,
              w,
              lmax,
              cap,
              total,
              hseed,
              strong ? rb.elig_strong : rb.elig_weak,
              strong ? &st_dev->n_elig_strong : &st_dev->n_elig_weak,
              body_ctr,
              st_dev,
              rb.key,
              rb.dest,
              rb.bw,
              var.j_rebalance ? 1 : 0,
              whist ? 1 : 0};
    auto kern = V == 2 ? k_reb_select<2> : k_reb_select<1>;
    const size_t lds = A.whist ? 4 * big_lds(h) : big_lds(h);
    hipEvent_t a = nullptr, b = nullptr;
    if (tl_timer) tl_timer->pair(KT_REB, a, b);
    if (a) hipExtLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), lds, s, a, b, 0, A);
    else hipLaunchKernelGGL(kern, dim3(nwg), dim3(kThreads), lds, s, A);
    PM_LAUNCH_CHECK();
    if (tl_timer)
      count_units(cl, g.xadj, CU_SOURCE, CountArgs{nullptr, nullptr, nullptr, rb.key, nullptr, nullptr},
                  tl_timer->counters(KT_REB), s);
  }
  KPArgs K{};
  K.n = (int32_t)n;
  K.ncodes = ncodes;
  K.tile = rb.tile;
  K.ntiles = rb.ntiles;
  K.pass = KP_SELECT;
  K.strong = strong ? 1 : 0;
  K.lmax = lmax;
  K.w = w;
  K.vwgt = g.c;
  K.key = rb.key;
  K.dest = rb.dest;
  K.bw = rb.bw;
  K.acc = rb.acc;
  K.crit = rb.crit;
  K.need = rb.need;
  K.tsum = rb.tsum;
  K.tcrit = rb.tcrit;
  K.tneed = rb.tneed;
  K.moved = moved;
  K.target = target;
  K.part = part;
  K.pn = pn;
  K.reject = rb.reject;
  keyed_prefix(K, s);
  if (!strong) return;
  K.pass = KP_ACCEPT;
  K.strong = 0;
  keyed_prefix(K, s);
  select_indices(ar, rb.reject, rb.rlist, rb.rcount, n, s);
  const size_t plds = ncodes <= kPlaceLdsCodes ? (size_t)ncodes * 20 : (size_t)ncodes * 4;
  hipLaunchKernelGGL(k_place_rejects, dim3(1), dim3(kPlaceThreads), plds, s, h, w, rb.acc, lmax,
                     rb.rlist, rb.rcount, g.c, rb.rweight, rb.resid, rb.rstart, target, moved,
                     pn);
  PM_LAUNCH_CHECK();
}

}  // namespace pm
