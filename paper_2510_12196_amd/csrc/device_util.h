// device_util.h -- wave/group/workgroup helpers for gfx950 (wave64).
#pragma once

#include "pm_internal.h"

namespace pm {

// ---- lane groups of G consecutive lanes inside a wave64 -------------------
template <int G>
__device__ __forceinline__ int32_t gshfl(int32_t x, int j) {
  return __shfl(x, j, G);
}
template <int G>
__device__ __forceinline__ int64_t gshfl64(int64_t x, int j) {
  int32_t lo = __shfl((int32_t)(uint32_t)(uint64_t)x, j, G);
  int32_t hi = __shfl((int32_t)((uint64_t)x >> 32), j, G);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int G>
__device__ __forceinline__ int64_t gxor64(int64_t x, int m) {
  int32_t lo = __shfl_xor((int32_t)(uint32_t)(uint64_t)x, m, G);
  int32_t hi = __shfl_xor((int32_t)((uint64_t)x >> 32), m, G);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Step K (1, 2, 4, ..., 32) of a group reduction: the value held by the other
// half of this lane's aligned 2K-lane block.  The steps run in increasing K,
// so every lane of a K-block already holds the same value and any pairing of
// the two halves works: DPP quad permutations for K = 1, 2 and the row
// mirrors for K = 4, 8 (VALU operand modifiers, no LDS round trip), a
// swizzle (xor 16 within 32 lanes) for K = 16, two lane reads for K = 32.
// Only lanes of the same group are read, so groups may differ in activity.
template <int K>
__device__ __forceinline__ int32_t xstep32(int32_t x) {
  if constexpr (K == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
  else if constexpr (K == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
  else if constexpr (K == 4) return __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);
  else if constexpr (K == 8) return __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false);
  else if constexpr (K == 16) return __builtin_amdgcn_ds_swizzle(x, 0x401F);
  else {
    static_assert(K == 32, "reduction step");
    const int32_t a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 32);
    return (threadIdx.x & 32) ? a : b;
  }
}
template <int K>
__device__ __forceinline__ int64_t xstep64(int64_t x) {
  const int32_t lo = xstep32<K>((int32_t)(uint32_t)(uint64_t)x);
  const int32_t hi = xstep32<K>((int32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int K> __device__ __forceinline__ int32_t xstep_any(int32_t x) { return xstep32<K>(x); }
template <int K> __device__ __forceinline__ uint32_t xstep_any(uint32_t x) {
  return (uint32_t)xstep32<K>((int32_t)x);
}
template <int K> __device__ __forceinline__ int64_t xstep_any(int64_t x) { return xstep64<K>(x); }
template <int K> __device__ __forceinline__ uint64_t xstep_any(uint64_t x) {
  return (uint64_t)xstep64<K>((int64_t)x);
}
// The value of lane (lane xor m) for m = 1, 2 (DPP quad permutations), 4, 8,
// 16 (swizzles within 32 lanes) or 32 (LDS permute): an exact exchange, for
// sorting networks.  m must fold to a constant (unrolled loops).
__device__ __forceinline__ int32_t xor_lane(int32_t x, int m) {
  switch (m) {
    case 1: return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_ds_swizzle(x, 0x101F);
    case 8: return __builtin_amdgcn_ds_swizzle(x, 0x201F);
    case 16: return __builtin_amdgcn_ds_swizzle(x, 0x401F);
    default: return __shfl_xor(x, m, 64);
  }
}

// Runs f(step) for the steps of a G-lane group reduction, K = 1 upwards.
template <int G, class F>
__device__ __forceinline__ void xsteps(F f) {
  if constexpr (G >= 2) f([](auto x) { return xstep_any<1>(x); });
  if constexpr (G >= 4) f([](auto x) { return xstep_any<2>(x); });
  if constexpr (G >= 8) f([](auto x) { return xstep_any<4>(x); });
  if constexpr (G >= 16) f([](auto x) { return xstep_any<8>(x); });
  if constexpr (G >= 32) f([](auto x) { return xstep_any<16>(x); });
  if constexpr (G >= 64) f([](auto x) { return xstep_any<32>(x); });
}
template <int G>
__device__ __forceinline__ int64_t gsum64(int64_t x) {
  xsteps<G>([&](auto st) { x += st(x); });
  return x;
}
template <int G>
__device__ __forceinline__ int32_t gor(int32_t x) {
  xsteps<G>([&](auto st) { x |= st(x); });
  return x;
}
// (value desc, key asc) argmax over the group; every lane gets the result.
template <int G>
__device__ __forceinline__ void gargmax(int64_t &val, uint32_t &key) {
  xsteps<G>([&](auto st) {
    const int64_t ov = st(val);
    const uint32_t ok = st(key);
    if (ov > val || (ov == val && ok < key)) {
      val = ov;
      key = ok;
    }
  });
}

// ---- whole workgroup (kThreads = 256, four waves) --------------------------
// LDS scratch for the block-level reductions below: 4 waves x 2 words.
struct BlockScratch {
  int64_t v[kThreads / 64];
  uint32_t k[kThreads / 64];
  uint32_t u[kThreads / 64];
};

__device__ __forceinline__ int64_t block_sum64(int64_t x, BlockScratch &sc) {
  x = gsum64<64>(x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sc.v[wave] = x;
  __syncthreads();
  int64_t t = 0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) t += sc.v[i];
  return t;
}

__device__ __forceinline__ void block_argmax(int64_t &val, uint32_t &key, BlockScratch &sc) {
  gargmax<64>(val, key);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sc.v[wave] = val;
    sc.k[wave] = key;
  }
  __syncthreads();
  val = sc.v[0];
  key = sc.k[0];
#pragma unroll
  for (int i = 1; i < kThreads / 64; ++i)
    if (sc.v[i] > val || (sc.v[i] == val && sc.k[i] < key)) {
      val = sc.v[i];
      key = sc.k[i];
    }
}

// exclusive scan of one uint32 per thread over the workgroup
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, BlockScratch &sc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int32_t)incl, o, 64);
    if (lane >= o) incl += y;
  }
  __syncthreads();
  if (lane == 63) sc.u[wave] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int i = 0; i < wave; ++i) off += sc.u[i];
  return off + incl - x;
}

// In-place inclusive scan of a[0..m) held in LDS.
__device__ __forceinline__ void block_scan_lds(uint32_t *a, int m, BlockScratch &sc) {
  const int per = (m + kThreads - 1) / kThreads;
  const int lo = threadIdx.x * per;
  const int hi = lo + per < m ? lo + per : m;
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) {
    s += a[i];
    a[i] = s;
  }
  uint32_t off = block_excl_scan(s, sc);
  for (int i = lo; i < hi; ++i) a[i] += off;
  __syncthreads();
}

// ---- one wave working alone on its own LDS slice ------------------------------
// The LDS instructions of one wave are performed in issue order, so a wave
// needs no barrier between its own LDS phases; this keeps the compiler from
// moving LDS accesses across the phase boundary.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
// Inclusive prefix sum over a[0..m) in LDS by the 64 lanes of one wave: a
// contiguous run of ceil(m/64) entries per lane, then a scan of the run
// totals by shuffles.
__device__ __forceinline__ void wave_scan_lds(uint32_t *a, int m) {
  const int lane = threadIdx.x & 63;
  const int per = (m + 63) / 64;
  const int lo = lane * per;
  const int hi = lo + per < m ? lo + per : m;
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) {
    s += a[i];
    a[i] = s;
  }
  uint32_t incl = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int32_t)incl, d, 64);
    if (lane >= d) incl += y;
  }
  const uint32_t off = incl - s;
  for (int i = lo; i < hi; ++i) a[i] += off;
}

// ---- striped accumulators ---------------------------------------------------
// A global sum updated by thousands of workgroups is spread over kStripes
// counters one cache line apart (atomics on a single address serialise);
// fold_stripes() adds them up afterwards and clears them.
constexpr int kStripes = 256;
constexpr int kStripeStride = 16;  // int64 words: 128 bytes
constexpr int kStripeWords = kStripes * kStripeStride;
__device__ __forceinline__ void stripe_add(int64_t *stripes, int64_t x) {
  if (x != 0)
    atomicAdd((unsigned long long *)&stripes[(blockIdx.x & (kStripes - 1)) * kStripeStride],
              (unsigned long long)x);
}

// ---- arcs of one high-degree vertex over a whole workgroup -------------------
// For the arcs e in [beg, end) owned by this thread (stride kThreads), calls
// use(e, load(e)).  load() may only read memory; kArcBatch loads are issued
// before their uses, so that that many arcs' gathers are in flight together.
constexpr int kArcBatch = 8;
template <class L, class U>
__device__ __forceinline__ void big_arcs(int64_t beg, int64_t end, L load, U use) {
  int64_t e = beg + threadIdx.x;
  for (; e + (kArcBatch - 1) * kThreads < end; e += kArcBatch * kThreads) {
    decltype(load(e)) a[kArcBatch];
#pragma unroll
    for (int i = 0; i < kArcBatch; ++i) a[i] = load(e + i * kThreads);
#pragma unroll
    for (int i = 0; i < kArcBatch; ++i) use(e + i * kThreads, a[i]);
  }
  for (; e < end; e += kThreads) use(e, load(e));
}

// ---- keyed adds aggregated over a wave ----------------------------------------
__device__ __forceinline__ void atomic_add_any(int32_t *p, int64_t x) { atomicAdd(p, (int32_t)x); }
__device__ __forceinline__ void atomic_add_any(int64_t *p, int64_t x) {
  atomicAdd((unsigned long long *)p, (unsigned long long)x);
}
// For every lane with `has`, adds val to *addr(key).  The keys of the first
// two leaders are summed over the wave (one atomic each: the common case of
// neighbouring vertices in one block); lanes with any other key add on their
// own, since a wave of many distinct keys would otherwise pay a wave-wide
// sum per key.  Integer adds: the totals do not depend on the grouping.
// Every lane of the wave must call it (no lane may have left the kernel).
template <class AddrF>
__device__ __forceinline__ void wave_keyed_add(bool has, uint32_t key, int64_t val, AddrF addr) {
  unsigned long long left = __ballot(has);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    if (!left) return;
    const int leader = __ffsll((long long)left) - 1;
    const uint32_t lk = (uint32_t)__shfl((int32_t)key, leader, 64);
    const bool in = has && key == lk;
    const int64_t sum = gsum64<64>(in ? val : 0);
    if ((int)(threadIdx.x & 63) == leader && sum != 0) atomic_add_any(addr(lk), sum);
    left &= ~__ballot(in);
  }
  if (((left >> (threadIdx.x & 63)) & 1ull) && val != 0) atomic_add_any(addr(key), val);
}

// ---- classed launches --------------------------------------------------------
// Classed kernels run a capped grid; every workgroup walks the class tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...
constexpr int kMaxGrid = 2048;
// (CL: Classes, or any view with the members list, off[] and wg[])
template <class CL>
__device__ __forceinline__ int find_class(const CL &cl, int b) {
  int c = 0;
  while (c < NCLS - 1 && b >= cl.wg[c + 1]) ++c;
  return c;
}

// Vertex handled by this lane group (G lanes per vertex) in class cls.
template <int G, class CL>
__device__ __forceinline__ bool group_vertex(const CL &cl, int cls, int local, int32_t &v) {
  const int idx = local * (kThreads / G) + (int)threadIdx.x / G;
  const int cnt = cl.off[cls + 1] - cl.off[cls];
  if (idx >= cnt) return false;
  v = cl.list[cl.off[cls] + idx];
  return true;
}

// W tiles: one vertex per wave, kThreads / 64 vertices per tile.
template <class CL>
__device__ __forceinline__ bool w_vertex(const CL &cl, int local, int32_t &v) {
  const int idx = local * (kThreads / 64) + (int)(threadIdx.x >> 6);
  if (idx >= cl.off[CLS_W + 1] - cl.off[CLS_W]) return false;
  v = cl.list[cl.off[CLS_W] + idx];
  return true;
}

// The arcs [beg, end) of one vertex over the 64 lanes of a wave: lane l takes
// beg + l, beg + l + 64, ...; B arcs per lane are loaded before any is used
// (indices past the row are clamped to its last arc, so that no load sits
// behind a branch, and their uses skipped).  Every lane gets the same number
// of rounds.
template <int B, class L, class U>
__device__ __forceinline__ void wave_arcs(int64_t beg, int64_t end, L load, U use) {
  const int lane = threadIdx.x & 63;
  for (int64_t e0 = beg; e0 < end; e0 += 64 * B) {
    decltype(load(e0)) a[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int64_t e = e0 + lane + 64 * i;
      a[i] = load(e < end ? e : end - 1);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int64_t e = e0 + lane + 64 * i;
      if (e < end) use(e, a[i]);
    }
  }
}

// ISO tiles: V vertices per thread.
template <int V, class CL, class F>
__device__ __forceinline__ void iso_tiles(const CL &cl, int local, F f) {
  const int cnt = cl.off[CLS_ISO + 1] - cl.off[CLS_ISO];
#pragma unroll
  for (int r = 0; r < V; ++r) {
    const int idx = (local * V + r) * kThreads + threadIdx.x;
    if (idx < cnt) f(cl.list[cl.off[CLS_ISO] + idx]);
  }
}

// ---- staged tiles: V vertices per lane group -------------------------------
// A tile of class cls (G lanes per vertex, deg <= G) holds V * (kThreads / G)
// vertices; lane group q handles slots r = 0..V-1, vertex index
// (local * V + r) * (kThreads / G) + q of the class list.  The loads of the V
// slots are issued level by level -- list entries; vload(v, act) and the row
// bounds; the arc (adj, then nload(u, e)) of every active slot -- before any
// slot is used, so that V dependent chains are in flight together.  use(r,
// ok, v, vv, act, deg, valid, nv) runs per slot r with ok = the slot holds a
// vertex, valid = this lane holds an arc of an active vertex; every lane of
// the workgroup reaches it for every slot (group shuffles are allowed).
template <int G, int V, class CL, class VL, class NL, class U>
__device__ __forceinline__ void group_tiles(const int64_t *xadj, const int32_t *adj,
                                            const CL &cl, int cls, int local, VL vload,
                                            NL nload, U use) {
  constexpr int GPW = kThreads / G;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  const int cnt = cl.off[cls + 1] - cl.off[cls];
  const int32_t *list = cl.list + cl.off[cls];
  int32_t v[V];
  bool ok[V];
#pragma unroll
  for (int r = 0; r < V; ++r) {
    const int idx = (local * V + r) * GPW + grp;
    ok[r] = idx < cnt;
    v[r] = ok[r] ? list[idx] : 0;
  }
  decltype(vload(0, ok[0])) vv[V];
  bool act[V];
  int64_t beg[V];
  int deg[V];
#pragma unroll
  for (int r = 0; r < V; ++r) {
    act[r] = false;
    deg[r] = 0;
    beg[r] = 0;
    if (ok[r]) {
      vv[r] = vload(v[r], act[r]);
      beg[r] = xadj[v[r]];
      deg[r] = (int)(xadj[v[r] + 1] - beg[r]);
    }
  }
  decltype(nload(0, (int64_t)0)) nv[V];
  bool valid[V];
#pragma unroll
  for (int r = 0; r < V; ++r) {
    valid[r] = act[r] && lane < deg[r];
    if (valid[r]) nv[r] = nload(adj[beg[r] + lane], beg[r] + lane);
  }
#pragma unroll
  for (int r = 0; r < V; ++r) use(r, ok[r], v[r], vv[r], act[r], deg[r], valid[r], nv[r]);
}

}  // namespace pm
