// twohop.hip -- two-hop matching (leaf, twin and relative categories) that
// follows heavy-edge matching while 75 % or fewer of the vertices are matched
// (Section 4.2, Matching).  Every category forms groups of unmatched vertices
// -- leaves by their only neighbour, twins by their neighbourhood, relatives
// by a common "matchmaker" neighbour of smallest (degree, id) -- and pairs
// the members of each group in id order.
#include "device_util.h"
#include "kernels.h"
#include "prim.h"

namespace pm {

static inline unsigned grid_for(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

struct TwoHopArgs {
  DGraph g;
  Classes cl;
  int32_t mode;       // TWOHOP_LEAF / TWOHOP_TWIN / TWOHOP_RELATIVE
  uint64_t tseed;     // twin neighbourhood hash seed
  const int32_t *match;
  uint64_t *key;
  uint8_t *flag;
};

// (degree << 32 | id) of u: the matchmaker is the neighbour minimising it
__device__ __forceinline__ uint64_t mm_code(const DGraph &g, int32_t u) {
  return ((uint64_t)(g.xadj[u + 1] - g.xadj[u]) << 32) | (uint32_t)u;
}

__device__ __forceinline__ void th_write(const TwoHopArgs &A, int32_t v, bool f, uint64_t k) {
  A.flag[v] = f ? 1 : 0;
  if (f) A.key[v] = k;
}

template <int G>
__device__ __forceinline__ void th_group(const TwoHopArgs &A, int cls, int local) {
  int32_t v;
  if (!group_vertex<G>(A.cl, cls, local, v)) return;
  const int lane = threadIdx.x % G;
  const int64_t beg = A.g.xadj[v];
  const int deg = (int)(A.g.xadj[v + 1] - beg);
  const bool free_v = A.match[v] < 0;
  if (!free_v || (A.mode == TWOHOP_LEAF && deg != 1)) {
    if (lane == 0) A.flag[v] = 0;
    return;
  }
  const int32_t u = lane < deg ? A.g.adj[beg + lane] : -1;
  if (A.mode == TWOHOP_LEAF) {
    if (lane == 0) th_write(A, v, true, (uint64_t)(uint32_t)u);
  } else if (A.mode == TWOHOP_TWIN) {
    const int64_t h = gsum64<G>(u >= 0 ? (int64_t)mix_hash(A.tseed, (uint64_t)(uint32_t)u) : 0);
    if (lane == 0) th_write(A, v, true, mix_hash((uint64_t)h, (uint64_t)deg));
  } else {
    int64_t m = u >= 0 ? (int64_t)mm_code(A.g, u) : INT64_MAX;
#pragma unroll
    for (int s = G / 2; s > 0; s >>= 1) {
      const int64_t o = gxor64<G>(m, s);
      m = o < m ? o : m;
    }
    if (lane == 0) th_write(A, v, true, (uint64_t)(uint32_t)(m & 0xffffffffll));
  }
}

struct MinScratch {
  int64_t m[kThreads / 64];
};

__global__ __launch_bounds__(kThreads) void k_twohop_keys(TwoHopArgs A) {
  __shared__ BlockScratch sc;
  __shared__ MinScratch ms;
  const int cls = find_class(A.cl, blockIdx.x);
  const int local = blockIdx.x - A.cl.wg[cls];
  switch (cls) {
    case CLS_ISO: {
      const int idx = local * kThreads + threadIdx.x;
      if (idx < A.cl.off[CLS_ISO + 1] - A.cl.off[CLS_ISO]) {
        const int32_t v = A.cl.list[A.cl.off[CLS_ISO] + idx];
        // isolated vertices are twins of each other (empty neighbourhood)
        const bool f = A.mode == TWOHOP_TWIN && A.match[v] < 0;
        th_write(A, v, f, mix_hash(0, 0));
      }
      break;
    }
    case CLS_G8: th_group<8>(A, cls, local); break;
    case CLS_G16: th_group<16>(A, cls, local); break;
    case CLS_G32: th_group<32>(A, cls, local); break;
    case CLS_G64: th_group<64>(A, cls, local); break;
    case CLS_W: {
      int32_t v;
      if (!w_vertex(A.cl, local, v)) break;
      const int lane = threadIdx.x & 63;
      if (A.match[v] >= 0 || A.mode == TWOHOP_LEAF) {  // degree > 64: never a leaf
        if (lane == 0) A.flag[v] = 0;
        break;
      }
      const int64_t beg = A.g.xadj[v], end = A.g.xadj[v + 1];
      if (A.mode == TWOHOP_TWIN) {
        int64_t h = 0;
        for (int64_t e = beg + lane; e < end; e += 64)
          h += (int64_t)mix_hash(A.tseed, (uint64_t)(uint32_t)A.g.adj[e]);
        h = gsum64<64>(h);
        if (lane == 0) th_write(A, v, true, mix_hash((uint64_t)h, (uint64_t)(end - beg)));
      } else {
        int64_t m = INT64_MAX;
        for (int64_t e = beg + lane; e < end; e += 64) {
          const int64_t c = (int64_t)mm_code(A.g, A.g.adj[e]);
          m = c < m ? c : m;
        }
        for (int sh = 32; sh > 0; sh >>= 1) {
          const int64_t o = gxor64<64>(m, sh);
          m = o < m ? o : m;
        }
        if (lane == 0) th_write(A, v, true, (uint64_t)(uint32_t)(m & 0xffffffffll));
      }
      break;
    }
    default: {
      const int32_t v = A.cl.list[A.cl.off[CLS_BIG] + local];
      if (A.match[v] >= 0 || A.mode == TWOHOP_LEAF) {  // degree > 64: never a leaf
        if (threadIdx.x == 0) A.flag[v] = 0;
        break;
      }
      const int64_t beg = A.g.xadj[v], end = A.g.xadj[v + 1];
      if (A.mode == TWOHOP_TWIN) {
        int64_t h = 0;
        for (int64_t e = beg + threadIdx.x; e < end; e += kThreads)
          h += (int64_t)mix_hash(A.tseed, (uint64_t)(uint32_t)A.g.adj[e]);
        h = block_sum64(h, sc);
        if (threadIdx.x == 0) th_write(A, v, true, mix_hash((uint64_t)h, (uint64_t)(end - beg)));
      } else {
        int64_t m = INT64_MAX;
        for (int64_t e = beg + threadIdx.x; e < end; e += kThreads) {
          const int64_t c = (int64_t)mm_code(A.g, A.g.adj[e]);
          m = c < m ? c : m;
        }
        for (int s = 32; s > 0; s >>= 1) {
          const int64_t o = gxor64<64>(m, s);
          m = o < m ? o : m;
        }
        if ((threadIdx.x & 63) == 0) ms.m[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
          int64_t b = ms.m[0];
          for (int i = 1; i < kThreads / 64; ++i) b = ms.m[i] < b ? ms.m[i] : b;
          th_write(A, v, true, (uint64_t)(uint32_t)(b & 0xffffffffll));
        }
      }
      break;
    }
  }
}

__global__ void k_gather_u64(int32_t m, const int32_t *list, const uint64_t *key, uint64_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = key[list[i]];
}

// run starts: head index for the first element of every run of equal keys
__global__ void k_run_heads(int32_t m, const uint64_t *key, int32_t *head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) head[i] = (i == 0 || key[i] != key[i - 1]) ? (int32_t)i : 0;
}

// pairs the 1st and 2nd, 3rd and 4th, ... member of every run
__global__ __launch_bounds__(kThreads) void k_pair_runs(int32_t m, const uint64_t *key,
                                                        const int32_t *ids,
                                                        const int32_t *runstart,
                                                        const int32_t *vwgt, int64_t lmax,
                                                        int32_t *match, int64_t *stripes) {
  __shared__ BlockScratch sc;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t paired = 0;
  if (i + 1 < m && ((i - runstart[i]) & 1) == 0 && key[i + 1] == key[i]) {
    const int32_t a = ids[i], b = ids[i + 1];
    if ((int64_t)vwgt[a] + vwgt[b] <= lmax) {
      match[a] = b;
      match[b] = a;
      paired = 2;
    }
  }
  paired = block_sum64(paired, sc);
  if (threadIdx.x == 0) stripe_add(stripes, paired);
}

int64_t two_hop_step(Arena &ar, const DGraph &g, const Classes &cl, int mode, uint64_t tseed,
                     int64_t lmax, int32_t *match, int64_t *stripes, Status *st_dev,
                     Status *st_host, hipStream_t s) {
  const int64_t n = g.n;
  const unsigned nwg = classed_grid(cl);
  if (n <= 0 || nwg == 0) return 0;
  const size_t mark = ar.mark();
  uint64_t *key = ar.alloc_n<uint64_t>(n);
  uint8_t *flag = ar.alloc_n<uint8_t>(n);
  int32_t *list = ar.alloc_n<int32_t>(n);
  int32_t *ids = ar.alloc_n<int32_t>(n);
  uint64_t *skey = ar.alloc_n<uint64_t>(n);
  uint64_t *skey2 = ar.alloc_n<uint64_t>(n);
  int32_t *head = ar.alloc_n<int32_t>(n);
  int32_t *runstart = ar.alloc_n<int32_t>(n);
  TwoHopArgs A{g, cl, mode, tseed, match, key, flag};
  hipLaunchKernelGGL(k_twohop_keys, dim3(nwg), dim3(kThreads), 0, s, A);
  PM_LAUNCH_CHECK();
  select_indices(ar, flag, list, &st_dev->count, n, s);
  PM_HIP(hipMemcpyAsync(&st_host->count, &st_dev->count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  const int32_t m = st_host->count;
  int64_t added = 0;
  if (m >= 2) {
    hipLaunchKernelGGL(k_gather_u64, dim3(grid_for(m)), dim3(kThreads), 0, s, m, list, key, skey);
    PM_LAUNCH_CHECK();
    int bits = 64;
    if (mode != TWOHOP_TWIN) {
      bits = 1;
      while (bits < 63 && (int64_t(1) << bits) < n) ++bits;
    }
    sort_pairs(ar, skey, skey2, list, ids, m, bits, s);
    hipLaunchKernelGGL(k_run_heads, dim3(grid_for(m)), dim3(kThreads), 0, s, m, skey2, head);
    PM_LAUNCH_CHECK();
    scan_incl_max(ar, head, runstart, m, s);
    hipLaunchKernelGGL(k_pair_runs, dim3(grid_for(m)), dim3(kThreads), 0, s, m, skey2, ids,
                       runstart, g.c, lmax, match, stripes);
    PM_LAUNCH_CHECK();
    fold_stripes(stripes, &st_dev->aux, nullptr, s);
    PM_HIP(hipMemcpyAsync(&st_host->aux, &st_dev->aux, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    added = st_host->aux;
  }
  ar.rewind(mark);
  return added;
}

}  // namespace pm
