// hm.hip -- induced subgraphs of a partition on the GPU (Section 4.1,
// Algorithm 1), for hierarchical multisection.
//
// All blocks are built at once: a stable radix sort of the vertex ids by
// block gives every block's vertices in ascending id order (the local id of
// a vertex is its rank there); per position the number of neighbours in the
// same block, one scan, then every row is emitted in the original neighbour
// order.  No atomics: every output slot has exactly one writer.
#include "device_util.h"
#include "kernels.h"
#include "prim.h"

namespace pm {

static inline unsigned grid_of(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : b);
}

__global__ void k_sub_iota(int32_t n, int32_t *ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ids[i] = (int32_t)i;
}

// vstart[b] = first position of block b (key[] sorted); one writer per b
__global__ void k_sub_starts(int32_t n, int32_t parts, const uint32_t *key, int32_t *vstart) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > n) return;
  const int64_t prev = j > 0 ? (int64_t)key[j - 1] : -1;
  const int64_t cur = j < n ? (int64_t)key[j] : (int64_t)parts;
  for (int64_t b = prev + 1; b <= cur; ++b) vstart[b] = (int32_t)j;
}

__global__ void k_sub_local(int32_t n, const uint32_t *key, const int32_t *order,
                            const int32_t *vstart, int32_t *local) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) local[order[j]] = (int32_t)(j - vstart[key[j]]);
}

// rowcnt[j]: neighbours of order[j] in its block; rowcnt[n] = 0
__global__ void k_sub_rowcnt(DGraph g, const int32_t *part, const uint32_t *key,
                             const int32_t *order, int32_t *rowcnt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > g.n) return;
  if (j == g.n) {
    rowcnt[j] = 0;
    return;
  }
  const int32_t v = order[j];
  const int32_t b = (int32_t)key[j];
  int32_t c = 0;
  for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) c += part[g.adj[e]] == b ? 1 : 0;
  rowcnt[j] = c;
}

__global__ void k_sub_estart(int32_t parts, const int32_t *vstart, const int64_t *G,
                             int64_t *estart) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= parts) estart[b] = G[vstart[b]];
}

// block b's row offsets live at xadj[vstart[b] + b .. vstart[b+1] + b]
__global__ void k_sub_xadj(int32_t n, int32_t parts, const uint32_t *key, const int32_t *vstart,
                           const int64_t *estart, const int64_t *G, int64_t *xadj) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const int32_t b = (int32_t)key[j];
    xadj[j + b] = G[j] - estart[b];
  }
  if (j < parts) xadj[vstart[j + 1] + j] = estart[j + 1] - estart[j];
}

__global__ void k_sub_emit(DGraph g, const int32_t *part, const uint32_t *key,
                           const int32_t *order, const int32_t *local, const int64_t *G,
                           int32_t *adj_out, int32_t *w_out, int32_t *vwgt_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.n) return;
  const int32_t v = order[j];
  const int32_t b = (int32_t)key[j];
  vwgt_out[j] = g.c[v];
  int64_t pos = G[j];
  for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
    const int32_t u = g.adj[e];
    if (part[u] != b) continue;
    adj_out[pos] = local[u];
    w_out[pos] = g.w[e];
    ++pos;
  }
}

// one workgroup per block: the block's vertex weight
__global__ __launch_bounds__(kThreads) void k_sub_weight(const int32_t *vstart,
                                                         const int32_t *vwgt, int64_t *wsum) {
  __shared__ BlockScratch sc;
  const int32_t b = blockIdx.x;
  int64_t x = 0;
  for (int64_t j = vstart[b] + threadIdx.x; j < vstart[b + 1]; j += kThreads) x += vwgt[j];
  x = block_sum64(x, sc);
  if (threadIdx.x == 0) wsum[b] = x;
}

void subgraphs(Arena &ar, const DGraph &g, const int32_t *part, int32_t parts,
               const SubgraphOut &o, hipStream_t s) {
  const int32_t n = g.n;
  uint32_t *key = ar.alloc_n<uint32_t>((size_t)n + 1);
  int32_t *iota = ar.alloc_n<int32_t>((size_t)n + 1);
  int32_t *local = ar.alloc_n<int32_t>((size_t)n + 1);
  int32_t *rowcnt = ar.alloc_n<int32_t>((size_t)n + 1);
  int64_t *G = ar.alloc_n<int64_t>((size_t)n + 1);
  int bits = 1;
  while ((1ll << bits) < (int64_t)parts) ++bits;
  if (n > 0) {
    hipLaunchKernelGGL(k_sub_iota, dim3(grid_of(n)), dim3(kThreads), 0, s, n, iota);
    PM_LAUNCH_CHECK();
    // part is non-negative (checked by the caller): its bits are the keys
    sort_pairs(ar, reinterpret_cast<const uint32_t *>(part), key, iota, o.order, n, bits, s);
  }
  hipLaunchKernelGGL(k_sub_starts, dim3(grid_of((int64_t)n + 1)), dim3(kThreads), 0, s, n, parts,
                     key, o.vstart);
  PM_LAUNCH_CHECK();
  if (n > 0) {
    hipLaunchKernelGGL(k_sub_local, dim3(grid_of(n)), dim3(kThreads), 0, s, n, key, o.order,
                       o.vstart, local);
    PM_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_sub_rowcnt, dim3(grid_of((int64_t)n + 1)), dim3(kThreads), 0, s, g, part,
                     key, o.order, rowcnt);
  PM_LAUNCH_CHECK();
  scan_excl_widen(ar, rowcnt, G, (int64_t)n + 1, s);
  hipLaunchKernelGGL(k_sub_estart, dim3(grid_of((int64_t)parts + 1)), dim3(kThreads), 0, s,
                     parts, o.vstart, G, o.estart);
  PM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sub_xadj, dim3(grid_of(n > parts ? n : parts)), dim3(kThreads), 0, s, n,
                     parts, key, o.vstart, o.estart, G, o.xadj);
  PM_LAUNCH_CHECK();
  if (n > 0) {
    hipLaunchKernelGGL(k_sub_emit, dim3(grid_of(n)), dim3(kThreads), 0, s, g, part, key, o.order,
                       local, G, o.adjncy, o.adjwgt, o.vwgt);
    PM_LAUNCH_CHECK();
  }
  if (o.wsum && parts > 0) {
    hipLaunchKernelGGL(k_sub_weight, dim3(parts), dim3(kThreads), 0, s, o.vstart, o.vwgt, o.wsum);
    PM_LAUNCH_CHECK();
  }
}

__global__ void k_sub_check(const int32_t *part, int32_t n, int32_t parts, int32_t *bad) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && (part[v] < 0 || part[v] >= parts)) atomicOr(bad, 1);
}
void check_parts(const int32_t *part, int32_t n, int32_t parts, int32_t *bad, hipStream_t s) {
  PM_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub_check, dim3(grid_of(n)), dim3(kThreads), 0, s, part, n, parts, bad);
  PM_LAUNCH_CHECK();
}

// out[j] = orig ? orig[order[j]] : order[j]
__global__ void k_sub_compose(int32_t n, const int32_t *orig, const int32_t *order, int32_t *out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = orig ? orig[order[j]] : order[j];
}
void compose_ids(int32_t n, const int32_t *orig, const int32_t *order, int32_t *out,
                 hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub_compose, dim3(grid_of(n)), dim3(kThreads), 0, s, n, orig, order, out);
  PM_LAUNCH_CHECK();
}

// part_out[orig ? orig[v] : v] = base + part[v]
__global__ void k_sub_scatter(int32_t n, const int32_t *orig, const int32_t *part, int32_t base,
                              int32_t *part_out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) part_out[orig ? orig[v] : (int32_t)v] = base + part[v];
}
void scatter_blocks(int32_t n, const int32_t *orig, const int32_t *part, int32_t base,
                    int32_t *part_out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub_scatter, dim3(grid_of(n)), dim3(kThreads), 0, s, n, orig, part, base,
                     part_out);
  PM_LAUNCH_CHECK();
}

}  // namespace pm
