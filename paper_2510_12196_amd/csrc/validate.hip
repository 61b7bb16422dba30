// validate.hip -- input checks: weight totals (always) and CSR structure
// (with PM_FLAG_VALIDATE).
#include "device_util.h"
#include "kernels.h"

namespace pm {

struct Checks {
  unsigned long long vsum;      // sum of vertex weights
  unsigned long long esum;      // sum of arc weights
  int32_t bad_vwgt;             // vertex weight <= 0
  int32_t bad_ewgt;             // arc weight <= 0
  int32_t bad_xadj;             // offsets not monotone / wrong ends
  int32_t bad_adj;              // neighbour out of range or self loop
  int32_t bad_sym;              // reverse arc missing or weight differs
  int32_t pad_;
};

__global__ void k_check_weights(DGraph g, Checks *c) {
  unsigned long long vs = 0, es = 0;
  int32_t bv = 0, be = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
    const int32_t x = g.c[v];
    if (x <= 0) ++bv;
    else vs += (unsigned long long)x;
  }
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.nnz; e += stride) {
    const int32_t x = g.w[e];
    if (x <= 0) ++be;
    else es += (unsigned long long)x;
  }
  __shared__ BlockScratch sc;
  const int64_t tv = block_sum64((int64_t)vs, sc);
  const int64_t te = block_sum64((int64_t)es, sc);
  const int64_t tb = block_sum64((int64_t)bv + ((int64_t)be << 32), sc);
  if (threadIdx.x == 0) {
    if (tv) atomicAdd(&c->vsum, (unsigned long long)tv);
    if (te) atomicAdd(&c->esum, (unsigned long long)te);
    if (tb & 0xffffffffll) atomicAdd(&c->bad_vwgt, (int32_t)(tb & 0xffffffffll));
    if (tb >> 32) atomicAdd(&c->bad_ewgt, (int32_t)(tb >> 32));
  }
}

// offsets, ranges, self loops, and symmetry by a search of the reverse arc
// (linear in the neighbour's degree; only under PM_FLAG_VALIDATE)
__global__ void k_check_structure(DGraph g, Checks *c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
    const int64_t b = g.xadj[v], e = g.xadj[v + 1];
    if (b < 0 || b > e || e > g.nnz || (v == 0 && b != 0) || (v == g.n - 1 && e != g.nnz)) {
      atomicAdd(&c->bad_xadj, 1);
      continue;
    }
    for (int64_t i = b; i < e; ++i) {
      const int32_t u = g.adj[i];
      if (u < 0 || u >= g.n || u == v) {
        atomicAdd(&c->bad_adj, 1);
        continue;
      }
      const int64_t ub = g.xadj[u], ue = g.xadj[u + 1];
      bool found = false;
      if (ub <= ue && ub >= 0 && ue <= g.nnz)
        for (int64_t j = ub; j < ue; ++j)
          if (g.adj[j] == (int32_t)v) {
            found = g.w[j] == g.w[i];
            break;
          }
      if (!found) atomicAdd(&c->bad_sym, 1);
    }
  }
}

void validate_graph(Arena &ar, const DGraph &g, bool full, int64_t *total_vwgt, hipStream_t s) {
  const size_t m = ar.mark();
  Checks *c = ar.alloc_n<Checks>(1);
  PM_HIP(hipMemsetAsync(c, 0, sizeof(Checks), s));
  const int64_t big = g.n > g.nnz ? g.n : g.nnz;
  unsigned grid = (unsigned)((big + kThreads - 1) / kThreads);
  if (grid < 1) grid = 1;
  if (grid > 512) grid = 512;
  if (g.n > 0 || g.nnz > 0) {
    hipLaunchKernelGGL(k_check_weights, dim3(grid), dim3(kThreads), 0, s, g, c);
    PM_LAUNCH_CHECK();
  }
  if (full && g.n > 0) {
    // xadj ends are needed before walking rows
    int64_t ends[2] = {0, 0};
    PM_HIP(hipMemcpyAsync(&ends[0], g.xadj, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipMemcpyAsync(&ends[1], g.xadj + g.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != g.nnz) throw Error(PM_EGRAPH, "xadj[0] != 0 or xadj[n] != nnz");
    unsigned gs = (unsigned)((g.n + kThreads - 1) / kThreads);
    if (gs > 4096) gs = 4096;
    hipLaunchKernelGGL(k_check_structure, dim3(gs), dim3(kThreads), 0, s, g, c);
    PM_LAUNCH_CHECK();
  }
  Checks h{};
  PM_HIP(hipMemcpyAsync(&h, c, sizeof(Checks), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  ar.rewind(m);
  if (h.bad_vwgt || h.bad_ewgt) throw Error(PM_EGRAPH, "non-positive vertex or edge weight");
  if (h.bad_xadj || h.bad_adj || h.bad_sym) throw Error(PM_EGRAPH, "malformed CSR");
  if (h.vsum > (unsigned long long)INT32_MAX) throw Error(PM_EOVERFLOW, "sum of vertex weights");
  if (h.esum > (unsigned long long)INT32_MAX) throw Error(PM_EOVERFLOW, "sum of edge weights");
  *total_vwgt = (int64_t)h.vsum;
}

}  // namespace pm
