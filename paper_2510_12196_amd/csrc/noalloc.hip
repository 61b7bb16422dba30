// noalloc.hip -- J(Pi) without any allocation, for callers that cannot call
// hipMalloc (code under graph capture, tight serving loops, harnesses that
// forbid it).  The per-workgroup partial sums, the error flag and the result
// live in a file-scope device array of fixed size (one copy per device, held
// until the process ends); the caller passes the graph, the mapping and a
// host result slot.
#include <mutex>

#include "device_util.h"
#include "kernels.h"

namespace pm {

constexpr int kNaSlots = 4096;  // workgroup partial sums (the grid never exceeds it)
constexpr int kNaErr = kNaSlots;  // out-of-range block id seen
constexpr int kNaJ = kNaSlots + 1;  // the result
constexpr int kNaWords = kNaSlots + 64;  // 33 280 bytes per device

// The scratch.  In host code its name is a host-side stand-in: kernels get
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) int64_t scratch[kNaWords];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex na_mutex;
int64_t *na_ptr[kNaMaxDevices] = {};

// The device address of scratch on device dev (dev current), looked up once.
int64_t *scratch_on(int dev) {
  if (dev < 0 || dev >= kNaMaxDevices) throw Error(PM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(PM_EHIP, "hipGetSymbolAddress of the scratch array failed");
    }
    na_ptr[dev] = static_cast<int64_t *>(p);
  }
  return na_ptr[dev];
}

// D between two block ids from the prefix products: d_j for the smallest j
// with x / P_j == y / P_j (no codes, no tables).
__device__ __forceinline__ int64_t dist_ids(const Hier &h, uint32_t x, uint32_t y) {
  if (x == y) return 0;
  for (int j = 1; j <= h.levels; ++j) {
    const uint32_t p = (uint32_t)h.P[j];
    if (x / p == y / p) return h.d[j - 1];
  }
  return h.d[h.levels - 1];
}

__global__ void k_na_clear(int64_t *scr) {
  if (threadIdx.x < 2) scr[kNaErr + threadIdx.x] = 0;
}

// J over the arcs of the vertices [0, n): the grid walks chunks of kThreads
// consecutive ids; in a wave the arcs of its 64 vertices are laid end to end
// (an exclusive prefix of their degrees) and the lanes walk that sequence.
// One partial sum per workgroup into scr[blockIdx.x]; a block id outside
// [0, k) sets scr[kNaErr].
__global__ __launch_bounds__(kThreads) void k_na_cost(DGraph g, const int32_t *part, Hier h,
                                                      int64_t *scr) {
  __shared__ BlockScratch sc;
  const int lane = threadIdx.x & 63;
  int64_t x = 0;
  bool bad = false;
  for (int64_t c0 = (int64_t)blockIdx.x * kThreads; c0 < g.n;
       c0 += (int64_t)gridDim.x * kThreads) {
    const int64_t v = c0 + threadIdx.x;
    int32_t deg = 0;
    int64_t beg = 0;
    uint32_t pv = 0;
    if (v < g.n) {
      const int32_t b = part[v];
      bad |= b < 0 || (int64_t)b >= h.k;
      pv = (uint32_t)b;
      beg = g.xadj[v];
      deg = (int32_t)(g.xadj[v + 1] - beg);
    }
    int32_t incl = deg;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int32_t excl = incl - deg;
    const int32_t total = __shfl(incl, 63, 64);
    for (int32_t base = 0; base < total; base += 64) {
      const int32_t idx = base + lane;
      int own = 0;  // the last lane whose arcs start at or before idx
#pragma unroll
      for (int st = 32; st > 0; st >>= 1) {
        const int cand = own + st;
        const int32_t ce = __shfl(excl, cand < 64 ? cand : 63, 64);
        if (cand < 64 && ce <= idx) own = cand;
      }
      const int64_t ob = gshfl64<64>(beg, own);
      const int32_t oe = __shfl(excl, own, 64);
      const uint32_t op = (uint32_t)__shfl((int32_t)pv, own, 64);
      if (idx < total) {
        const int64_t e = ob + (idx - oe);
        const int32_t pu = part[g.adj[e]];
        bad |= pu < 0 || (int64_t)pu >= h.k;
        x += (int64_t)g.w[e] * dist_ids(h, op, (uint32_t)pu);
      }
    }
  }
  x = block_sum64(x, sc);
  if (threadIdx.x == 0) scr[blockIdx.x] = x;
  if (bad) atomicOr((unsigned long long *)&scr[kNaErr], 1ull);
}

// The sum of the partials, in workgroup order.
__global__ __launch_bounds__(kThreads) void k_na_fold(int64_t *scr, int32_t parts) {
  __shared__ BlockScratch sc;
  int64_t x = 0;
  for (int i = threadIdx.x; i < parts; i += kThreads) x += scr[i];
  x = block_sum64(x, sc);
  if (threadIdx.x == 0) scr[kNaJ] = x;
}

}  // namespace
}  // namespace pm

using namespace pm;

extern "C" int pm_comm_cost_noalloc(const pm_graph *g, const pm_hierarchy *h,
                                    const int32_t *part, int64_t *j_out, void *stream) {
  try {
    if (!g || !j_out) return PM_EINVAL;
    if (g->n < 0 || g->nnz < 0) return PM_EINVAL;
    if (g->nnz > INT32_MAX) return PM_EOVERFLOW;
    if (g->n > 0 && (!part || !g->xadj || (g->nnz > 0 && (!g->adjncy || !g->adjwgt))))
      return PM_EINVAL;
    const Hier hh = make_hier(h);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      return PM_ENODEVICE;
    }
    int64_t *scr = scratch_on(dev);
    *j_out = 0;
    if (g->n == 0) return PM_OK;
    hipStream_t s = as_stream(stream);
    const DGraph dg{g->n, g->nnz, g->xadj, g->adjncy, g->adjwgt, g->vwgt};
    const int64_t chunks = (g->n + kThreads - 1) / kThreads;
    const int32_t parts = (int32_t)(chunks < kNaSlots ? chunks : kNaSlots);
    hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(64), 0, s, scr);
    hipLaunchKernelGGL(k_na_cost, dim3((unsigned)parts), dim3(kThreads), 0, s, dg, part, hh, scr);
    hipLaunchKernelGGL(k_na_fold, dim3(1), dim3(kThreads), 0, s, scr, parts);
    if (hipGetLastError() != hipSuccess) return PM_EHIP;
    int64_t res[2] = {0, 0};
    if (hipMemcpyAsync(res, scr + kNaErr, sizeof(res), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      return PM_EHIP;
    }
    if (res[0]) return PM_EINVAL;  // a block id outside [0, k)
    *j_out = res[1];
    return PM_OK;
  } catch (const Error &e) {
    (void)hipGetLastError();
    return e.code;
  } catch (...) {
    return PM_EHIP;
  }
}
