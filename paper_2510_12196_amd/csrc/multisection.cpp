// multisection.cpp -- hierarchical multisection on the GPU (Section 4.1,
// Algorithm 2): split the graph into a_l blocks with the adaptive imbalance
// of equation (2), build the induced subgraphs, split each into a_{l-1}
// blocks, and so on down to a_1.  The graph partitioner is the multilevel
// mapper itself with the one-level hierarchy (a_i) and d = 1, for which J is
// twice the edge cut.
//
// The recursion runs breadth first: every subgraph of one hierarchy level is
// an independent instance, and the instances of a level run concurrently on
// worker threads that own a stream each.  All subgraphs of a level sit in
// level-wide arrays (positions in block order, arcs in row order), so a
// subgraph is a view (offsets) into them and the next level's subgraphs of
// one instance land in the slice of the instance that produced them.
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "kernels.h"

namespace pm {

int64_t adaptive_eps_ppm(int64_t eps_ppm, int64_t kp, int64_t k, int64_t cv, int64_t cvp,
                         int32_t d) {
  if (cvp <= 0 || d <= 0) return eps_ppm;
  const double eps = (double)eps_ppm / 1e6;
  const double base = ((1.0 + eps) * (double)kp) * (double)cv / ((double)k * (double)cvp);
  const double e = std::pow(base, 1.0 / (double)d) - 1.0;
  const int64_t ppm = (int64_t)std::llround(e * 1e6);
  return ppm > 0 ? ppm : 0;
}

namespace {

// One subgraph: a view into its level's arrays.
struct Task {
  int32_t n = 0;
  int64_t nnz = 0;
  const int64_t *xadj = nullptr;  // relative to adj
  const int32_t *adj = nullptr, *w = nullptr, *c = nullptr;
  const int32_t *orig = nullptr;  // input vertex id per vertex (nullptr: identity)
  int64_t base = 0;               // first block of this subgraph's range
  int64_t cvp = 0;                // vertex weight
  int64_t voff = 0, eoff = 0;     // position of its vertices / arcs in the level
};

struct Streams {
  std::vector<hipStream_t> s;
  Streams(int count) {
    for (int i = 0; i < count; ++i) {
      hipStream_t x = nullptr;
      if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(PM_EHIP, "stream creation failed");
      }
      s.push_back(x);
    }
  }
  ~Streams() {
    for (auto x : s) (void)hipStreamDestroy(x);
  }
};

}  // namespace

int hm_impl(const DGraph &dg, const int32_t *a, int32_t levels, double eps, uint64_t seed,
            int32_t *part_out, int32_t workers, int32_t *calls_out, hipStream_t s,
            const Variants &var) {
  if (calls_out) *calls_out = 0;
  if (levels < 1 || levels > PM_MAX_LEVELS) throw Error(PM_EINVAL, "bad hierarchy depth");
  int64_t k = 1;
  for (int i = 0; i < levels; ++i) {
    if (a[i] < 1) throw Error(PM_EINVAL, "hierarchy factor below 1");
    k *= a[i];
    if (k > (int64_t(1) << kMaxCodeBits)) throw Error(PM_EOVERFLOW, "too many blocks");
  }
  if (!(eps >= 0.0) || eps > 1e6) throw Error(PM_EINVAL, "bad imbalance");
  const int64_t eps_ppm = (int64_t)std::llround(eps * 1e6);
  if (dg.n == 0) return PM_OK;
  if (!part_out) throw Error(PM_EINVAL, "NULL output");
  int dev = 0;
  PM_HIP(hipGetDevice(&dev));

  ArenaLease lease(s);  // level-wide arrays of every level
  Arena &ar = *lease;
  int64_t cv = 0;
  validate_graph(ar, dg, false, &cv, s);
  PM_HIP(hipStreamSynchronize(s));

  if (workers <= 0) workers = 8;
  Streams pool(workers);

  std::vector<Task> tasks(1);
  tasks[0].n = dg.n;
  tasks[0].nnz = dg.nnz;
  tasks[0].xadj = dg.xadj;
  tasks[0].adj = dg.adj;
  tasks[0].w = dg.w;
  tasks[0].c = dg.c;
  tasks[0].cvp = cv;
  const int64_t level_nnz = dg.nnz;
  const int32_t n = dg.n;
  int32_t status = PM_OK;
  int32_t calls = 0;

  for (int i = levels; i >= 1; --i) {
    const int32_t ai = a[i - 1];
    int64_t kp = 1;
    for (int j = 0; j < i; ++j) kp *= a[j];
    const int64_t pstride = kp / ai;  // P_{i-1}
    const int64_t T = (int64_t)tasks.size();
    int32_t *part = ar.alloc_n<int32_t>(n);
    // next level's arrays (i > 1)
    int32_t *vstart = nullptr, *order = nullptr, *adj = nullptr, *wgt = nullptr, *vw = nullptr,
            *orig = nullptr;
    int64_t *estart = nullptr, *xadj = nullptr, *wsum = nullptr;
    if (i > 1) {
      vstart = ar.alloc_n<int32_t>(T * (ai + 1));
      estart = ar.alloc_n<int64_t>(T * (ai + 1));
      wsum = ar.alloc_n<int64_t>(T * ai);
      order = ar.alloc_n<int32_t>(n);
      orig = ar.alloc_n<int32_t>(n);
      xadj = ar.alloc_n<int64_t>(n + T * ai);
      adj = ar.alloc_n<int32_t>(level_nnz);
      wgt = ar.alloc_n<int32_t>(level_nnz);
      vw = ar.alloc_n<int32_t>(n);
    }
    std::vector<int32_t> rc(T, PM_OK);
    std::atomic<int64_t> next{0};
    auto run = [&](hipStream_t ws) {
      (void)hipSetDevice(dev);
      for (;;) {
        const int64_t t = next.fetch_add(1);
        if (t >= T) break;
        const Task &tk = tasks[t];
        try {
          const int64_t ppm = adaptive_eps_ppm(eps_ppm, kp, k, cv, tk.cvp, i);
          pm_graph pg{};
          pg.n = tk.n;
          pg.nnz = tk.nnz;
          pg.xadj = tk.xadj;
          pg.adjncy = tk.adj;
          pg.adjwgt = tk.w;
          pg.vwgt = tk.c;
          pm_hierarchy h1{};
          h1.levels = 1;
          h1.a[0] = ai;
          h1.d[0] = 1;
          int32_t *pt = part + tk.voff;
          rc[t] = map_impl(&pg, &h1, (double)ppm / 1e6, seed, pt, nullptr, 0, ws, var);
          if (i == 1) {
            scatter_blocks(tk.n, tk.orig, pt, (int32_t)tk.base, part_out, ws);
            PM_HIP(hipStreamSynchronize(ws));
          } else {
            ArenaLease tmp(ws);
            const DGraph g{tk.n, tk.nnz, tk.xadj, tk.adj, tk.w, tk.c};
            SubgraphOut o{vstart + t * (ai + 1), estart + t * (ai + 1), order + tk.voff,
                          xadj + tk.voff + t * ai, adj + tk.eoff, wgt + tk.eoff, vw + tk.voff,
                          wsum + t * ai};
            subgraphs(*tmp, g, pt, ai, o, ws);
            compose_ids(tk.n, tk.orig, order + tk.voff, orig + tk.voff, ws);
            PM_HIP(hipStreamSynchronize(ws));
          }
        } catch (const Error &e) {
          (void)hipGetLastError();
          rc[t] = e.code;
        } catch (const std::bad_alloc &) {
          rc[t] = PM_ENOMEM;
        } catch (...) {
          rc[t] = PM_EHIP;
        }
      }
    };
    const int nw = (int)std::min<int64_t>(workers, T);
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w) th.emplace_back(run, pool.s[w]);
    for (auto &x : th) x.join();
    calls += (int32_t)T;
    for (int64_t t = 0; t < T; ++t) {
      if (rc[t] < 0) throw Error(rc[t], "subgraph partitioning failed");
      if (rc[t] > status) status = rc[t];
    }
    if (i == 1) break;

    // children, in block order within each instance (empty ones dropped:
    // they have nothing to place)
    std::vector<int32_t> hv(T * (ai + 1));
    std::vector<int64_t> he(T * (ai + 1)), hw(T * ai);
    PM_HIP(hipMemcpyAsync(hv.data(), vstart, sizeof(int32_t) * hv.size(), hipMemcpyDeviceToHost, s));
    PM_HIP(hipMemcpyAsync(he.data(), estart, sizeof(int64_t) * he.size(), hipMemcpyDeviceToHost, s));
    PM_HIP(hipMemcpyAsync(hw.data(), wsum, sizeof(int64_t) * hw.size(), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    std::vector<Task> kids;
    for (int64_t t = 0; t < T; ++t) {
      const Task &tk = tasks[t];
      for (int32_t b = 0; b < ai; ++b) {
        const int32_t v0 = hv[t * (ai + 1) + b], v1 = hv[t * (ai + 1) + b + 1];
        const int64_t e0 = he[t * (ai + 1) + b], e1 = he[t * (ai + 1) + b + 1];
        if (v1 == v0) continue;
        Task c;
        c.n = v1 - v0;
        c.nnz = e1 - e0;
        c.xadj = xadj + tk.voff + t * ai + v0 + b;
        c.adj = adj + tk.eoff + e0;
        c.w = wgt + tk.eoff + e0;
        c.c = vw + tk.voff + v0;
        c.orig = orig + tk.voff + v0;
        c.base = tk.base + (int64_t)b * pstride;
        c.cvp = hw[t * ai + b];
        c.voff = tk.voff + v0;
        c.eoff = tk.eoff + e0;
        kids.push_back(c);
      }
    }
    tasks.swap(kids);
  }
  if (calls_out) *calls_out = calls;
  return status;
}

}  // namespace pm
