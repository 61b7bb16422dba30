// timer.cpp -- optional per-launch device timing and unit counts of selected
// kernels.
#include <cstring>
#include <mutex>

#include "kernels.h"

namespace pm {

thread_local KernelTimer *tl_timer = nullptr;

namespace {

// Events of finished timers are kept for the next ones: creating an event
// costs far more host time than recording one, and timed maps launch
// hundreds of timed kernels.
std::mutex pool_mutex;
std::vector<std::pair<int, hipEvent_t>> pool;  // (device, event)

hipEvent_t take_event() {
  int dev = 0;
  PM_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lock(pool_mutex);
    for (size_t i = pool.size(); i-- > 0;)
      if (pool[i].first == dev) {
        hipEvent_t e = pool[i].second;
        pool[i] = pool.back();
        pool.pop_back();
        return e;
      }
  }
  hipEvent_t e = nullptr;
  PM_HIP(hipEventCreate(&e));
  return e;
}

void give_events(std::vector<hipEvent_t> &evs) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    for (auto e : evs) (void)hipEventDestroy(e);
    evs.clear();
    return;
  }
  std::lock_guard<std::mutex> lock(pool_mutex);
  for (auto e : evs) pool.emplace_back(dev, e);
  evs.clear();
}

constexpr int kCountStride = 16;  // int64 words between counters (one cache line)
constexpr size_t kCountWords = (size_t)NKT * 3 * kCountStripes * kCountStride;

// Algorithmic bytes of kernel id from its units (tiled vertices, active
// vertices, arcs of the active vertices), as documented in pm.h.
double algorithmic_bytes(int id, const int64_t *u) {
  const double nt = (double)u[0], na = (double)u[1], ar = (double)u[2];
  switch (id) {
    case KT_LP1: return 12.0 * ar + 25.0 * nt;
    case KT_LP2: return 24.0 * ar + 16.0 * na + 9.0 * nt;
    case KT_APPLY: return 16.0 * ar + 24.0 * na;
    case KT_HEM: return 12.0 * ar + 12.0 * nt;
    default: return 12.0 * ar + 24.0 * na;  // KT_REB
  }
}
}  // namespace

void KernelTimer::pair(int id, hipEvent_t &a, hipEvent_t &b) {
  a = b = nullptr;
  if (!timing) return;
  a = take_event();
  start[id].push_back(a);
  b = take_event();
  stop[id].push_back(b);
}

int64_t *KernelTimer::counters(int id) {
  if (!counting) return nullptr;
  if (!dcount) {
    PM_HIP(hipMalloc(&dcount, kCountWords * sizeof(int64_t)));
    PM_HIP(hipMemset(dcount, 0, kCountWords * sizeof(int64_t)));
  }
  return dcount + (size_t)id * 3 * kCountStripes * kCountStride;
}

void KernelTimer::finish(int64_t *launches, double *ms, double *bytes_out, int64_t (*units)[3]) {
  std::vector<int64_t> h;
  if (dcount) {
    h.resize(kCountWords);
    PM_HIP(hipMemcpy(h.data(), dcount, kCountWords * sizeof(int64_t), hipMemcpyDeviceToHost));
  }
  for (int id = 0; id < NKT; ++id) {
    double sum = 0.0;
    for (size_t i = 0; i < start[id].size(); ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, start[id][i], stop[id][i]) == hipSuccess) sum += t;
    }
    launches[id] = (int64_t)start[id].size();
    ms[id] = sum;
    int64_t u[3] = {0, 0, 0};
    if (dcount)
      for (int j = 0; j < 3; ++j)
        for (int st = 0; st < kCountStripes; ++st)
          u[j] += h[(((size_t)id * 3 + j) * kCountStripes + st) * kCountStride];
    for (int j = 0; j < 3; ++j) units[id][j] = u[j];
    bytes_out[id] = dcount ? algorithmic_bytes(id, u) : 0.0;
  }
}

KernelTimer::~KernelTimer() {
  // (a call that ends normally has synchronised its stream; after an error an
  // event may still be pending, and recording it again replaces that record)
  for (int id = 0; id < NKT; ++id) {
    give_events(start[id]);
    give_events(stop[id]);
  }
  if (dcount) (void)hipFree(dcount);
}

}  // namespace pm
