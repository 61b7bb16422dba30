// timer.cpp -- optional per-launch device timing of selected kernels.
#include "kernels.h"

namespace pm {

thread_local KernelTimer *tl_timer = nullptr;

void KernelTimer::pair(int id, hipEvent_t &a, hipEvent_t &b) {
  PM_HIP(hipEventCreate(&a));
  PM_HIP(hipEventCreate(&b));
  start[id].push_back(a);
  stop[id].push_back(b);
}

void KernelTimer::finish(int64_t *launches, double *ms, double *bytes_out) {
  for (int id = 0; id < NKT; ++id) {
    double sum = 0.0;
    for (size_t i = 0; i < start[id].size(); ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, start[id][i], stop[id][i]) == hipSuccess) sum += t;
    }
    launches[id] = (int64_t)start[id].size();
    ms[id] = sum;
    bytes_out[id] = bytes[id];
  }
}

KernelTimer::~KernelTimer() {
  for (int id = 0; id < NKT; ++id) {
    for (auto e : start[id]) (void)hipEventDestroy(e);
    for (auto e : stop[id]) (void)hipEventDestroy(e);
  }
}

}  // namespace pm
