// batch.cpp -- many mapping instances at once: the batched executor and the
// continuous-batching server.  Both run every instance through map_impl (the
// code path of pm_map) on worker threads that own a HIP stream each, so the
// result of an instance never depends on what runs beside it.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "kernels.h"

namespace pm {
namespace {

using Clock = std::chrono::steady_clock;

int run_job(pm_map_job &job, hipStream_t s) {
  const auto t0 = Clock::now();
  int rc;
  pm_map_stats st;
  try {
    rc = map_impl(&job.graph, &job.hierarchy, job.eps, job.seed, job.part_out, &st, 0, s);
  } catch (const Error &e) {
    (void)hipGetLastError();
    rc = e.code;
  } catch (const std::bad_alloc &) {
    rc = PM_ENOMEM;
  } catch (...) {
    rc = PM_EHIP;
  }
  job.status = rc;
  job.levels = rc >= 0 ? st.levels : 0;
  job.j_final = rc >= 0 ? st.j_final : 0;
  job.ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  return rc;
}

// A worker's stream at default priority, created and destroyed on its thread.
struct WorkerStream {
  hipStream_t s = nullptr;
  explicit WorkerStream(int dev) {
    (void)hipSetDevice(dev);
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      s = nullptr;
    }
  }
  ~WorkerStream() {
    if (s) (void)hipStreamDestroy(s);
  }
};

int64_t footprint(const pm_graph *g, const pm_hierarchy *h) {
  if (!g || !h || g->n < 0 || g->nnz < 0) return -1;
  int bits = 0;
  for (int i = 0; i < h->levels && i < PM_MAX_LEVELS; ++i) {
    int w = 0;
    while ((1 << w) < h->a[i]) ++w;
    bits += w;
  }
  const int64_t codes = int64_t(1) << (bits < kMaxCodeBits ? bits : kMaxCodeBits);
  // coarse levels (at most the input again), sort buffers, refinement state,
  // rebalancing tables; the arena hands out at least one 64 MiB chunk
  const int64_t est = 72 * g->nnz + 128 * (int64_t)g->n +
                      codes * kBuckets * 8 * (kBucketStripes + 1) + (int64_t(8) << 20);
  const int64_t chunk = int64_t(64) << 20;
  return est > chunk ? est : chunk;
}

}  // namespace

// ---------------------------------------------------------------------------
// server
// ---------------------------------------------------------------------------
struct Server {
  struct Req {
    pm_map_job job;
    int64_t fp = 0;
    Clock::time_point submitted;
    double latency_ms = 0.0;
    bool done = false;
  };
  int dev = 0;
  int64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;          // FIFO of tickets not yet admitted
  std::map<int64_t, Req> reqs;
  int64_t next_ticket = 0;
  int64_t in_flight_bytes = 0;
  int64_t running = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  void worker_loop() {
    WorkerStream ws(dev);
    for (;;) {
      int64_t t;
      {
        std::unique_lock<std::mutex> lk(mu);
        // admission: the head of the queue, once its footprint fits
        cv_work.wait(lk, [&] {
          if (queue.empty()) return stop;
          const Req &r = reqs.at(queue.front());
          return in_flight_bytes + r.fp <= budget || running == 0;
        });
        if (queue.empty()) return;  // stop requested and nothing left
        t = queue.front();
        queue.pop_front();
        Req &r = reqs.at(t);
        in_flight_bytes += r.fp;
        ++running;
      }
      pm_map_job job;
      {
        std::lock_guard<std::mutex> lk(mu);
        job = reqs.at(t).job;
      }
      if (ws.s) run_job(job, ws.s);
      else job.status = PM_EHIP;
      {
        std::lock_guard<std::mutex> lk(mu);
        Req &r = reqs.at(t);
        r.job = job;
        r.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.submitted).count();
        r.done = true;
        in_flight_bytes -= r.fp;
        --running;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

}  // namespace pm

using namespace pm;

extern "C" {

int64_t pm_job_footprint(const pm_graph *g, const pm_hierarchy *h) {
  const int64_t f = footprint(g, h);
  return f < 0 ? PM_EINVAL : f;
}

int pm_map_batch(pm_map_job *jobs, int32_t count, int32_t workers, void *stream) {
  if (count < 0 || (count > 0 && !jobs)) return PM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return PM_ENODEVICE;
  }
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
    (void)hipGetLastError();
    return PM_EHIP;
  }
  if (workers <= 0) workers = 8;
  if (workers > count) workers = count > 0 ? count : 1;
  // largest first, so that the long instances do not end the batch alone
  std::vector<int32_t> order(count);
  for (int32_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return jobs[a].graph.nnz + jobs[a].graph.n > jobs[b].graph.nnz + jobs[b].graph.n;
  });
  std::atomic<int32_t> next{0};
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w)
    pool.emplace_back([&] {
      WorkerStream ws(dev);
      for (;;) {
        const int32_t i = next.fetch_add(1);
        if (i >= count) break;
        pm_map_job &job = jobs[order[i]];
        if (ws.s) run_job(job, ws.s);
        else job.status = PM_EHIP;
      }
    });
  for (auto &t : pool) t.join();
  for (int32_t i = 0; i < count; ++i)
    if (jobs[i].status < 0) return jobs[i].status;
  return PM_OK;
}

pm_server *pm_server_create(int64_t hbm_budget_bytes, int32_t workers) {
  if (hbm_budget_bytes <= 0) return nullptr;
  Server *srv = new (std::nothrow) Server();
  if (!srv) return nullptr;
  if (hipGetDevice(&srv->dev) != hipSuccess) {
    (void)hipGetLastError();
    delete srv;
    return nullptr;
  }
  srv->budget = hbm_budget_bytes;
  if (workers <= 0) workers = 8;
  for (int w = 0; w < workers; ++w) srv->workers.emplace_back([srv] { srv->worker_loop(); });
  return reinterpret_cast<pm_server *>(srv);
}

int64_t pm_server_submit(pm_server *s, const pm_map_job *job) {
  Server *srv = reinterpret_cast<Server *>(s);
  if (!srv || !job) return PM_EINVAL;
  const int64_t fp = footprint(&job->graph, &job->hierarchy);
  if (fp < 0) return PM_EINVAL;
  if (fp > srv->budget) return PM_ENOMEM;
  int64_t t;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return PM_EINVAL;
    t = srv->next_ticket++;
    Server::Req &r = srv->reqs[t];
    r.job = *job;
    r.job.status = 0;
    r.fp = fp;
    r.submitted = Clock::now();
    srv->queue.push_back(t);
  }
  srv->cv_work.notify_all();
  return t;
}

int pm_server_poll(pm_server *s, int64_t ticket) {
  Server *srv = reinterpret_cast<Server *>(s);
  if (!srv) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return PM_EINVAL;
  return it->second.done ? 1 : 0;
}

int pm_server_wait(pm_server *s, int64_t ticket, pm_map_job *out, double *latency_ms) {
  Server *srv = reinterpret_cast<Server *>(s);
  if (!srv) return PM_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return PM_EINVAL;
  srv->cv_done.wait(lk, [&] { return it->second.done; });
  if (out) *out = it->second.job;
  if (latency_ms) *latency_ms = it->second.latency_ms;
  const int rc = it->second.job.status;
  srv->reqs.erase(it);
  return rc;
}

void pm_server_destroy(pm_server *s) {
  Server *srv = reinterpret_cast<Server *>(s);
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto &t : srv->workers) t.join();
  delete srv;
}

}  // extern "C"
