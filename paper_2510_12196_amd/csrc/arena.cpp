// arena.cpp -- per-call scratch memory for the process-mapping library.
#include <cstring>
#include <map>

#include "pm_internal.h"

namespace pm {

static constexpr size_t kAlign = 256;
static constexpr size_t kMinChunk = size_t(64) << 20;

Arena::~Arena() { release(); }

void Arena::release() {
  for (auto &c : chunks_) (void)hipFree(c.ptr);
  chunks_.clear();
  top_ = 0;
  if (host_) (void)hipHostFree(host_);
  host_ = nullptr;
  host_size_ = 0;
  if (mapped_) (void)hipHostFree(mapped_);
  mapped_ = nullptr;
  mapped_dev_ = nullptr;
}

void *Arena::host_mapped(void **dev_view) {
  if (!mapped_) {
    void *p = nullptr;
    if (hipHostMalloc(&p, kMappedBytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(PM_ENOMEM, "hipHostMalloc of mapped status memory failed");
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(p);
      throw Error(PM_EHIP, "hipHostGetDevicePointer failed");
    }
    std::memset(p, 0, kMappedBytes);
    mapped_ = p;
    mapped_dev_ = d;
  }
  *dev_view = mapped_dev_;
  return mapped_;
}

void *Arena::alloc(size_t bytes) {
  bytes = bytes ? (bytes + kAlign - 1) & ~(kAlign - 1) : kAlign;
  for (auto &c : chunks_) {
    if (top_ >= c.base && top_ < c.base + c.size) {
      if (top_ + bytes <= c.base + c.size) {
        void *p = c.ptr + (top_ - c.base);
        top_ += bytes;
        return p;
      }
      top_ = c.base + c.size;  // the tail of this chunk stays unused
    }
  }
  size_t base = chunks_.empty() ? 0 : chunks_.back().base + chunks_.back().size;
  size_t total = base;
  size_t size = bytes > kMinChunk ? bytes : kMinChunk;
  if (size < total / 2) size = (total / 2 + kAlign - 1) & ~(kAlign - 1);
  char *p = nullptr;
  if (hipMalloc(&p, size) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(PM_ENOMEM, "hipMalloc of scratch memory failed");
  }
  chunks_.push_back({p, size, base});
  top_ = base + bytes;
  return p;
}

void Arena::rewind(size_t m) {
  if (m < top_) top_ = m;
}

void *Arena::host_stage(size_t bytes) {
  if (bytes > host_size_) {
    if (host_) (void)hipHostFree(host_);
    host_ = nullptr;
    size_t sz = bytes < 4096 ? 4096 : bytes;
    if (hipHostMalloc(&host_, sz, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      host_size_ = 0;
      throw Error(PM_ENOMEM, "hipHostMalloc of staging memory failed");
    }
    host_size_ = sz;
  }
  return host_;
}

namespace {
std::mutex g_pool_mutex;
std::map<int, std::vector<Arena *>> g_free;   // idle arenas per device
std::vector<Arena *> g_all;                   // every arena ever made
}  // namespace

ArenaLease::ArenaLease(hipStream_t s) : s_(s) {
  int dev = 0;
  PM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  auto &fl = g_free[dev];
  if (!fl.empty()) {
    arena_ = fl.back();
    fl.pop_back();
  } else {
    arena_ = new Arena(dev);
    g_all.push_back(arena_);
  }
  arena_->reset();
}

ArenaLease::~ArenaLease() {
  if (hipStreamSynchronize(s_) != hipSuccess) (void)hipGetLastError();
  arena_->reset();
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  g_free[arena_->device()].push_back(arena_);
}

void release_all_arenas() {
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : g_free) {
    (void)hipSetDevice(kv.first);
    for (Arena *a : kv.second) a->release();
  }
  (void)hipSetDevice(cur);
}

}  // namespace pm
