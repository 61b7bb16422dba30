// pm_internal.h -- shared definitions of the gfx950 process-mapping library.
//
// Block ids inside the library are "codes": the mixed-radix digits of a PE id
// (digit i in [0, a_i), a_1 least significant) packed into bit fields of
// width ceil(log2 a_i).  The packing keeps the order of ids, and two PEs share
// their level-j component (Section 2, hierarchy H = a_1:...:a_l) iff their
// codes agree above bit shift[j].  The distance D(x,y) of the hierarchical
// process-mapping problem then depends only on the bit length of x ^ y:
// D = d_j for the smallest j with bitlen(x ^ y) <= shift[j], and 0 if x == y.
// When every a_i is a power of two, code == id.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "pm.h"

namespace pm {

constexpr int kMaxCodeBits = 13;     // LDS histograms hold 2^13 entries
constexpr int kThreads = 256;        // threads per workgroup
constexpr int64_t kNotInX = INT64_MIN;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

#define PM_HIP(expr)                                                         \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::pm::Error(PM_EHIP, std::string(#expr) + ": " +                 \
                                     hipGetErrorString(e_));                 \
  } while (0)

#define PM_LAUNCH_CHECK() PM_HIP(hipGetLastError())

// Hierarchy as passed to kernels (by value, lives in kernel arguments).
struct Hier {
  int32_t levels;
  int32_t bits;                        // shift[levels]
  int32_t pow2;                        // all a_i powers of two (code == id)
  int32_t pad_;
  int64_t k;                           // number of PEs
  int32_t shift[PM_MAX_LEVELS + 1];    // shift[0] = 0, cumulative bit widths
  int32_t d[PM_MAX_LEVELS];
  int32_t a[PM_MAX_LEVELS];
  int64_t P[PM_MAX_LEVELS + 1];        // prefix products, P[0] = 1
};

Hier make_hier(const pm_hierarchy *h);  // throws Error(PM_EINVAL/EOVERFLOW)

__host__ __device__ inline int32_t dist(const Hier &h, uint32_t x, uint32_t y) {
  uint32_t z = x ^ y;
  if (z == 0) return 0;
  int32_t len = 32 - __builtin_clz(z);
  int32_t D = h.d[0];
  for (int j = 1; j < h.levels; ++j)
    if (len > h.shift[j]) D = h.d[j];
  return D;
}

__host__ __device__ inline uint32_t id_to_code(const Hier &h, int64_t id) {
  uint32_t c = 0;
  for (int i = 0; i < h.levels; ++i) {
    int64_t digit = (id / h.P[i]) % h.a[i];
    c |= (uint32_t)digit << h.shift[i];
  }
  return c;
}

__host__ __device__ inline int32_t code_to_id(const Hier &h, uint32_t c) {
  int64_t id = 0;
  for (int i = 0; i < h.levels; ++i) {
    uint32_t width = (uint32_t)(h.shift[i + 1] - h.shift[i]);
    uint32_t digit = width ? (c >> h.shift[i]) & ((1u << width) - 1u) : 0u;
    id += (int64_t)digit * h.P[i];
  }
  return (int32_t)id;
}

// A code is valid iff every digit is below its a_i.
__host__ __device__ inline bool code_valid(const Hier &h, uint32_t c) {
  if (c >> h.bits) return false;
  for (int i = 0; i < h.levels; ++i) {
    uint32_t width = (uint32_t)(h.shift[i + 1] - h.shift[i]);
    uint32_t digit = width ? (c >> h.shift[i]) & ((1u << width) - 1u) : 0u;
    if (digit >= (uint32_t)h.a[i]) return false;
  }
  return true;
}

// The (word+1)-th output of a splitmix64 stream started at `seed`
// (Steele, Lea, Flood, OOPSLA 2014): a counter-based hash.
__host__ __device__ inline uint64_t mix_hash(uint64_t seed, uint64_t word) {
  uint64_t z = seed + (word + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kTagMatch = 0x48454D31ull;
constexpr uint64_t kTagRebalance = 0x5245424Cull;
constexpr uint64_t kTagTwin = 0x5457494Eull;

// Graph view (device pointers).
struct DGraph {
  int32_t n;
  int64_t nnz;
  const int64_t *xadj;
  const int32_t *adj;
  const int32_t *w;
  const int32_t *c;
};

// Degree classes: vertices are processed by groups of G lanes (one arc per
// lane) when deg <= G (G = 8, 16, 32, 64), by one wave with up to
// kWaveMaxDeg / 64 arcs per lane when deg <= kWaveMaxDeg (W), by a whole
// workgroup otherwise (BIG).  The enumeration order is the launch order of
// the class tiles: the longest tiles (high degree) start first, so that they
// overlap with the rest.
enum { CLS_BIG = 0, CLS_W, CLS_G64, CLS_G32, CLS_G16, CLS_G8, CLS_ISO, NCLS };
constexpr int kWaveMaxDeg = 512;
constexpr int kWaveMinCount = 8192;  // fewer W vertices: they go to BIG
constexpr int32_t kHemCompactMinN = 1 << 18;  // matching rounds tile only active vertices
constexpr int32_t kRebCompactMinN = 1 << 19;  // rebalancing tiles only overloaded blocks
constexpr int32_t kContractRowsMinNnz = 1 << 20;  // row-local contraction from this many arcs
constexpr int32_t kContractRowsLongPct = 100;     // ... while rows above 64 hold <= this % of them
constexpr int kHemRoundsPerRead = 4;  // matching rounds between status read-backs (small levels)

// Process-wide launch parameters (pm_set_tuning); read at each call.
struct TuningValues {
  int32_t group_v, wave_min_count, hem_compact_min_n, reb_compact_min_n, contract_rows_min_nnz,
      contract_rows_long_pct, lp_cache, graph_bodies;
};
TuningValues tuning();
void set_tuning(const TuningValues &t);
__host__ __device__ constexpr int class_group(int cls) {
  return cls == CLS_G8 ? 8 : cls == CLS_G16 ? 16 : cls == CLS_G32 ? 32
       : (cls == CLS_G64 || cls == CLS_W) ? 64 : 1;
}
// vertices handled by one workgroup in each class
__host__ __device__ constexpr int class_per_wg(int cls) {
  return cls == CLS_BIG ? 1 : cls == CLS_ISO ? kThreads : kThreads / class_group(cls);
}

struct Classes {
  const int32_t *list;        // all n vertices, grouped by class, id order inside
  int32_t off[NCLS + 1];      // class c occupies list[off[c] .. off[c+1])
  int32_t wg[NCLS + 1];       // workgroup prefix: class c uses blocks wg[c]..wg[c+1)
};

// ---------------------------------------------------------------------------
// Scratch memory: a stack arena over hipMalloc'd chunks, one per call.
// ---------------------------------------------------------------------------
class Arena {
 public:
  explicit Arena(int device) : device_(device) {}
  ~Arena();
  void *alloc(size_t bytes);
  template <class T> T *alloc_n(size_t n) { return static_cast<T *>(alloc(n * sizeof(T))); }
  size_t mark() const { return top_; }
  void rewind(size_t m);    // frees everything allocated after mark m
  void reset() { rewind(0); }
  void release();           // returns all chunks to HIP
  int device() const { return device_; }
  // pinned host staging for small read-backs
  void *host_stage(size_t bytes);
  // Coherent host memory mapped into the device (kMappedBytes): kernels store
  // into it through *dev_view; the host reads it while they run.
  static constexpr size_t kMappedBytes = 4096;
  void *host_mapped(void **dev_view);
  int64_t next_publish() { return ++publish_seq_; }
  int64_t publish_seq() const { return publish_seq_; }

 private:
  struct Chunk { char *ptr; size_t size; size_t base; };
  int device_;
  std::vector<Chunk> chunks_;
  size_t top_ = 0;          // global offset over concatenated chunks
  void *host_ = nullptr;
  size_t host_size_ = 0;
  void *mapped_ = nullptr;
  void *mapped_dev_ = nullptr;
  int64_t publish_seq_ = 0;
};

// Acquire an arena for the current device for the duration of a call whose
// work runs on stream s.  On release (also when the call throws) the stream
// is synchronised first, so no queued kernel still writes into the arena when
// another call leases it.
class ArenaLease {
 public:
  explicit ArenaLease(hipStream_t s);
  ~ArenaLease();
  ArenaLease(const ArenaLease &) = delete;
  ArenaLease &operator=(const ArenaLease &) = delete;
  Arena &operator*() { return *arena_; }
  Arena *operator->() { return arena_; }
 private:
  Arena *arena_;
  hipStream_t s_;
};

// Events that are destroyed with their owner (also on an exception).
struct EventSet {
  std::vector<hipEvent_t> ev;
  hipEvent_t make() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(PM_EHIP, "hipEventCreate failed");
    }
    ev.push_back(e);
    return e;
  }
  ~EventSet() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

void release_all_arenas();

// Stream helper
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace pm
