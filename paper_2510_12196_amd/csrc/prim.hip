// prim.hip -- device-wide scan / select / radix sort via rocPRIM.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "prim.h"

namespace pm {
namespace {

template <class F>
void run_two_phase(Arena &ar, F f) {
  size_t bytes = 0;
  PM_HIP(f(nullptr, bytes));
  size_t m = ar.mark();
  void *tmp = ar.alloc(bytes ? bytes : 1);
  PM_HIP(f(tmp, bytes));
  ar.rewind(m);  // later work on the same stream runs after this one
}

struct GatherWeight {
  const int32_t *vwgt;
  __host__ __device__ int64_t operator()(int32_t v) const { return (int64_t)vwgt[v]; }
};

struct MaskedWeight {
  const uint8_t *flags;
  const int32_t *vwgt;
  __host__ __device__ int64_t operator()(int32_t i) const {
    return flags[i] ? (int64_t)vwgt[i] : 0;
  }
};

struct Widen {
  __host__ __device__ int64_t operator()(int32_t x) const { return (int64_t)x; }
};

// flag of the vertex at position i of a list
struct ListFlag {
  const uint8_t *flag;
  const int32_t *list;
  __host__ __device__ uint8_t operator()(int32_t i) const { return flag[list[i]]; }
};

}  // namespace

void scan_excl(Arena &ar, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::exclusive_scan(t, b, in, out, int32_t(0), (size_t)n,
                                   rocprim::plus<int32_t>(), s);
  });
}

void scan_excl(Arena &ar, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::exclusive_scan(t, b, in, out, int64_t(0), (size_t)n,
                                   rocprim::plus<int64_t>(), s);
  });
}

void scan_excl_widen(Arena &ar, const int32_t *in, int64_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  auto it = rocprim::make_transform_iterator(in, Widen{});
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::exclusive_scan(t, b, it, out, int64_t(0), (size_t)n,
                                   rocprim::plus<int64_t>(), s);
  });
}

void scan_excl_gather(Arena &ar, const int32_t *idx, const int32_t *vwgt, int64_t *out,
                      int64_t n, hipStream_t s) {
  if (n <= 0) return;
  auto it = rocprim::make_transform_iterator(idx, GatherWeight{vwgt});
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::exclusive_scan(t, b, it, out, int64_t(0), (size_t)n,
                                   rocprim::plus<int64_t>(), s);
  });
}

void scan_incl_max(Arena &ar, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::inclusive_scan(t, b, in, out, (size_t)n, rocprim::maximum<int32_t>(), s);
  });
}

void scan_excl_masked(Arena &ar, const uint8_t *flags, const int32_t *vwgt, int64_t *out,
                      int64_t n, hipStream_t s) {
  if (n <= 0) return;
  auto it = rocprim::make_transform_iterator(rocprim::counting_iterator<int32_t>(0),
                                             MaskedWeight{flags, vwgt});
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::exclusive_scan(t, b, it, out, int64_t(0), (size_t)n,
                                   rocprim::plus<int64_t>(), s);
  });
}

void select_indices(Arena &ar, const uint8_t *flags, int32_t *out, int32_t *count_dev,
                    int64_t n, hipStream_t s) {
  if (n <= 0) {
    PM_HIP(hipMemsetAsync(count_dev, 0, sizeof(int32_t), s));
    return;
  }
  rocprim::counting_iterator<int32_t> ids(0);
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::select(t, b, ids, flags, out, count_dev, (size_t)n, s);
  });
}

void select_list_flagged(Arena &ar, const uint8_t *flag, const int32_t *list, int32_t *out,
                         int32_t *count_dev, int64_t n, hipStream_t s) {
  if (n <= 0) {
    PM_HIP(hipMemsetAsync(count_dev, 0, sizeof(int32_t), s));
    return;
  }
  rocprim::counting_iterator<int32_t> ids(0);
  rocprim::transform_iterator<rocprim::counting_iterator<int32_t>, ListFlag, uint8_t> fl(
      ids, ListFlag{flag, list});
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::select(t, b, ids, fl, out, count_dev, (size_t)n, s);
  });
}

void sort_pairs(Arena &ar, const uint32_t *kin, uint32_t *kout, const int32_t *vin,
                int32_t *vout, int64_t n, int bits, hipStream_t s) {
  if (n <= 0) return;
  if (bits < 1) bits = 1;
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::radix_sort_pairs(t, b, kin, kout, vin, vout, (size_t)n, 0u,
                                     (unsigned)bits, s);
  });
}

void sort_pairs(Arena &ar, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                int32_t *vout, int64_t n, int bits, hipStream_t s) {
  if (n <= 0) return;
  if (bits < 1) bits = 1;
  run_two_phase(ar, [&](void *t, size_t &b) {
    return rocprim::radix_sort_pairs(t, b, kin, kout, vin, vout, (size_t)n, 0u,
                                     (unsigned)bits, s);
  });
}

}  // namespace pm
