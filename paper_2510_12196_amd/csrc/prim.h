// prim.h -- device-wide scan / select / radix-sort building blocks.
// Thin wrappers over rocPRIM (AMD's device primitive library), compiled in
// their own translation unit; scratch comes from the caller's arena.
#pragma once

#include "pm_internal.h"

namespace pm {

// out[i] = sum_{j<i} in[j]
void scan_excl(Arena &ar, const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
void scan_excl(Arena &ar, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
void scan_excl_widen(Arena &ar, const int32_t *in, int64_t *out, int64_t n, hipStream_t s);
// out[i] = sum_{j<i} vwgt[idx[j]] (int64)
void scan_excl_gather(Arena &ar, const int32_t *idx, const int32_t *vwgt, int64_t *out,
                      int64_t n, hipStream_t s);

// out[i] = max_{j<=i} in[j]
void scan_incl_max(Arena &ar, const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
// out[i] = sum_{j<i, flags[j] != 0} vwgt[j] (int64)
void scan_excl_masked(Arena &ar, const uint8_t *flags, const int32_t *vwgt, int64_t *out,
                      int64_t n, hipStream_t s);

// Stable compaction of the indices i in [0,n) with flags[i] != 0 (ascending).
// *count_dev receives the number selected.
void select_indices(Arena &ar, const uint8_t *flags, int32_t *out, int32_t *count_dev,
                    int64_t n, hipStream_t s);
// The same with flags[i] = flag[list[i]] (a gather through the list).
void select_list_flagged(Arena &ar, const uint8_t *flag, const int32_t *list, int32_t *out,
                         int32_t *count_dev, int64_t n, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
void sort_pairs(Arena &ar, const uint32_t *kin, uint32_t *kout, const int32_t *vin,
                int32_t *vout, int64_t n, int bits, hipStream_t s);
void sort_pairs(Arena &ar, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                int32_t *vout, int64_t n, int bits, hipStream_t s);

}  // namespace pm
