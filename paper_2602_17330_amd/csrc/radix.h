// Device-wide stable LSD radix sort of 64-bit records and an exclusive scan of 32-bit counts.
#pragma once

#include "common.h"

namespace subquad {

constexpr int kRadixBits = 8;
constexpr int kRadixBuckets = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // records per block

// Scratch bytes for sorting up to n_cap records.
size_t radix_scratch_bytes(int64_t n_cap);

// Stable sort of records [0, n) of `a` by bits [lo_bit, lo_bit + key_bits) using `b` as the
// second buffer.  n = n_cap, or min(*n_dev, n_cap) when n_dev is non-null (read on the
// device, so the call never synchronises).  *result receives a or b: the sorted buffer.
// few_live: the device count is expected to be zero or small against a large capacity, so
// the passes launch few blocks that loop over the tiles (cheap when empty, slower when full).
int radix_sort_u64(uint64_t *a, uint64_t *b, int64_t n_cap, const int64_t *n_dev, int lo_bit,
                   int key_bits, void *scratch, size_t scratch_bytes, hipStream_t st,
                   uint64_t **result, const char *tag = "radix", bool few_live = false);

// In-place exclusive prefix sum of `count` 32-bit values (sum must fit in 32 bits).
size_t scan_scratch_bytes(int64_t count);
int scan_exclusive_u32(uint32_t *data, int64_t count, void *scratch, hipStream_t st);

// In-place exclusive prefix sum of 64-bit values; the count of values is read from
// count_dev when non-null (bounded by count_cap).
size_t scan64_scratch_bytes(int64_t count_cap);
int scan_exclusive_u64(uint64_t *data, int64_t count_cap, const uint64_t *count_dev, void *scratch, hipStream_t st);

}  // namespace subquad
