// Radix-sort entry points (primitives.hip) whose first pass takes its
// per-tile digit counts from the kernel that wrote the keys, so that pass
// needs no histogram kernel of its own.  Used by build.hip.
#pragma once

#include "internal.hpp"

namespace bfc {

// Keys per tile of every radix-sort pass.
constexpr int kSortTileKeys = 4096;

inline int64_t sort_tiles(int64_t n) { return (n + kSortTileKeys - 1) / kSortTileKeys; }

// As radix_sort_u64_keys_any and radix_sort_u64_any, where first_counts
// holds, for tiles = sort_tiles(n), counts[d * tiles + t] = the number of
// keys of tile t (keys [t * kSortTileKeys, (t + 1) * kSortTileKeys) of the
// input) whose bits [lo_bit, lo_bit + 8) equal d (lo_bit 0 for the second
// form).  The buffer is scanned in place.
bool radix_sort_u64_keys_counted(uint64_t* keys, uint64_t* keys_tmp, int64_t n, int lo_bit, int bits,
                                 uint32_t* first_counts, hipStream_t s);
bool radix_sort_u64_counted(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                            int bits, uint32_t* first_counts, hipStream_t s);

}  // namespace bfc
