// Sort-based total count (sorted.hip), used by api.hip.
#pragma once

#include "internal.hpp"

namespace bfc {

// B_G of a built graph by Algorithm 6's pair sort over the wedges of
// Algorithm 2 (direction 0) or Algorithm 3 (direction 1), in chunks of at
// most max_pairs pairs (<= 0: 2^31) plus one start's wedges.  Waits on s.
void count_total_sorted(bfc_graph_s* g, int direction, int64_t max_pairs, hipStream_t s, int64_t* total_host,
                        int64_t* pairs_host, int64_t* chunks_host);

}  // namespace bfc
