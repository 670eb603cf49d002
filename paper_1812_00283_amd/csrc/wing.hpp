// Declarations shared by api.hip and wing.hip (k-wing peeling).
#pragma once

#include "internal.hpp"

namespace bfc {

// bfc_build's argument checks (sizes, null edges, more edges than pairs);
// throws Error.  They touch no device state.
void check_graph_args(const int32_t* edges, int64_t m, int32_t n_upper, int32_t n_lower);
// A graph handle built from device edges with bfc_build's checks and steps
// (throws Error: invalid argument, id out of range, duplicate edge, ...).
bfc_graph_s* new_graph(const int32_t* edges, int64_t m, int32_t n_upper, int32_t n_lower, hipStream_t s);
// Frees a handle whose queued work has completed.
void delete_idle_graph(bfc_graph_s* g);

// The k-wing of the input graph: in_wing[i] (uint8) and counts[i] (int64,
// may be null) for every input edge; returns the wing's edge count and the
// number of count rounds.  Waits on s.
void k_wing(const int32_t* edges, int64_t m, int32_t n_upper, int32_t n_lower, int64_t k, hipStream_t s,
            uint8_t* in_wing, int64_t* counts, int64_t* wing_edges, int32_t* rounds);

}  // namespace bfc
