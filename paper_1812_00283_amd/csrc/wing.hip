// k-wing by batched peeling on exact per-edge counts.
//
// Section 1 defines the k-wing of a bipartite graph as its largest subgraph in
// which every edge lies in at least k butterflies, and describes computing it
// from exact per-edge counts (Eq. 8) by removing low-count edges until every
// remaining edge is in at least k butterflies.  Butterfly counts only fall when
// edges go, so an edge below k in any subgraph that contains the k-wing is not
// in the k-wing: all of them can leave together.  Each round therefore counts
// every remaining edge exactly (the per-edge path of Algorithm 2), drops every
// edge below k in one stable compaction and rebuilds the relabelled graph of
// the rest; the first round in which no edge is below k leaves the k-wing and
// its counts.  One read-back per round (the number of kept edges) decides
// whether to go on.
#include "wing.hpp"

namespace bfc {
namespace {

__global__ void wing_iota_kernel(int32_t* id, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    id[i] = (int32_t)i;
}

__global__ void wing_clear_kernel(uint8_t* in_wing, int64_t* counts, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    in_wing[i] = 0;
    if (counts) counts[i] = 0;
  }
}

__global__ void wing_keep_kernel(const int64_t* __restrict__ cnt, int64_t n, int64_t k, int32_t* __restrict__ keep) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keep[i] = cnt[i] >= k ? 1 : 0;
}

// pos: exclusive prefix sum of the keep flags, so kept edges keep their order
__global__ void wing_compact_kernel(const int2* __restrict__ e, const int32_t* __restrict__ id,
                                    const int64_t* __restrict__ cnt, const int32_t* __restrict__ pos, int64_t n,
                                    int64_t k, int2* __restrict__ e_out, int32_t* __restrict__ id_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (cnt[i] >= k) {
      const int32_t p = pos[i];
      e_out[p] = e[i];
      id_out[p] = id[i];
    }
  }
}

__global__ void wing_result_kernel(const int32_t* __restrict__ id, const int64_t* __restrict__ cnt, int64_t n,
                                   uint8_t* __restrict__ in_wing, int64_t* __restrict__ counts) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = id[i];
    in_wing[j] = 1;
    if (counts) counts[j] = cnt[i];
  }
}

unsigned grid_of(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Owns one round's graph handle; on an early exit it waits for the work
// queued on the handle's stream before freeing it.
struct GraphHold {
  bfc_graph_s* g = nullptr;
  hipStream_t s = nullptr;
  ~GraphHold() {
    if (g) (void)hipStreamSynchronize(s);
    reset();
  }
  void reset() {
    if (g) delete_idle_graph(g);
    g = nullptr;
  }
};

}  // namespace

void k_wing(const int32_t* edges, int64_t m, int32_t n_upper, int32_t n_lower, int64_t k, hipStream_t s,
            uint8_t* in_wing, int64_t* counts, int64_t* wing_edges, int32_t* rounds) {
  *wing_edges = 0;
  *rounds = 0;
  check_graph_args(edges, m, n_upper, n_lower);
  if (m > 0) {
    wing_clear_kernel<<<grid_of(m), 256, 0, s>>>(in_wing, counts, m);
    BFC_LAUNCH_CHECK();
  }
  // edges and input indices of the remaining graph, in two ping-pong pairs;
  // the first round reads the caller's edges
  TmpBuf ebuf[2], ibuf[2], cnt, pos, total;
  const int64_t cap = m > 0 ? m : 1;
  ibuf[0].alloc(cap * sizeof(int32_t), s);
  cnt.alloc(cap * sizeof(int64_t), s);
  pos.alloc((cap + 1) * sizeof(int32_t), s);
  total.alloc(sizeof(int32_t), s);
  if (m > 0) {
    wing_iota_kernel<<<grid_of(m), 256, 0, s>>>(ibuf[0].as<int32_t>(), m);
    BFC_LAUNCH_CHECK();
  }
  const int32_t* cur_e = edges;
  int cur = 0;
  int64_t n = m;
  GraphHold hold;
  hold.s = s;
  while (n > 0) {
    hold.g = new_graph(cur_e, n, n_upper, n_lower, s);
    count(hold.g, kEdge, nullptr, cnt.as<int64_t>(), nullptr, s);
    ++*rounds;
    wing_keep_kernel<<<grid_of(n), 256, 0, s>>>(cnt.as<int64_t>(), n, k, pos.as<int32_t>());
    BFC_LAUNCH_CHECK();
    exclusive_scan_i32(pos.as<int32_t>(), pos.as<int32_t>(), n, total.as<int32_t>(), s);
    int32_t kept = 0, st = 0;
    BFC_HIP(hipMemcpyAsync(&kept, total.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipMemcpyAsync(&st, count_status(hold.g), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    if (st) throw Error{BFC_ERR_DEVICE, "internal error: a counting window could not be sized"};
    hold.reset();
    if (kept == n) break;  // every remaining edge is in at least k butterflies
    const int nxt = cur ^ 1;
    if (!ebuf[nxt].p) ebuf[nxt].alloc(cap * sizeof(int2), s);
    if (!ibuf[nxt].p) ibuf[nxt].alloc(cap * sizeof(int32_t), s);
    wing_compact_kernel<<<grid_of(n), 256, 0, s>>>(reinterpret_cast<const int2*>(cur_e), ibuf[cur].as<int32_t>(),
                                                   cnt.as<int64_t>(), pos.as<int32_t>(), n, k,
                                                   ebuf[nxt].as<int2>(), ibuf[nxt].as<int32_t>());
    BFC_LAUNCH_CHECK();
    cur = nxt;
    cur_e = ebuf[cur].as<int32_t>();
    n = kept;
  }
  if (n > 0) {
    wing_result_kernel<<<grid_of(n), 256, 0, s>>>(ibuf[cur].as<int32_t>(), cnt.as<int64_t>(), n, in_wing, counts);
    BFC_LAUNCH_CHECK();
  }
  BFC_HIP(hipStreamSynchronize(s));
  *wing_edges = n;
}

}  // namespace bfc
