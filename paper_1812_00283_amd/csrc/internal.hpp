// Internal declarations shared by the HIP translation units of libbfc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>
#include <string>

#include "bfc.h"

namespace bfc {

constexpr int kWave = 64;
// Window-boundary tables: entries every 2^kWinShift end ranks, rows for the
// middles of degree >= max(2 x row length, kWinMinDegree).
constexpr int kWinShift = 15;
// Medium heavy starts (256-thread workgroups) have at most this many middles.
constexpr int32_t kMediumMaxPre = 512;
constexpr int32_t kWinMinDegree = 64;
// byte offset of the caterpillar partial sums (64 int64 slots) in a graph's
// info block (past the status words and the schedule totals), and its size
constexpr int kInfoCaterpillars = 192;
// int32 index in the info block of the count status word (bit 0: a counting
// window could not be sized); zeroed by the build, set by the count kernels
// and never cleared, so any later call that waits can report it
constexpr int kInfoCountStatus = 6;
constexpr int kInfoBytes = kInfoCaterpillars + 64 * 8;
// Light starts of at most kSmallMax wedges use the small-table kernel, those
// of at most kLightMidMax the mid-table one, the rest (to light_max) the
// large-table one.
constexpr int32_t kSmallMax = 256;
constexpr int32_t kLightMidMax = 1024;

// ------------------------------------------------------------ errors
struct Error {
  bfc_status status;
  std::string what;
};

void set_error(bfc_status s, const std::string& what);

#define BFC_HIP(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) throw ::bfc::Error{e_ == hipErrorOutOfMemory ? BFC_ERR_OUT_OF_MEMORY \
                                                                       : BFC_ERR_DEVICE,     \
                                             std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define BFC_LAUNCH_CHECK() BFC_HIP(hipGetLastError())

// ------------------------------------------------------------ memory
// Caching device allocator (alloc.hip).  cache_alloc returns a block of at
// least `bytes` on the current device, usable by work queued on `s` from now
// on.  cache_free hands it back once the work queued on `s` so far no longer
// needs it (the block is reused by `s` at once and by other streams after
// that work completes); cache_free_idle when no queued work uses it.  None
// may be called for a stream that is being captured.
void* cache_alloc(size_t bytes, hipStream_t s);
// Installs the source of new blocks (null functions: hipMalloc / hipFree),
// after returning every idle cached block to the allocator that made it.
void set_allocator(bfc_alloc_fn alloc_fn, bfc_free_fn free_fn, void* ctx);
// Returns every idle cached block to its allocator; the bytes freed.
int64_t trim_cache();
// Bytes held in idle cached blocks.
int64_t cached_bytes();
void cache_free(void* p, hipStream_t s);
void cache_free_idle(void* p);
// A pinned host buffer of at least `bytes` owned by the calling thread, for
// read-backs that the thread waits for before its next call.
void* pinned_stage(size_t bytes);

// A device buffer owned by a graph handle.  Work on a handle is ordered
// (each count call waits for the previous one), so a buffer replaced by a
// call on stream s is freed in order on s; the handle's destructor runs
// after all its work has completed.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) cache_free_idle(p);
  }
  void alloc(size_t n, hipStream_t s) {
    if (p) cache_free(p, s);
    p = nullptr;
    bytes = 0;
    if (n == 0) n = 256;
    p = cache_alloc(n, s);
    bytes = n;
  }
  void release(hipStream_t s) {
    if (p) cache_free(p, s);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// A stream-ordered temporary: allocated and freed in order on one stream,
// so it may go out of scope while kernels that use it are still queued.
struct TmpBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  TmpBuf() = default;
  TmpBuf(const TmpBuf&) = delete;
  TmpBuf& operator=(const TmpBuf&) = delete;
  ~TmpBuf() { release(); }
  void alloc(size_t n, hipStream_t stream) {
    release();
    if (n == 0) n = 256;
    s = stream;
    p = cache_alloc(n, s);
    bytes = n;
  }
  void release() {
    if (p) cache_free(p, s);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------ graph
// One layer's side of the relabelled graph: vertices of this layer in
// ascending priority (local rank r), each with its neighbours' local ranks
// in the other layer, ascending (so ascending priority).
struct Side {
  int32_t n = 0;
  DevBuf off;      // int32 [n+1] CSR offsets by local rank
  DevBuf adj;      // int32 [m] neighbour local ranks (other layer)
  DevBuf rev;      // int32 [m] slot of the reverse arc in the other side's adj
  DevBuf lo;       // int32 [n] number of neighbours with lower priority (a prefix of the list)
  DevBuf id_of;    // int32 [n] local rank -> input id
  DevBuf work;     // int64 [n] wedges Algorithm 2 processes from this start
  DevBuf wpp;      // int64 [n] wedges Algorithm 3 processes from this start (computed when first needed)
  // Top band of this layer (tuning top_band): ranks [band_lo, n).  A pair of
  // this layer whose lower vertex lies below the band while the higher one
  // lies in it is counted from the lower vertex with Algorithm 3's wedges
  // into the band; every other pair from its higher vertex with Algorithm
  // 2's wedges, which then end inside the start's own part (band or below).
  int32_t band_lo = 0;  // 0: no band (Algorithm 2's wedges from every start)
  DevBuf band_lb;  // int32 [n of the other layer]: first slot of each other-layer list whose end rank is >= band_lo
  DevBuf wband;    // int64 [n]: Algorithm 2 wedges of each start, ends within its part
  DevBuf wtop;     // int64 [n]: Algorithm 3 wedges from each start below the band into the band
};

struct Schedule {
  int32_t n_light = 0;   // starts counted by one wavefront
  int32_t n_small = 0;   // of those, the first n_small have at most kSmallMax wedges,
  int32_t n_mid = 0;     // the next n_mid at most kLightMidMax, the rest more
  int32_t n_heavy = 0;   // starts counted by one workgroup
  int32_t n_medium = 0;  // of those, the last n_medium use the 256-thread shape
  DevBuf light;          // int4 {code (band item << 31 | side << 30 | rank), off[rank], middles, wedges}
  DevBuf heavy;          // int4 entries as in `light`, by decreasing work
  int64_t wedges = 0;    // |W|
  int32_t max_prefix = 0;
  int64_t wedges_light = 0, wedges_heavy = 0;
  int64_t middles_light = 0, middles_heavy = 0;
  int64_t max_start_wedges = 0;
  int32_t light_max = 0; // thresholds the lists were built with
  int32_t medium_max = 0;
  int32_t vpp = 0;       // bit x: the lists hold Algorithm 3's starts of layer x (entry = {code, off, degree, wedges})
  int32_t band = 0;      // bit x: layer x has a top band (its band items carry code bit 31)
};

struct Tuning {
  int32_t light_max_wedges = 2048;  // used up to light_max_cap()
  int32_t dense_min_ratio = 4;
  int32_t window_mode = 1;  // 1 auto, 2 dense only, 3 hash only
  int32_t hash_window_wedges = 8192;
  int32_t dense_block = 0;
  int32_t dense_min_wedges = 8192;
  int32_t medium_max_wedges = 0;  // 256-thread workgroups measured slower on the degree-skewed workloads
  int32_t vpp = 0;                // bit x: layer x's starts count Algorithm 3's wedges (BFC-VP++), else Algorithm 2's
  int32_t top_band = 0;           // width of each layer's top band of ranks (0: none); layers in vpp take none
};

// Dense block of top-priority vertices (int8 MFMA, see dense.hip).
struct DenseBlock {
  int32_t KU = 0, KL = 0;  // block sizes per layer (0: disabled)
  int32_t PU = 0, PL = 0;  // padded to multiples of 32
  DevBuf buf;              // XU, YU, XL, YL (int8) then CU [PU][PU], CL [PL][PL] (int32)
  int32_t* CU() const { return reinterpret_cast<int32_t*>(buf.as<int8_t>() + 4 * (size_t)PU * (size_t)PL); }
  int32_t* CL() const { return CU() + (size_t)PU * (size_t)PU; }
};

}  // namespace bfc

struct bfc_graph_s {
  int64_t m = 0;
  int32_t n_upper = 0, n_lower = 0;
  bfc::Side side[2];      // 0 = upper layer, 1 = lower layer
  bfc::DevBuf edge0;      // int32 [m] input edge index of each side[0].adj slot
  // window-boundary tables, one per middle layer o: for the ranks
  // v >= wt_first[o] (the vertices of degree >= wt_min_degree), row v holds
  // wt_row[o] slots; entry w is the first slot of N(v) whose end rank is
  // >= w * 2^15 (end ranks are ranks of the other layer)
  bfc::DevBuf wt[2];
  int32_t wt_first[2] = {0, 0};
  int32_t wt_row[2] = {0, 0};
  // batches: graph index of every rank (per layer) and per-graph |W|
  int32_t n_graphs = 1;
  bfc::DevBuf gid[2];
  bfc::DevBuf grank[2];   // per layer: first rank of each graph (G + 1), batches only
  // build status (int32 [10]: [8 + x] the first rank of degree >= 256 in layer x)
  // and schedule totals (int64 [16] from byte 64),
  // the caterpillar partial sums (from byte kInfoCaterpillars), read back once
  // when the build is complete
  bfc::DevBuf info;
  int64_t caterpillars = 0;  // three-paths, sum over edges of (d_u - 1)(d_v - 1)
  // light tables pack (end - first rank of its graph + 1) << 12 | count
  // when every graph's layers have fewer than 2^20 vertices; light starts
  // then go up to 2048 wedges, else 1024
  bool light_packed = false;
  int32_t key_span[2] = {-1, -1};  // largest layer of one graph of a batch (-1: one graph)
  int32_t light_max_cap() const { return light_packed ? 2048 : 1024; }
  int64_t rows_max[2] = {0, 0};  // window-table rows allocated per layer
  // per layer: the vertices of rank below byte_rank have degree < 256, so as
  // ends their counts fit 8-bit dense counters (0 in a batch, whose ranks
  // do not follow degree across graphs)
  int32_t byte_rank[2] = {0, 0};
  int32_t max_deg[2] = {0, 0};   // largest degree per layer
  // per-edge counts accumulate in 32-bit words while every B_e fits:
  // B_e <= (d_u - 1)(d_v - 1) <= (max_deg[0] - 1)(max_deg[1] - 1) < 2^32
  bool edge_acc32() const {
    const uint64_t a = max_deg[0] > 1 ? (uint64_t)(max_deg[0] - 1) : 0;
    const uint64_t b = max_deg[1] > 1 ? (uint64_t)(max_deg[1] - 1) : 0;
    return a * b < (uint64_t(1) << 32);
  }
  std::vector<int64_t> graph_wedges;
  // per-graph settings of a batch (bfc_set_graph_tuning): light_max per
  // graph (int32 [G]) and {dense ratio, window mode, hash window wedges,
  // dense min wedges} per graph (int4 [G]); empty when not set
  bfc::DevBuf glight, gtune;
  // captured total count
  hipGraph_t cap_graph = nullptr;
  hipGraphExec_t cap_exec = nullptr;
  bfc::Schedule sched;
  bfc::Tuning tune;
  bfc::DenseBlock dense;
  bfc::DevBuf scratch;    // per-workgroup cursors and the work ticket of the count kernels
  size_t scratch_bytes = 0;
  bfc::DevBuf acc;        // int64 [2m] per-arc accumulators of the per-edge count (allocated on first use)
  bfc::DevBuf vacc;       // int64 [n_upper + n_lower] per-rank accumulators of the per-vertex count
  int device = 0;
  // count calls share scratch: they are serialised on the device with `done`
  std::mutex mu;
  hipEvent_t done = nullptr;
  hipStream_t last = nullptr;
  bool used = false;
  // optional kernel timing: events around the count kernels of each call
  bool timing = false;
  struct TimedCall { hipEvent_t ev[5]; };
  std::vector<TimedCall> timed;
  int64_t timed_calls = 0;
  double light_ms = 0, heavy_ms = 0, other_ms = 0;
  int64_t device_bytes() const;
};

namespace bfc {

// ------------------------------------------------------------ primitives
// Exclusive prefix sum of n values; `out` may alias `in`.  Returns the
// total through total_dev (device, may be null).
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev, hipStream_t s);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total_dev, hipStream_t s);
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on bits [0, bits).  Sorted
// output ends in keys/vals; tmp buffers must hold n elements.
void radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int bits,
                    hipStream_t s);
void radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int bits,
                    hipStream_t s);
// As radix_sort_u64, but leaves the result where the last pass wrote it:
// returns true when that is (keys_tmp, vals_tmp).
bool radix_sort_u64_any(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int bits,
                        hipStream_t s);
// Keys only, on key bits [lo_bit, lo_bit + bits) (lower bits ride along);
// same return convention.
bool radix_sort_u64_keys_any(uint64_t* keys, uint64_t* keys_tmp, int64_t n, int lo_bit, int bits, hipStream_t s);

// ------------------------------------------------------------ build and count
// groups (batches): per layer, G + 1 device offsets of each graph's ids;
// vertices are then ranked by (graph, degree, id) so each graph's ranks are
// contiguous.
void build_graph(bfc_graph_s* g, const int32_t* edges, hipStream_t s, const int32_t* const* groups = nullptr,
                 int32_t G = 0);
void build_schedule(bfc_graph_s* g, hipStream_t s);
// Wedges Algorithm 3 processes from every start of layer x (int64 [n_x]):
// each neighbour v contributes the part of N(v) above both the start and v.
void vpp_work(const bfc_graph_s* g, int x, int64_t* work, hipStream_t s);
// Waits for the build and schedule queued on s and reads their results
// (throws on a duplicate edge).  The only wait after the degree check.
void finish_schedule(bfc_graph_s* g, hipStream_t s);

enum CountMode { kTotal = 0, kVertex = 1, kEdge = 2 };
// Runs the wedge kernels.  kTotal: adds B_G into total_dev.  kVertex: writes
// per-vertex counts into out0 (upper, by id) and out1 (lower, by id).
// kEdge: writes per-edge counts into out0 (int64 [m]).
// gtotals (kTotal only): per-graph totals [n_graphs] instead of total_dev.
// static_scratch: the kernels' cursors and tickets live in the library's
// fixed device array instead of the handle's scratch (nothing is allocated;
// BFC_ERR_TOO_LARGE when one workgroup's cursors do not fit it).
void count(bfc_graph_s* g, CountMode mode, int64_t* total_dev, int64_t* out0, int64_t* out1, hipStream_t s,
           int64_t* gtotals = nullptr, bool static_scratch = false);
// Size of the fixed scratch array, and the least scratch a count of g needs.
size_t static_scratch_bytes();
size_t min_count_scratch_bytes(const bfc_graph_s* g);
// Batch build: shifts each graph's ids into the union, validates them per
// graph and builds the union; fills gid[] and graph_wedges.
void build_batch(bfc_graph_s* g, const int32_t* edges, const int64_t* eoff_host, const int32_t* nu_host,
                 const int32_t* nl_host, int32_t G, hipStream_t s);
// Allocates the count kernels' scratch for the current schedule on stream s
// (not capture-safe; called when a schedule is built).
void prepare_count(bfc_graph_s* g, hipStream_t s);
// Device status word of the count kernels on this handle (0 = fine): set by
// any count call that failed internally, never cleared.
int32_t* count_status(bfc_graph_s* g);
// Sums the durations of timed count calls (waits for them).
void collect_times(bfc_graph_s* g);
// Dense block: sizes and buffers for the current tuning, and the MFMA
// products for one count call.
void prepare_dense(bfc_graph_s* g, hipStream_t s);
void dense_block(bfc_graph_s* g, hipStream_t s);
// Zero fill by kernel (safe inside captured graphs, unlike a memset node).
void zero_u64(void* p, int64_t n, hipStream_t s);

inline int bits_for(uint64_t x) {
  int b = 0;
  while (b < 64 && (x >> b)) ++b;
  return b < 1 ? 1 : b;
}

inline unsigned grid_for(int64_t n, int per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace bfc
