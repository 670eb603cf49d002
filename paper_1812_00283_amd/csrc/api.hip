// C-ABI entry points of libbfc (declared in include/bfc.h).
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "sorted.hpp"
#include "wing.hpp"

namespace {
thread_local std::string g_last_error;
}

namespace bfc {

void set_error(bfc_status, const std::string& what) { g_last_error = what; }

namespace {

template <typename F>
bfc_status guard(F&& f) {
  g_last_error.clear();
  try {
    f();
    return BFC_OK;
  } catch (const Error& e) {
    set_error(e.status, e.what);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error(BFC_ERR_OUT_OF_MEMORY, "host allocation failed");
    return BFC_ERR_OUT_OF_MEMORY;
  } catch (...) {
    set_error(BFC_ERR_DEVICE, "unexpected internal error");
    return BFC_ERR_DEVICE;
  }
}

// Restores the caller's current device on scope exit.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) BFC_HIP(hipSetDevice(dev));
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void zero_i64(int64_t* p, int64_t n, hipStream_t s) { zero_u64(p, n, s); }


bfc_graph_s* checked(bfc_graph g) {
  if (!g) throw Error{BFC_ERR_INVALID_ARGUMENT, "null graph handle"};
  return g;
}

}  // namespace
}  // namespace bfc

int64_t bfc_graph_s::device_bytes() const {
  int64_t b = 0;
  for (int x = 0; x < 2; ++x) {
    const bfc::Side& s = side[x];
    b += s.off.bytes + s.adj.bytes + s.rev.bytes + s.lo.bytes + s.id_of.bytes + s.work.bytes + s.wpp.bytes +
         s.band_lb.bytes + s.wband.bytes + s.wtop.bytes;
  }
  b += edge0.bytes + wt[0].bytes + wt[1].bytes + sched.light.bytes + sched.heavy.bytes + scratch.bytes + acc.bytes +
       vacc.bytes;
  return b;
}

namespace {

// Orders this count call after the previous one on the handle when the
// streams differ, and records its completion for the next one.
struct CountSection {
  bfc_graph_s* g;
  hipStream_t s;
  std::unique_lock<std::mutex> hold;
  bool capturing = false;
  CountSection(bfc_graph_s* h, hipStream_t stream) : g(h), s(stream), hold(h->mu) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    BFC_HIP(hipStreamIsCapturing(s, &cs));
    capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && g->used && g->last != s) BFC_HIP(hipStreamWaitEvent(s, g->done, 0));
  }
  void finish() {
    if (capturing) return;
    BFC_HIP(hipEventRecord(g->done, s));
    g->last = s;
    g->used = true;
  }
};

}  // namespace

namespace bfc {

void check_graph_args(const int32_t* edges_dev, int64_t m, int32_t n_upper, int32_t n_lower) {
  if (m < 0 || n_upper < 0 || n_lower < 0) throw Error{BFC_ERR_INVALID_ARGUMENT, "negative size"};
  if (m > 0 && !edges_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "edges_dev is null"};
  if (m >= (int64_t(1) << 30) || n_upper >= (1 << 30) || n_lower >= (1 << 30))
    throw Error{BFC_ERR_TOO_LARGE, "m and each layer size must be below 2^30"};
  if (m > (int64_t)n_upper * (int64_t)n_lower)
    throw Error{BFC_ERR_DUPLICATE_EDGE, "more edges than (upper, lower) pairs: some pair repeats"};
}

bfc_graph_s* new_graph(const int32_t* edges_dev, int64_t m, int32_t n_upper, int32_t n_lower, hipStream_t s) {
  check_graph_args(edges_dev, m, n_upper, n_lower);
  bfc_graph_s* g = new bfc_graph_s();
  try {
    BFC_HIP(hipGetDevice(&g->device));
    BFC_HIP(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
    g->m = m;
    g->n_upper = n_upper;
    g->n_lower = n_lower;
    build_graph(g, edges_dev, s);
    build_schedule(g, s);
    finish_schedule(g, s);
    prepare_count(g, s);
  } catch (...) {
    // let queued build work finish before its buffers return to the cache
    (void)hipStreamSynchronize(s);
    (void)hipGetLastError();
    if (g->done) (void)hipEventDestroy(g->done);
    delete g;
    throw;
  }
  return g;
}

void delete_idle_graph(bfc_graph_s* g) {
  if (g->done) (void)hipEventDestroy(g->done);
  delete g;
}

}  // namespace bfc

using namespace bfc;

extern "C" {

const char* bfc_last_error(void) { return g_last_error.c_str(); }

const char* bfc_version(void) { return "bfc-mi355x 0.1 (gfx950)"; }

int64_t bfc_estimate_device_bytes(int64_t m, int32_t n_upper, int32_t n_lower) {
  if (m < 0 || n_upper < 0 || n_lower < 0) return 0;
  const int64_t n = (int64_t)n_upper + n_lower;
  // resident: 2 sides x (adj + rev) + edge0 + per-vertex arrays and the two
  // start lists (16 bytes per vertex each) + window tables (at most 2 bytes
  // per edge each)
  const int64_t resident = m * 4 * 5 + m * 4 + n * (4 + 4 + 4 + 8 + 32) + 2 * 4 * (int64_t)2 + 4096;
  // build peak: resident + sort buffers (2 x (8 + 4) bytes per edge) + slots
  const int64_t build_peak = resident + m * (24 + 8) + n * 16;
  // per-edge and per-vertex counting: 2 accumulators per edge, 1 per vertex
  const int64_t edge_peak = resident + m * 16 + n * 8;
  return build_peak > edge_peak ? build_peak : edge_peak;
}

bfc_status bfc_build(const int32_t* edges_dev, int64_t m, int32_t n_upper, int32_t n_lower, void* stream,
                     bfc_graph* out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!out) throw Error{BFC_ERR_INVALID_ARGUMENT, "out is null"};
    *out = new_graph(edges_dev, m, n_upper, n_lower, static_cast<hipStream_t>(stream));
  });
}

bfc_status bfc_count_total(bfc_graph g, void* stream, int64_t* total_host, int64_t* wedges_host) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!total_host) throw Error{BFC_ERR_INVALID_ARGUMENT, "total_host is null"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    TmpBuf tot;
    tot.alloc(sizeof(int64_t), s);
    {
      CountSection cs(h, s);
      zero_i64(tot.as<int64_t>(), 1, s);
      count(h, kTotal, tot.as<int64_t>(), nullptr, nullptr, s);
      cs.finish();
    }
    int64_t* rb = static_cast<int64_t*>(pinned_stage(2 * sizeof(int64_t)));
    BFC_HIP(hipMemcpyAsync(rb, tot.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipMemcpyAsync(rb + 1, count_status(h), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    const int64_t v = rb[0];
    const int32_t st = *reinterpret_cast<const int32_t*>(rb + 1);
    if (st) throw Error{BFC_ERR_DEVICE, "internal error: a counting window could not be sized (counts are inexact)"};
    *total_host = v;
    if (wedges_host) *wedges_host = h->sched.wedges;
  });
}

bfc_status bfc_build_batch(const int32_t* edges_dev, const int64_t* edge_offsets_host, const int32_t* n_upper_host,
                           const int32_t* n_lower_host, int32_t G, void* stream, bfc_graph* out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!out || !edge_offsets_host || !n_upper_host || !n_lower_host || G < 1)
      throw Error{BFC_ERR_INVALID_ARGUMENT, "null batch description or G < 1"};
    if (edge_offsets_host[0] != 0) throw Error{BFC_ERR_INVALID_ARGUMENT, "edge_offsets[0] must be 0"};
    const int64_t m = edge_offsets_host[G];
    if (m < 0) throw Error{BFC_ERR_INVALID_ARGUMENT, "negative edge count"};
    if (m > 0 && !edges_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "edges_dev is null"};
    if (m >= (int64_t(1) << 30)) throw Error{BFC_ERR_TOO_LARGE, "total edges must be below 2^30"};
    hipStream_t s = static_cast<hipStream_t>(stream);
    bfc_graph_s* g = new bfc_graph_s();
    try {
      BFC_HIP(hipGetDevice(&g->device));
      BFC_HIP(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
      build_batch(g, edges_dev, edge_offsets_host, n_upper_host, n_lower_host, G, s);
      build_schedule(g, s);
      finish_schedule(g, s);
      prepare_count(g, s);
    } catch (...) {
      // let queued build work finish before its buffers return to the cache
      (void)hipStreamSynchronize(s);
      (void)hipGetLastError();
      if (g->done) (void)hipEventDestroy(g->done);
      delete g;
      throw;
    }
    *out = g;
  });
}

bfc_status bfc_count_total_batch(bfc_graph g, void* stream, int64_t* totals_dev) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!totals_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "totals_dev is null"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    zero_i64(totals_dev, h->n_graphs, s);
    count(h, kTotal, nullptr, nullptr, nullptr, s, totals_dev);
    cs.finish();
  });
}

bfc_status bfc_batch_wedges(bfc_graph g, int64_t* wedges_host) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!wedges_host) throw Error{BFC_ERR_INVALID_ARGUMENT, "wedges_host is null"};
    if (h->graph_wedges.empty()) wedges_host[0] = h->sched.wedges;
    else for (int32_t i = 0; i < h->n_graphs; ++i) wedges_host[i] = h->graph_wedges[i];
  });
}

bfc_status bfc_graph_count(bfc_graph g, int32_t* graphs) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!graphs) throw Error{BFC_ERR_INVALID_ARGUMENT, "graphs is null"};
    *graphs = h->n_graphs;
  });
}

bfc_status bfc_graph_capture_total(bfc_graph g, void* stream, int64_t* totals_dev) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!totals_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "totals_dev is null"};
    if (!stream) throw Error{BFC_ERR_INVALID_ARGUMENT, "capture needs a created stream (the default stream cannot be captured)"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> hold(h->mu);
    if (h->used) BFC_HIP(hipEventSynchronize(h->done));
    if (h->cap_exec) { (void)hipGraphExecDestroy(h->cap_exec); h->cap_exec = nullptr; }
    if (h->cap_graph) { (void)hipGraphDestroy(h->cap_graph); h->cap_graph = nullptr; }
    const bool timing = h->timing;
    h->timing = false;
    BFC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      zero_i64(totals_dev, h->n_graphs, s);
      count(h, kTotal, nullptr, nullptr, nullptr, s, totals_dev);
    } catch (...) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(s, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      h->timing = timing;
      throw;
    }
    h->timing = timing;
    BFC_HIP(hipStreamEndCapture(s, &h->cap_graph));
    BFC_HIP(hipGraphInstantiate(&h->cap_exec, h->cap_graph, nullptr, nullptr, 0));
  });
}

bfc_status bfc_graph_replay(bfc_graph g, void* stream) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!h->cap_exec) throw Error{BFC_ERR_INVALID_ARGUMENT, "nothing captured on this handle"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    BFC_HIP(hipGraphLaunch(h->cap_exec, s));
    cs.finish();
  });
}

bfc_status bfc_count_total_async(bfc_graph g, void* stream, int64_t* total_dev) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!total_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "total_dev is null"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    zero_i64(total_dev, 1, s);
    count(h, kTotal, total_dev, nullptr, nullptr, s);
    cs.finish();
  });
}

bfc_status bfc_count_total_static(bfc_graph g, void* stream, int64_t* total_dev) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!total_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "total_dev is null"};
    if (min_count_scratch_bytes(h) > static_scratch_bytes())
      throw Error{BFC_ERR_TOO_LARGE, "the count needs " + std::to_string(min_count_scratch_bytes(h)) +
                                         " bytes of scratch; the static buffer holds " +
                                         std::to_string(static_scratch_bytes())};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    zero_i64(total_dev, 1, s);
    count(h, kTotal, total_dev, nullptr, nullptr, s, nullptr, true);
    cs.finish();
  });
}

int64_t bfc_static_scratch_bytes(void) { return (int64_t)static_scratch_bytes(); }

bfc_status bfc_count_per_vertex(bfc_graph g, void* stream, int64_t* upper_dev, int64_t* lower_dev) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if ((h->n_upper > 0 && !upper_dev) || (h->n_lower > 0 && !lower_dev))
      throw Error{BFC_ERR_INVALID_ARGUMENT, "output pointer is null"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    count(h, kVertex, nullptr, upper_dev, lower_dev, s);
    cs.finish();
  });
}

bfc_status bfc_caterpillars(bfc_graph g, int64_t* caterpillars_host) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!caterpillars_host) throw Error{BFC_ERR_INVALID_ARGUMENT, "caterpillars_host is null"};
    *caterpillars_host = h->caterpillars;
  });
}

bfc_status bfc_clustering_coefficient(bfc_graph g, void* stream, double* coefficient_host) {
  int64_t total = 0;
  if (coefficient_host) {
    const bfc_status st = bfc_count_total(g, stream, &total, nullptr);
    if (st != BFC_OK) return st;
  }
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!coefficient_host) throw Error{BFC_ERR_INVALID_ARGUMENT, "coefficient_host is null"};
    *coefficient_host = h->caterpillars > 0 ? 4.0 * (double)total / (double)h->caterpillars : 0.0;
  });
}

bfc_status bfc_count_per_edge(bfc_graph g, void* stream, int64_t* edge_dev) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (h->m > 0 && !edge_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "edge_dev is null"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    count(h, kEdge, nullptr, edge_dev, nullptr, s);
    cs.finish();
  });
}

bfc_status bfc_count_total_sorted(bfc_graph g, void* stream, int32_t direction, int64_t max_pairs,
                                  int64_t* total_host, int64_t* pairs_host, int64_t* chunks_host) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!total_host) throw Error{BFC_ERR_INVALID_ARGUMENT, "total_host is null"};
    if (direction != 0 && direction != 1) throw Error{BFC_ERR_INVALID_ARGUMENT, "direction must be 0 or 1"};
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CountSection cs(h, s);
    if (cs.capturing) throw Error{BFC_ERR_INVALID_ARGUMENT, "the sorted count waits on the stream: not capturable"};
    count_total_sorted(h, direction, max_pairs, s, total_host, pairs_host, chunks_host);
    cs.finish();
  });
}

bfc_status bfc_k_wing(const int32_t* edges_dev, int64_t m, int32_t n_upper, int32_t n_lower, int64_t k,
                      void* stream, uint8_t* in_wing_dev, int64_t* counts_dev, int64_t* wing_edges_host,
                      int32_t* rounds_host) {
  return guard([&] {
    check_graph_args(edges_dev, m, n_upper, n_lower);  // before any device work
    if (m > 0 && !in_wing_dev) throw Error{BFC_ERR_INVALID_ARGUMENT, "in_wing_dev is null"};
    int64_t w = 0;
    int32_t r = 0;
    k_wing(edges_dev, m, n_upper, n_lower, k, static_cast<hipStream_t>(stream), in_wing_dev, counts_dev, &w, &r);
    if (wing_edges_host) *wing_edges_host = w;
    if (rounds_host) *rounds_host = r;
  });
}

bfc_status bfc_graph_info(bfc_graph g, int64_t* m, int32_t* n_upper, int32_t* n_lower, int64_t* wedges,
                          int64_t* device_bytes) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (m) *m = h->m;
    if (n_upper) *n_upper = h->n_upper;
    if (n_lower) *n_lower = h->n_lower;
    if (wedges) *wedges = h->sched.wedges;
    if (device_bytes) *device_bytes = h->device_bytes();
  });
}

bfc_status bfc_destroy(bfc_graph g) {
  if (!g) return BFC_OK;
  return guard([&] {
    {
      DeviceScope ds(g->device);
      if (g->used) BFC_HIP(hipEventSynchronize(g->done));
      collect_times(g);
      if (g->cap_exec) (void)hipGraphExecDestroy(g->cap_exec);
      if (g->cap_graph) (void)hipGraphDestroy(g->cap_graph);
      (void)hipEventDestroy(g->done);
      delete g;
    }
  });
}

bfc_status bfc_set_tuning(bfc_graph g, const bfc_tuning* t) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!t) throw Error{BFC_ERR_INVALID_ARGUMENT, "tuning is null"};
    DeviceScope ds(h->device);
    std::lock_guard<std::mutex> hold(h->mu);
    // a captured count holds the old schedule's buffers and settings: drop it
    // (replay fails until the caller captures again)
    if (h->cap_exec || h->cap_graph) {
      if (h->used) BFC_HIP(hipEventSynchronize(h->done));
      if (h->cap_exec) (void)hipGraphExecDestroy(h->cap_exec);
      if (h->cap_graph) (void)hipGraphDestroy(h->cap_graph);
      h->cap_exec = nullptr;
      h->cap_graph = nullptr;
    }
    if (t->light_max_wedges > 2048)
      throw Error{BFC_ERR_INVALID_ARGUMENT, "light_max_wedges must be at most 2048"};
    if (t->dense_block > 0 && (t->dense_block % 64 || t->dense_block > 32768))
      throw Error{BFC_ERR_INVALID_ARGUMENT, "dense_block must be a multiple of 64 and at most 32768"};
    if (t->window_mode > 3) throw Error{BFC_ERR_INVALID_ARGUMENT, "window_mode must be 1, 2 or 3"};
    Tuning nt = h->tune;
    if (t->light_max_wedges > 0) nt.light_max_wedges = t->light_max_wedges;
    if (t->dense_min_ratio > 0) nt.dense_min_ratio = t->dense_min_ratio;
    if (t->window_mode > 0) nt.window_mode = t->window_mode;
    if (t->hash_window_wedges > 0) nt.hash_window_wedges = t->hash_window_wedges;
    if (t->dense_block >= 0) nt.dense_block = t->dense_block;
    if (t->dense_min_wedges > 0) nt.dense_min_wedges = t->dense_min_wedges;
    if (t->medium_max_wedges >= 0) nt.medium_max_wedges = t->medium_max_wedges;
    if (t->vpp > 3) throw Error{BFC_ERR_INVALID_ARGUMENT, "vpp must be 0 to 3"};
    if (t->vpp >= 0) nt.vpp = t->vpp;
    if (t->top_band >= 0) nt.top_band = t->top_band;
    const bool resched = nt.light_max_wedges != h->tune.light_max_wedges || nt.dense_block != h->tune.dense_block ||
                         nt.medium_max_wedges != h->tune.medium_max_wedges || nt.vpp != h->tune.vpp ||
                         nt.top_band != h->tune.top_band;
    h->tune = nt;
    if (resched) {
      if (h->used) BFC_HIP(hipEventSynchronize(h->done));
      BFC_HIP(hipDeviceSynchronize());
      build_schedule(h, nullptr);
      finish_schedule(h, nullptr);
      prepare_count(h, nullptr);
      BFC_HIP(hipStreamSynchronize(nullptr));
    }
  });
}

bfc_status bfc_sync(bfc_graph g, void* stream) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    DeviceScope ds(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t* rb = static_cast<int32_t*>(pinned_stage(sizeof(int32_t)));
    {
      CountSection cs(h, s);
      if (cs.capturing) throw Error{BFC_ERR_INVALID_ARGUMENT, "bfc_sync waits on the stream: not capturable"};
      BFC_HIP(hipMemcpyAsync(rb, count_status(h), sizeof(int32_t), hipMemcpyDeviceToHost, s));
      cs.finish();
    }
    BFC_HIP(hipStreamSynchronize(s));
    if (*rb) throw Error{BFC_ERR_DEVICE, "internal error: a counting window could not be sized (counts are inexact)"};
  });
}

bfc_status bfc_set_allocator(bfc_alloc_fn alloc_fn, bfc_free_fn free_fn, void* ctx) {
  return guard([&] {
    if (!alloc_fn != !free_fn)
      throw Error{BFC_ERR_INVALID_ARGUMENT, "alloc_fn and free_fn must both be set or both be null"};
    set_allocator(alloc_fn, free_fn, ctx);
  });
}

int64_t bfc_trim_cache(void) {
  try {
    return trim_cache();
  } catch (...) {
    return 0;
  }
}

int64_t bfc_cached_bytes(void) {
  try {
    return cached_bytes();
  } catch (...) {
    return 0;
  }
}

bfc_status bfc_set_graph_tuning(bfc_graph g, const bfc_tuning* tunings_host, int32_t count) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (count != 0 && count != h->n_graphs)
      throw Error{BFC_ERR_INVALID_ARGUMENT, "count must be 0 or the handle's number of graphs"};
    if (count > 0 && !tunings_host) throw Error{BFC_ERR_INVALID_ARGUMENT, "tunings_host is null"};
    if (count > 0 && !h->gid[0].bytes)
      throw Error{BFC_ERR_INVALID_ARGUMENT, "per-graph settings need a batch handle (else use bfc_set_tuning)"};
    DeviceScope ds(h->device);
    std::lock_guard<std::mutex> hold(h->mu);
    if (h->cap_exec || h->cap_graph) {
      if (h->used) BFC_HIP(hipEventSynchronize(h->done));
      if (h->cap_exec) (void)hipGraphExecDestroy(h->cap_exec);
      if (h->cap_graph) (void)hipGraphDestroy(h->cap_graph);
      h->cap_exec = nullptr;
      h->cap_graph = nullptr;
    }
    if (h->used) BFC_HIP(hipEventSynchronize(h->done));
    BFC_HIP(hipDeviceSynchronize());
    if (count == 0) {
      // back to the handle's settings (the device is idle: free at once)
      for (DevBuf* b : {&h->glight, &h->gtune}) {
        if (b->p) cache_free_idle(b->p);
        b->p = nullptr;
        b->bytes = 0;
      }
    } else {
      const int32_t cap = h->light_max_cap();
      std::vector<int32_t> lm(count);
      std::vector<int4> gt(count);
      for (int32_t i = 0; i < count; ++i) {
        const bfc_tuning& t = tunings_host[i];
        if (t.light_max_wedges > 2048 || t.window_mode > 3)
          throw Error{BFC_ERR_INVALID_ARGUMENT, "light_max_wedges above 2048 or window_mode above 3"};
        const int32_t l = t.light_max_wedges > 0 ? t.light_max_wedges : h->tune.light_max_wedges;
        lm[i] = l < cap ? l : cap;
        gt[i] = make_int4(t.dense_min_ratio > 0 ? t.dense_min_ratio : h->tune.dense_min_ratio,
                          t.window_mode > 0 ? t.window_mode : h->tune.window_mode,
                          t.hash_window_wedges > 0 ? t.hash_window_wedges : h->tune.hash_window_wedges,
                          t.dense_min_wedges > 0 ? t.dense_min_wedges : h->tune.dense_min_wedges);
      }
      h->glight.alloc(sizeof(int32_t) * (size_t)count, nullptr);
      h->gtune.alloc(sizeof(int4) * (size_t)count, nullptr);
      BFC_HIP(hipMemcpy(h->glight.p, lm.data(), sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice));
      BFC_HIP(hipMemcpy(h->gtune.p, gt.data(), sizeof(int4) * (size_t)count, hipMemcpyHostToDevice));
    }
    build_schedule(h, nullptr);
    finish_schedule(h, nullptr);
    prepare_count(h, nullptr);
    BFC_HIP(hipStreamSynchronize(nullptr));
  });
}

bfc_status bfc_get_schedule_info(bfc_graph g, bfc_schedule_info* out) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!out) throw Error{BFC_ERR_INVALID_ARGUMENT, "out is null"};
    const Schedule& sc = h->sched;
    out->wedges = sc.wedges;
    out->starts_light = sc.n_light;
    out->starts_heavy = sc.n_heavy;
    out->wedges_light = sc.wedges_light;
    out->wedges_heavy = sc.wedges_heavy;
    out->middles_light = sc.middles_light;
    out->middles_heavy = sc.middles_heavy;
    out->max_start_wedges = sc.max_start_wedges;
    out->starts_medium = sc.n_medium;
    out->starts_small = sc.n_small;
  });
}

bfc_status bfc_set_kernel_timing(bfc_graph g, int32_t enable) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    DeviceScope ds(h->device);
    std::lock_guard<std::mutex> hold(h->mu);
    collect_times(h);
    h->timing = enable != 0;
    h->timed_calls = 0;
    h->light_ms = h->heavy_ms = h->other_ms = 0;
  });
}

bfc_status bfc_get_kernel_times(bfc_graph g, bfc_kernel_times* out) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!out) throw Error{BFC_ERR_INVALID_ARGUMENT, "out is null"};
    DeviceScope ds(h->device);
    std::lock_guard<std::mutex> hold(h->mu);
    collect_times(h);
    out->calls = h->timed_calls;
    out->light_ms = h->light_ms;
    out->heavy_ms = h->heavy_ms;
    out->other_ms = h->other_ms;
  });
}

bfc_status bfc_get_tuning(bfc_graph g, bfc_tuning* t) {
  return guard([&] {
    bfc_graph_s* h = checked(g);
    if (!t) throw Error{BFC_ERR_INVALID_ARGUMENT, "tuning is null"};
    t->light_max_wedges = h->tune.light_max_wedges;
    t->dense_min_ratio = h->tune.dense_min_ratio;
    t->window_mode = h->tune.window_mode;
    t->hash_window_wedges = h->tune.hash_window_wedges;
    t->dense_block = h->tune.dense_block;
    t->dense_min_wedges = h->tune.dense_min_wedges;
    t->medium_max_wedges = h->tune.medium_max_wedges;
    t->vpp = h->tune.vpp;
    t->top_band = h->tune.top_band;
  });
}

}  // extern "C"
