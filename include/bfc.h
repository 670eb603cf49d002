/*
 * bfc.h -- exact butterfly counting on one MI355X (gfx950) GPU.
 *
 * C ABI of libbfc.so.  Method: vertex-priority butterfly counting (BFC-VP,
 * Algorithm 2 of Wang, Lin, Qin, Zhang, Zhang, "Efficient Butterfly Counting
 * for Large Bipartite Networks") on the priority-relabelled graph of its
 * cache-aware graph projection (Definition 4), with the per-edge extension
 * of Algorithm 4 and per-vertex counts by Lemma 1.
 *
 * Problem (Section 2): G = (U, L, E) is a bipartite graph, E a subset of
 * U x L.  A butterfly is a 2x2 biclique (Definition 2).  The library returns
 *   - B_G, the number of butterflies                       (bfc_count_total)
 *   - B_x for every vertex x of U and of L                 (bfc_count_per_vertex)
 *   - B_e for every edge e, in input order                 (bfc_count_per_edge)
 * as exact int64 values.
 *
 * Conventions shared by every call:
 *   - Vertex ids are 0-based per layer: upper ids in [0, n_upper), lower ids
 *     in [0, n_lower).  For Definition 3's tie-break the library uses the
 *     global id (lower v -> v, upper u -> n_lower + u), so every upper id is
 *     larger than every lower id, as Section 2 assumes.
 *   - "dev" pointers are HIP device memory on the current device; "host"
 *     pointers are host memory.  `stream` is a hipStream_t (NULL = default
 *     stream).  Work is ordered on that stream.
 *   - Every call returns a bfc_status; on failure no output is written, a
 *     failed bfc_build leaves *out NULL, and bfc_last_error() describes the
 *     failure.  No C++ exception crosses this interface.
 *   - Counts are exact: the whole path is integer arithmetic (int32 wedge
 *     counters, int64 sums; C(c,2) = c(c-1)/2 in int64).
 */
#ifndef BFC_H_
#define BFC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BFC_OK = 0,
  BFC_ERR_INVALID_ARGUMENT = 1,    /* null pointer, negative size, bad handle or option */
  BFC_ERR_VERTEX_OUT_OF_RANGE = 2, /* an upper id outside [0,n_upper) or a lower id outside [0,n_lower) */
  BFC_ERR_DUPLICATE_EDGE = 3,      /* E is a set (Section 2): a repeated (upper, lower) pair is rejected */
  BFC_ERR_TOO_LARGE = 4,           /* m >= 2^30 or a layer with 2^30 or more vertices */
  BFC_ERR_OUT_OF_MEMORY = 5,       /* a device allocation failed */
  BFC_ERR_DEVICE = 6               /* a HIP runtime or kernel error */
} bfc_status;

/* Opaque handle: the priority-relabelled CSR of one graph and its schedule,
 * resident in device memory until bfc_destroy.  A built handle is read-only
 * for the count calls; concurrent count calls on one handle must use
 * different streams and are serialised by the library. */
typedef struct bfc_graph_s* bfc_graph;

/*
 * Builds the relabelled graph (Algorithm 2's first two steps, Definition 3,
 * Definition 4, and the per-start wedge counts used for scheduling).
 *   edges_dev  device int32 [m][2], row i = (upper id, lower id) of edge i.
 *              Read only; the caller keeps ownership.  May be NULL if m == 0.
 *   m          number of edges, 0 <= m < 2^30.
 *   n_upper, n_lower  layer sizes, each in [0, 2^30).  Isolated vertices allowed.
 *   stream     hipStream_t for the build kernels.
 *   out        receives the handle (owned by the caller; free with bfc_destroy).
 * Validates ids and distinctness on the device.  Synchronises `stream`.
 */
bfc_status bfc_build(const int32_t* edges_dev, int64_t m, int32_t n_upper, int32_t n_lower, void* stream,
                     bfc_graph* out);

/*
 * B_G (Lemma 1 Eq. 2, computed as in Algorithm 2): each butterfly is counted
 * once, from the two wedges through its vertex of highest priority.
 *   total_host   host int64, receives B_G.
 *   wedges_host  host int64 or NULL; receives |W|, the number of wedges
 *                Algorithm 2 processes (Theorem 2's work measure).
 * Synchronises `stream`.
 */
bfc_status bfc_count_total(bfc_graph g, void* stream, int64_t* total_host, int64_t* wedges_host);

/*
 * Device-output variant of bfc_count_total: writes B_G to total_dev (device
 * int64 [1]) without synchronising.  For graph capture and pipelining.
 */
bfc_status bfc_count_total_async(bfc_graph g, void* stream, int64_t* total_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count
 * of bfc_count_total_async, whose kernels here keep their scratch (per-start
 * cursors and work tickets) in a fixed array of bfc_static_scratch_bytes()
 * bytes (64 MiB) that the library holds on each device it runs on until the
 * process ends.  The call allocates and frees nothing, creates no event and
 * records no memset (kernel timing is not applied), so it may be captured.
 *   total_dev  device int64 [1], receives B_G (same value as bfc_count_total).
 * When the full grid's cursors do not fit the array the count runs on fewer
 * workgroups (slower, same result); BFC_ERR_TOO_LARGE when not even one
 * workgroup's cursors fit (28 bytes per middle: a start with more than
 * about 2.4 million lower-priority neighbours).  The array is shared by every call on a
 * device and keeps the last call's contents (the call clears what must
 * start at zero): calls that overlap on one device, on different streams
 * or from different threads, race and give wrong results; order them.
 * Asynchronous on `stream`; internal failures are reported like those of
 * bfc_count_per_vertex.
 */
bfc_status bfc_count_total_static(bfc_graph g, void* stream, int64_t* total_dev);
int64_t bfc_static_scratch_bytes(void);

/*
 * B_x for every vertex (Lemma 1 Eq. 1).  Each pair (start, end) with c
 * common lower-priority middles adds C(c,2) to both, and each of its c
 * wedges adds c-1 to its middle.
 *   upper_dev  device int64 [n_upper], B_u by upper id (overwritten).
 *   lower_dev  device int64 [n_lower], B_v by lower id (overwritten).
 * Asynchronous on `stream`: an internal failure of its kernels is reported
 * by the next call on the handle that waits (bfc_sync, bfc_count_total).
 */
bfc_status bfc_count_per_vertex(bfc_graph g, void* stream, int64_t* upper_dev, int64_t* lower_dev);

/*
 * B_e for every edge (Eq. 8 evaluated as in Algorithm 4): a second walk over
 * the same wedges adds count - 1 to both of each wedge's edges.
 *   edge_dev  device int64 [m], B_e in the input order of bfc_build (overwritten).
 * Asynchronous on `stream`, reported like bfc_count_per_vertex.
 */
bfc_status bfc_count_per_edge(bfc_graph g, void* stream, int64_t* edge_dev);

/*
 * Waits on `stream` (after the handle's previous count call, whatever its
 * stream) until every count queued on the handle has finished, and reports
 * whether any of them failed internally.  The count kernels flag a start
 * whose end range could not be cut into windows that fit on chip (which the
 * window halving rules out; the flag guards against a logic error): that
 * start's wedges were skipped, so the outputs of that call are inexact.  The
 * flag is sticky: from then on bfc_sync and bfc_count_total on the handle
 * return BFC_ERR_DEVICE.  Not for use while `stream` is being captured
 * (BFC_ERR_INVALID_ARGUMENT).
 */
bfc_status bfc_sync(bfc_graph g, void* stream);

/*
 * Caterpillars C_G (Section 1): the three-paths of the graph, walks x-y-z-t
 * over four distinct vertices, each path counted once.  A three-path has one
 * middle edge (y, z) and extends it in (d_y - 1)(d_z - 1) ways, so C_G is the
 * sum of that over the edges.  bfc_build computes it with the per-start
 * wedge counts; for a batch handle it is the sum over the graphs.  Writes
 * the int64 value to *caterpillars_host (exact while the sum fits in int64).
 */
bfc_status bfc_caterpillars(bfc_graph g, int64_t* caterpillars_host);

/*
 * Bipartite clustering coefficient 4 B_G / C_G (Section 1; 0 when the graph
 * has no three-path).  Runs bfc_count_total on `stream` under the same rules
 * and waits for it; writes the coefficient (double) to *coefficient_host.
 */
bfc_status bfc_clustering_coefficient(bfc_graph g, void* stream, double* coefficient_host);

/*
 * B_G by sorting vertex pairs (Section 6.3, Algorithm 6, with device memory in
 * the place of disk): every processed wedge gives the pair (end, start);
 * equal pairs are brought together by a radix sort and every run of c equal
 * pairs adds C(c, 2) (Lemma 1).
 *   direction    0: the wedges of Algorithm 2 (BFC-VP: the start outranks the
 *                middle and the end); 1: those of Algorithm 3 (BFC-VP++,
 *                Section 5: the end outranks the start and the middle).  Both
 *                give B_G over the same number of wedges (Lemma 3, Theorem 4).
 *   max_pairs    pairs per chunk: chunks are consecutive start ranks of one
 *                layer holding at most max_pairs pairs (<= 0 or above 2^31:
 *                2^31) plus the wedges of one start; the call needs 16 bytes
 *                of device memory per pair of its largest chunk plus 16 per
 *                middle arc of it
 *   total_host   B_G (int64)
 *   pairs_host   may be NULL: the number of pairs (processed wedges)
 *   chunks_host  may be NULL: the number of chunks
 * Same result as bfc_count_total.  Blocking: waits on `stream` (not for
 * stream capture).  BFC_ERR_TOO_LARGE if one start has so many wedges that
 * its chunk would hold 2^32 pairs or more; BFC_ERR_INVALID_ARGUMENT for
 * another direction.
 */
bfc_status bfc_count_total_sorted(bfc_graph g, void* stream, int32_t direction, int64_t max_pairs,
                                  int64_t* total_host, int64_t* pairs_host, int64_t* chunks_host);

/*
 * k-wing (Section 1, computing k-wing in bipartite graphs): the largest
 * subgraph in which every edge lies in at least k butterflies, as the peeling
 * the paper describes defines it.  Edges below k in a subgraph that contains
 * the k-wing are outside it, so each round counts every remaining edge
 * exactly (bfc_count_per_edge), removes all edges below k at once and
 * rebuilds the rest, until no edge is below k.
 *   edges_dev, m, n_upper, n_lower  as in bfc_build (same checks and errors)
 *   k               the threshold; k <= 0 keeps every edge
 *   in_wing_dev     device uint8 [m]: 1 for the input edges of the k-wing, else 0
 *   counts_dev      device int64 [m] or NULL: butterflies of each edge within
 *                   the k-wing, 0 for the edges outside it
 *   wing_edges_host, rounds_host  may be NULL: edges in the k-wing, count rounds
 * Outputs are in the input edge order.  Blocking: returns after the outputs
 * are written (waits on `stream`, once per round).  Device memory: one build
 * of the remaining edges at a time plus 28 bytes per input edge.
 */
bfc_status bfc_k_wing(const int32_t* edges_dev, int64_t m, int32_t n_upper, int32_t n_lower, int64_t k,
                      void* stream, uint8_t* in_wing_dev, int64_t* counts_dev, int64_t* wing_edges_host,
                      int32_t* rounds_host);

/*
 * Batched form: G independent graphs built into one handle and counted by
 * one set of kernel launches.  Graph g's edges are rows
 * [edge_offsets[g], edge_offsets[g+1]) of edges_dev, with its own 0-based
 * ids (upper < n_upper[g], lower < n_lower[g]).  The handle stores the
 * disjoint union of the graphs (graph g's ids shifted past those of graphs
 * 0..g-1); Definition 3's order restricted to one graph is the same in the
 * union, so every per-graph count and wedge total equals that of building
 * the graph alone.  bfc_count_per_vertex / bfc_count_per_edge on a batch
 * handle return the concatenation of the per-graph outputs (graph order).
 *   edge_offsets_host  host int64 [G+1], non-decreasing, edge_offsets[0] = 0.
 *   n_upper_host, n_lower_host  host int32 [G].
 *   G >= 1; the total edge and vertex counts obey the limits of bfc_build.
 * Synchronises `stream`.
 */
bfc_status bfc_build_batch(const int32_t* edges_dev, const int64_t* edge_offsets_host, const int32_t* n_upper_host,
                           const int32_t* n_lower_host, int32_t G, void* stream, bfc_graph* out);

/* Per-graph totals of a batch handle: totals_dev (device int64 [G], or [1]
 * for a handle from bfc_build) receives B_G of every graph.  Asynchronous. */
bfc_status bfc_count_total_batch(bfc_graph g, void* stream, int64_t* totals_dev);

/* Per-graph processed-wedge counts |W| (host int64 [G]). */
bfc_status bfc_batch_wedges(bfc_graph g, int64_t* wedges_host);

/*
 * Graph capture of the total count: records one bfc_count_total_batch(g, .,
 * totals_dev) into a HIP graph owned by the handle (replacing an earlier
 * one); bfc_graph_replay launches it on `stream`.  The captured work
 * allocates nothing and records no memset nodes.  totals_dev must stay valid
 * while the capture is in use.  `stream` must be a created stream (the
 * default stream cannot be captured): BFC_ERR_INVALID_ARGUMENT otherwise.
 * bfc_set_tuning discards the capture (its kernels hold the old schedule):
 * bfc_graph_replay then returns BFC_ERR_INVALID_ARGUMENT until the next
 * bfc_graph_capture_total.
 */
bfc_status bfc_graph_capture_total(bfc_graph g, void* stream, int64_t* totals_dev);
bfc_status bfc_graph_replay(bfc_graph g, void* stream);

/* Number of graphs in a handle (1 for bfc_build). */
bfc_status bfc_graph_count(bfc_graph g, int32_t* graphs);

/* Sizes of a built graph.  Any output pointer may be NULL.
 *   device_bytes  device memory the handle holds (CSR, maps, schedule, scratch). */
bfc_status bfc_graph_info(bfc_graph g, int64_t* m, int32_t* n_upper, int32_t* n_lower, int64_t* wedges,
                          int64_t* device_bytes);

/* Device memory bfc_build would need for a graph of this size (an upper
 * bound, for admission control).  Returns 0 on bad sizes. */
int64_t bfc_estimate_device_bytes(int64_t m, int32_t n_upper, int32_t n_lower);

/* Frees the handle and its device memory.  NULL is a no-op. */
bfc_status bfc_destroy(bfc_graph g);

/*
 * Device memory.  The library takes its device buffers (graph arrays,
 * schedules, scratch and temporaries) from an internal cache: a freed buffer
 * is kept with the stream and an event of its last use and handed out again,
 * so repeated builds and counts make no allocator calls once warm.  The
 * cache gets new blocks from hipMalloc, or, after bfc_set_allocator, from
 * the caller's functions (for example a framework's caching allocator, so
 * the library's memory is counted in that framework's pool):
 *   alloc_fn(bytes, stream, ctx)  returns `bytes` of device memory on the
 *                 current device, usable by work queued on `stream` (a
 *                 hipStream_t), or NULL when it has none;
 *   free_fn(p, stream, ctx)       takes back a block alloc_fn returned; the
 *                 library calls it only once all work using p has completed.
 * Both NULL restores hipMalloc / hipFree; one NULL is BFC_ERR_INVALID_ARGUMENT.
 * Process-wide.  Before switching, every idle cached block goes back to the
 * allocator that made it; blocks still in use go back to theirs when freed.
 * When an allocation fails the cache returns its idle blocks and retries once;
 * if that fails too the call returns BFC_ERR_OUT_OF_MEMORY (a failed build
 * leaves *out NULL and writes nothing).  Not to be called while other
 * threads are inside library calls.
 */
typedef void* (*bfc_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*bfc_free_fn)(void* p, void* stream, void* ctx);
bfc_status bfc_set_allocator(bfc_alloc_fn alloc_fn, bfc_free_fn free_fn, void* ctx);

/* Returns every idle cached block to its allocator (blocks whose last use
 * has not completed stay); returns the number of bytes released. */
int64_t bfc_trim_cache(void);

/* Bytes held in idle cached blocks (device memory the library holds beyond
 * its live handles and calls in progress). */
int64_t bfc_cached_bytes(void);

/*
 * Tuning knobs for one handle.  None of them changes any count; they choose
 * which kernel path handles each start vertex.  A field <= 0 keeps the
 * current setting (except dense_block and medium_max_wedges, where 0
 * disables and < 0 keeps).
 *   light_max_wedges   starts with at most this many wedges (<= 2048) are
 *                      counted by one wavefront with an LDS hash table;
 *                      larger ones by a workgroup.  Default 2048; values
 *                      above 1024 apply only while both layers have fewer
 *                      than 2^20 vertices (the wavefront tables pack an end
 *                      and its count into one word), else 1024 is used.
 *   dense_min_ratio    a workgroup start uses dense LDS counter windows when
 *                      wedges * dense_min_ratio >= its end-rank range, else LDS
 *                      hash windows.  Default 4.
 *   window_mode        1 = automatic (default), 2 = always dense windows,
 *                      3 = always hash windows.
 *   dense_min_wedges   in automatic mode a start also uses dense windows when
 *                      it has more than this many wedges.  Default 8192.
 *   hash_window_wedges wedges aimed at per hash window (the window is halved
 *                      when its distinct ends overfill the table).  In
 *                      automatic mode a dense start's low end ranks, up to
 *                      the longest multiple of the dense width expected to
 *                      hold this many wedges, form one hash window.  Default
 *                      8192.
 *   dense_block        vertices per layer in the top-priority block counted
 *                      with int8 MFMA (0 disables it; multiple of 64).
 *   medium_max_wedges  workgroup starts with at most this many wedges and at
 *                      most 512 middles (outside the dense block) use
 *                      256-thread workgroups with a 32 KB LDS table, four to
 *                      a CU; the others 1024 threads and 128 KB.  0 puts
 *                      every workgroup start on 1024 threads.  Default 0.
 *   vpp                which wedges the hash / counter kernels process, per
 *                      layer of the start (< 0 keeps; at most 3): bit 0 for
 *                      upper starts, bit 1 for lower starts; a clear bit
 *                      takes Algorithm 2's wedges (BFC-VP: the start
 *                      outranks the middle and the end; default 0), a set
 *                      bit Algorithm 3's (BFC-VP++, Section 5: the end
 *                      outranks the start and the middle, so a start's ends
 *                      are the ranks above it).  The two are the same wedges
 *                      walked from opposite ends, and a butterfly's counted
 *                      pair lies in the layer of its top vertex, so any mix
 *                      gives the same counts and the same |W| (Lemma 3); the
 *                      lists, light / heavy split and per-start work follow
 *                      the chosen wedges.  With vpp != 0 the dense block and
 *                      the 256-thread shape are not used (dense_block and
 *                      medium_max_wedges are kept but ignored).
 *   top_band           width T of each layer's top band of priority ranks
 *                      (< 0 keeps; 0, the default, disables; ignored for a
 *                      layer in vpp, a layer of at most T vertices and a
 *                      batch handle).  A pair of same-layer vertices is
 *                      counted once, from one of its two vertices (Theorem
 *                      1): from the higher one with Algorithm 2's wedges
 *                      when both lie in the band or both below it, and from
 *                      the lower one with Algorithm 3's wedges (Section 5)
 *                      when only the higher one lies in the band.  The two
 *                      walks see the same wedges of the pair, so the counts
 *                      and |W| are those of Algorithm 2 alone.  Every end
 *                      range then lies inside one part: band starts and the
 *                      band wedges of lower starts end within the T top
 *                      ranks (one dense LDS window when T <= 65536).  A start
 *                      below the band becomes two list items (its own part,
 *                      then the band); the dense block and the 256-thread
 *                      shape are not used while a band is set.
 */
typedef struct {
  int32_t light_max_wedges;
  int32_t dense_min_ratio;
  int32_t window_mode;
  int32_t hash_window_wedges;
  int32_t dense_block;
  int32_t dense_min_wedges;
  int32_t medium_max_wedges;
  int32_t vpp;
  int32_t top_band;
} bfc_tuning;

bfc_status bfc_set_tuning(bfc_graph g, const bfc_tuning* t);

/*
 * Per-graph settings of a batch handle (bfc_build_batch), for an autotuner
 * that picks settings per kind of graph while every graph is still counted
 * by the same launches: tunings_host[g] (host array of `count` =
 * the handle's number of graphs) applies to the starts of graph g.  Used
 * fields: light_max_wedges (which kernel takes a start), dense_min_ratio,
 * window_mode, hash_window_wedges and dense_min_wedges (how its end range
 * is cut); a field <= 0 takes the handle's setting; other fields are
 * ignored (they stay per handle).  count = 0 returns every graph to the
 * handle's settings.  No count changes.  Rebuilds the schedule and discards
 * a captured count, as bfc_set_tuning does.  BFC_ERR_INVALID_ARGUMENT for a
 * handle from bfc_build, another count, or a field out of range.
 */
bfc_status bfc_set_graph_tuning(bfc_graph g, const bfc_tuning* tunings_host, int32_t count);
bfc_status bfc_get_tuning(bfc_graph g, bfc_tuning* t);

/*
 * Work split of a built graph (for reporting; all counts are exact integers).
 *   wedges          |W|, the wedges Algorithm 2 processes (Theorem 2's measure)
 *   starts_*        start vertices handed to the wavefront (light) and
 *                   workgroup (heavy) kernels; starts_medium of the heavy
 *                   ones run on 256-thread workgroups; starts_small of the
 *                   light ones (at most 256 wedges) use the small-table kernel
 *   wedges_*        wedges those starts process
 *   middles_*       lower-priority neighbours (middle vertices) they walk
 *   max_start_wedges  the largest per-start wedge count
 */
typedef struct {
  int64_t wedges;
  int64_t starts_light, starts_heavy;
  int64_t wedges_light, wedges_heavy;
  int64_t middles_light, middles_heavy;
  int64_t max_start_wedges;
  int64_t starts_medium;
  int64_t starts_small;
} bfc_schedule_info;

bfc_status bfc_get_schedule_info(bfc_graph g, bfc_schedule_info* out);

/*
 * Kernel timing with HIP events recorded on the caller's stream around the
 * count kernels of every later count call on this handle.  enable != 0
 * turns it on and resets the sums; 0 turns it off.  Not for use while the
 * stream is being captured into a graph.
 *   calls      count calls timed since the reset
 *   light_ms   summed duration of the light-start (wavefront) kernel
 *   heavy_ms   summed duration of the heavy-start (workgroup) kernel
 *   other_ms   summed duration of the remaining count kernels (fold, dense block)
 * bfc_get_kernel_times waits for the timed calls to finish.
 */
typedef struct {
  int64_t calls;
  double light_ms;
  double heavy_ms;
  double other_ms;
} bfc_kernel_times;

bfc_status bfc_set_kernel_timing(bfc_graph g, int32_t enable);
bfc_status bfc_get_kernel_times(bfc_graph g, bfc_kernel_times* out);

/* Text of the last error on the calling thread ("" if none).  Valid until the
 * next call from that thread. */
const char* bfc_last_error(void);

/* Library version string. */
const char* bfc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BFC_H_ */
