// Graph build: validation, priorities (Definition 3), the relabelled CSR of
// the graph projection (Definition 4) and the per-start wedge counts that
// drive the schedule of the counting kernels.
//
// Layout produced (per layer X in {upper, lower}, "other" = the other layer):
//   rank_X(x)   position of x in ascending priority among the vertices of X.
//               Definition 3 orders by degree, ties by id; restricted to one
//               layer this is a stable sort of the layer's ids by degree.
//   off_X, adj_X  CSR by rank; adj holds the neighbours' ranks in the other
//               layer in ascending order (the sorted neighbour lists of
//               Algorithm 2, built by sorting (rank, neighbour rank) keys).
//   rev_X[k]    slot, in adj_other, of the reverse of arc k.
//   lo_X[r]     number of neighbours of r with lower priority than r; they
//               form a prefix of r's list.  Across layers the global id makes
//               every upper id larger than every lower id, so for an edge
//               (u upper, v lower): p(v) < p(u)  <=>  deg(v) <= deg(u).
//   work_X[r]   wedges Algorithm 2 processes from start r: for each middle v
//               in the prefix, the ends are the entries of N(v) before r,
//               i.e. rev[k] - off_other[v] of them.
#include <algorithm>
#include <vector>

#include "device.hpp"
#include "internal.hpp"
#include "sort.hpp"

namespace bfc {

namespace {

// Degree histogram.  Each workgroup first counts in a small LDS table of
// hashed slots, each claimed by the first id that lands in it, so the many
// increments of a hub vertex reach global memory about once per workgroup
// (same-address global atomics serialise); an id whose slot another id holds
// is counted in global memory directly.
constexpr int kDegNT = 256;
constexpr int kDegSlotBits = 11;
constexpr int kDegSlots = 1 << kDegSlotBits;

__device__ __forceinline__ void degree_add(int32_t* key, int32_t* cnt, int32_t* deg, int32_t v) {
  const uint32_t h = ((uint32_t)v * 0x9E3779B1u) >> (32 - kDegSlotBits);
  int32_t k = key[h];
  if (k == -1) {
    k = atomicCAS(&key[h], -1, v);
    if (k == -1) k = v;
  }
  if (k == v) atomicAdd(&cnt[h], 1);
  else atomicAdd(&deg[v], 1);
}

__global__ __launch_bounds__(kDegNT) void degree_kernel(const int32_t* __restrict__ edges, int64_t m, int32_t nU,
                                                        int32_t nL, int32_t* __restrict__ degU,
                                                        int32_t* __restrict__ degL, int32_t* __restrict__ status) {
  __shared__ int32_t skey[2][kDegSlots];
  __shared__ int32_t scnt[2][kDegSlots];
  for (int i = threadIdx.x; i < kDegSlots; i += kDegNT) {
    skey[0][i] = skey[1][i] = -1;
    scnt[0][i] = scnt[1][i] = 0;
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int2 e = reinterpret_cast<const int2*>(edges)[i];
    if (e.x < 0 || e.x >= nU || e.y < 0 || e.y >= nL) {
      atomicOr(&status[0], 1);
      continue;
    }
    degree_add(skey[0], scnt[0], degU, e.x);
    degree_add(skey[1], scnt[1], degL, e.y);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDegSlots; i += kDegNT) {
    if (scnt[0][i]) atomicAdd(&degU[skey[0][i]], scnt[0][i]);
    if (scnt[1][i]) atomicAdd(&degL[skey[1][i]], scnt[1][i]);
  }
}

// Degrees by partition (no global atomics per endpoint): ids are grouped
// into buckets of 2^shift consecutive ids -- bucket totals per tile, a
// scatter of each id into its bucket's region (order inside a bucket is
// irrelevant), then kDegSplit workgroups per bucket count its ids in LDS.
// Both layers at once.  The bucket width is the smallest of 2^13 .. 2^14
// ids that leaves each layer at most kMaxBuckets buckets (layers up to
// 2^26 ids: batches of thousands of graphs have tens of millions); wider
// layers fall back to one atomic per endpoint.
constexpr int kPartNT = 512;
constexpr int64_t kPartTile = 16384;  // edges per workgroup
constexpr int kMinBucketShift = 13;
constexpr int kMaxBucketShift = 14;  // 64 KB of dynamic LDS in part_degree_kernel
constexpr int kMaxBuckets = 4096;

__global__ __launch_bounds__(kPartNT) void part_count_kernel(const int32_t* __restrict__ edges, int64_t m,
                                                             int32_t nU, int32_t nL, int32_t BU, int32_t BL,
                                                             int shift, uint32_t* __restrict__ cnt,
                                                             int32_t* __restrict__ status) {
  __shared__ uint32_t h[2 * kMaxBuckets];
  const int nb = BU + BL;
  for (int i = threadIdx.x; i < nb; i += kPartNT) h[i] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * kPartTile;
  const int64_t e1 = e0 + kPartTile < m ? e0 + kPartTile : m;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kPartNT) {
    const int2 e = reinterpret_cast<const int2*>(edges)[i];
    if (e.x < 0 || e.x >= nU || e.y < 0 || e.y >= nL) {
      atomicOr(&status[0], 1);
      continue;
    }
    atomicAdd(&h[e.x >> shift], 1u);
    atomicAdd(&h[BU + (e.y >> shift)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kPartNT)
    if (h[i]) atomicAdd(&cnt[i], h[i]);
}

__global__ __launch_bounds__(kPartNT) void part_scatter_kernel(const int32_t* __restrict__ edges, int64_t m,
                                                               int32_t nU, int32_t nL, int32_t BU, int32_t BL,
                                                               int shift, const uint32_t* __restrict__ off,
                                                               uint32_t* __restrict__ fill,
                                                               int32_t* __restrict__ part) {
  __shared__ uint32_t h[2 * kMaxBuckets];
  __shared__ uint32_t base[2 * kMaxBuckets];
  const int nb = BU + BL;
  for (int i = threadIdx.x; i < nb; i += kPartNT) h[i] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * kPartTile;
  const int64_t e1 = e0 + kPartTile < m ? e0 + kPartTile : m;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kPartNT) {
    const int2 e = reinterpret_cast<const int2*>(edges)[i];
    if (e.x < 0 || e.x >= nU || e.y < 0 || e.y >= nL) continue;
    atomicAdd(&h[e.x >> shift], 1u);
    atomicAdd(&h[BU + (e.y >> shift)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kPartNT) {
    base[i] = h[i] ? off[i] + atomicAdd(&fill[i], h[i]) : 0u;
    h[i] = 0;
  }
  __syncthreads();
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kPartNT) {
    const int2 e = reinterpret_cast<const int2*>(edges)[i];
    if (e.x < 0 || e.x >= nU || e.y < 0 || e.y >= nL) continue;
    const int bu = e.x >> shift, bl = BU + (e.y >> shift);
    part[base[bu] + atomicAdd(&h[bu], 1u)] = e.x;
    part[base[bl] + atomicAdd(&h[bl], 1u)] = e.y;
  }
}

// kDegSplit workgroups share a bucket: each counts a slice of its ids in
// LDS and adds its non-zero counts to the (zeroed) degrees.
constexpr int kDegSplit = 8;
// (dynamic LDS: 4 bytes per id of a bucket)
__global__ __launch_bounds__(kPartNT) void part_degree_kernel(const int32_t* __restrict__ part,
                                                              const uint32_t* __restrict__ off, int32_t BU,
                                                              int32_t nU, int32_t nL, int shift,
                                                              int32_t* __restrict__ degU,
                                                              int32_t* __restrict__ degL) {
  extern __shared__ uint32_t h[];
  const int32_t bucket_ids = 1 << shift;
  const int b = blockIdx.x / kDegSplit;
  const int sp = blockIdx.x % kDegSplit;
  const bool lower = b >= BU;
  const int32_t id0 = (lower ? b - BU : b) << shift;
  const int32_t n = lower ? nL : nU;
  const int32_t w = n - id0 < bucket_ids ? n - id0 : bucket_ids;
  for (int i = threadIdx.x; i < w; i += kPartNT) h[i] = 0;
  __syncthreads();
  const uint32_t a0 = off[b], len = off[b + 1] - a0;
  const uint32_t s0 = a0 + (uint32_t)((uint64_t)len * sp / kDegSplit);
  const uint32_t s1 = a0 + (uint32_t)((uint64_t)len * (sp + 1) / kDegSplit);
  for (uint32_t i = s0 + threadIdx.x; i < s1; i += kPartNT) atomicAdd(&h[part[i] - id0], 1u);
  __syncthreads();
  int32_t* deg = lower ? degL : degU;
  for (int i = threadIdx.x; i < w; i += kPartNT)
    if (h[i]) atomicAdd(&deg[id0 + i], (int32_t)h[i]);
}

__global__ void iota_kernel(uint32_t* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (uint32_t)i;
}

__global__ void invert_kernel(const uint32_t* __restrict__ id_of, int32_t* __restrict__ rank_of, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    rank_of[id_of[r]] = (int32_t)r;
}

// keys for one side's CSR sort: (rank of source) << bits_other | rank of neighbour
// Arc keys (rank_u << bits_dst | rank_v).  bits_idx > 0: the key is shifted
// up by bits_idx and the edge index fills the low bits (no value array);
// otherwise vals receives the edge index.
// The key kernels below write one radix-sort tile per workgroup
// (kSortTileKeys keys, 512 threads) and count the tile's first sort digit,
// bits [shift, shift + 8) of each key, into counts[d * tiles + tile].
constexpr int kKeyNT = 512;

__device__ __forceinline__ void tile_digit_counts(uint32_t* h, uint32_t* __restrict__ counts, int64_t tiles) {
  __syncthreads();
  if (threadIdx.x < 256) counts[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kKeyNT) void arc_keys_kernel(const int32_t* __restrict__ edges, int64_t m, int src_col,
                                                          const int32_t* __restrict__ rank_src,
                                                          const int32_t* __restrict__ rank_dst, int bits_dst,
                                                          int bits_idx, uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals, int shift,
                                                          uint32_t* __restrict__ counts, int64_t tiles) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTileKeys;
#pragma unroll
  for (int j = 0; j < kSortTileKeys / kKeyNT; ++j) {
    const int64_t i = base + j * kKeyNT + threadIdx.x;
    if (i >= m) break;
    const int2 e = reinterpret_cast<const int2*>(edges)[i];
    const int32_t a = src_col == 0 ? e.x : e.y;
    const int32_t b = src_col == 0 ? e.y : e.x;
    uint64_t key = ((uint64_t)(uint32_t)rank_src[a] << bits_dst) | (uint64_t)(uint32_t)rank_dst[b];
    if (bits_idx > 0) {
      key = (key << bits_idx) | (uint64_t)i;
    } else {
      vals[i] = (uint32_t)i;
    }
    keys[i] = key;
    atomicAdd(&h[(uint32_t)(key >> shift) & 255u], 1u);
  }
  tile_digit_counts(h, counts, tiles);
}

__global__ void arc_unpack_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t m,
                                  int bits_dst, int bits_idx, int32_t* __restrict__ adj, int32_t* __restrict__ src,
                                  int32_t* __restrict__ edge_of_slot, int32_t* __restrict__ status) {
  const uint64_t mask = (1ull << bits_dst) - 1ull;
  const uint64_t imask = bits_idx > 0 ? (1ull << bits_idx) - 1ull : 0ull;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t packed = keys[k];
    const uint64_t key = packed >> bits_idx;
    adj[k] = (int32_t)(key & mask);
    src[k] = (int32_t)(key >> bits_dst);
    edge_of_slot[k] = bits_idx > 0 ? (int32_t)(packed & imask) : (int32_t)vals[k];
    if (k > 0 && (keys[k - 1] >> bits_idx) == key) atomicOr(&status[1], 1);
  }
}

// Side 1 from side 0: key = rank_v of side-0 slot k, value = k.
__global__ void transpose_keys_kernel(const int32_t* __restrict__ adj0, int64_t m, uint32_t* __restrict__ key,
                                      uint32_t* __restrict__ val) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    key[k] = (uint32_t)adj0[k];
    val[k] = (uint32_t)k;
  }
}

// Side-1 slot k1 holds the arc of side-0 slot s0 = val[k1]: start rank_v =
// key[k1], neighbour rank_u = src0[s0]; the two reverse slots point at each
// other.
// Packed transpose: key (v << (bu + bs)) | (u << bs) | s0 per side-0 slot
// s0 = (u, v); sorted on its v bits, it yields side 1 without gathers.
__global__ __launch_bounds__(kKeyNT) void transpose_keys_packed_kernel(const int32_t* __restrict__ adj0,
                                                                       const int32_t* __restrict__ src0, int64_t m,
                                                                       int bu, int bs, uint64_t* __restrict__ key,
                                                                       uint32_t* __restrict__ counts, int64_t tiles) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTileKeys;
#pragma unroll
  for (int j = 0; j < kSortTileKeys / kKeyNT; ++j) {
    const int64_t k = base + j * kKeyNT + threadIdx.x;
    if (k >= m) break;
    const uint32_t v = (uint32_t)adj0[k];
    key[k] = ((uint64_t)v << (bu + bs)) | ((uint64_t)(uint32_t)src0[k] << bs) | (uint64_t)k;
    atomicAdd(&h[v & 255u], 1u);  // the sort's first digit: the low 8 bits of v
  }
  tile_digit_counts(h, counts, tiles);
}
__global__ void transpose_unpack_packed_kernel(const uint64_t* __restrict__ key, int64_t m, int bu, int bs,
                                               int32_t* __restrict__ adj1, int32_t* __restrict__ src1,
                                               int32_t* __restrict__ rev1, int32_t* __restrict__ rev0) {
  const uint64_t smask = (1ull << bs) - 1ull, umask = (1ull << bu) - 1ull;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t kk = key[k];
    const int32_t s0 = (int32_t)(kk & smask);
    src1[k] = (int32_t)(kk >> (bu + bs));
    adj1[k] = (int32_t)((kk >> bs) & umask);
    rev1[k] = s0;
    rev0[s0] = (int32_t)k;
  }
}
__global__ void transpose_unpack_kernel(const uint32_t* __restrict__ key, const uint32_t* __restrict__ val,
                                        const int32_t* __restrict__ src0, int64_t m, int32_t* __restrict__ adj1,
                                        int32_t* __restrict__ src1, int32_t* __restrict__ rev1,
                                        int32_t* __restrict__ rev0) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s0 = (int32_t)val[k];
    src1[k] = (int32_t)key[k];
    adj1[k] = src0[s0];
    rev1[k] = s0;
    rev0[s0] = (int32_t)k;
  }
}

// Per arc k of side X (source rank src[k], neighbour rank adj[k]): is the
// neighbour a middle of the source (lower priority), and if so how many
// wedges it gives: the entries of N(neighbour) before the source, i.e.
// rev[k] - off_other[neighbour].  With the global id putting every upper
// vertex above every lower one, for an upper u and lower v:
// p(v) < p(u)  <=>  deg(v) <= deg(u).
// Per start r of side x: lo[r] = its middles (the neighbours v of lower
// priority, a prefix of N(r): deg(v) <= deg(r) across the layers, ties to
// the lower layer) and work[r] = the wedges Algorithm 2 walks from r, the
// sum over middles of v's neighbours below r (rev[k] - off_other[v]).
constexpr int kCatSlots = 64;

// Degrees are differences of adjacent CSR offsets, so the other layer's
// offset and degree come from one cache line per arc.
// Arc-parallel over the side's CSR, whose starts ascend: a wavefront sums
// its 64 arcs per run of equal start (segmented scan) and the run's last
// lane adds the sums with one atomic each (lo and work start at zero).
// With cat non-null it also adds the caterpillars (three-paths) of the
// graph, sum over its edges of (d_u - 1)(d_v - 1) (Section 1), into
// cat[0 .. kCatSlots): one atomic per workgroup, spread over the slots.
__global__ void start_stats_kernel(int64_t m, int x, const int32_t* __restrict__ src,
                                   const int32_t* __restrict__ adj, const int32_t* __restrict__ rev,
                                   const int32_t* __restrict__ off_self, const int32_t* __restrict__ off_other,
                                   int32_t* __restrict__ lo, unsigned long long* __restrict__ work,
                                   unsigned long long* __restrict__ cat) {
  __shared__ unsigned long long s_paths[4];
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long paths = 0;
  for (int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ll; b < m; b += stride) {
    const int64_t k = b + lane;
    int32_t r = -1, f = 0;
    unsigned long long w = 0;
    if (k < m) {
      r = src[k];
      const int32_t v = adj[k];
      const int32_t rk = rev[k];
      const int32_t ov = off_other[v];
      const int32_t ds = off_self[r + 1] - off_self[r], dv = off_other[v + 1] - ov;
      paths += (unsigned long long)(uint32_t)(ds - 1) * (uint32_t)(dv - 1);  // degrees >= 1: a 32x32-bit product
      if (x == 0 ? dv <= ds : dv < ds) {
        f = 1;
        w = (unsigned long long)(rk - ov);
      }
    }
    // run boundaries: a lane heads a run when its start differs from the lane below
    const int32_t r_prev = __shfl_up(r, 1, 64);
    const int32_t r_next = __shfl_down(r, 1, 64);
    const bool head = lane == 0 || r_prev != r;
    const bool tail = lane == 63 || r_next != r;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? heads : heads & ((2ull << lane) - 1ull);
    const int s0 = 63 - (int)__builtin_clzll(upto);  // first lane of this lane's run
    const int32_t inc_f = wave_inclusive_scan(f);
    const unsigned long long inc_w = wave_inclusive_scan(w);
    const int src_lane = s0 > 0 ? s0 - 1 : 0;
    const int32_t pf = __shfl(inc_f, src_lane, 64);
    const unsigned long long pw = __shfl(inc_w, src_lane, 64);
    if (tail && r >= 0) {
      const int32_t sf = inc_f - (s0 > 0 ? pf : 0);
      const unsigned long long sw = inc_w - (s0 > 0 ? pw : 0ull);
      if (sf) {
        atomicAdd(&lo[r], sf);
        atomicAdd(&work[r], sw);
      }
    }
  }
  if (cat) {
    paths = wave_sum(paths);
    if (lane == 0) s_paths[threadIdx.x >> 6] = paths;
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long b = s_paths[0] + s_paths[1] + s_paths[2] + s_paths[3];
      if (b) atomicAdd(&cat[blockIdx.x % kCatSlots], b);
    }
  }
}

unsigned grid_1d(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

// largest g in [0, G) with off[g] <= x (off non-decreasing, off[0] <= x)
template <typename T>
__device__ __forceinline__ int32_t graph_of(const T* __restrict__ off, int32_t G, T x) {
  int32_t lo = 0, hi = G;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Batch priority keys: (graph << db) | degree, so a stable sort by key
// ranks each graph's vertices contiguously, in Definition 3's order inside
// the graph (ids of one graph are consecutive, ties keep id order).
__global__ void group_key_kernel(const int32_t* __restrict__ deg, int64_t n, const int32_t* __restrict__ goff,
                                 int32_t G, int db, uint64_t* __restrict__ key) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = ((uint64_t)graph_of<int32_t>(goff, G, (int32_t)i) << db) | (uint32_t)deg[i];
}

__global__ void low_bits_kernel(const uint64_t* __restrict__ key, int64_t n, int db, uint32_t* __restrict__ out) {
  const uint64_t mask = (1ull << db) - 1ull;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)(key[i] & mask);
}

// ---- window-boundary tables
// Degrees do not decrease with rank, so the vertices of degree >= D are the
// ranks from the first such one up.
__global__ void first_rank_kernel(const int32_t* __restrict__ off, int32_t n, int32_t D, int32_t* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid + 1] - off[mid] >= D) hi = mid; else lo = mid + 1;
  }
  *out = lo;
}

// Row of rank v (v >= first): entry w = first slot of N(v) with end rank
// >= w << kWinShift (a binary search over the ascending list).
__global__ void window_table_kernel(const int32_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t n,
                                    int32_t R, int64_t rows_max, const int32_t* __restrict__ first_p,
                                    int32_t* __restrict__ tab) {
  int32_t first = *first_p;
  if ((int64_t)n - first > rows_max) first = (int32_t)(n - rows_max);
  const int64_t total = ((int64_t)n - first) * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = first + (int32_t)(i / R);
    const int32_t key = (int32_t)(i % R) << kWinShift;
    int32_t a = off[v], b = off[v + 1];
    while (a < b) {
      const int32_t mid = (a + b) >> 1;
      if (adj[mid] < key) a = mid + 1; else b = mid;
    }
    tab[i] = a;
  }
}

// Largest of n degrees into *out (one atomic max per workgroup of 256
// threads; *out starts at 0).
__global__ __launch_bounds__(256) void max_kernel(const int32_t* __restrict__ a, int64_t n,
                                                  int32_t* __restrict__ out) {
  __shared__ int32_t red[4];
  int32_t mx = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mx = a[i] > mx ? a[i] : mx;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int32_t o = __shfl_xor(mx, d, 64);
    mx = o > mx ? o : mx;
  }
  if (__lane_id() == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t m0 = red[0] > red[1] ? red[0] : red[1], m1 = red[2] > red[3] ? red[2] : red[3];
    const int32_t m = m0 > m1 ? m0 : m1;
    if (m) atomicMax(out, m);
  }
}

}  // namespace

void build_graph(bfc_graph_s* g, const int32_t* edges, hipStream_t s, const int32_t* const* groups, int32_t G) {
  const int64_t m = g->m;
  const int32_t n[2] = {g->n_upper, g->n_lower};
  const int32_t span0 = g->key_span[0] >= 0 ? g->key_span[0] : n[0];
  const int32_t span1 = g->key_span[1] >= 0 ? g->key_span[1] : n[1];
  g->light_packed = span0 < (1 << 20) && span1 < (1 << 20);

  // status: [0] id out of range, [1] duplicate edge, [2 + o] first table row of layer o,
  // [4 + x] largest degree of layer x
  g->info.alloc(kInfoBytes, s);
  BFC_HIP(hipMemsetAsync(g->info.p, 0, kInfoBytes, s));
  DevBuf& status = g->info;
  TmpBuf deg[2];
  for (int x = 0; x < 2; ++x) {
    deg[x].alloc(sizeof(int32_t) * (size_t)(n[x] + 1), s);
    BFC_HIP(hipMemsetAsync(deg[x].p, 0, sizeof(int32_t) * (size_t)(n[x] + 1), s));
  }
  int shift = kMinBucketShift;
  while (shift < kMaxBucketShift && (((int64_t)(n[0] > n[1] ? n[0] : n[1]) + (1 << shift) - 1) >> shift) > kMaxBuckets)
    ++shift;
  const int32_t BU = (int32_t)(((int64_t)n[0] + (1 << shift) - 1) >> shift);
  const int32_t BL = (int32_t)(((int64_t)n[1] + (1 << shift) - 1) >> shift);
  if (m > 0 && BU <= kMaxBuckets && BL <= kMaxBuckets) {
    const int nb = BU + BL;
    TmpBuf cnt, fill, part;
    cnt.alloc(sizeof(uint32_t) * (size_t)(nb + 1), s);
    fill.alloc(sizeof(uint32_t) * (size_t)nb, s);
    part.alloc(sizeof(int32_t) * 2 * (size_t)m, s);
    BFC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t) * (size_t)(nb + 1), s));
    BFC_HIP(hipMemsetAsync(fill.p, 0, sizeof(uint32_t) * (size_t)nb, s));
    const unsigned tiles = (unsigned)((m + kPartTile - 1) / kPartTile);
    part_count_kernel<<<tiles, kPartNT, 0, s>>>(edges, m, n[0], n[1], BU, BL, shift, cnt.as<uint32_t>(),
                                                status.as<int32_t>());
    BFC_LAUNCH_CHECK();
    exclusive_scan_u32(cnt.as<uint32_t>(), cnt.as<uint32_t>(), nb + 1, s);
    part_scatter_kernel<<<tiles, kPartNT, 0, s>>>(edges, m, n[0], n[1], BU, BL, shift, cnt.as<uint32_t>(),
                                                  fill.as<uint32_t>(), part.as<int32_t>());
    BFC_LAUNCH_CHECK();
    if (nb > 0) {
      part_degree_kernel<<<(unsigned)nb * kDegSplit, kPartNT, sizeof(uint32_t) << shift, s>>>(
          part.as<int32_t>(), cnt.as<uint32_t>(), BU, n[0], n[1], shift,
                                                          deg[0].as<int32_t>(), deg[1].as<int32_t>());
      BFC_LAUNCH_CHECK();
    }
  } else if (m > 0) {
    int64_t grid = (m + kDegNT - 1) / kDegNT;
    if (grid > 2048) grid = 2048;
    degree_kernel<<<(unsigned)grid, kDegNT, 0, s>>>(edges, m, n[0], n[1], deg[0].as<int32_t>(), deg[1].as<int32_t>(),
                                                   status.as<int32_t>());
    BFC_LAUNCH_CHECK();
  }
  for (int x = 0; x < 2; ++x) {
    if (n[x] == 0) continue;
    const int64_t grid = n[x] / 256 + 1 < 256 ? n[x] / 256 + 1 : 256;
    max_kernel<<<(unsigned)grid, 256, 0, s>>>(deg[x].as<int32_t>(), n[x], status.as<int32_t>() + 4 + x);
    BFC_LAUNCH_CHECK();
  }
  int32_t* st = static_cast<int32_t*>(pinned_stage(8 * sizeof(int32_t)));
  BFC_HIP(hipMemcpyAsync(st, status.p, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BFC_HIP(hipStreamSynchronize(s));
  if (st[0]) throw Error{BFC_ERR_VERTEX_OUT_OF_RANGE, "an edge has an upper id outside [0,n_upper) or a lower id outside [0,n_lower)"};
  g->max_deg[0] = st[4];
  g->max_deg[1] = st[5];

  // ---- priorities: stable sort of each layer's ids by degree
  TmpBuf rank_of[2], deg_rank[2];
  for (int x = 0; x < 2; ++x) {
    Side& sd = g->side[x];
    sd.n = n[x];
    const int64_t nx = n[x];
    TmpBuf ktmp, vtmp;
    sd.id_of.alloc(sizeof(uint32_t) * (size_t)nx, s);
    DevBuf& vals = sd.id_of;
    deg_rank[x].alloc(sizeof(uint32_t) * (size_t)nx, s);
    ktmp.alloc(sizeof(uint32_t) * (size_t)nx, s);
    vtmp.alloc(sizeof(uint32_t) * (size_t)nx, s);
    if (nx > 0) {
      iota_kernel<<<grid_1d(nx), 256, 0, s>>>(vals.as<uint32_t>(), nx);
      BFC_LAUNCH_CHECK();
      // the priority keys are the degrees: sort on the bits of the largest
      const int db = bits_for((uint64_t)st[4 + x]);
      if (groups && G > 1) {
        // batch: sort by (graph, degree); the degrees in rank order are the keys' low bits
        TmpBuf key, key_tmp;
        key.alloc(sizeof(uint64_t) * (size_t)nx, s);
        key_tmp.alloc(sizeof(uint64_t) * (size_t)nx, s);
        group_key_kernel<<<grid_1d(nx), 256, 0, s>>>(deg[x].as<int32_t>(), nx, groups[x], G, db, key.as<uint64_t>());
        BFC_LAUNCH_CHECK();
        radix_sort_u64(key.as<uint64_t>(), vals.as<uint32_t>(), key_tmp.as<uint64_t>(), vtmp.as<uint32_t>(), nx,
                       db + bits_for((uint64_t)(G - 1)), s);
        low_bits_kernel<<<grid_1d(nx), 256, 0, s>>>(key.as<uint64_t>(), nx, db, deg_rank[x].as<uint32_t>());
        BFC_LAUNCH_CHECK();
      } else {
        BFC_HIP(hipMemcpyAsync(deg_rank[x].p, deg[x].p, sizeof(uint32_t) * (size_t)nx, hipMemcpyDeviceToDevice, s));
        radix_sort_u32(deg_rank[x].as<uint32_t>(), vals.as<uint32_t>(), ktmp.as<uint32_t>(), vtmp.as<uint32_t>(), nx,
                       db, s);
      }
    }
    // deg_rank = degrees in rank order; id_of = ids in rank order
    rank_of[x].alloc(sizeof(int32_t) * (size_t)nx, s);
    if (nx > 0) {
      invert_kernel<<<grid_1d(nx), 256, 0, s>>>(sd.id_of.as<uint32_t>(), rank_of[x].as<int32_t>(), nx);
      BFC_LAUNCH_CHECK();
    }
    sd.off.alloc(sizeof(int32_t) * (size_t)(nx + 1), s);
    exclusive_scan_i32(deg_rank[x].as<int32_t>(), sd.off.as<int32_t>(), nx, sd.off.as<int32_t>() + nx, s);
  }

  // ---- per-side CSR.  Side 0: sort (rank_u, rank_v) keys; the sort's
  // values give edge0 (side-0 slot -> input edge index).  Side 1 is side 0 transposed: side 0's arcs
  // are in ascending (u, v) order, so a stable sort of them by v alone lists
  // each v's neighbours u in ascending order.  The sort's values are side-0
  // slots, which are side 1's reverse slots.
  TmpBuf src[2];
  for (int x = 0; x < 2; ++x) g->side[x].rev.alloc(sizeof(int32_t) * (size_t)m, s);
  g->edge0.alloc(sizeof(int32_t) * (size_t)m, s);
  const int bits[2] = {bits_for((uint64_t)(n[0] > 1 ? n[0] - 1 : 1)), bits_for((uint64_t)(n[1] > 1 ? n[1] - 1 : 1))};
  for (int x = 0; x < 2; ++x) {
    g->side[x].adj.alloc(sizeof(int32_t) * (size_t)m, s);
    src[x].alloc(sizeof(int32_t) * (size_t)m, s);
  }
  if (m > 0) {
    TmpBuf keys, vals, ktmp, vtmp;
    keys.alloc(sizeof(uint64_t) * (size_t)m, s);
    vals.alloc(sizeof(uint32_t) * (size_t)m, s);
    ktmp.alloc(sizeof(uint64_t) * (size_t)m, s);
    vtmp.alloc(sizeof(uint32_t) * (size_t)m, s);
    // when the key and the edge index fit 64 bits together the sort moves
    // keys only (8 bytes per arc and pass instead of 12)
    const int bits_idx = bits_for((uint64_t)(m - 1));
    const bool packed = bits[0] + bits[1] + bits_idx <= 64;
    // the key kernels also count each sort tile's first digit, which
    // spares each sort its first histogram pass
    const int64_t tiles = sort_tiles(m);
    TmpBuf counts;
    counts.alloc(sizeof(uint32_t) * 256 * (size_t)tiles, s);
    arc_keys_kernel<<<(unsigned)tiles, kKeyNT, 0, s>>>(edges, m, 0, rank_of[0].as<int32_t>(),
                                                       rank_of[1].as<int32_t>(), bits[1], packed ? bits_idx : 0,
                                                       keys.as<uint64_t>(), vals.as<uint32_t>(),
                                                       packed ? bits_idx : 0, counts.as<uint32_t>(), tiles);
    BFC_LAUNCH_CHECK();
    const bool in_tmp =
        packed ? radix_sort_u64_keys_counted(keys.as<uint64_t>(), ktmp.as<uint64_t>(), m, bits_idx,
                                             bits[0] + bits[1], counts.as<uint32_t>(), s)
               : radix_sort_u64_counted(keys.as<uint64_t>(), vals.as<uint32_t>(), ktmp.as<uint64_t>(),
                                        vtmp.as<uint32_t>(), m, bits[0] + bits[1], counts.as<uint32_t>(), s);
    arc_unpack_kernel<<<grid_1d(m), 256, 0, s>>>(in_tmp ? ktmp.as<uint64_t>() : keys.as<uint64_t>(),
                                                 in_tmp ? vtmp.as<uint32_t>() : vals.as<uint32_t>(), m, bits[1],
                                                 packed ? bits_idx : 0, g->side[0].adj.as<int32_t>(),
                                                 src[0].as<int32_t>(), g->edge0.as<int32_t>(),
                                                 status.as<int32_t>());
    BFC_LAUNCH_CHECK();
    if (packed) {
      // side 1: one 64-bit key per side-0 slot carrying (v, u, slot), sorted on v
      transpose_keys_packed_kernel<<<(unsigned)tiles, kKeyNT, 0, s>>>(g->side[0].adj.as<int32_t>(),
                                                                      src[0].as<int32_t>(), m, bits[0], bits_idx,
                                                                      keys.as<uint64_t>(), counts.as<uint32_t>(),
                                                                      tiles);
      BFC_LAUNCH_CHECK();
      const bool t_tmp = radix_sort_u64_keys_counted(keys.as<uint64_t>(), ktmp.as<uint64_t>(), m, bits[0] + bits_idx,
                                                     bits[1], counts.as<uint32_t>(), s);
      transpose_unpack_packed_kernel<<<grid_1d(m), 256, 0, s>>>(
          t_tmp ? ktmp.as<uint64_t>() : keys.as<uint64_t>(), m, bits[0], bits_idx, g->side[1].adj.as<int32_t>(),
          src[1].as<int32_t>(), g->side[1].rev.as<int32_t>(), g->side[0].rev.as<int32_t>());
      BFC_LAUNCH_CHECK();
    } else {
      // side 1: keys = rank_v of each side-0 slot, values = the slot
      uint32_t* k1 = reinterpret_cast<uint32_t*>(keys.p);
      uint32_t* v1 = vals.as<uint32_t>();
      uint32_t* k1t = reinterpret_cast<uint32_t*>(ktmp.p);
      uint32_t* v1t = vtmp.as<uint32_t>();
      transpose_keys_kernel<<<grid_1d(m), 256, 0, s>>>(g->side[0].adj.as<int32_t>(), m, k1, v1);
      BFC_LAUNCH_CHECK();
      radix_sort_u32(k1, v1, k1t, v1t, m, bits[1], s);
      transpose_unpack_kernel<<<grid_1d(m), 256, 0, s>>>(k1, v1, src[0].as<int32_t>(), m,
                                                         g->side[1].adj.as<int32_t>(), src[1].as<int32_t>(),
                                                         g->side[1].rev.as<int32_t>(), g->side[0].rev.as<int32_t>());
      BFC_LAUNCH_CHECK();
    }
  }

  // ---- per start: lower-priority prefix length and wedges
  for (int x = 0; x < 2; ++x) {
    Side& sd = g->side[x];
    sd.lo.alloc(sizeof(int32_t) * (size_t)sd.n, s);
    sd.work.alloc(sizeof(int64_t) * (size_t)sd.n, s);
    if (sd.n > 0) {
      BFC_HIP(hipMemsetAsync(sd.lo.p, 0, sizeof(int32_t) * (size_t)sd.n, s));
      BFC_HIP(hipMemsetAsync(sd.work.p, 0, sizeof(int64_t) * (size_t)sd.n, s));
    }
    if (m > 0) {
      int64_t grid = (m + 255) / 256;
      if (grid > 8192) grid = 8192;
      start_stats_kernel<<<(unsigned)grid, 256, 0, s>>>(m, x, src[x].as<int32_t>(), sd.adj.as<int32_t>(),
                                                        sd.rev.as<int32_t>(), sd.off.as<int32_t>(),
                                                        g->side[1 - x].off.as<int32_t>(), sd.lo.as<int32_t>(),
                                                        sd.work.as<unsigned long long>(),
                                                        x == 0 ? reinterpret_cast<unsigned long long*>(
                                                                     g->info.as<char>() + kInfoCaterpillars)
                                                               : nullptr);
      BFC_LAUNCH_CHECK();
    }
  }
  // window-boundary tables of both middle layers (first row rank -> status[2 + o])
  int64_t rows_max[2] = {0, 0};
  for (int o = 0; o < 2; ++o) {
    const int32_t no = n[o];
    const int32_t R = (n[1 - o] >> kWinShift) + 2;
    const int32_t D = 2 * R > kWinMinDegree ? 2 * R : kWinMinDegree;
    rows_max[o] = m / D < no ? m / D : no;
    g->wt_row[o] = R;
    g->wt_first[o] = no;
    if (rows_max[o] <= 0) continue;
    g->wt[o].alloc(sizeof(int32_t) * (size_t)rows_max[o] * (size_t)R, s);
    first_rank_kernel<<<1, 64, 0, s>>>(g->side[o].off.as<int32_t>(), no, D, status.as<int32_t>() + 2 + o);
    BFC_LAUNCH_CHECK();
    window_table_kernel<<<grid_1d(rows_max[o] * R), 256, 0, s>>>(
        g->side[o].off.as<int32_t>(), g->side[o].adj.as<int32_t>(), no, R, rows_max[o],
        status.as<int32_t>() + 2 + o, g->wt[o].as<int32_t>());
    BFC_LAUNCH_CHECK();
  }
  // first rank of degree >= 256 per layer (status words 8 and 9)
  if (!groups) {
    for (int x = 0; x < 2; ++x) {
      first_rank_kernel<<<1, 64, 0, s>>>(g->side[x].off.as<int32_t>(), n[x], 256, status.as<int32_t>() + 8 + x);
      BFC_LAUNCH_CHECK();
    }
  }
  // duplicates, the tables' first rows and the byte ranks are read by finish_schedule
  g->rows_max[0] = rows_max[0];
  g->rows_max[1] = rows_max[1];
}

// ---------------------------------------------------------------- schedule
namespace {

// deg[r] = off[r + 1] - off[r]
__global__ void degree_of_kernel(const int32_t* __restrict__ off, int32_t n, int32_t* __restrict__ deg) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    deg[r] = off[r + 1] - off[r];
}

// The schedule's items: segment q < 2 holds layer q's starts with
// Algorithm 2's wedges (or Algorithm 3's for a layer in vpp), segment 2 + x
// the band items of layer x (Algorithm 3's wedges from a start below the
// top band into it; empty without a band).  Item i of the concatenation is
// start i - first[q] of segment q.
struct Segs {
  const int64_t* work[4];  // wedges per start
  const int32_t* pre[4];   // middles per start
  const int32_t* off[2];   // first slot of each start's list, per layer
  int64_t first[5];        // first item of each segment; first[4] = item count
};

__device__ __forceinline__ int seg_of(const Segs& g, int64_t i) {
  return (int)(i >= g.first[1]) + (int)(i >= g.first[2]) + (int)(i >= g.first[3]);
}

// item code: band item << 31 | layer << 30 | rank
__device__ __forceinline__ int32_t item_code(int q, int32_t r) {
  return (int32_t)(((uint32_t)(q >> 1) << 31) | ((uint32_t)(q & 1) << 30) | (uint32_t)r);
}

// Classifies item i: 0 = no pair can reach a count of 2, 1 = light, 2 = heavy.
// sums: [0] |W|, [1] max prefix of a heavy start, [2] light wedges,
// [3] heavy wedges, [4] light middles, [5] heavy middles, [6] max start wedges
// Starts in the dense block (the top KU / KL ranks) always go to the
// workgroup kernel, which seeds them with the block's MFMA products.
constexpr int kClassifyNT = 256;

__global__ __launch_bounds__(kClassifyNT) void classify_kernel(Segs sg,
                                int64_t light_max, const int32_t* __restrict__ glight,
                                const int32_t* __restrict__ gid0, const int32_t* __restrict__ gid1,
                                int32_t KU, int32_t KL, int64_t* __restrict__ is_light,
                                int64_t* __restrict__ is_heavy, unsigned long long* __restrict__ sums) {
  const int64_t n = sg.first[4];
  const int32_t n0 = (int32_t)sg.first[1], n1 = (int32_t)(sg.first[2] - sg.first[1]);
  unsigned long long s_all = 0, s_lw = 0, s_hw = 0, s_lm = 0, s_hm = 0, max_w = 0;
  int32_t max_pre = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int q = seg_of(sg, i);
    const int32_t r = (int32_t)(i - sg.first[q]);
    const int x = q & 1;
    const int64_t w = sg.work[q][r];
    const int32_t pre = sg.pre[q][r];
    const bool in_block = q < 2 && (x == 0 ? r >= n0 - KU : r >= n1 - KL);
    // a tuned batch: this start's graph's cutoff
    const int64_t lm = glight ? (int64_t)glight[x == 0 ? gid0[r] : gid1[r]] : light_max;
    const bool heavy = w > lm || (in_block && w >= 2);
    const bool light = w >= 2 && !heavy;
    s_all += (unsigned long long)w;
    // light starts: small ones count in is_light's low word, mid ones in its
    // high word, large ones in is_heavy's high word (heavy starts: low word)
    const bool large = light && w > kLightMidMax;
    is_light[i] = light && !large ? (w <= kSmallMax ? 1ll : (1ll << 32)) : 0ll;
    is_heavy[i] = heavy ? 1ll : (large ? (1ll << 32) : 0ll);
    if (light) { s_lw += (unsigned long long)w; s_lm += (unsigned long long)pre; }
    if (heavy) {
      s_hw += (unsigned long long)w;
      s_hm += (unsigned long long)pre;
      max_pre = pre > max_pre ? pre : max_pre;
    }
    max_w = (unsigned long long)w > max_w ? (unsigned long long)w : max_w;
  }
  // workgroup totals, then one atomic per workgroup
  __shared__ unsigned long long red[5][kClassifyNT / 64];
  __shared__ unsigned long long rmax[2][kClassifyNT / 64];
  s_all = wave_sum(s_all);
  s_lw = wave_sum(s_lw);
  s_hw = wave_sum(s_hw);
  s_lm = wave_sum(s_lm);
  s_hm = wave_sum(s_hm);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int32_t op = __shfl_xor(max_pre, d, 64);
    const unsigned long long ow = __shfl_xor(max_w, d, 64);
    max_pre = op > max_pre ? op : max_pre;
    max_w = ow > max_w ? ow : max_w;
  }
  const int wv = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    red[0][wv] = s_all;
    red[1][wv] = s_lw;
    red[2][wv] = s_hw;
    red[3][wv] = s_lm;
    red[4][wv] = s_hm;
    rmax[0][wv] = (unsigned long long)max_pre;
    rmax[1][wv] = max_w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t[5] = {0, 0, 0, 0, 0}, mp = 0, mw = 0;
    for (int w = 0; w < kClassifyNT / 64; ++w) {
      for (int q = 0; q < 5; ++q) t[q] += red[q][w];
      mp = rmax[0][w] > mp ? rmax[0][w] : mp;
      mw = rmax[1][w] > mw ? rmax[1][w] : mw;
    }
    const int slot[5] = {0, 2, 3, 4, 5};
    for (int q = 0; q < 5; ++q)
      if (t[q]) atomicAdd(&sums[slot[q]], t[q]);
    if (mp) atomicMax(&sums[1], mp);
    if (mw) atomicMax(&sums[6], mw);
  }
}

// Light and heavy lists.  A heavy start is medium (256-thread workgroup)
// when it has at most medium_max wedges and kMediumMaxPre middles and lies
// outside the dense block; the key orders big starts first, each class by
// decreasing work.  n_medium counts the medium starts.
__global__ void compact_kernel(const int64_t* __restrict__ is_light, const int64_t* __restrict__ is_heavy,
                               const int64_t* __restrict__ pos_light, const int64_t* __restrict__ pos_heavy,
                               Segs sg, int64_t medium_max, int32_t KU, int32_t KL,
                               int4* __restrict__ light, int32_t* __restrict__ heavy,
                               uint32_t* __restrict__ heavy_key, unsigned long long* __restrict__ n_medium,
                               long long* __restrict__ counts) {
  const int64_t n = sg.first[4];
  const int32_t n0 = (int32_t)sg.first[1], n1 = (int32_t)(sg.first[2] - sg.first[1]);
  // the small light starts come first, then the mid ones, then the large ones
  const int32_t n_small = (int32_t)(pos_light[n] & 0xFFFFFFFFll);
  const int32_t n_mid = (int32_t)(pos_light[n] >> 32);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counts[0] = pos_light[n];
    counts[1] = pos_heavy[n];
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int q = seg_of(sg, i);
    const int32_t r = (int32_t)(i - sg.first[q]);
    const int x = q & 1;
    const int32_t code = item_code(q, r);
    const int64_t fl = is_light[i];
    const int64_t fh = is_heavy[i];
    const int64_t w = sg.work[q][r];
    const int32_t pre = sg.pre[q][r];
    if (fl || (fh >> 32)) {
      const int64_t pl = pos_light[i];
      const int32_t at = (fl & 0xFFFFFFFFll)   ? (int32_t)(pl & 0xFFFFFFFFll)
                         : fl                  ? n_small + (int32_t)(pl >> 32)
                                               : n_small + n_mid + (int32_t)(pos_heavy[i] >> 32);
      light[at] = make_int4(code, sg.off[x][r], pre, (int32_t)w);
    }
    bool med = false;
    if (fh & 0xFFFFFFFFll) {
      const bool in_block = q < 2 && (x == 0 ? r > n0 - KU : r > n1 - KL);
      med = medium_max > 0 && w <= medium_max && pre <= kMediumMaxPre && !in_block;
      // ascending keys: big starts by decreasing work (steps of 2^(1/512)), then medium ones
      const int32_t lg = (int32_t)(512.0f * log2f((float)w));
      const int32_t at = (int32_t)(pos_heavy[i] & 0xFFFFFFFFll);
      heavy[at] = code;
      heavy_key[at] = (med ? 0x8000u : 0u) | (uint32_t)(32767 - (lg < 32767 ? lg : 32767));
    }
    const uint64_t mb = __ballot(med);
    if (__lane_id() == 0 && mb) atomicAdd(n_medium, (unsigned long long)__popcll(mb));
  }
}

// Heavy list entries {code, off[rank], middles, wedges (clamped to int32)}
// in the sorted order of the codes.
__global__ void heavy_entries_kernel(const uint32_t* __restrict__ codes, const int64_t* __restrict__ n_dev, Segs sg,
                                     int4* __restrict__ out) {
  const int32_t n = (int32_t)(*n_dev & 0xFFFFFFFFll);  // heavy starts: the low word
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t code = codes[i];
    const int x = (int)((code >> 30) & 1u);
    const int q = (int)(code >> 31) * 2 + x;
    const int32_t r = (int32_t)(code & ((1u << 30) - 1u));
    const int64_t w = sg.work[q][r];
    out[i] = make_int4((int32_t)code, sg.off[x][r], sg.pre[q][r], w < 0x7FFFFFFF ? (int32_t)w : 0x7FFFFFFF);
  }
}

// First slot of each list of the other layer whose end rank is >= lo (a
// binary search per list; lists ascend).
__global__ void band_lb_kernel(const int32_t* __restrict__ off_o, const int32_t* __restrict__ adj_o, int32_t n_o,
                               int32_t lo, int32_t* __restrict__ out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n_o; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = off_o[v], b = off_o[v + 1];
    while (a < b) {
      const int32_t mid = a + ((b - a) >> 1);
      if (adj_o[mid] < lo) a = mid + 1; else b = mid;
    }
    out[v] = a;
  }
}

// Per start r of a layer with a top band [band_lo, n) (one wavefront per
// start):
//   wband[r] = Algorithm 2's wedges through its lower-priority middles that
//              end in the start's own part: ranks [band_lo, r) for a band
//              start, [0, r) below the band;
//   wtop[r]  = for a start below the band, Algorithm 3's wedges that end in
//              the band: per middle v, the entries of N(v) above both r and
//              v and >= band_lo (0 for band starts).
__global__ void band_work_kernel(const int32_t* __restrict__ off_x, const int32_t* __restrict__ adj_x,
                                 const int32_t* __restrict__ rev_x, const int32_t* __restrict__ lo_x,
                                 const int32_t* __restrict__ off_o, const int32_t* __restrict__ lo_o,
                                 const int32_t* __restrict__ blb, int32_t n, int32_t band_lo,
                                 int64_t* __restrict__ wband, int64_t* __restrict__ wtop) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t wi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wi < n; wi += waves) {
    const int32_t r = (int32_t)wi;
    const int32_t a0 = off_x[r], lo = lo_x[r], d = off_x[r + 1] - a0;
    const bool top = r >= band_lo;
    unsigned long long t0 = 0, t1 = 0;
    for (int32_t j = lane; j < d; j += 64) {
      const int32_t a = a0 + j;
      const int32_t v = adj_x[a];
      const int32_t b = blb[v];
      if (j < lo) {
        const int32_t s0 = top ? b : off_o[v];
        const int32_t e0 = rev_x[a];
        t0 += (unsigned long long)(e0 > s0 ? e0 - s0 : 0);
      }
      if (!top) {
        int32_t s0 = j < lo ? rev_x[a] + 1 : off_o[v] + lo_o[v];
        s0 = s0 > b ? s0 : b;
        const int32_t e0 = off_o[v + 1];
        t1 += (unsigned long long)(e0 > s0 ? e0 - s0 : 0);
      }
    }
    t0 = wave_sum(t0);
    t1 = wave_sum(t1);
    if (lane == 0) {
      wband[r] = (int64_t)t0;
      wtop[r] = (int64_t)t1;
    }
  }
}

}  // namespace

void build_schedule(bfc_graph_s* g, hipStream_t s) {
  Schedule& sc = g->sched;
  const int32_t n0 = g->side[0].n, n1 = g->side[1].n;
  // Algorithm 2: a start's middles are its lower-priority prefix (lo) and its
  // work the wedges through them.  Algorithm 3: every neighbour is a middle
  // (the degree) and the work is Algorithm 3's count for the start.  A top
  // band splits a layer's pairs between the two (band_work_kernel).
  const bool vpp = g->tune.vpp != 0;  // Algorithm 3 in at least one layer
  const bool batch = g->grank[0].bytes != 0;
  TmpBuf degs[2];
  Segs sg{};
  int32_t band = 0;
  for (int x = 0; x < 2; ++x) {
    Side& sd = g->side[x];
    sg.work[x] = sd.work.as<int64_t>();
    sg.pre[x] = sd.lo.as<int32_t>();
    sg.off[x] = sd.off.as<int32_t>();
    const bool layer_vpp = (g->tune.vpp >> x) & 1;
    const int64_t T = g->tune.top_band;
    sd.band_lo = (!layer_vpp && !batch && T > 0 && sd.n > T) ? (int32_t)(sd.n - T) : 0;
    if (layer_vpp || sd.band_lo > 0) {
      degs[x].alloc(sizeof(int32_t) * (size_t)sd.n, s);
      degree_of_kernel<<<grid_1d(sd.n), 256, 0, s>>>(sd.off.as<int32_t>(), sd.n, degs[x].as<int32_t>());
      BFC_LAUNCH_CHECK();
    }
    if (layer_vpp) {
      if (sd.wpp.bytes < sizeof(int64_t) * (size_t)sd.n) {
        sd.wpp.alloc(sizeof(int64_t) * (size_t)sd.n, s);
        vpp_work(g, x, sd.wpp.as<int64_t>(), s);
      }
      sg.work[x] = sd.wpp.as<int64_t>();
      sg.pre[x] = degs[x].as<int32_t>();
    } else if (sd.band_lo > 0) {
      const Side& od = g->side[1 - x];
      sd.band_lb.alloc(sizeof(int32_t) * (size_t)od.n, s);
      sd.wband.alloc(sizeof(int64_t) * (size_t)sd.n, s);
      sd.wtop.alloc(sizeof(int64_t) * (size_t)sd.n, s);
      if (od.n > 0) {
        band_lb_kernel<<<grid_1d(od.n), 256, 0, s>>>(od.off.as<int32_t>(), od.adj.as<int32_t>(), od.n, sd.band_lo,
                                                     sd.band_lb.as<int32_t>());
        BFC_LAUNCH_CHECK();
      }
      const int64_t wg = ((int64_t)sd.n + 3) / 4;
      band_work_kernel<<<(unsigned)(wg < 65536 ? wg : 65536), 256, 0, s>>>(
          sd.off.as<int32_t>(), sd.adj.as<int32_t>(), sd.rev.as<int32_t>(), sd.lo.as<int32_t>(),
          od.off.as<int32_t>(), od.lo.as<int32_t>(), sd.band_lb.as<int32_t>(), sd.n, sd.band_lo,
          sd.wband.as<int64_t>(), sd.wtop.as<int64_t>());
      BFC_LAUNCH_CHECK();
      sg.work[x] = sd.wband.as<int64_t>();
      sg.work[2 + x] = sd.wtop.as<int64_t>();
      sg.pre[2 + x] = degs[x].as<int32_t>();
      band |= 1 << x;
    } else {
      sd.band_lb.release(s);
      sd.wband.release(s);
      sd.wtop.release(s);
    }
  }
  sc.vpp = g->tune.vpp;
  sc.band = band;
  sg.first[0] = 0;
  sg.first[1] = n0;
  sg.first[2] = (int64_t)n0 + n1;
  sg.first[3] = sg.first[2] + ((band & 1) ? n0 : 0);
  sg.first[4] = sg.first[3] + ((band & 2) ? n1 : 0);
  const int64_t n = sg.first[4];
  // Algorithm 3's heavy starts all take the 1024-thread shape: the 256-thread
  // shape hung on them (kept off until its cause is found)
  // totals go to g->info from byte 64: [0..7] the classify sums, [7] medium
  // starts, [8] light counts (small | mid << 32), [9] heavy | large light << 32
  unsigned long long* sums = reinterpret_cast<unsigned long long*>(g->info.as<char>() + 64);
  BFC_HIP(hipMemsetAsync(sums, 0, 16 * sizeof(int64_t), s));
  TmpBuf flags_l, flags_h, pos_l, pos_h;
  flags_l.alloc(sizeof(int64_t) * (size_t)n, s);
  flags_h.alloc(sizeof(int64_t) * (size_t)n, s);
  pos_l.alloc(sizeof(int64_t) * (size_t)(n + 1), s);
  pos_h.alloc(sizeof(int64_t) * (size_t)(n + 1), s);
  const int64_t light_max =
      g->tune.light_max_wedges < g->light_max_cap() ? g->tune.light_max_wedges : g->light_max_cap();
  // the dense block seeds Algorithm 2's windows over whole layers only
  const int32_t K = (vpp || band) ? 0 : g->tune.dense_block;
  int32_t KU = K > 0 ? (K < n0 ? K : n0) : 0;
  int32_t KL = K > 0 ? (K < n1 ? K : n1) : 0;
  if (KU == 0 || KL == 0) KU = KL = 0;
  if (n > 0) {
    classify_kernel<<<grid_1d(n) < 1024 ? grid_1d(n) : 1024, kClassifyNT, 0, s>>>(
        sg, light_max, g->glight.bytes ? g->glight.as<int32_t>() : nullptr, g->gid[0].as<int32_t>(),
        g->gid[1].as<int32_t>(), KU, KL, flags_l.as<int64_t>(), flags_h.as<int64_t>(), sums);
    BFC_LAUNCH_CHECK();
  }
  exclusive_scan_i64(flags_l.as<int64_t>(), pos_l.as<int64_t>(), n, pos_l.as<int64_t>() + n, s);
  exclusive_scan_i64(flags_h.as<int64_t>(), pos_h.as<int64_t>(), n, pos_h.as<int64_t>() + n, s);
  // the list sizes are known only once the build is read back: each list
  // holds every item (32 bytes per item for both; shrinking them would
  // take a copy and a wait at the end of every build)
  sc.light.alloc(sizeof(int4) * (size_t)n, s);
  sc.heavy.alloc(sizeof(int4) * (size_t)n, s);
  TmpBuf hkey, hkey_tmp, hval_tmp, hcode;
  hcode.alloc(sizeof(uint32_t) * (size_t)n, s);
  hkey.alloc(sizeof(uint32_t) * (size_t)n, s);
  hkey_tmp.alloc(sizeof(uint32_t) * (size_t)n, s);
  hval_tmp.alloc(sizeof(uint32_t) * (size_t)n, s);
  if (n > 0) {
    BFC_HIP(hipMemsetAsync(hkey.p, 0xFF, sizeof(uint32_t) * (size_t)n, s));  // past the heavy starts: key 0xFFFF...
    // the 256-thread shape walks Algorithm 2's wedges of whole layers only
    compact_kernel<<<grid_1d(n), 256, 0, s>>>(flags_l.as<int64_t>(), flags_h.as<int64_t>(), pos_l.as<int64_t>(),
                                               pos_h.as<int64_t>(), sg,
                                               (vpp || band) ? 0 : (int64_t)g->tune.medium_max_wedges, KU, KL,
                                               sc.light.as<int4>(), hcode.as<int32_t>(), hkey.as<uint32_t>(),
                                               sums + 7, reinterpret_cast<long long*>(sums + 8));
    BFC_LAUNCH_CHECK();
    // heavy starts first, in key order (16-bit keys)
    if (n > 1)
      radix_sort_u32(hkey.as<uint32_t>(), hcode.as<uint32_t>(), hkey_tmp.as<uint32_t>(), hval_tmp.as<uint32_t>(), n,
                     16, s);
    heavy_entries_kernel<<<grid_1d(n), 256, 0, s>>>(hcode.as<uint32_t>(), pos_h.as<int64_t>() + n, sg,
                                                    sc.heavy.as<int4>());
    BFC_LAUNCH_CHECK();
  }
}

namespace {
// Replaces b's block by a copy of its first `bytes` bytes (stream-ordered).
}  // namespace

void finish_schedule(bfc_graph_s* g, hipStream_t s) {
  Schedule& sc = g->sched;
  // the whole info block in one read-back: status words, schedule totals,
  // caterpillar slots
  char* info = static_cast<char*>(pinned_stage(kInfoBytes));
  BFC_HIP(hipMemcpyAsync(info, g->info.p, kInfoBytes, hipMemcpyDeviceToHost, s));
  BFC_HIP(hipStreamSynchronize(s));
  const int32_t* st = reinterpret_cast<const int32_t*>(info);
  const int64_t* t = reinterpret_cast<const int64_t*>(info + 64);
  const int64_t* cat_slots = reinterpret_cast<const int64_t*>(info + kInfoCaterpillars);
  if (st[1]) throw Error{BFC_ERR_DUPLICATE_EDGE, "the edge list repeats an (upper, lower) pair"};
  const int32_t nn[2] = {g->side[0].n, g->side[1].n};
  for (int o = 0; o < 2; ++o) {
    if (g->rows_max[o] <= 0) continue;
    const int32_t lo = (int32_t)(nn[o] - g->rows_max[o]);
    g->wt_first[o] = st[2 + o] > lo ? st[2 + o] : lo;
  }
  g->byte_rank[0] = st[8];
  g->byte_rank[1] = st[9];
  sc.wedges = t[0];
  sc.max_prefix = (int32_t)t[1];
  sc.wedges_light = t[2];
  sc.wedges_heavy = t[3];
  sc.middles_light = t[4];
  sc.middles_heavy = t[5];
  sc.max_start_wedges = t[6];
  sc.n_medium = (int32_t)t[7];
  sc.n_small = (int32_t)(t[8] & 0xFFFFFFFFll);
  sc.n_mid = (int32_t)(t[8] >> 32);
  sc.n_light = sc.n_small + sc.n_mid + (int32_t)(t[9] >> 32);
  sc.n_heavy = (int32_t)(t[9] & 0xFFFFFFFFll);
  sc.light_max = g->tune.light_max_wedges < g->light_max_cap() ? g->tune.light_max_wedges : g->light_max_cap();
  sc.medium_max = g->tune.medium_max_wedges;
  int64_t cat = 0;
  for (int i = 0; i < kCatSlots; ++i) cat += cat_slots[i];
  g->caterpillars = cat;
}

// ---------------------------------------------------------------- batches
namespace {

// Edges come grouped by graph, so a tile of consecutive edges spans few
// graphs: one binary search finds the tile's first graph, and each edge
// steps forward from it (usually not at all).
constexpr int kShiftNT = 256;
constexpr int kShiftTile = 4 * kShiftNT;
__global__ __launch_bounds__(kShiftNT) void shift_kernel(const int32_t* __restrict__ edges, int64_t m,
                                                         const int64_t* __restrict__ eoff, int32_t G,
                                                         const int32_t* __restrict__ uoff,
                                                         const int32_t* __restrict__ loff, int32_t* __restrict__ out,
                                                         int32_t* __restrict__ status) {
  __shared__ int32_t s_g0;
  const int64_t t0 = (int64_t)blockIdx.x * kShiftTile;
  if (threadIdx.x == 0) s_g0 = graph_of<int64_t>(eoff, G, t0);
  __syncthreads();
  const int32_t g0 = s_g0;
  for (int64_t i = t0 + threadIdx.x; i < m && i < t0 + kShiftTile; i += kShiftNT) {
    int32_t gi = g0;
    while (gi + 1 < G && eoff[gi + 1] <= i) ++gi;
    const int2 e = reinterpret_cast<const int2*>(edges)[i];
    const int32_t nu = uoff[gi + 1] - uoff[gi];
    const int32_t nl = loff[gi + 1] - loff[gi];
    int2 o;
    if (e.x < 0 || e.x >= nu || e.y < 0 || e.y >= nl) {
      atomicOr(&status[0], 1);
      o.x = 0;
      o.y = 0;
    } else {
      o.x = e.x + uoff[gi];
      o.y = e.y + loff[gi];
    }
    reinterpret_cast<int2*>(out)[i] = o;
  }
}

// Graph of every rank (a graph's ranks are contiguous, [voff[g], voff[g+1]),
// as its ids are) and per-graph wedge sums: per wavefront, each run of
// lanes in one graph adds its sum with one atomic.
__global__ void gid_kernel(int32_t n, const int32_t* __restrict__ voff, int32_t G, int32_t* __restrict__ gid,
                           const int64_t* __restrict__ work, unsigned long long* __restrict__ gw) {
  const int lane = __lane_id();
  for (int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ll; b < n;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = b + lane;
    int32_t gi = -1;
    unsigned long long w = 0;
    if (r < n) {
      gi = graph_of<int32_t>(voff, G, (int32_t)r);
      gid[r] = gi;
      w = (unsigned long long)work[r];
    }
    // runs of equal graph over the lanes: the last lane of a run adds the run's sum
    const int32_t g_prev = __shfl_up(gi, 1, 64);
    const int32_t g_next = __shfl_down(gi, 1, 64);
    const bool head = lane == 0 || g_prev != gi;
    const bool tail = lane == 63 || g_next != gi;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? heads : heads & ((2ull << lane) - 1ull);
    const int s0 = 63 - (int)__builtin_clzll(upto);
    const unsigned long long inc = wave_inclusive_scan(w);
    const unsigned long long before = __shfl(inc, s0 > 0 ? s0 - 1 : 0, 64);
    if (tail && gi >= 0) {
      const unsigned long long run = inc - (s0 > 0 ? before : 0ull);
      if (run) atomicAdd(&gw[gi], run);
    }
  }
}

}  // namespace

void build_batch(bfc_graph_s* g, const int32_t* edges, const int64_t* eoff_host, const int32_t* nu_host,
                 const int32_t* nl_host, int32_t G, hipStream_t s) {
  std::vector<int32_t> uoff(G + 1, 0), loff(G + 1, 0);
  int64_t su = 0, sl = 0;
  for (int32_t i = 0; i < G; ++i) {
    if (nu_host[i] < 0 || nl_host[i] < 0) throw Error{BFC_ERR_INVALID_ARGUMENT, "negative layer size in batch"};
    if (eoff_host[i + 1] < eoff_host[i]) throw Error{BFC_ERR_INVALID_ARGUMENT, "edge offsets must not decrease"};
    if (eoff_host[i + 1] - eoff_host[i] > (int64_t)nu_host[i] * nl_host[i])
      throw Error{BFC_ERR_DUPLICATE_EDGE, "a graph of the batch has more edges than (upper, lower) pairs"};
    su += nu_host[i];
    sl += nl_host[i];
    if (su >= (1 << 30) || sl >= (1 << 30)) throw Error{BFC_ERR_TOO_LARGE, "batch layers must stay below 2^30"};
    uoff[i + 1] = (int32_t)su;
    loff[i + 1] = (int32_t)sl;
  }
  const int64_t m = eoff_host[G];
  g->m = m;
  g->n_upper = (int32_t)su;
  g->n_lower = (int32_t)sl;
  g->n_graphs = G;
  g->key_span[0] = G > 0 ? *std::max_element(nu_host, nu_host + G) : 0;
  g->key_span[1] = G > 0 ? *std::max_element(nl_host, nl_host + G) : 0;
  TmpBuf d_eoff, d_uoff, d_loff, shifted, status;
  d_eoff.alloc(sizeof(int64_t) * (size_t)(G + 1), s);
  d_uoff.alloc(sizeof(int32_t) * (size_t)(G + 1), s);
  d_loff.alloc(sizeof(int32_t) * (size_t)(G + 1), s);
  shifted.alloc(sizeof(int32_t) * 2 * (size_t)m, s);
  status.alloc(4 * sizeof(int32_t), s);
  BFC_HIP(hipMemcpyAsync(d_eoff.p, eoff_host, sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
  BFC_HIP(hipMemcpyAsync(d_uoff.p, uoff.data(), sizeof(int32_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
  BFC_HIP(hipMemcpyAsync(d_loff.p, loff.data(), sizeof(int32_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
  BFC_HIP(hipMemsetAsync(status.p, 0, 4 * sizeof(int32_t), s));
  if (m > 0) {
    shift_kernel<<<(unsigned)((m + kShiftTile - 1) / kShiftTile), kShiftNT, 0, s>>>(
        edges, m, d_eoff.as<int64_t>(), G, d_uoff.as<int32_t>(), d_loff.as<int32_t>(), shifted.as<int32_t>(),
        status.as<int32_t>());
    BFC_LAUNCH_CHECK();
  }
  int32_t st[4] = {0, 0, 0, 0};
  BFC_HIP(hipMemcpyAsync(st, status.p, sizeof(st), hipMemcpyDeviceToHost, s));
  BFC_HIP(hipStreamSynchronize(s));
  if (st[0]) throw Error{BFC_ERR_VERTEX_OUT_OF_RANGE, "a batch edge has an id outside its graph's layers"};
  const int32_t* groups[2] = {d_uoff.as<int32_t>(), d_loff.as<int32_t>()};
  build_graph(g, shifted.as<int32_t>(), s, groups, G);
  // graph i's vertices of layer x hold ranks [off_x[i], off_x[i+1]) of that layer
  for (int x = 0; x < 2; ++x) {
    g->grank[x].alloc(sizeof(int32_t) * (size_t)(G + 1), s);
    BFC_HIP(hipMemcpyAsync(g->grank[x].p, groups[x], sizeof(int32_t) * (size_t)(G + 1), hipMemcpyDeviceToDevice, s));
  }
  TmpBuf gw;
  gw.alloc(sizeof(int64_t) * (size_t)G, s);
  BFC_HIP(hipMemsetAsync(gw.p, 0, sizeof(int64_t) * (size_t)G, s));
  const TmpBuf* voff[2] = {&d_uoff, &d_loff};
  for (int x = 0; x < 2; ++x) {
    Side& sd = g->side[x];
    g->gid[x].alloc(sizeof(int32_t) * (size_t)sd.n, s);
    if (sd.n > 0) {
      gid_kernel<<<grid_1d(sd.n), 256, 0, s>>>(sd.n, voff[x]->as<int32_t>(), G, g->gid[x].as<int32_t>(),
                                                sd.work.as<int64_t>(), gw.as<unsigned long long>());
      BFC_LAUNCH_CHECK();
    }
  }
  g->graph_wedges.assign(G, 0);
  BFC_HIP(hipMemcpyAsync(g->graph_wedges.data(), gw.p, sizeof(int64_t) * (size_t)G, hipMemcpyDeviceToHost, s));
  BFC_HIP(hipStreamSynchronize(s));
}

}  // namespace bfc
