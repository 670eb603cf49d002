// Wedge enumeration and counting: the hot loop of BFC-VP (Algorithm 2), its
// per-edge second pass (Algorithm 4) and per-vertex counts (Lemma 1).
//
// For a start r of layer X (rank r in X's ascending priority order):
//   middles  = the first lo_X[r] entries of N(r)             (p(v) < p(r))
//   ends     = for middle v reached through slot k, the entries of N(v)
//              before r, i.e. adj_other[off_other[v] .. rev_X[k])  (p(w) < p(r))
// count_wedge(w) is accumulated on chip and each distinct end adds
// C(count,2) = count(count-1)/2 (int64) to the total.  Ends are ranks of X,
// all below r, so a window [lo, hi) of end ranks selects, in every middle's
// (sorted) list, one contiguous sub-slice.
//
// Work split (from the per-start wedge counts computed at build time):
//   light starts (2 <= wedges <= light_max): one wavefront each, with a
//     wavefront-private LDS hash table of >= 2x the start's wedges.
//   heavy starts (> light_max), in decreasing order of wedges: one 1024-thread
//     workgroup each, taken from a global ticket.  The workgroup walks end-rank
//     windows; per window it either keeps dense LDS counters (32K int32, when
//     wedges >= range / dense_min_ratio) or an LDS hash table (16K entries;
//     a window whose distinct ends would overfill it is halved and redone).
//     Middles are processed 1024 at a time; a workgroup prefix sum of their
//     slice lengths spreads the wedges evenly over the threads and each
//     thread finds its middle by binary search in LDS, so global reads of
//     end ids stay coalesced.
// The count of a pair is final once its window has been walked, so the
// per-edge and per-vertex second pass runs window by window.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace bfc {

namespace {

struct SideView {
  const int32_t* off;
  const int32_t* adj;
  const int32_t* rev;
  const int32_t* lo;
  const int32_t* id_of;
  const int64_t* work;
};

struct CountParams {
  SideView sv[2];
  const int4* list;            // heavy starts: {code, off[rank], lo[rank], wedges clamped to int32}
  int32_t n_list;
  int32_t mode;
  unsigned long long* total;
  unsigned long long* vout[2];  // per-vertex: accumulators by rank, per layer
  unsigned long long* acc[2];
  uint32_t* acc32[2];          // per-edge: 32-bit accumulators when every B_e fits (else null)
  int32_t* cursor;
  int64_t cursor_stride;
  unsigned int* ticket;
  int32_t* status;             // bit 0: a window could not be made to fit (internal error)
  int32_t dense_ratio;
  int32_t window_mode;
  int32_t hash_window_wedges;
  int32_t dense_min_wedges;
  unsigned long long* gtotal;  // per-graph totals of a batch (kTotal), else null
  const int32_t* gid[2];       // graph index of every rank, per layer (null: one graph)
  const int32_t* grank[2];     // first rank of each graph, per layer (null: one graph)
  int32_t dtop[2];             // first rank of the dense block per layer (n_X when disabled)
  const int32_t* dC[2];        // MFMA products CU, CL (row-major)
  int32_t dld[2];              // their row strides
  const int32_t* wt[2];        // window-boundary tables per middle layer (rows for ranks >= wt_first)
  int32_t wt_first[2];
  int32_t wt_row[2];
  int32_t vpp;                 // bit x: layer x's starts take Algorithm 3's wedges (ends above the start and the middle)
  const int4* gtune;           // per graph {dense ratio, window mode, hash window wedges, dense min wedges}, or null
  int32_t nX[2];               // layer sizes (the end of Algorithm 3's end ranges)
  int32_t q8[2];               // per layer: ends below this rank have degree < 256 (8-bit dense counters)
  int32_t band_lo[2];          // first rank of each layer's top band (0: no band)
  const int32_t* blb[2];       // per layer x with a band: first slot >= band_lo[x] of each other-layer list
  const int64_t* wtop[2];      // per layer x with a band: band-item wedges per start
};

__device__ __forceinline__ int32_t graph_index(const CountParams& p, int x, int32_t r) {
  const int32_t* g = x ? p.gid[1] : p.gid[0];
  return g ? g[r] : 0;
}

__device__ __forceinline__ SideView pick(const CountParams& p, int x) {
  SideView s;
  s.off = x ? p.sv[1].off : p.sv[0].off;
  s.adj = x ? p.sv[1].adj : p.sv[0].adj;
  s.rev = x ? p.sv[1].rev : p.sv[0].rev;
  s.lo = x ? p.sv[1].lo : p.sv[0].lo;
  s.id_of = x ? p.sv[1].id_of : p.sv[0].id_of;
  s.work = x ? p.sv[1].work : p.sv[0].work;
  return s;
}

__device__ __forceinline__ unsigned long long* pick_ptr(unsigned long long* const* a, int x) { return x ? a[1] : a[0]; }

// Middle j of a start (its slot k = base + j in the start's list; lo_r =
// the start's lower-priority prefix) and the slice [s0, e0) of adj_other
// holding the ends of its wedges, ascending by end rank:
//   Algorithm 2: the entries of N(v) before the start, [off(v), rev(k));
//   Algorithm 3: the entries of N(v) above both the start and v: past the
//   start's slot when v ranks below the start, else past v's own
//   lower-priority prefix (which then holds the start).
// clb (non-null for a band start and for a band item): the slice also
// keeps to end ranks >= the band's first rank, clb[v] being N(v)'s first
// slot there.
__device__ __forceinline__ void mid_slice(bool vpp, const SideView& S, const SideView& O, int32_t k, int32_t j,
                                          int32_t lo_r, const int32_t* clb, int32_t& v, int32_t& s0, int32_t& e0) {
  v = S.adj[k];
  if (!vpp) {
    s0 = O.off[v];
    e0 = S.rev[k];
  } else {
    s0 = j < lo_r ? S.rev[k] + 1 : O.off[v] + O.lo[v];
    e0 = O.off[v + 1];
  }
  if (clb) {
    const int32_t b = clb[v];
    s0 = s0 > b ? s0 : b;
  }
}

// The band part of a list item: clb for mid_slice (null: none) and the end
// ranks [elo, ehi) of the item's wedges when it has a band part (band
// start: [band_lo, r); band item: [band_lo, n)).
struct BandPart {
  const int32_t* clb;
  bool band_item;
};

__device__ __forceinline__ BandPart band_part(const CountParams& p, int32_t code, int x, int32_t r) {
  BandPart b;
  b.band_item = (uint32_t)code >> 31;
  const int32_t lo = x ? p.band_lo[1] : p.band_lo[0];
  b.clb = (lo > 0 && (b.band_item || r >= lo)) ? (x ? p.blb[1] : p.blb[0]) : nullptr;
  return b;
}

// Adds d to per-arc accumulator i of side x.  Every partial sum is at most
// its edge's B_e <= (d_u - 1)(d_v - 1), so while the largest degrees keep
// that below 2^32 the accumulators are 32-bit words: half the atomic traffic.
__device__ __forceinline__ void acc_add(const CountParams& p, int x, int64_t i, unsigned long long d) {
  if (p.acc32[0]) atomicAdd(&(x ? p.acc32[1] : p.acc32[0])[i], (uint32_t)d);
  else atomicAdd(&(x ? p.acc[1] : p.acc[0])[i], d);
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x *= 0x9E3779B1u;
  return x ^ (x >> 15);
}

__device__ __forceinline__ unsigned long long choose2(int32_t c) {
  return (unsigned long long)c * (unsigned long long)(c - 1) / 2ull;
}

// first index in [lo, hi) with a[index] >= key (a ascending), by galloping from lo
__device__ __forceinline__ int32_t gallop_lower_bound(const int32_t* __restrict__ a, int32_t lo, int32_t hi,
                                                      int32_t key) {
  if (lo >= hi || a[lo] >= key) return lo;
  int32_t prev = lo;  // a[prev] < key
  int32_t step = 1;
  while (prev + step < hi && a[prev + step] < key) {
    prev += step;
    step <<= 1;
  }
  int32_t l = prev + 1;
  int32_t h = prev + step < hi ? prev + step : hi;
  while (l < h) {
    const int32_t mid = (l + h) >> 1;
    if (a[mid] < key) l = mid + 1; else h = mid;
  }
  return l;
}

constexpr int32_t kNoEnd = 0x7FFFFFFF;  // "no further end" (no rank reaches it)

// First index in [lo, hi) with a[index] >= key when the answer is usually
// within a few entries of lo: four probes, then a gallop.  Also returns
// a[index] in val (kNoEnd when index == hi).  (Probes made unconditional, or
// more of them, measured slower: more loads and registers in the window
// set-up than the latency they save.)
__device__ __forceinline__ int32_t near_lower_bound_v(const int32_t* __restrict__ a, int32_t lo, int32_t hi,
                                                      int32_t key, int32_t& val) {
  const int32_t n = hi - lo;
  val = kNoEnd;
  if (n <= 0) return lo;
  const int32_t a0 = a[lo];
  const int32_t a1 = n > 1 ? a[lo + 1] : kNoEnd;
  const int32_t a2 = n > 2 ? a[lo + 2] : kNoEnd;
  const int32_t a3 = n > 3 ? a[lo + 3] : kNoEnd;
  if (a0 >= key) { val = a0; return lo; }
  if (a1 >= key) { val = a1; return lo + 1; }
  if (a2 >= key) { val = a2; return lo + 2; }
  if (a3 >= key) { val = a3; return lo + 3; }
  const int32_t i = gallop_lower_bound(a, lo + 4, hi, key);
  if (i < hi) val = a[i];
  return i;
}

__device__ __forceinline__ int32_t near_lower_bound(const int32_t* __restrict__ a, int32_t lo, int32_t hi,
                                                    int32_t key) {
  int32_t val;
  return near_lower_bound_v(a, lo, hi, key, val);
}

// First slot of a table middle's list (row `rowp` of the window-boundary
// table) whose end rank is >= key: the table entry of key's 2^kWinShift
// block, then a gallop inside that block when key is not a block start.
__device__ __forceinline__ int32_t table_lb(const int32_t* __restrict__ oadj, const int32_t* __restrict__ rowp,
                                            int32_t key) {
  const int32_t w = key >> kWinShift;
  const int32_t a = rowp[w];
  if ((key & ((1 << kWinShift) - 1)) == 0) return a;
  return gallop_lower_bound(oadj, a, rowp[w + 1], key);
}

// ------------------------------------------------------------ wavefront helpers
// end id at slot (a 32-bit byte offset from a wavefront-uniform base)
__device__ __forceinline__ int32_t load_end(const int32_t* __restrict__ oadj, int32_t slot) {
  return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(oadj) + ((uint32_t)slot << 2));
}

// number of set bits of m in lanes below this one, plus add
__device__ __forceinline__ int32_t mbcnt(uint64_t m, int32_t add) {
  return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)add));
}

// Inclusive prefix maximum over the lanes of non-negative values: shifts of
// 1, 2, 4 and 8 lanes inside each row of 16, then the row broadcasts of
// lanes 15 and 31 (lanes a shift moves out of range read 0).
__device__ __forceinline__ int32_t wave_prefix_max(int32_t v) {
  int32_t t;
  t = __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v = v > t ? v : t;
  t = __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v = v > t ? v : t;
  t = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v = v > t ? v : t;
  t = __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v = v > t ? v : t;
  t = __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1 and 3
  v = v > t ? v : t;
  t = __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2 and 3
  v = v > t ? v : t;
  return v;
}

// ------------------------------------------------------------ wavefront walk
// Steps of 64 positions each lane loads before using any of them.
constexpr int kLightSteps = 4;

// Visits every wedge of a group of up to 64 middles; lane j holds middle
// j's end slice [cs, cs + len) in adj_other.  Wedges are numbered 0..tot-1
// in middle order and position f is taken by lane f mod 64.  The middle of
// position f is the last non-empty middle whose first position is <= f: per
// step of 64 positions, a ballot finds the last one starting at or before
// the step, the middles starting inside the step mark their first lane
// (ds_permute; non-empty middles start at distinct positions) and a prefix
// maximum over the lanes picks the latest mark.  fn(middle lane, slot, end)
// is called per wedge.
template <typename Fn>
__device__ __forceinline__ void light_walk(const int32_t* __restrict__ oadj, int32_t cs, int32_t len, Fn&& fn) {
  const int lane = __lane_id();
  const int32_t inc = wave_inclusive_scan(len);
  const int32_t tot = __shfl(inc, 63, 64);
  const int32_t exc = inc - len;
  const int32_t delta = cs - exc;  // slot of position f in this middle: delta + f
  for (int32_t f0 = 0; f0 < tot; f0 += 64 * kLightSteps) {
    int32_t slot[kLightSteps], w[kLightSteps], mid[kLightSteps];
#pragma unroll
    for (int q = 0; q < kLightSteps; ++q) {
      const int32_t fq = f0 + 64 * q;
      w[q] = -1;
      slot[q] = 0;
      mid[q] = 0;
      if (fq < tot) {
        // the middle holding position fq starts at or before it, so the ballot is non-empty
        const uint64_t before = __ballot(len > 0 && exc <= fq);
        const int32_t carry = 63 - (int32_t)__builtin_clzll(before);
        const int32_t e = exc - fq;
        const bool mk = len > 0 && e > 0 && e < 64;
        const int32_t mark = __builtin_amdgcn_ds_permute(mk ? e << 2 : 0, mk ? lane + 1 : 0);
        int32_t m = wave_prefix_max(mark) - 1;
        m = m > carry ? m : carry;
        const int32_t dm = __builtin_amdgcn_ds_bpermute(m << 2, delta);
        const int32_t f = fq + lane;
        if (f < tot) {
          slot[q] = dm + f;
          mid[q] = m;
          w[q] = load_end(oadj, slot[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kLightSteps; ++q)
      if (w[q] >= 0) fn(mid[q], slot[q], w[q]);
  }
}

// ------------------------------------------------------------ hash tables
// Counts one wedge to end w in a wavefront's table (keys hold w + 1, 0 when
// empty); returns the end's count before this wedge.  Summed over all
// wedges, the returned counts give sum over ends of C(count, 2).
__device__ __forceinline__ int32_t wave_hash_inc(int32_t* keys, int32_t* cnt, uint32_t mask, int32_t w) {
  const int32_t key = w + 1;
  uint32_t h = mix32((uint32_t)w) & mask;
  for (;;) {
    const int32_t cur = keys[h];
    if (cur == key) return atomicAdd(&cnt[h], 1);
    if (cur == 0) {
      const int32_t old = atomicCAS(&keys[h], 0, key);
      if (old == 0 || old == key) return atomicAdd(&cnt[h], 1);
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int32_t hash_get(const int32_t* keys, const int32_t* cnt, uint32_t mask, int32_t w) {
  const int32_t key = w + 1;
  uint32_t h = mix32((uint32_t)w) & mask;
  while (keys[h] != key) h = (h + 1) & mask;
  return cnt[h];
}

// Packed wavefront tables: one word per entry, (w + 1) << kLightCountBits |
// count, for keys w below 2^(32 - kLightCountBits) (a layer's rank, or in a
// batch its offset from the first rank of its graph) and starts of fewer
// than 2^kLightCountBits wedges.  Same probing and return
// value as wave_hash_inc.
constexpr int kLightCountBits = 12;
constexpr uint32_t kLightCountMask = (1u << kLightCountBits) - 1u;

__device__ __forceinline__ int32_t wave_packed_inc(uint32_t* tab, uint32_t mask, int32_t w) {
  const uint32_t key = (uint32_t)w + 1u;
  uint32_t h = mix32((uint32_t)w) & mask;
  for (;;) {
    const uint32_t cur = tab[h];
    if ((cur >> kLightCountBits) == key) return (int32_t)(atomicAdd(&tab[h], 1u) & kLightCountMask);
    if (cur == 0) {
      const uint32_t old = atomicCAS(&tab[h], 0u, (key << kLightCountBits) | 1u);
      if (old == 0) return 0;
      if ((old >> kLightCountBits) == key) return (int32_t)(atomicAdd(&tab[h], 1u) & kLightCountMask);
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int32_t wave_packed_get(const uint32_t* tab, uint32_t mask, int32_t w) {
  const uint32_t key = (uint32_t)w + 1u;
  uint32_t h = mix32((uint32_t)w) & mask;
  while ((tab[h] >> kLightCountBits) != key) h = (h + 1) & mask;
  return (int32_t)(tab[h] & kLightCountMask);
}

// ------------------------------------------------------------ light
// Light starts come in three classes by wedge count: up to kSmallMax wedges
// (a 512-entry table per wavefront, so a CU holds 32 wavefronts), up to
// kLightMidMax (2,048 entries: packed, 8 KB, about 20 wavefronts per CU, or
// key and count, 16 KB, 8 per CU) and, where the layers allow packing, up to
// light_max = 2048 (packed 4,096 entries, 16 KB, 8 per CU).  A table has at
// least twice as many entries as its start has wedges.
constexpr int kLightNT = 256;
constexpr int kLightWaves = kLightNT / 64;
constexpr int kLightCap = 2048;        // mid class: kLightMidMax <= kLightCap / 2
constexpr int kLightPackedCap = 4096;  // packed: light_max <= kLightPackedCap / 2
constexpr int kSmallCap = 2 * kSmallMax;
static_assert(kLightPackedCap / 2 < (1 << kLightCountBits), "packed counts must fit");
static_assert(kLightMidMax <= kLightCap / 2, "mid starts must fit the mid table");

// Each entry of the light list is {code, first slot of N(r), middles, wedges}.
// kVpp: some layer's starts take Algorithm 3's wedges (compiled out when not).
template <int kMode, int kCap, bool kPacked, bool kVpp>
__global__ __launch_bounds__(kLightNT) void light_kernel(CountParams p, const int4* __restrict__ list,
                                                         int32_t n_list) {
  // packed: kCap words; else kCap keys then kCap counts
  constexpr int kWordsPerWave = kPacked ? kCap : 2 * kCap;
  __shared__ uint32_t ttab[kLightWaves][kWordsPerWave];
  __shared__ unsigned long long tdelta[kLightWaves][kMode == kTotal ? 1 : 64];
  const int lane = __lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* ptab = ttab[wv];
  int32_t* keys = reinterpret_cast<int32_t*>(ptab);
  int32_t* cnt = keys + kCap;
  unsigned long long* dsum = tdelta[wv];
  for (int h = lane; h < kWordsPerWave; h += 64) ptab[h] = 0u;
  if (kMode != kTotal) dsum[lane] = 0;
  unsigned long long acc_total = 0;
  const int64_t stride = (int64_t)gridDim.x * kLightWaves;
  int64_t idx = (int64_t)blockIdx.x * kLightWaves + wv;
  int4 next = idx < n_list ? list[idx] : make_int4(0, 0, 0, 0);
  for (; idx < n_list; idx += stride) {
    const int4 cur = next;
    if (idx + stride < n_list) next = list[idx + stride];
    const int x = (int)(((uint32_t)cur.x >> 30) & 1u);
    const int32_t r = cur.x & ((1 << 30) - 1);
    const int32_t base = cur.y;
    const int32_t pre = cur.z;
    const SideView S = pick(p, x);
    const SideView O = pick(p, 1 - x);
    // (bands need the kVpp instantiation: band items take Algorithm 3's wedges)
    const BandPart bp = band_part(p, cur.x, x, r);
    const int32_t* clb = kVpp ? bp.clb : nullptr;
    const bool vpp = kVpp && (bp.band_item || ((p.vpp >> x) & 1));
    const int32_t lo_r = vpp ? S.lo[r] : 0;
    // packed keys of a batch count from the first rank of the start's graph
    // (every end lies in that graph's part of layer x)
    const int32_t* grank = x ? p.grank[1] : p.grank[0];
    const int32_t wlo = (kPacked && grank) ? __builtin_amdgcn_readfirstlane(grank[graph_index(p, x, r)]) : 0;
    uint32_t cap = 64;
    while ((int32_t)cap < 2 * cur.w) cap <<= 1;
    const uint32_t mask = cap - 1;
    unsigned long long a = 0;
    for (int32_t j0 = 0; j0 < pre; j0 += 64) {
      const int32_t j = j0 + lane;
      int32_t cs = 0, len = 0;
      if (j < pre) {
        int32_t v, e;
        mid_slice(vpp, S, O, base + j, j, lo_r, clb, v, cs, e);
        len = e - cs;
      }
      light_walk(O.adj, cs, len, [&](int, int32_t, int32_t w) {
        a += (unsigned)(kPacked ? wave_packed_inc(ptab, mask, w - wlo) : wave_hash_inc(keys, cnt, mask, w));
      });
    }
    if (kMode == kTotal) {
      if (p.gtotal) {
        a = wave_sum(a);
        if (lane == 0 && a) atomicAdd(&p.gtotal[graph_index(p, x, r)], a);
      } else {
        acc_total += a;
      }
    } else {
      if (kMode == kVertex) {
        // each end w gains C(count_w, 2); the start gains their sum
        unsigned long long* vs = pick_ptr(p.vout, x);
        for (uint32_t h = lane; h < cap; h += 64) {
          const uint32_t word = ptab[h];
          const int32_t c = kPacked ? (int32_t)(word & kLightCountMask) : cnt[h];
          const int32_t key = kPacked ? (int32_t)(word >> kLightCountBits) + wlo : keys[h];
          if (c > 1) atomicAdd(&vs[key - 1], choose2(c));
        }
        a = wave_sum(a);
        if (lane == 0 && a) atomicAdd(&vs[r], a);
      }
      // second pass: every wedge (r, v, w) adds count_w - 1 to the middle v
      // (Lemma 1) and, per edge, to the arcs (r, v) and (v, w) (Algorithm 4)
      unsigned long long* vmid = pick_ptr(p.vout, 1 - x);
      for (int32_t j0 = 0; j0 < pre; j0 += 64) {
        const int32_t j = j0 + lane;
        int32_t cs = 0, len = 0, v = 0;
        if (j < pre) {
          int32_t e;
          mid_slice(vpp, S, O, base + j, j, lo_r, clb, v, cs, e);
          len = e - cs;
        }
        light_walk(O.adj, cs, len, [&](int mid, int32_t slot, int32_t w) {
          const int32_t c = kPacked ? wave_packed_get(ptab, mask, w - wlo) : hash_get(keys, cnt, mask, w);
          if (c > 1) {
            const unsigned long long d = (unsigned long long)(c - 1);
            if (kMode == kEdge) acc_add(p, 1 - x, slot, d);
            atomicAdd(&dsum[mid], d);
          }
        });
        __builtin_amdgcn_wave_barrier();
        const unsigned long long d = dsum[lane];
        if (d) {
          if (kMode == kEdge) acc_add(p, x, base + j, d);
          else atomicAdd(&vmid[v], d);
          dsum[lane] = 0;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t h = lane; h < cap; h += 64) {
      if (kPacked) {
        ptab[h] = 0u;
      } else {
        keys[h] = 0;
        cnt[h] = 0;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (kMode == kTotal && p.total) {
    acc_total = wave_sum(acc_total);
    if (lane == 0 && acc_total) atomicAdd(p.total, acc_total);
  }
}

// ------------------------------------------------------------ heavy
// Workgroup shapes of the heavy kernel: big starts take 1024 threads and a
// 128 KB LDS table; medium starts (few wedges and at most kMedPre middles)
// take 256 threads and a 32 KB table, four workgroups to a CU, so their
// per-window barriers and scans occupy a quarter of the wavefronts.
constexpr int kBigNT = 1024;
constexpr int kBigWords = 32768;
constexpr int kMedNT = 256;
constexpr int kMedWords = 8192;
constexpr int kMedPre = kMediumMaxPre;  // middles of a medium start (its cursor stride)
constexpr int32_t kNone = 0x7FFFFFFF;       // "no further end" in a middle's cursor

// Inserts end w into the workgroup hash table (count 1, or bumps its count).
// Returns 1 when w is a new key, 0 when it was present, and kOverfull when
// its probe sequence reached kMaxProbe slots without finding w or a free
// slot (nothing is inserted): the caller then flags the window, which is
// halved and walked again, so an overfull table never turns into long scans.
constexpr uint32_t kMaxProbe = 64;
constexpr int kOverfull = 2;

__device__ __forceinline__ int block_hash_add(int32_t* table, uint32_t cap, int32_t w) {
  int32_t* keys = table;
  int32_t* cnt = table + cap;
  const int32_t key = w + 1;
  const uint32_t mask = cap - 1;
  uint32_t h = mix32((uint32_t)w) & mask;
  for (uint32_t probe = 0; probe < kMaxProbe; ++probe) {
    const int32_t cur = keys[h];
    if (cur == key) { atomicAdd(&cnt[h], 1); return 0; }
    if (cur == 0) {
      const int32_t old = atomicCAS(&keys[h], 0, key);
      if (old == 0) { atomicAdd(&cnt[h], 1); return 1; }
      if (old == key) { atomicAdd(&cnt[h], 1); return 0; }
    }
    h = (h + 1) & mask;
  }
  return kOverfull;
}

// Dense window counters: 32-bit, two 16-bit counters per word when every
// count fits (a count is at most the start's number of middles), or four
// 8-bit counters per word for ends of degree below 256 (an end's count is at
// most its degree: each of its wedges has its own middle in N(end)).
__device__ __forceinline__ void dense_add(int32_t* table, int32_t i, bool half) {
  if (half) atomicAdd(reinterpret_cast<uint32_t*>(&table[i >> 1]), 1u << ((i & 1) << 4));
  else atomicAdd(&table[i], 1);
}

__device__ __forceinline__ int32_t dense_get(const int32_t* table, int32_t i, bool half, bool quarter) {
  if (quarter) return (int32_t)((reinterpret_cast<const uint32_t*>(table)[i >> 2] >> ((i & 3) << 3)) & 0xFFu);
  if (half) return (int32_t)((reinterpret_cast<const uint32_t*>(table)[i >> 1] >> ((i & 1) << 4)) & 0xFFFFu);
  return table[i];
}

// Packed hash entries, for starts whose counts fit kPackBits bits (fewer
// middles than 2^kPackBits) in windows narrower than kPackMaxWidth ranks:
// one 32-bit word holds (end - lo_w + 1) << kPackBits | count, so the LDS
// table holds twice as many entries.  Same probing and overflow rules as
// block_hash_add.
constexpr int kPackBits = 12;
constexpr uint32_t kPackMask = (1u << kPackBits) - 1u;
constexpr int32_t kPackMaxPre = 1 << kPackBits;
constexpr int32_t kPackMaxWidth = (1 << (32 - kPackBits)) - 1;

__device__ __forceinline__ int packed_hash_add(uint32_t* tab, uint32_t cap, uint32_t key) {
  const uint32_t mask = cap - 1;
  uint32_t h = mix32(key) & mask;
  for (uint32_t probe = 0; probe < kMaxProbe; ++probe) {
    const uint32_t cur = tab[h];
    if ((cur >> kPackBits) == key) { atomicAdd(&tab[h], 1u); return 0; }
    if (cur == 0) {
      const uint32_t old = atomicCAS(&tab[h], 0u, (key << kPackBits) | 1u);
      if (old == 0) return 1;
      if ((old >> kPackBits) == key) { atomicAdd(&tab[h], 1u); return 0; }
    }
    h = (h + 1) & mask;
  }
  return kOverfull;
}

__device__ __forceinline__ int32_t packed_hash_get(const uint32_t* tab, uint32_t mask, uint32_t key) {
  uint32_t h = mix32(key) & mask;
  while ((tab[h] >> kPackBits) != key) h = (h + 1) & mask;
  return (int32_t)(tab[h] & kPackMask);
}


// ------------------------------------------------------------ flattened walk
// A batch of (middle, window) slices is held in LDS as a segment list:
// se[i] = exclusive prefix of the slice lengths (strictly increasing, every
// slice is non-empty; se[n] = total), sd[i] = slice start slot - se[i], so
// the slot of flattened position f inside segment i is sd[i] + f.

// Visits positions [F0, F1) of a segment list of n entries (n < 4096).
// Lane l takes positions F0 + l, F0 + 64 + l, ...; an iteration covers
// kSegSteps steps of 64 positions.  The wavefront loads the next 64 segment
// starts; a start d positions into a step marks lane d (ds_permute), and a
// lane's segment is the current one plus the starts at or below its
// position (ballot + mbcnt).  When the 64 loaded starts reach past the
// iteration (segments averaging 8 positions or more) every step is located
// from them independently and without branches; otherwise the starts are
// reloaded per step.  End ids of the next iteration are loaded before this
// one's are used.  fn(segment, slot, end) is called per wedge; stop() is
// polled (uniformly) once per iteration.
constexpr int kSegSteps = 8;

template <typename Fn, typename Stop>
__device__ __forceinline__ void seg_walk(const int32_t* __restrict__ oadj, const int32_t* se, const int32_t* sd,
                                         int32_t n, int32_t F0, int32_t F1, Fn&& fn, Stop&& stop) {
  if (F0 >= F1) return;
  const int lane = __lane_id();
  // segment holding F0: largest s with se[s] <= F0 (se[0] = 0), by two
  // rounds of a 64-way search over se[0..n]
  int32_t s0;
  {
    const int32_t n1 = n + 1;
    const int32_t stride = (n1 + 63) >> 6;
    int32_t i = lane * stride;
    const int32_t c1 = __popcll(__ballot(i < n1 && se[i] <= F0)) - 1;
    const int32_t lo = c1 * stride;
    i = lo + lane;
    s0 = lo + __popcll(__ballot(lane < stride && i < n1 && se[i] <= F0)) - 1;
  }
  int32_t sd0 = sd[s0];
  // Positions f0 + 64 q + lane (q < kSegSteps): slot, segment and end id
  // (-1: position >= F1).  Returns true when every position is < F1.
  auto gen = [&](int32_t f0, int32_t* slot, int32_t* sg, int32_t* w) -> bool {
    const int32_t fend = f0 + 64 * kSegSteps;
    int32_t idx = s0 + 1 + lane;
    int32_t b = idx <= n ? se[idx] : 0x7FFFFFFF;
    int32_t g = idx < n ? sd[idx] : 0;
    const bool full = fend <= F1;
    if (full && __shfl(b, 63, 64) >= fend) {
      // every segment start below fend is among b (ascending over lanes):
      // the steps are independent
      const int32_t e0 = b - f0 - 1;  // start offset - 1 relative to step 0
      const int32_t pos0 = f0 + lane;
      // lane 63's start lies beyond the iteration, so its bias is never
      // read (c <= 63): it carries the current segment's bias instead, which
      // c = 0 reads (byte address -4 selects lane 63)
      const int32_t g63 = lane == 63 ? sd0 : g;
#pragma unroll
      for (int q = 0; q < kSegSteps; ++q) {
        const int32_t e = e0 - 64 * q;
        const bool mk = (uint32_t)e < 63u;  // start inside (f, f + 64)
        const int32_t mark = __builtin_amdgcn_ds_permute(mk ? (e + 1) << 2 : 0, mk ? 1 : 0);
        const int32_t cb = __popcll(__ballot(e < 0));  // starts at or before f
        // lane 0 is never marked (a start at f counts in cb), so the marks
        // at or below this lane are the marks shifted down one lane below it
        const int32_t c = mbcnt(__ballot(mark != 0) >> 1, cb);
        slot[q] = __builtin_amdgcn_ds_bpermute((c << 2) - 4, g63) + pos0 + 64 * q;
        sg[q] = s0 + c;
        w[q] = load_end(oadj, slot[q]);
      }
      const int32_t cn = __popcll(__ballot(b <= fend));
      if (cn > 0) {
        sd0 = __builtin_amdgcn_readlane(g, cn - 1);
        s0 += cn;
      }
      return true;
    }
#pragma unroll
    for (int q = 0; q < kSegSteps; ++q) {
      const int32_t f = f0 + 64 * q;
      w[q] = -1;
      slot[q] = 0;
      sg[q] = 0;
      if (f < F1) {
        // invariant: se[s0] <= f < se[s0 + 1], so every loaded start is > f
        if (q > 0) {
          idx = s0 + 1 + lane;
          b = idx <= n ? se[idx] : 0x7FFFFFFF;
          g = idx < n ? sd[idx] : 0;
        }
        const int32_t d = b - f;
        const int32_t mark = __builtin_amdgcn_ds_permute(d < 64 ? 4 * d : 0, d < 64 ? 1 : 0);
        // as above: lane 0 is never marked (d >= 1), and at most 63 starts
        // fall inside the step, so lane 63 may carry the current bias
        const int32_t c = mbcnt(__ballot(mark != 0) >> 1, 0);
        const int32_t gc = __builtin_amdgcn_ds_bpermute((c << 2) - 4, lane == 63 ? sd0 : g);
        if (f + lane < F1) {
          slot[q] = gc + f + lane;
          sg[q] = s0 + c;
          w[q] = load_end(oadj, slot[q]);
        }
        const int32_t cn = __popcll(__ballot(d <= 64));
        if (cn > 0) {
          sd0 = __builtin_amdgcn_readlane(g, cn - 1);
          s0 += cn;
        }
      }
    }
    return full;
  };
  int32_t slot_a[kSegSteps], sg_a[kSegSteps], w_a[kSegSteps];
  bool full_a = gen(F0, slot_a, sg_a, w_a);
  for (int32_t f0 = F0; f0 < F1; f0 += 64 * kSegSteps) {
    int32_t slot_b[kSegSteps], sg_b[kSegSteps], w_b[kSegSteps];
    const bool more = f0 + 64 * kSegSteps < F1;
    bool full_b = false;
    if (more) full_b = gen(f0 + 64 * kSegSteps, slot_b, sg_b, w_b);
    if (full_a) {
#pragma unroll
      for (int q = 0; q < kSegSteps; ++q) fn(sg_a[q], slot_a[q], w_a[q]);
    } else {
#pragma unroll
      for (int q = 0; q < kSegSteps; ++q)
        if (w_a[q] >= 0) fn(sg_a[q], slot_a[q], w_a[q]);
    }
    if (!more || stop()) break;
    full_a = full_b;
#pragma unroll
    for (int q = 0; q < kSegSteps; ++q) {
      slot_a[q] = slot_b[q];
      sg_a[q] = sg_b[q];
      w_a[q] = w_b[q];
    }
  }
}

// Walks all T positions of a segment list, the workgroup's `waves`
// wavefronts taking chunks of whole iterations from an LDS cursor (the next
// position, 0 on entry).  Chunks shrink as the list drains (about the rest
// over twice the wavefronts, 512 to 8,192 positions), so the wavefronts
// finish close together and one that meets a slow stretch (short segments)
// takes fewer positions.
template <typename Fn, typename Stop>
__device__ __forceinline__ void chunk_walk(const int32_t* __restrict__ oadj, const int32_t* se, const int32_t* sd,
                                           int32_t n, int32_t T, int32_t* ticket, int waves, Fn&& fn,
                                           Stop&& stop) {
  bool stopped = false;
  for (;;) {
    int32_t F0 = 0, c = 0;
    if (__lane_id() == 0) {
      const int32_t seen = __hip_atomic_load(ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      c = ((T - seen) / (2 * waves)) & ~511;
      c = c < 512 ? 512 : (c > 8192 ? 8192 : c);
      F0 = atomicAdd(ticket, c);
    }
    F0 = __shfl(F0, 0, 64);
    c = __shfl(c, 0, 64);
    if (F0 >= T) break;
    const int32_t F1 = T - F0 > c ? F0 + c : T;
    seg_walk(oadj, se, sd, n, F0, F1, fn, [&] { stopped = stop(); return stopped; });
    if (stopped) break;
  }
}

// A dense window of a total count whose wedges fit one batch and number
// fewer than this is finalized by walking its wedges again (each end's
// counter read and cleared once) instead of scanning every counter.
constexpr int32_t kRewalkMax = 8192;

// One instantiation per count mode (the total count carries no second pass)
// and per workgroup shape: kNT threads and an LDS table of kWords words.
// kVpp: some layer's starts take Algorithm 3's wedges (compiled out when not).
template <int kMode, int kNT, int kWords, bool kVpp>
__global__ __launch_bounds__(kNT) void heavy_kernel(CountParams p) {
  constexpr int kWaves = kNT / 64;
  constexpr int kCap = kWords / 2;          // hash entries (keys | counts)
  constexpr int kSingleMax = kCap / 2;      // one hash window suffices below this many wedges
  constexpr int kS1 = 2 * kNT;              // segment list capacity, pass 1
  constexpr int kS2 = kNT;                  // segment list capacity, pass 2
  constexpr int kFill = 2;                  // middles per thread and sweep of a segment-list fill (4 measured slower: sweeps past the list capacity redo their cut middles)
  constexpr int kSW = ((2 * kS1 + 1 > 5 * kS2 + 2 ? 2 * kS1 + 1 : 5 * kS2 + 2) + 3) / 4 * 4;
  __shared__ __align__(16) int32_t table[kWords];
  __shared__ __align__(16) int32_t segbuf[kSW];
  __shared__ unsigned long long s_red64[kWaves + 1];
  __shared__ int32_t s_fill, s_over, s_cut_j, s_cut_lex;
  __shared__ int4 s_entry;      // the next start's list entry (code -1: none left)
  __shared__ int32_t s_ticket;  // chunk ticket of the dense walk
  __shared__ unsigned long long s_emit;  // batch emission: count << 32 | total length

  const int t = threadIdx.x;
  const int lane = __lane_id();
  const int wv = t >> 6;
  constexpr int mode = kMode;
  // per-middle cursor state of multi-window starts, one 16-byte record per
  // middle: {middle, end of its slice, next slot (the slice's first slot for
  // a table middle), end id at that slot (kNone when exhausted)}, so a sweep
  // reads each middle's state with one coalesced load; and the window's end
  // slot per middle
  int4* rec = reinterpret_cast<int4*>(p.cursor + (int64_t)blockIdx.x * 7 * p.cursor_stride);
  int32_t* cend = reinterpret_cast<int32_t*>(rec + p.cursor_stride);
  // a window's non-empty slices [cs, ce) of such a start, in any order
  int2* act = reinterpret_cast<int2*>(cend + p.cursor_stride);
  for (int i = t; i < kWords; i += kNT) table[i] = 0;
  unsigned long long acc_total = 0;

  // Starts come from a global ticket, taken two starts ahead by thread 0:
  // when a start begins, thread 0 loads the entry of the next start (its
  // ticket taken one start earlier) and takes the ticket of the one after,
  // so neither round trip delays the workgroup between starts.
  // (code -1: none left; a real code has rank < 2^30 - 1)
  auto entry_of = [&](uint32_t i) { return (int32_t)i < p.n_list ? p.list[i] : make_int4(-1, 0, 0, 0); };
  uint32_t ticket_next = 0;
  if (t == 0) {
    s_entry = entry_of(atomicAdd(p.ticket, 1u));
    ticket_next = atomicAdd(p.ticket, 1u);
  }
  for (;;) {
    __syncthreads();
    const int4 ent = s_entry;
    __syncthreads();
    if (ent.x == -1) break;
    int4 next_entry = make_int4(-1, 0, 0, 0);
    if (t == 0) {
      next_entry = entry_of(ticket_next);
      ticket_next = atomicAdd(p.ticket, 1u);
    }
    // the entry is the same in every lane: keep it (and what derives from
    // it) in scalar registers
    const int32_t code = __builtin_amdgcn_readfirstlane(ent.x);
    const int x = (int)(((uint32_t)code >> 30) & 1u);
    const int32_t r = code & ((1 << 30) - 1);
    const SideView S = pick(p, x);
    const SideView O = pick(p, 1 - x);
    const int32_t base = __builtin_amdgcn_readfirstlane(ent.y);
    const int32_t pre = __builtin_amdgcn_readfirstlane(ent.z);
    const int32_t ew = __builtin_amdgcn_readfirstlane(ent.w);
    // (bands need the kVpp instantiation: band items take Algorithm 3's wedges)
    const BandPart bp = band_part(p, code, x, r);
    const int32_t* clb = kVpp ? bp.clb : nullptr;
    const bool band_item = kVpp && bp.band_item;
    int64_t W = ew;
    if (ew == 0x7FFFFFFF) {
      const int64_t w = band_item ? (x ? p.wtop[1] : p.wtop[0])[r] : S.work[r];
      W = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(w >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)w));
    }
    const bool vpp = kVpp && (band_item || ((p.vpp >> x) & 1));
    const int32_t lo_r = vpp ? __builtin_amdgcn_readfirstlane(S.lo[r]) : 0;
    // End ranks lie in [elo, ehi): below the start under Algorithm 2, above
    // it under Algorithm 3, within the start's graph (a batch ranks each
    // graph's vertices contiguously).  elo is rounded down to even because
    // dense counters pair ranks (rank r itself is never an end).
    const int32_t* grank = x ? p.grank[1] : p.grank[0];
    const int32_t gi = (grank || p.gtune) ? __builtin_amdgcn_readfirstlane(graph_index(p, x, r)) : 0;
    // window settings: the handle's, or this start's graph's in a tuned batch
    // (uniform: scalar registers)
    int32_t window_mode = p.window_mode, dense_ratio = p.dense_ratio;
    int32_t hash_window_wedges = p.hash_window_wedges, dense_min_wedges = p.dense_min_wedges;
    if (p.gtune) {
      const int4 gt = p.gtune[gi];
      dense_ratio = __builtin_amdgcn_readfirstlane(gt.x);
      window_mode = __builtin_amdgcn_readfirstlane(gt.y);
      hash_window_wedges = __builtin_amdgcn_readfirstlane(gt.z);
      dense_min_wedges = __builtin_amdgcn_readfirstlane(gt.w);
    }
    // With a band part the ends lie in [band_lo, r) (band start) or
    // [band_lo, n_X) (band item).
    const int32_t elo = clb ? ((x ? p.band_lo[1] : p.band_lo[0]) & ~1)
                        : vpp ? ((r + 1) & ~1)
                              : (grank ? (__builtin_amdgcn_readfirstlane(grank[gi]) & ~1) : 0);
    const int32_t ehi = (clb && !band_item) ? r
                        : vpp ? (grank ? __builtin_amdgcn_readfirstlane(grank[gi + 1]) : (x ? p.nX[1] : p.nX[0]))
                              : r;
    const int32_t span = ehi - elo;
    // middles of rank >= tfirst find their window slices in the table and
    // keep no cursor
    const int32_t* tab = x ? p.wt[0] : p.wt[1];
    const int32_t tfirst = tab ? (x ? p.wt_first[0] : p.wt_first[1]) : 0x7FFFFFFF;
    const int32_t trow = x ? p.wt_row[0] : p.wt_row[1];
    // A start whose counts fit kPackBits bits packs each hash entry into one
    // word, so one hash window over its whole end range holds up to 5/8 of
    // the table's words in distinct ends.
    const bool packable = pre < kPackMaxPre && span < kPackMaxWidth;
    const int64_t psingle = (int64_t)kWords / 8 * 5;
    const bool dense =
        window_mode == 2 ||
        (window_mode == 1 && ((W > dense_min_wedges && !(packable && W <= psingle)) ||
                              W * (int64_t)dense_ratio >= (int64_t)span));
    const bool half = pre < 65536;
    // Starts in the dense block: the last window covers the block's end ranks
    // [top, r); its counters start from the MFMA products and its first pass
    // walks only middles outside the other layer's block (a prefix).
    const int32_t top = x ? p.dtop[1] : p.dtop[0];
    const bool in_block = r > top;
    const int32_t sparse_end = in_block ? top : ehi;
    // Windows: hash windows over [0, hash_end) (width hwidth, adapted as they
    // go), then dense windows of `width` ranks up to sparse_end.
    int32_t width = half ? 2 * kWords : kWords;
    // dense windows below q8 hold 8-bit counters: four ranks per word (q8
    // rounded down to even: the 16-bit windows that follow pair ranks from
    // an even first rank)
    int32_t q8 = (x ? p.q8[1] : p.q8[0]) & ~1;
    auto dense_hi = [&](int32_t lo) -> int32_t {
      const int64_t h = lo < q8 ? (int64_t)lo + 4 * kWords : (int64_t)lo + width;
      const int32_t h8 = lo < q8 && h > q8 ? q8 : (int32_t)(h < 0x7FFFFFFF ? h : 0x7FFFFFFF);
      return h8 >= sparse_end ? sparse_end : h8;
    };
    int32_t hwidth = 0, hash_end = 0;
    uint32_t cap = kCap;
    if (dense) {
      const int32_t base_lo = __builtin_amdgcn_readfirstlane(S.off[elo]);
      const int32_t base_hi = vpp ? __builtin_amdgcn_readfirstlane(S.off[ehi]) : base;  // (Algorithm 2: ehi = r)
      hash_end = elo;
      if (window_mode == 1 && base_hi > base_lo) {
        // Sparse prefix of a dense start: the ends of its wedges are
        // neighbours of its middles, which in a degree-driven graph fall on
        // the start layer's vertices in proportion to their degree, so about
        // W * (off_X[x] - off_X[elo]) / (off_X[ehi] - off_X[elo]) wedges end
        // below rank x.  The prefix is the
        // longest multiple of the dense width expected to hold at most
        // hash_window_wedges of them (one 64-lane probe of off_X); a wrong
        // guess costs time only (an overfull hash window is split).
        const int32_t step0 = (sparse_end - elo + 63) / 64;
        const int32_t step = (step0 + 2 * kWords - 1) / (2 * kWords) * (2 * kWords);
        const int64_t xl = elo + (int64_t)(lane + 1) * step;
        const bool ok = xl < sparse_end && (double)W * (double)(S.off[xl] - base_lo) <=
                                               (double)hash_window_wedges * (double)(base_hi - base_lo);
        hash_end = elo + __popcll(__ballot(ok)) * step;
        hwidth = hash_end - elo;
      }
    } else {
      hash_end = sparse_end;
      const uint32_t cmax = packable ? (uint32_t)kWords : (uint32_t)kCap;
      if (W <= (packable ? psingle : (int64_t)kSingleMax)) {
        hwidth = span;
        cap = 512;
        while (cap < cmax && (int64_t)cap < 2 * W) cap <<= 1;
      } else {
        const int64_t wd = (int64_t)span * hash_window_wedges / W;
        hwidth = (int32_t)(wd < 256 ? 256 : (wd > span ? span : wd));
        cap = cmax;
      }
    }
    // The last 8-bit window stops at q8, so a short stretch below q8 can
    // cost a window more than wider-counter windows over the whole dense
    // range; and four counters to a word put more of a start's LDS atomics
    // on the same word.  So the 8-bit windows are kept only when they save
    // at least one window.
    if (hash_end < q8 && hash_end < sparse_end) {
      const int64_t e8 = q8 < sparse_end ? q8 : sparse_end;
      const int64_t n8 = (e8 - hash_end + 4 * kWords - 1) / (4 * kWords);
      const int64_t nw = q8 < sparse_end ? ((int64_t)sparse_end - q8 + width - 1) / width : 0;
      const int64_t n1 = ((int64_t)sparse_end - hash_end + width - 1) / width;
      if (n8 + nw >= n1) q8 = 0;
    }
    int32_t pre_out = pre;
    if (in_block) {
      const int32_t otop = x ? p.dtop[0] : p.dtop[1];
      int32_t a = 0, b = pre;
      while (a < b) {
        const int32_t mid = (a + b) >> 1;
        if (S.adj[base + mid] < otop) a = mid + 1; else b = mid;
      }
      pre_out = a;
    }
    // one window over [elo, ehi) needs no cursors; otherwise every middle
    // below tfirst keeps its next slot and next end id in scratch
    auto init_cursors = [&] {
      for (int32_t j = t; j < pre; j += kNT) {
        int32_t v, ps, pe;
        mid_slice(vpp, S, O, base + j, j, lo_r, clb, v, ps, pe);
        rec[j] = make_int4(v, pe, ps, v >= tfirst ? 0 : (ps < pe ? O.adj[ps] : kNone));
      }
    };
    bool cursors = !(sparse_end == ehi && (hash_end >= ehi ? hwidth >= span : (hash_end == elo && dense_hi(elo) >= ehi)));
    if (cursors) init_cursors();
    unsigned long long start_acc = 0;
    int32_t lo_w = elo;
    for (;;) {
      int32_t hi_w;
      bool wdense = lo_w >= hash_end;
      const bool seeded = lo_w >= sparse_end;
      bool wquarter = wdense && !seeded && lo_w < q8;
      bool whalf = half && wdense && !wquarter;
      if (!seeded) {
        if (wdense) hi_w = dense_hi(lo_w);
        else hi_w = (int64_t)lo_w + hwidth >= hash_end ? hash_end : lo_w + hwidth;
      } else if (in_block && lo_w < ehi) {
        hi_w = ehi;
        wdense = true;
        whalf = false;
        wquarter = false;
      } else {
        break;
      }
      const int32_t pre1 = seeded ? pre_out : pre;
      const bool wpacked = !wdense && packable;  // hash entries of this window: key | count words
      if (seeded) {
        const int32_t* crow = (x ? p.dC[1] : p.dC[0]) + (int64_t)(r - top) * (x ? p.dld[1] : p.dld[0]);
        for (int32_t i = t; i < ehi - top; i += kNT) table[i] = crow[i];
      }
      // cursors advance during pass 1 only for dense windows of a total count
      // (a hash window may have to be redone; pass 2 needs the old cursors)
      const bool advance_now = wdense && mode == kTotal;

      // Fills the segment list with the non-empty slices [cs, ce) of window
      // [lo_w, hi_w) of middles rj, rj+1, ... < npre, up to `segcap` of
      // them, kFill * kNT middles per sweep in middle order (one packed
      // workgroup scan of (active, length)).  Leaves rj at the first middle
      // not taken and returns the segment count and total length; the cursors
      // of taken middles advance (or record the window end, cend) here.
      auto fill = [&](int32_t npre, int32_t segcap, bool second, int32_t* se, int32_t* sd, int32_t* sj,
                      unsigned long long* sdel, int32_t& rj, int32_t& nseg, int32_t& T) {
        nseg = 0;
        T = 0;
        // cursor records of this sweep's middles, and of the next sweep's,
        // loaded before this one is compacted (the usual next sweep)
        int4 pf[kFill];
        auto load_rec = [&](int32_t j0) {
#pragma unroll
          for (int h = 0; h < kFill; ++h) {
            const int32_t j = j0 + kFill * t + h;
            pf[h] = (cursors && j < npre) ? rec[j] : make_int4(0, 0, 0, 0);
          }
        };
        load_rec(rj);
        while (nseg < segcap && rj < npre) {
          int32_t jv[kFill], csv[kFill], cev[kFill], ev[kFill], vv[kFill];
          bool actv[kFill];
          int4 rc[kFill];
#pragma unroll
          for (int h = 0; h < kFill; ++h) rc[h] = pf[h];
          if (cursors && npre - rj > kFill * kNT) load_rec(rj + kFill * kNT);
#pragma unroll
          for (int h = 0; h < kFill; ++h) {
            const int32_t j = rj + kFill * t + h;
            jv[h] = j;
            actv[h] = false;
            csv[h] = cev[h] = ev[h] = vv[h] = 0;
            if (j < npre) {
              int32_t v, s0, e, pj = 0, nj = kNone;  // cursor state (meaningful below tfirst)
              if (cursors) {
                v = rc[h].x;
                e = rc[h].y;
                pj = rc[h].z;
                nj = rc[h].w;
                s0 = rc[h].z;  // (a table middle's record keeps its first slot)
              } else {
                mid_slice(vpp, S, O, base + j, j, lo_r, clb, v, s0, e);
              }
              ev[h] = e;
              vv[h] = v;
              if (!cursors) {
                csv[h] = s0;
                cev[h] = e;
                actv[h] = e > s0;
              } else if (v >= tfirst) {
                // the table finds the window's slots in the whole list; the
                // slice keeps to [s0, e)
                const int32_t* rowp = tab + (int64_t)(v - tfirst) * trow;
                int32_t cs = table_lb(O.adj, rowp, lo_w);
                if (vpp || clb) cs = cs > s0 ? cs : s0;  // (Algorithm 2 alone: the table's slot is never before s0)
                int32_t ce = e;
                if (hi_w < ehi) {
                  const int32_t c2 = table_lb(O.adj, rowp, hi_w);
                  ce = c2 < e ? c2 : e;
                }
                csv[h] = cs;
                cev[h] = ce;
                actv[h] = ce > cs;
              } else if (nj < hi_w) {
                const int32_t cs = pj;  // O.adj[cs] = nj < hi_w
                actv[h] = true;
                csv[h] = cs;
                cev[h] = hi_w >= ehi ? e : (second ? cend[j] : near_lower_bound(O.adj, cs + 1, e, hi_w));
              }
            }
          }
          int32_t na = 0, ln = 0;
#pragma unroll
          for (int h = 0; h < kFill; ++h) {
            na += (int)actv[h];
            ln += actv[h] ? cev[h] - csv[h] : 0;
          }
          const unsigned long long packed = ((unsigned long long)na << 32) | (uint32_t)ln;
          unsigned long long tot;
          const unsigned long long ex = block_exclusive_scan<unsigned long long, kNT>(packed, s_red64, &tot);
          const int32_t room = segcap - nseg;
          const int32_t nact = (int32_t)(tot >> 32);
          int32_t ia = (int32_t)(ex >> 32);
          int32_t lex = (int32_t)(uint32_t)ex;
#pragma unroll
          for (int h = 0; h < kFill; ++h) {
            if (!actv[h]) continue;
            if (ia < room) {
              const int32_t ps = nseg + ia;
              se[ps] = T + lex;
              sd[ps] = csv[h] - (T + lex);
              if (second) {
                sj[ps] = jv[h];
                sdel[ps] = 0ull;
              }
              if (cursors && vv[h] < tfirst) {
                if (second || advance_now) {
                  *reinterpret_cast<int2*>(&rec[jv[h]].z) =
                      make_int2(cev[h], cev[h] < ev[h] ? O.adj[cev[h]] : kNone);
                } else {
                  cend[jv[h]] = cev[h];
                }
              }
            } else if (ia == room) {
              s_cut_j = jv[h];
              s_cut_lex = lex;
            }
            ++ia;
            lex += cev[h] - csv[h];
          }
          if (nact <= room) {
            nseg += nact;
            T += (int32_t)(uint32_t)tot;
            rj = npre - rj > kFill * kNT ? rj + kFill * kNT : npre;
          } else {
            __syncthreads();
            rj = s_cut_j;
            T += s_cut_lex;
            nseg = segcap;
          }
        }
        if (t == 0) { se[nseg] = T; s_ticket = 0; }
        __syncthreads();
      };
      // this wavefront's share of the batch's positions
      auto share = [&](int32_t T, int32_t& F0, int32_t& F1) {
        F0 = (int32_t)((int64_t)T * wv / kWaves);
        F1 = (int32_t)((int64_t)T * (wv + 1) / kWaves);
      };

      // ---- pass 1: count the wedges whose end lies in [lo_w, hi_w)
      int32_t halvings = 0;
      int32_t batches = 0, last_n = 0, last_t = 0;
      for (;;) {
        if (t == 0) { s_fill = 0; s_over = 0; s_emit = 0ull; }
        __syncthreads();
        int32_t* se = segbuf;
        int32_t* sd = segbuf + kS1 + 1;
        int32_t rj = 0;
        bool over = false;
        batches = 0;
        // A cursor start's window: every middle's slice in one barrier-free
        // pass (kA middles per thread and round, their loads issued
        // together).  Each wavefront reserves positions for its non-empty
        // slices with one LDS atomic per round (count and total length): the
        // first kS1 go straight into the segment list as the first batch,
        // the rest to `act`, from which later batches take kS1 each.
        const bool compact = cursors && !seeded;
        int32_t n_act = 0, nseg0 = 0, T0 = 0;
        if (compact) {
          constexpr int kA = 2;
          for (int32_t j0 = 0; j0 < pre1; j0 += kA * kNT) {
            int4 rc[kA];
#pragma unroll
            for (int a = 0; a < kA; ++a) {
              const int32_t j = j0 + a * kNT + t;
              rc[a] = j < pre1 ? rec[j] : make_int4(0, 0, 0, kNone);
            }
#pragma unroll
            for (int a = 0; a < kA; ++a) {
              const int32_t j = j0 + a * kNT + t;
              const int32_t v = rc[a].x, e = rc[a].y;
              int32_t cs = 0, ce = 0;
              bool ac = false;
              if (j < pre1) {
                if (v >= tfirst) {
                  const int32_t* rowp = tab + (int64_t)(v - tfirst) * trow;
                  cs = table_lb(O.adj, rowp, lo_w);
                  if (vpp || clb) cs = cs > rc[a].z ? cs : rc[a].z;  // (rc.z: the slice's first slot)
                  ce = e;
                  if (hi_w < ehi) {
                    const int32_t c2 = table_lb(O.adj, rowp, hi_w);
                    ce = c2 < e ? c2 : e;
                  }
                  ac = ce > cs;
                } else if (rc[a].w < hi_w) {
                  cs = rc[a].z;  // O.adj[cs] = rc.w < hi_w
                  int32_t nv = kNone;  // end id at ce (the search returns it)
                  if (hi_w >= ehi) {
                    ce = e;
                  } else {
                    ce = near_lower_bound_v(O.adj, cs + 1, e, hi_w, nv);
                    if (ce >= e) nv = kNone;
                  }
                  ac = true;
                  if (advance_now) *reinterpret_cast<int2*>(&rec[j].z) = make_int2(ce, nv);
                  else cend[j] = ce;
                }
              }
              const unsigned long long pv = ac ? (1ull << 32) | (uint32_t)(ce - cs) : 0ull;
              const unsigned long long inc = wave_inclusive_scan(pv);
              const unsigned long long wt = __shfl(inc, 63, 64);
              unsigned long long wb = 0;
              if (lane == 63 && wt) wb = atomicAdd(&s_emit, wt);
              wb = __shfl(wb, 63, 64);
              if (ac) {
                const unsigned long long at = wb + inc - pv;
                const int32_t ps = (int32_t)(at >> 32), L = (int32_t)(uint32_t)at;
                if (ps < kS1) {
                  se[ps] = L;
                  sd[ps] = cs - L;
                } else {
                  act[ps - kS1] = make_int2(cs, ce);
                  if (ps == kS1) s_cut_lex = L;  // the first batch's total length
                }
              }
            }
          }
          __syncthreads();
          const unsigned long long all = s_emit;
          n_act = (int32_t)(all >> 32);
          nseg0 = n_act < kS1 ? n_act : kS1;
          T0 = n_act <= kS1 ? (int32_t)(uint32_t)all : s_cut_lex;
          if (t == 0) {
            se[nseg0] = T0;
            s_ticket = 0;
          }
          __syncthreads();
        }
        while (compact ? rj < n_act : rj < pre1) {
          int32_t nseg, T;
          if (compact && rj == 0) {
            // the first batch, emitted by the pass
            nseg = nseg0;
            T = T0;
            rj = nseg0;
          } else if (compact) {
            // batch [rj, rj + kS1) of the window's slices (act holds those
            // from kS1 on): two per thread, positions from a wavefront scan
            // and one LDS atomic per wavefront
            if (t == 0) s_emit = 0ull;
            __syncthreads();
            const int32_t i0 = rj + 2 * t, i1 = i0 + 1;
            const int32_t lim = n_act - rj < kS1 ? n_act : rj + kS1;
            int2 c0 = make_int2(0, 0), c1 = make_int2(0, 0);
            if (i0 < lim) c0 = act[i0 - kS1];
            if (i1 < lim) c1 = act[i1 - kS1];
            const uint32_t l0 = (uint32_t)(c0.y - c0.x), l1 = (uint32_t)(c1.y - c1.x);
            const unsigned long long v =
                ((unsigned long long)((int)(i0 < lim) + (int)(i1 < lim)) << 32) | (l0 + l1);
            const unsigned long long inc = wave_inclusive_scan(v);
            const unsigned long long wt = __shfl(inc, 63, 64);
            unsigned long long wb = 0;
            if (lane == 63 && wt) wb = atomicAdd(&s_emit, wt);
            wb = __shfl(wb, 63, 64);
            unsigned long long at = wb + inc - v;
            if (i0 < lim) {
              const int32_t ps = (int32_t)(at >> 32), L = (int32_t)(uint32_t)at;
              se[ps] = L;
              sd[ps] = c0.x - L;
              at += (1ull << 32) | l0;
            }
            if (i1 < lim) {
              const int32_t ps = (int32_t)(at >> 32), L = (int32_t)(uint32_t)at;
              se[ps] = L;
              sd[ps] = c1.x - L;
            }
            __syncthreads();
            const unsigned long long all = s_emit;
            nseg = (int32_t)(all >> 32);
            T = (int32_t)(uint32_t)all;
            if (t == 0) {
              se[nseg] = T;
              s_ticket = 0;
            }
            __syncthreads();
            rj = lim;
          } else {
            fill(pre1, kS1, false, se, sd, nullptr, nullptr, rj, nseg, T);
          }
          ++batches;
          last_n = nseg;
          last_t = T;
          int32_t F0, F1;
          share(T, F0, F1);
          if (wquarter) {
            // counter w - lo_w: byte (w - lo_w) & 3 of word (w - lo_w) >> 2
            char* tb = reinterpret_cast<char*>(table);
            chunk_walk(O.adj, se, sd, nseg, T, &s_ticket, kWaves,
                       [&](int32_t, int32_t, int32_t w) {
                         const uint32_t i = (uint32_t)(w - lo_w);
                         atomicAdd(reinterpret_cast<uint32_t*>(tb + (i & ~3u)), 1u << ((i & 3u) << 3));
                       },
                       [] { return false; });
          } else if (wdense && whalf) {
            // lo_w is even: counter pair (w >> 1) - (lo_w >> 1), half (w & 1):
            // byte offset (w & ~1) * 2 from tw, add 1 or 1 << 16
            char* tw = reinterpret_cast<char*>(table) - 2 * lo_w;
            chunk_walk(O.adj, se, sd, nseg, T, &s_ticket, kWaves,
                       [&](int32_t, int32_t, int32_t w) {
                         atomicAdd(reinterpret_cast<uint32_t*>(tw + ((uint32_t)(w & ~1) << 1)),
                                   __umul24((uint32_t)w & 1u, 65535u) + 1u);
                       },
                       [] { return false; });
          } else if (wdense) {
            int32_t* tw = table - lo_w;
            seg_walk(O.adj, se, sd, nseg, F0, F1, [&](int32_t, int32_t, int32_t w) { atomicAdd(&tw[w], 1); },
                     [] { return false; });
          } else {
            // this lane's new keys since the last poll, and whether a probe overran
            int32_t fresh = 0;
            bool overran = false;
            auto poll = [&] {
              const bool ovf = __ballot(overran) != 0;
              const int32_t fw = wave_sum(fresh);
              fresh = 0;
              if (lane == 0 && (ovf || (fw && atomicAdd(&s_fill, fw) + fw > (int32_t)(cap / 8 * 5)))) s_over = 1;
              // a plain LDS read of the flag (other wavefronts may have set it)
              return __builtin_amdgcn_readfirstlane(
                         __hip_atomic_load(&s_over, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0;
            };
            if (wpacked) {
              uint32_t* pt = reinterpret_cast<uint32_t*>(table);
              const int32_t kb = lo_w - 1;  // key = end - lo_w + 1
              seg_walk(O.adj, se, sd, nseg, F0, F1,
                       [&](int32_t, int32_t, int32_t w) {
                         const int res = packed_hash_add(pt, cap, (uint32_t)(w - kb));
                         fresh += res & 1;
                         overran |= res == kOverfull;
                       },
                       poll);
            } else {
              seg_walk(O.adj, se, sd, nseg, F0, F1,
                       [&](int32_t, int32_t, int32_t w) {
                         const int res = block_hash_add(table, cap, w);
                         fresh += res & 1;
                         overran |= res == kOverfull;
                       },
                       poll);
            }
            poll();  // the walk does not poll after its last iteration
          }
          __syncthreads();
          if (!wdense && s_over) {
            over = true;
            break;
          }
        }
        if (!over) break;
        // the window holds too many distinct ends for the table: halve it and
        // redo.  A start walked without cursors (one window over its whole
        // end range) switches to cursors first, so the smaller window applies.
        for (int i = t; i < (int)(wpacked ? cap : 2 * cap); i += kNT) table[i] = 0;
        if (!cursors) {
          init_cursors();
          cursors = true;
        }
        __syncthreads();
        // a window of one end rank holds one distinct end, so this ends after
        // at most 31 halvings; the cap only guards against a logic error
        if (++halvings > 40) {
          if (t == 0) atomicOr(p.status, 1);
          break;
        }
        hi_w = lo_w + ((hi_w - lo_w) > 1 ? (hi_w - lo_w) / 2 : 1);
      }
      // ---- pass 2 (per-vertex / per-edge): count - 1 to both edges of every
      // wedge; also advances the cursors past this window
      if (mode != kTotal) {
        unsigned long long* vmid = pick_ptr(p.vout, 1 - x);
        int32_t* se = segbuf;
        int32_t* sd = segbuf + kS2 + 1;
        int32_t* sj = sd + kS2;
        unsigned long long* sdel = reinterpret_cast<unsigned long long*>(segbuf + 3 * kS2 + 2);
        int32_t rj = 0;
        while (rj < pre) {
          int32_t nseg, T;
          fill(pre, kS2, true, se, sd, sj, sdel, rj, nseg, T);
          int32_t F0, F1;
          share(T, F0, F1);
          // a lane's segments only increase along its positions: sum its
          // deltas per segment in a register and add them to LDS on a change
          int32_t cur = -1;
          unsigned long long run = 0;
          seg_walk(O.adj, se, sd, nseg, F0, F1,
                   [&](int32_t sg, int32_t slot, int32_t w) {
                     const int32_t c =
                         wdense ? dense_get(table, w - lo_w, whalf, wquarter)
                                : (wpacked ? packed_hash_get(reinterpret_cast<const uint32_t*>(table), cap - 1,
                                                             (uint32_t)(w - lo_w + 1))
                                           : hash_get(table, table + cap, cap - 1, w));
                     if (c > 1) {
                       const unsigned long long d = (unsigned long long)(c - 1);
                       if (mode == kEdge) acc_add(p, 1 - x, slot, d);
                       if (sg != cur) {
                         if (run) atomicAdd(&sdel[cur], run);
                         cur = sg;
                         run = 0;
                       }
                       run += d;
                     }
                   },
                   [] { return false; });
          if (run) atomicAdd(&sdel[cur], run);
          __syncthreads();
          for (int32_t i = t; i < nseg; i += kNT) {
            const unsigned long long d = sdel[i];
            if (d) {
              const int32_t k = base + sj[i];
              if (mode == kEdge) acc_add(p, x, k, d);
              else atomicAdd(&vmid[S.adj[k]], d);
            }
          }
          __syncthreads();
        }
      } else if (cursors && !advance_now) {
        // hash window of a total count: advance the cursors now that the window is final
        for (int32_t j = t; j < pre1; j += kNT) {
          const int4 r4 = rec[j];
          if (r4.x < tfirst && r4.w < hi_w) {
            const int32_t ce = cend[j];
            *reinterpret_cast<int2*>(&rec[j].z) = make_int2(ce, ce < r4.y ? O.adj[ce] : kNone);
          }
        }
      }
      // ---- finalize the window: C(count,2) per end, then clear the table
      unsigned long long* vs = pick_ptr(p.vout, x);
      if (mode == kTotal && wdense && !seeded && batches == 1 && last_t < kRewalkMax) {
        // the window's segment list is still in LDS: visit its wedges again
        int32_t F0, F1;
        share(last_t, F0, F1);
        seg_walk(O.adj, segbuf, segbuf + kS1 + 1, last_n, F0, F1,
                 [&](int32_t, int32_t, int32_t w) {
                   const int32_t i = w - lo_w;
                   int32_t c;
                   if (wquarter) {
                     const uint32_t sh = (uint32_t)(i & 3) << 3;
                     const uint32_t old = atomicAnd(reinterpret_cast<uint32_t*>(&table[i >> 2]), ~(0xFFu << sh));
                     c = (int32_t)((old >> sh) & 0xFFu);
                   } else if (whalf) {
                     const uint32_t sh = (uint32_t)(i & 1) << 4;
                     const uint32_t old = atomicAnd(reinterpret_cast<uint32_t*>(&table[i >> 1]), ~(0xFFFFu << sh));
                     c = (int32_t)((old >> sh) & 0xFFFFu);
                   } else {
                     c = atomicExch(&table[i], 0);
                   }
                   if (c > 1) start_acc += choose2(c);
                 },
                 [] { return false; });
      } else if (wquarter && mode != kVertex) {
        // sum of c (c - 1) over the 8-bit counters, branch-free (c (c - 1)
        // is 0 for c = 0 or 1); the sum is even and halves exactly
        const int32_t words = (hi_w - lo_w + 3) >> 2;
        const int32_t quads = (words + 3) >> 2;
        uint4* t4 = reinterpret_cast<uint4*>(table);
        unsigned long long twice = 0;
        for (int32_t i4 = t; i4 < quads; i4 += kNT) {
          const uint4 q4 = t4[i4];
          if ((q4.x | q4.y | q4.z | q4.w) == 0u) continue;
          const uint32_t wd[4] = {q4.x, q4.y, q4.z, q4.w};
          uint32_t part = 0;  // at most 16 x 255 x 254 < 2^21
#pragma unroll
          for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const uint32_t n = (wd[c] >> (8 * b)) & 0xFFu;
              part += __umul24(n, n) - n;
            }
          }
          twice += part;
          t4[i4] = make_uint4(0u, 0u, 0u, 0u);
        }
        start_acc += twice >> 1;
      } else if (wdense && whalf && mode != kVertex) {
        // sum of c (c - 1) over the 16-bit counters: c (c - 1) < 2^32 is
        // exact in a 24-bit multiply and is 0 for c = 0 or 1, so no branch
        // per counter; the sum is even and halves exactly
        const int32_t words = (hi_w - lo_w + 1) >> 1;
        const int32_t quads = (words + 3) >> 2;
        uint4* t4 = reinterpret_cast<uint4*>(table);
        unsigned long long twice = 0;
        for (int32_t i4 = t; i4 < quads; i4 += kNT) {
          const uint4 q4 = t4[i4];
          if ((q4.x | q4.y | q4.z | q4.w) == 0u) continue;
          const uint32_t wd[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t c0 = wd[c] & 0xFFFFu, c1 = wd[c] >> 16;
            twice += (unsigned long long)(__umul24(c0, c0) - c0);
            twice += (unsigned long long)(__umul24(c1, c1) - c1);
          }
          t4[i4] = make_uint4(0u, 0u, 0u, 0u);
        }
        start_acc += twice >> 1;
      } else if (wdense) {
        const int32_t wn = hi_w - lo_w;
        const int32_t words = wquarter ? (wn + 3) >> 2 : whalf ? (wn + 1) >> 1 : wn;
        const int32_t quads = (words + 3) >> 2;
        uint4* t4 = reinterpret_cast<uint4*>(table);
        for (int32_t i4 = t; i4 < quads; i4 += kNT) {
          const uint4 q4 = t4[i4];
          if ((q4.x | q4.y | q4.z | q4.w) == 0u) continue;
          const uint32_t wd[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t word = wd[c];
            if (!word) continue;
            const int32_t i = 4 * i4 + c;
            if (wquarter) {
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                const int32_t cb = (int32_t)((word >> (8 * b)) & 0xFFu);
                if (cb > 1) {
                  const unsigned long long cc = choose2(cb);
                  start_acc += cc;
                  if (mode == kVertex) atomicAdd(&vs[lo_w + 4 * i + b], cc);
                }
              }
            } else if (whalf) {
              const int32_t c0 = (int32_t)(word & 0xFFFFu), c1 = (int32_t)(word >> 16);
              if (c0 > 1) {
                const unsigned long long cc = choose2(c0);
                start_acc += cc;
                if (mode == kVertex) atomicAdd(&vs[lo_w + 2 * i], cc);
              }
              if (c1 > 1) {
                const unsigned long long cc = choose2(c1);
                start_acc += cc;
                if (mode == kVertex) atomicAdd(&vs[lo_w + 2 * i + 1], cc);
              }
            } else if ((int32_t)word > 1) {
              const unsigned long long cc = choose2((int32_t)word);
              start_acc += cc;
              if (mode == kVertex) atomicAdd(&vs[lo_w + i], cc);
            }
          }
          t4[i4] = make_uint4(0u, 0u, 0u, 0u);
        }
      } else if (wpacked && mode != kVertex) {
        // c (c - 1) of the 12-bit counts, branch-free (see the dense case); cap >= 512 is a multiple of 4
        uint4* t4 = reinterpret_cast<uint4*>(table);
        unsigned long long twice = 0;
        for (uint32_t i4 = t; i4 < cap / 4; i4 += kNT) {
          const uint4 q4 = t4[i4];
          if ((q4.x | q4.y | q4.z | q4.w) == 0u) continue;
          const uint32_t wd[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t n = wd[c] & kPackMask;
            twice += (unsigned long long)(__umul24(n, n) - n);
          }
          t4[i4] = make_uint4(0u, 0u, 0u, 0u);
        }
        start_acc += twice >> 1;
      } else if (wpacked) {
        uint32_t* pt = reinterpret_cast<uint32_t*>(table);
        for (uint32_t h = t; h < cap; h += kNT) {
          const uint32_t word = pt[h];
          if (word) {
            const int32_t c = (int32_t)(word & kPackMask);
            if (c > 1) {
              const unsigned long long cc = choose2(c);
              start_acc += cc;
              if (mode == kVertex) atomicAdd(&vs[lo_w - 1 + (int32_t)(word >> kPackBits)], cc);
            }
            pt[h] = 0u;
          }
        }
      } else {
        for (uint32_t h = t; h < cap; h += kNT) {
          const int32_t key = table[h];
          if (key) {
            const int32_t c = table[cap + h];
            if (c > 1) {
              const unsigned long long cc = choose2(c);
              start_acc += cc;
              if (mode == kVertex) atomicAdd(&vs[key - 1], cc);
            }
            table[h] = 0;
            table[cap + h] = 0;
          }
        }
      }
      if (!wdense && cursors && !seeded) {
        // size the next hash window from this one's distinct ends (aim: a quarter of the table)
        const int64_t span = hi_w - lo_w;
        const int64_t fill_n = s_fill;
        int64_t next = fill_n > 0 ? span * (int64_t)(cap / 4) / fill_n : 2 * span;
        next = next < 64 ? 64 : next;
        hwidth = (int32_t)(next > span ? span : next);
      }
      __syncthreads();
      lo_w = hi_w;
    }
    if (mode == kVertex) {
      const unsigned long long sa = block_sum<unsigned long long, kNT>(start_acc, s_red64);
      if (t == 0 && sa) atomicAdd(&pick_ptr(p.vout, x)[r], sa);
    } else if (mode == kTotal && p.gtotal) {
      const unsigned long long sa = block_sum<unsigned long long, kNT>(start_acc, s_red64);
      if (t == 0 && sa) atomicAdd(&p.gtotal[graph_index(p, x, r)], sa);
    } else {
      acc_total += start_acc;
    }
    if (t == 0) s_entry = next_entry;
  }
  if (mode == kTotal && p.total) {
    const unsigned long long s = block_sum<unsigned long long, kNT>(acc_total, s_red64);
    if (t == 0 && s) atomicAdd(p.total, s);
  }
}

// B_e of the edge at side-0 slot k: its two arcs' accumulators, written to
// the edge's input position.
__global__ void fold_edges_kernel(const int32_t* __restrict__ edge0, const int32_t* __restrict__ rev0,
                                  const unsigned long long* __restrict__ acc0,
                                  const unsigned long long* __restrict__ acc1, int64_t m,
                                  unsigned long long* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    out[edge0[k]] = acc0[k] + acc1[rev0[k]];
}

// B_x of every vertex of one layer, from its rank-indexed accumulator to its
// input id.
__global__ void vertex_out_kernel(const unsigned long long* __restrict__ by_rank, const int32_t* __restrict__ id_of,
                                  int32_t n, unsigned long long* __restrict__ out) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    out[id_of[r]] = by_rank[r];
}

__global__ void fold_edges32_kernel(const int32_t* __restrict__ edge0, const int32_t* __restrict__ rev0,
                                    const uint32_t* __restrict__ acc0, const uint32_t* __restrict__ acc1, int64_t m,
                                    unsigned long long* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    out[edge0[k]] = (unsigned long long)acc0[k] + acc1[rev0[k]];
}

int num_cus() {
  int dev = 0;
  BFC_HIP(hipGetDevice(&dev));
  int cus = 0;
  BFC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus > 0 ? cus : 1;
}

}  // namespace

namespace {

// workgroups of the big and medium heavy launches
int big_grid_for(const bfc_graph_s* g) {
  const int cus = num_cus();
  const int n = g->sched.n_heavy - g->sched.n_medium;
  return n < cus ? n : cus;
}
int med_grid_for(const bfc_graph_s* g) {
  const int w = 4 * num_cus();
  return g->sched.n_medium < w ? g->sched.n_medium : w;
}

int64_t cursor_stride_for(const bfc_graph_s* g) { return ((int64_t)g->sched.max_prefix + 63) / 64 * 64; }

// scratch: three cursor arrays per big workgroup, three per medium workgroup
// (stride kMedPre), then 256 bytes: the two tickets
// per workgroup and middle: a 16-byte cursor record, a window end slot and
// an 8-byte slice of the window's compacted list
size_t big_wg_bytes(const bfc_graph_s* g) { return 7 * (size_t)cursor_stride_for(g) * sizeof(int32_t); }
size_t med_wg_bytes() { return 7 * (size_t)kMedPre * sizeof(int32_t); }
size_t big_cursor_bytes(const bfc_graph_s* g) { return (size_t)big_grid_for(g) * big_wg_bytes(g); }
size_t med_cursor_bytes(const bfc_graph_s* g) { return (size_t)med_grid_for(g) * med_wg_bytes(); }

// ------------------------------------------------------------ static scratch
// Scratch of bfc_count_total_static: a fixed array in device memory, so that
// call allocates nothing.  Each device holds its own copy, at its own
// address, for the life of the process.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
void* g_static_ptr[256] = {};

// Device address of this device's copy of `scratch` (the host-side name is
// only a stand-in for it), looked up once per device with it current.
void* static_scratch_ptr() {
  int dev = 0;
  BFC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) throw Error{BFC_ERR_DEVICE, "device index out of range"};
  std::lock_guard<std::mutex> hold(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    BFC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error{BFC_ERR_DEVICE, "no device address for the static scratch"};
    g_static_ptr[dev] = ptr;
  }
  return g_static_ptr[dev];
}

__global__ void fill_zero_kernel(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace

void zero_u64(void* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  fill_zero_kernel<<<(unsigned)grid, 256, 0, s>>>(static_cast<unsigned long long*>(p), n);
  BFC_LAUNCH_CHECK();
}

int32_t* count_status(bfc_graph_s* g) { return g->info.as<int32_t>() + kInfoCountStatus; }

void prepare_count(bfc_graph_s* g, hipStream_t s) {
  prepare_dense(g, s);
  const size_t need = big_cursor_bytes(g) + med_cursor_bytes(g) + 256;
  if (g->scratch_bytes < need) {
    g->scratch.alloc(need, s);
    g->scratch_bytes = need;
  }
}

template <int kCap, bool kPacked>
void launch_light(CountMode mode, bool vpp, unsigned grid, hipStream_t s, const CountParams& p, const int4* l,
                  int32_t n) {
  if (vpp) {
    if (mode == kTotal) light_kernel<kTotal, kCap, kPacked, true><<<grid, kLightNT, 0, s>>>(p, l, n);
    else if (mode == kVertex) light_kernel<kVertex, kCap, kPacked, true><<<grid, kLightNT, 0, s>>>(p, l, n);
    else light_kernel<kEdge, kCap, kPacked, true><<<grid, kLightNT, 0, s>>>(p, l, n);
  } else {
    if (mode == kTotal) light_kernel<kTotal, kCap, kPacked, false><<<grid, kLightNT, 0, s>>>(p, l, n);
    else if (mode == kVertex) light_kernel<kVertex, kCap, kPacked, false><<<grid, kLightNT, 0, s>>>(p, l, n);
    else light_kernel<kEdge, kCap, kPacked, false><<<grid, kLightNT, 0, s>>>(p, l, n);
  }
  BFC_LAUNCH_CHECK();
}

template <int kNT, int kWords, bool kVpp>
void launch_heavy(CountMode mode, int grid, hipStream_t s, const CountParams& p) {
  if (mode == kTotal) heavy_kernel<kTotal, kNT, kWords, kVpp><<<(unsigned)grid, kNT, 0, s>>>(p);
  else if (mode == kVertex) heavy_kernel<kVertex, kNT, kWords, kVpp><<<(unsigned)grid, kNT, 0, s>>>(p);
  else heavy_kernel<kEdge, kNT, kWords, kVpp><<<(unsigned)grid, kNT, 0, s>>>(p);
  BFC_LAUNCH_CHECK();
}

size_t static_scratch_bytes() { return kStaticScratchBytes; }

size_t min_count_scratch_bytes(const bfc_graph_s* g) {
  size_t b = 256;
  if (g->sched.n_heavy - g->sched.n_medium > 0) b += big_wg_bytes(g);
  if (g->sched.n_medium > 0) b += med_wg_bytes();
  return b;
}

void count(bfc_graph_s* g, CountMode mode, int64_t* total_dev, int64_t* out0, int64_t* out1, hipStream_t s,
           int64_t* gtotals, bool static_scratch) {
  const Schedule& sc = g->sched;
  const int cus = num_cus();
  int big_grid = big_grid_for(g);
  int med_grid = med_grid_for(g);
  const int64_t stride = cursor_stride_for(g);
  char* sbase = g->scratch.as<char>();
  size_t sbytes = g->scratch_bytes;
  if (static_scratch) {
    // the same layout in the static array, with fewer workgroups when the
    // full grid's cursors do not fit (the starts come from a ticket, so any
    // grid of at least one workgroup counts every start)
    const size_t need = min_count_scratch_bytes(g);
    if (need > kStaticScratchBytes)
      throw Error{BFC_ERR_TOO_LARGE, "the count needs " + std::to_string(need) +
                                         " bytes of scratch; the static buffer holds " +
                                         std::to_string(kStaticScratchBytes)};
    sbase = static_cast<char*>(static_scratch_ptr());
    sbytes = kStaticScratchBytes;
    size_t room = kStaticScratchBytes - 256;
    if (sc.n_medium > 0) {
      const int fit = (int)std::min<size_t>((size_t)med_grid, (room - (sc.n_heavy > sc.n_medium ? big_wg_bytes(g) : 0)) /
                                                                   med_wg_bytes());
      med_grid = fit;
      room -= (size_t)med_grid * med_wg_bytes();
    }
    if (sc.n_heavy - sc.n_medium > 0) big_grid = (int)std::min<size_t>((size_t)big_grid, room / big_wg_bytes(g));
  }
  int32_t* cursor = reinterpret_cast<int32_t*>(sbase);
  int32_t* med_cursor = reinterpret_cast<int32_t*>(sbase + (size_t)big_grid * big_wg_bytes(g));
  // tickets: [0] big heavy starts, [1] medium heavy starts
  unsigned int* ticket = reinterpret_cast<unsigned int*>(sbase + sbytes - 256);
  // sticky: set by any count on the handle, never cleared (read by the calls that wait)
  int32_t* status = count_status(g);

  CountParams p{};
  for (int x = 0; x < 2; ++x) {
    p.sv[x].off = g->side[x].off.as<int32_t>();
    p.sv[x].adj = g->side[x].adj.as<int32_t>();
    p.sv[x].rev = g->side[x].rev.as<int32_t>();
    p.sv[x].lo = g->side[x].lo.as<int32_t>();
    p.sv[x].id_of = g->side[x].id_of.as<int32_t>();
    p.sv[x].work = g->side[x].work.as<int64_t>();
  }
  p.mode = mode;
  p.total = reinterpret_cast<unsigned long long*>(total_dev);
  p.cursor = cursor;
  p.cursor_stride = stride;
  p.ticket = ticket;
  p.status = status;
  p.dense_ratio = g->tune.dense_min_ratio;
  p.window_mode = g->tune.window_mode;
  p.hash_window_wedges = g->tune.hash_window_wedges;
  p.dense_min_wedges = g->tune.dense_min_wedges;
  if (g->gtune.bytes && g->gid[0].bytes) {
    p.gtune = g->gtune.as<int4>();
    p.gid[0] = g->gid[0].as<int32_t>();
    p.gid[1] = g->gid[1].as<int32_t>();
  }
  p.vpp = sc.vpp;
  p.nX[0] = g->side[0].n;
  p.nX[1] = g->side[1].n;
  // Algorithm 3's per-start work (read when a list entry's clamps)
  if (sc.vpp & 1) p.sv[0].work = g->side[0].wpp.as<int64_t>();
  if (sc.vpp & 2) p.sv[1].work = g->side[1].wpp.as<int64_t>();
  p.q8[0] = g->byte_rank[0];
  p.q8[1] = g->byte_rank[1];
  // top bands: band starts' own-part work, band items' work and slice bounds
  for (int x = 0; x < 2; ++x) {
    p.band_lo[x] = 0;
    p.blb[x] = nullptr;
    p.wtop[x] = nullptr;
    if ((sc.band >> x) & 1) {
      const Side& sd = g->side[x];
      p.band_lo[x] = sd.band_lo;
      p.blb[x] = sd.band_lb.as<int32_t>();
      p.wtop[x] = sd.wtop.as<int64_t>();
      p.sv[x].work = sd.wband.as<int64_t>();
    }
  }
  for (int o = 0; o < 2; ++o) {
    p.wt[o] = g->wt[o].bytes ? g->wt[o].as<int32_t>() : nullptr;
    p.wt_first[o] = g->wt_first[o];
    p.wt_row[o] = g->wt_row[o];
  }
  if (g->grank[0].bytes && g->grank[1].bytes) {
    // a batch: each start's ends lie in its graph's rank range
    p.gid[0] = g->gid[0].as<int32_t>();
    p.gid[1] = g->gid[1].as<int32_t>();
    p.grank[0] = g->grank[0].as<int32_t>();
    p.grank[1] = g->grank[1].as<int32_t>();
  }
  if (gtotals) {
    p.total = nullptr;
    p.gtotal = reinterpret_cast<unsigned long long*>(gtotals);
    p.gid[0] = g->gid[0].as<int32_t>();
    p.gid[1] = g->gid[1].as<int32_t>();
  }
  if (mode == kVertex) {
    // accumulate by rank (an end's counter and its accumulator share an
    // index, so neighbouring counters add to neighbouring words), then
    // write each vertex's sum to its input id
    const int64_t nv = (int64_t)g->side[0].n + g->side[1].n;
    const size_t need = sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1);
    if (g->vacc.bytes < need) g->vacc.alloc(need, s);
    zero_u64(g->vacc.p, nv, s);
    p.vout[0] = g->vacc.as<unsigned long long>();
    p.vout[1] = g->vacc.as<unsigned long long>() + g->side[0].n;
  } else if (mode == kEdge) {
    const size_t need = sizeof(int64_t) * 2 * (size_t)(g->m > 0 ? g->m : 1);
    if (g->acc.bytes < need) g->acc.alloc(need, s);
    if (g->edge_acc32()) {
      zero_u64(g->acc.p, g->m, s);  // 2m 32-bit words
      p.acc32[0] = g->acc.as<uint32_t>();
      p.acc32[1] = g->acc.as<uint32_t>() + g->m;
    } else {
      zero_u64(g->acc.p, 2 * g->m, s);
      p.acc[0] = g->acc.as<unsigned long long>();
      p.acc[1] = g->acc.as<unsigned long long>() + g->m;
    }
  }
  const DenseBlock& d = g->dense;
  p.dtop[0] = g->side[0].n - d.KU;
  p.dtop[1] = g->side[1].n - d.KL;
  if (d.KU > 0) {
    p.dC[0] = d.CU();
    p.dC[1] = d.CL();
    p.dld[0] = d.PU;
    p.dld[1] = d.PL;
  }
  zero_u64(ticket, 1, s);      // both tickets
  // kernel timing creates events: not in the static-scratch call, which creates nothing
  const bool timing = g->timing && !static_scratch;
  // events: [0] dense block [1] light [2] heavy [3] fold [4]
  bfc_graph_s::TimedCall tc{};
  if (timing) {
    for (int i = 0; i < 5; ++i) BFC_HIP(hipEventCreate(&tc.ev[i]));
    BFC_HIP(hipEventRecord(tc.ev[0], s));
  }
  dense_block(g, s);
  if (timing) BFC_HIP(hipEventRecord(tc.ev[1], s));
  {
    // the light list holds the small starts, then the mid ones, then the large ones
    const int4* llist = g->sched.light.as<int4>();
    auto light_grid = [&](int32_t n) {
      int64_t grid = ((int64_t)n + kLightWaves - 1) / kLightWaves;
      return (unsigned)(grid > (int64_t)cus * 16 ? (int64_t)cus * 16 : grid);
    };
    const int32_t n_small = sc.n_small, n_mid = sc.n_mid, n_large = sc.n_light - sc.n_small - sc.n_mid;
    const bool vpp = sc.vpp != 0 || sc.band != 0;
    if (n_small > 0) {
      launch_light<kSmallCap, false>(mode, vpp, light_grid(n_small), s, p, llist, n_small);
    }
    if (n_mid > 0) {
      const int4* l = llist + n_small;
      if (g->light_packed) launch_light<kLightCap, true>(mode, vpp, light_grid(n_mid), s, p, l, n_mid);
      else launch_light<kLightCap, false>(mode, vpp, light_grid(n_mid), s, p, l, n_mid);
    }
    if (n_large > 0) {
      // only where the tables pack (light_max above 1024)
      launch_light<kLightPackedCap, true>(mode, vpp, light_grid(n_large), s, p, llist + n_small + n_mid, n_large);
    }
  }
  if (timing) BFC_HIP(hipEventRecord(tc.ev[2], s));
  // the heavy list holds the big starts (decreasing work), then the medium ones
  const int32_t n_big = sc.n_heavy - sc.n_medium;
  if (n_big > 0) {
    p.list = g->sched.heavy.as<int4>();
    p.n_list = n_big;
    if (sc.vpp || sc.band) launch_heavy<kBigNT, kBigWords, true>(mode, big_grid, s, p);
    else launch_heavy<kBigNT, kBigWords, false>(mode, big_grid, s, p);
  }
  if (sc.n_medium > 0) {
    // (the schedule has no medium starts when a layer takes Algorithm 3's wedges)
    p.list = g->sched.heavy.as<int4>() + n_big;
    p.n_list = sc.n_medium;
    p.ticket = ticket + 1;
    p.cursor = med_cursor;
    p.cursor_stride = kMedPre;
    launch_heavy<kMedNT, kMedWords, false>(mode, med_grid, s, p);
  }
  if (timing) BFC_HIP(hipEventRecord(tc.ev[3], s));
  if (mode == kVertex) {
    for (int x = 0; x < 2; ++x) {
      const int32_t n = g->side[x].n;
      if (n == 0) continue;
      const int64_t grid = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
      vertex_out_kernel<<<(unsigned)grid, 256, 0, s>>>(p.vout[x], g->side[x].id_of.as<int32_t>(), n,
                                                       reinterpret_cast<unsigned long long*>(x ? out1 : out0));
      BFC_LAUNCH_CHECK();
    }
  }
  if (mode == kEdge && g->m > 0) {
    int64_t grid = (g->m + 255) / 256;
    if (grid > 65536) grid = 65536;
    if (p.acc32[0])
      fold_edges32_kernel<<<(unsigned)grid, 256, 0, s>>>(g->edge0.as<int32_t>(), g->side[0].rev.as<int32_t>(),
                                                         p.acc32[0], p.acc32[1], g->m,
                                                         reinterpret_cast<unsigned long long*>(out0));
    else
      fold_edges_kernel<<<(unsigned)grid, 256, 0, s>>>(g->edge0.as<int32_t>(), g->side[0].rev.as<int32_t>(),
                                                       p.acc[0], p.acc[1], g->m,
                                                       reinterpret_cast<unsigned long long*>(out0));
    BFC_LAUNCH_CHECK();
  }
  if (timing) {
    BFC_HIP(hipEventRecord(tc.ev[4], s));
    g->timed.push_back(tc);
  }
}

void collect_times(bfc_graph_s* g) {
  for (auto& tc : g->timed) {
    BFC_HIP(hipEventSynchronize(tc.ev[4]));
    float dn = 0, a = 0, b = 0, c = 0;
    BFC_HIP(hipEventElapsedTime(&dn, tc.ev[0], tc.ev[1]));
    BFC_HIP(hipEventElapsedTime(&a, tc.ev[1], tc.ev[2]));
    BFC_HIP(hipEventElapsedTime(&b, tc.ev[2], tc.ev[3]));
    BFC_HIP(hipEventElapsedTime(&c, tc.ev[3], tc.ev[4]));
    g->light_ms += a;
    g->heavy_ms += b;
    g->other_ms += c + dn;
    g->timed_calls += 1;
    for (int i = 0; i < 5; ++i) (void)hipEventDestroy(tc.ev[i]);
  }
  g->timed.clear();
}

}  // namespace bfc
