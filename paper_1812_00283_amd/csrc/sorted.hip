// Sort-based total count: the external-memory algorithm of Section 6.3
// (Algorithm 6) with HBM in the place of disk.
//
// Algorithm 6 emits, for every wedge (u, v, w) whose end w has the highest
// priority of the three (the wedges Algorithm 2 processes, with w as their
// start), the vertex pair (u, w); sorts the pairs so equal pairs are adjacent;
// and adds C(c, 2) for every run of c equal pairs (Lemma 1).  Here the pairs
// of a contiguous range of start ranks of one layer form a chunk of at most
// max_pairs (plus one start's wedges) 64-bit keys (start rank - first rank of
// the chunk) << ebits | end rank; equal pairs never cross chunks because a
// pair holds its start.  A chunk is emitted start by start (its wedges are
// the prefix N(r) below r's priority, and for each such middle v the part of
// N(v) below r), so its keys are already ordered by start: a stable radix
// sort on the end bits alone (the build's sort) leaves each end's pairs in
// start order, so equal pairs end up adjacent.  The runs are then counted
// in one pass.
//
// The same machinery runs the wedges of Algorithm 3 (BFC-VP++, Section 5):
// there the end outranks both the start and the middle, every neighbour of a
// start is a middle, and the ends of middle v are the suffix of N(v) above
// max(p(start), p(v)): past the start's own slot when v ranks below the
// start, else past v's lower-priority prefix.  Same wedge count (Lemma 3),
// same pairs-and-runs count (Theorem 4).
#include "sorted.hpp"

namespace bfc {
namespace {

constexpr int kEmitNT = 256;
constexpr int kEmitTile = 4096;  // pairs per emitting workgroup
constexpr int kRunNT = 256;
constexpr int kRunPer = 16;
constexpr int kRunTile = kRunNT * kRunPer;

// bounds[c] = first rank r with offs[r] >= c * per (c < nch), bounds[nch] = n;
// firsts[c] = offs[bounds[c]], mids[c] = moff[bounds[c]]
__global__ void chunk_bounds_kernel(const int64_t* __restrict__ offs, const int32_t* __restrict__ moff, int32_t n,
                                    int64_t per, int32_t nch, int32_t* __restrict__ bounds,
                                    int64_t* __restrict__ firsts, int32_t* __restrict__ mids) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > nch) return;
  int32_t r = n;
  if (c < nch) {
    const int64_t want = (int64_t)c * per;
    int32_t lo = 0, hi = n;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (offs[mid] < want) lo = mid + 1; else hi = mid;
    }
    r = lo;
  }
  bounds[c] = r;
  firsts[c] = offs[r];
  mids[c] = moff[r];
}

// The middle arcs of the chunk's starts as one dense list: arc q of start r
// (its j-th middle) sits at q = moff[r] - q0 + j and records its slice of
// ends (first slot, length) and r - r0.  One wavefront per start.
// Algorithm 2 (kPlus false): the middles are the prefix lo[r] of N(r) and the
// ends of middle v are N(v) below r.  Algorithm 3 (kPlus true, moff = off_x):
// every neighbour is a middle and the ends are the suffix of N(v) above both.
template <bool kPlus>
__global__ void mid_fill_kernel(const int32_t* __restrict__ off_x, const int32_t* __restrict__ adj_x,
                                const int32_t* __restrict__ rev_x, const int32_t* __restrict__ lo_x,
                                const int32_t* __restrict__ off_o, const int32_t* __restrict__ lo_o,
                                const int32_t* __restrict__ moff, int32_t r0, int32_t r1,
                                int64_t* __restrict__ qlen, int32_t* __restrict__ qbeg,
                                int32_t* __restrict__ qsrc) {
  const int lane = threadIdx.x & 63;
  const int32_t q0 = moff[r0];
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < r1 - r0; w += waves) {
    const int32_t r = r0 + (int32_t)w;
    const int32_t a0 = off_x[r], lo = lo_x[r], qb = moff[r] - q0;
    const int32_t nm = kPlus ? off_x[r + 1] - a0 : lo;
    for (int32_t j = lane; j < nm; j += 64) {
      const int32_t a = a0 + j;
      const int32_t v = adj_x[a];
      int32_t beg, len;
      if (kPlus) {
        beg = j < lo ? rev_x[a] + 1 : off_o[v] + lo_o[v];
        len = off_o[v + 1] - beg;
      } else {
        beg = off_o[v];
        len = rev_x[a] - beg;
      }
      qlen[qb + j] = len;
      qbeg[qb + j] = beg;
      qsrc[qb + j] = r - r0;
    }
  }
}

// W of every start under Algorithm 3: the sum of its middles' suffix
// lengths.  One wavefront per start.
__global__ void vpp_work_kernel(const int32_t* __restrict__ off_x, const int32_t* __restrict__ adj_x,
                                const int32_t* __restrict__ rev_x, const int32_t* __restrict__ lo_x,
                                const int32_t* __restrict__ off_o, const int32_t* __restrict__ lo_o, int32_t n,
                                int64_t* __restrict__ work) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < n; w += waves) {
    const int32_t r = (int32_t)w;
    const int32_t a0 = off_x[r], lo = lo_x[r], d = off_x[r + 1] - a0;
    unsigned long long t = 0;
    for (int32_t j = lane; j < d; j += 64) {
      const int32_t a = a0 + j;
      const int32_t v = adj_x[a];
      const int32_t beg = j < lo ? rev_x[a] + 1 : off_o[v] + lo_o[v];
      t += (unsigned long long)(off_o[v + 1] - beg);
    }
    for (int s = 32; s > 0; s >>= 1) t += __shfl_down(t, s, 64);
    if (lane == 0) work[r] = (int64_t)t;
  }
}

// Each workgroup writes the pairs [P0, P0 + kEmitTile) of the chunk, in the
// order of the middle-arc list (qpos: exclusive prefix of the slice lengths):
// it finds the arc holding P0, then loads kEmitNT arcs at a time into LDS and
// each thread finds the arc of each of its positions by a binary search.
__global__ __launch_bounds__(kEmitNT) void pair_emit_kernel(const int64_t* __restrict__ qpos,
                                                            const int32_t* __restrict__ qbeg,
                                                            const int32_t* __restrict__ qsrc, int32_t nq,
                                                            int64_t np, const int32_t* __restrict__ adj_o,
                                                            int ebits, uint64_t* __restrict__ keys) {
  __shared__ int64_t s_pos[kEmitNT + 1];
  __shared__ int32_t s_beg[kEmitNT];
  __shared__ uint32_t s_src[kEmitNT];
  __shared__ int32_t s_q;
  const int tid = threadIdx.x;
  const int64_t P0 = (int64_t)blockIdx.x * kEmitTile;
  const int64_t P1 = P0 + kEmitTile < np ? P0 + kEmitTile : np;
  if (tid == 0) {
    int32_t lo = 0, hi = nq - 1;  // the last arc with qpos <= P0
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if (qpos[mid] <= P0) lo = mid; else hi = mid - 1;
    }
    s_q = lo;
  }
  __syncthreads();
  for (int32_t qb = s_q;; qb += kEmitNT) {
    const int32_t q = qb + tid;
    s_pos[tid] = q < nq ? qpos[q] : np;
    s_beg[tid] = q < nq ? qbeg[q] : 0;
    s_src[tid] = q < nq ? (uint32_t)qsrc[q] : 0u;
    if (tid == 0) s_pos[kEmitNT] = qb + kEmitNT < nq ? qpos[qb + kEmitNT] : np;
    __syncthreads();
    const int64_t a = P0 > s_pos[0] ? P0 : s_pos[0];
    const int64_t b = P1 < s_pos[kEmitNT] ? P1 : s_pos[kEmitNT];
    for (int64_t p = a + tid; p < b; p += kEmitNT) {
      int lo = 0, hi = kEmitNT - 1;  // the last arc with s_pos <= p
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pos[mid] <= p) lo = mid; else hi = mid - 1;
      }
      keys[p] = ((uint64_t)s_src[lo] << ebits) | (uint32_t)adj_o[s_beg[lo] + (p - s_pos[lo])];
    }
    const bool done = s_pos[kEmitNT] >= P1;
    __syncthreads();
    if (done) break;
  }
}

__device__ __forceinline__ int64_t choose2(int64_t c) { return c * (c - 1) / 2; }

// Sum of C(c, 2) over the runs of equal sorted keys whose first key lies in
// this workgroup's tile.  Each thread takes kRunPer consecutive keys; a run
// that leaves a thread's keys ends at the first run start of a later thread
// (a suffix minimum over the workgroup) or, past the tile, where a forward
// scan by the whole workgroup finds the key change.
__global__ __launch_bounds__(kRunNT) void run_count_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                           unsigned long long* __restrict__ total) {
  __shared__ int64_t s_first[kRunNT];
  __shared__ int64_t s_next;
  __shared__ unsigned long long s_sum[kRunNT / 64];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kRunTile;
  const int64_t t1 = t0 + kRunTile < n ? t0 + kRunTile : n;
  const int64_t b = t0 + (int64_t)tid * kRunPer;
  uint64_t k[kRunPer];
  uint64_t prev = 0;
  if (b < t1) {
    if (b + kRunPer <= t1) {
      const ulonglong2* v = reinterpret_cast<const ulonglong2*>(keys + b);
#pragma unroll
      for (int i = 0; i < kRunPer / 2; ++i) {
        const ulonglong2 x = v[i];
        k[2 * i] = x.x;
        k[2 * i + 1] = x.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kRunPer; ++i) k[i] = b + i < t1 ? keys[b + i] : 0;
    }
    prev = b > 0 ? keys[b - 1] : ~k[0];
  }
  // run starts among this thread's keys
  int64_t first = INT64_MAX, last = -1;
  unsigned long long sum = 0;
  if (b < t1) {
    uint64_t pk = prev;
#pragma unroll
    for (int i = 0; i < kRunPer; ++i) {
      if (b + i < t1 && k[i] != pk) {
        if (last >= 0) sum += (unsigned long long)choose2(b + i - last);
        else first = b + i;
        last = b + i;
      }
      pk = k[i];
    }
  }
  s_first[tid] = first;
  if (tid == 0) s_next = INT64_MAX;
  __syncthreads();
  // suffix minimum of the first run starts of the later threads
  for (int d = 1; d < kRunNT; d <<= 1) {
    const int64_t o = tid + d < kRunNT ? s_first[tid + d] : INT64_MAX;
    __syncthreads();
    if (o < s_first[tid]) s_first[tid] = o;
    __syncthreads();
  }
  int64_t after = tid + 1 < kRunNT ? s_first[tid + 1] : INT64_MAX;
  // the tile's last run: find where it ends past the tile
  // the run of the tile's last run start reaches the tile's end; it goes on
  // while the keys past the tile equal the tile's last key
  if (s_first[0] != INT64_MAX && t1 < n) {
    const uint64_t lastkey = keys[t1 - 1];
    for (int64_t base = t1; base < n; base += kRunNT) {
      const int64_t i = base + tid;
      if (i < n && keys[i] != lastkey) atomicMin(reinterpret_cast<unsigned long long*>(&s_next),
                                                 (unsigned long long)i);
      __syncthreads();
      if (s_next != INT64_MAX) break;
      __syncthreads();
    }
  }
  __syncthreads();
  const int64_t tail = s_next != INT64_MAX ? s_next : n;
  if (last >= 0) {
    const int64_t end = after != INT64_MAX ? after : tail;
    sum += (unsigned long long)choose2(end - last);
  }
  // workgroup sum
  for (int d = 32; d > 0; d >>= 1) sum += __shfl_down(sum, d, 64);
  if ((tid & 63) == 0) s_sum[tid >> 6] = sum;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kRunNT / 64; ++w) t += s_sum[w];
    if (t) atomicAdd(total, t);
  }
}

}  // namespace

void vpp_work(const bfc_graph_s* g, int x, int64_t* work, hipStream_t s) {
  const Side& S = g->side[x];
  const Side& O = g->side[1 - x];
  const int32_t n = S.n;
  if (n <= 0) return;
  const int64_t wg = ((int64_t)n + 3) / 4;
  vpp_work_kernel<<<(unsigned)(wg < 65536 ? wg : 65536), 256, 0, s>>>(
      S.off.as<int32_t>(), S.adj.as<int32_t>(), S.rev.as<int32_t>(), S.lo.as<int32_t>(), O.off.as<int32_t>(),
      O.lo.as<int32_t>(), n, work);
  BFC_LAUNCH_CHECK();
}

void count_total_sorted(bfc_graph_s* g, int direction, int64_t max_pairs, hipStream_t s, int64_t* total_host,
                        int64_t* pairs_host, int64_t* chunks_host) {
  // the radix sort ranks keys with 32-bit offsets
  constexpr int64_t kMaxChunk = int64_t(1) << 31, kSortLimit = int64_t(1) << 32;
  const bool plus = direction == 1;
  if (max_pairs <= 0 || max_pairs > kMaxChunk) max_pairs = kMaxChunk;
  TmpBuf tot;
  tot.alloc(sizeof(int64_t), s);
  zero_u64(tot.p, 1, s);
  int64_t chunks = 0, all_pairs = 0;
  TmpBuf keys, ktmp, qlen, qbeg, qsrc;
  size_t key_cap = 0, q_cap = 0;
  for (int x = 0; x < 2; ++x) {
    const Side& S = g->side[x];
    const Side& O = g->side[x ^ 1];
    const int32_t n = S.n;
    if (n == 0) continue;
    // per start: first pair (prefix of W) and first middle arc (prefix of lo,
    // or the CSR offsets when every neighbour is a middle)
    TmpBuf offs, moff_buf, work_plus;
    offs.alloc(sizeof(int64_t) * ((size_t)n + 1), s);
    const int64_t* work = S.work.as<int64_t>();
    if (plus) {
      work_plus.alloc(sizeof(int64_t) * (size_t)n, s);
      vpp_work(g, x, work_plus.as<int64_t>(), s);
      work = work_plus.as<int64_t>();
    }
    exclusive_scan_i64(work, offs.as<int64_t>(), n, offs.as<int64_t>() + n, s);
    const int32_t* moff = S.off.as<int32_t>();
    if (!plus) {
      moff_buf.alloc(sizeof(int32_t) * ((size_t)n + 1), s);
      exclusive_scan_i32(S.lo.as<int32_t>(), moff_buf.as<int32_t>(), n, moff_buf.as<int32_t>() + n, s);
      moff = moff_buf.as<int32_t>();
    }
    int64_t pairs = 0;
    BFC_HIP(hipMemcpyAsync(&pairs, offs.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    all_pairs += pairs;
    if (pairs == 0) continue;
    const int32_t nch = (int32_t)((pairs + max_pairs - 1) / max_pairs);
    TmpBuf bnd, fst, mst;
    bnd.alloc(sizeof(int32_t) * ((size_t)nch + 1), s);
    fst.alloc(sizeof(int64_t) * ((size_t)nch + 1), s);
    mst.alloc(sizeof(int32_t) * ((size_t)nch + 1), s);
    chunk_bounds_kernel<<<grid_for(nch + 1, 256), 256, 0, s>>>(offs.as<int64_t>(), moff, n, max_pairs, nch,
                                                                bnd.as<int32_t>(), fst.as<int64_t>(),
                                                                mst.as<int32_t>());
    BFC_LAUNCH_CHECK();
    std::vector<int32_t> b(nch + 1), mq(nch + 1);
    std::vector<int64_t> f(nch + 1);
    BFC_HIP(hipMemcpyAsync(b.data(), bnd.p, sizeof(int32_t) * (nch + 1), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipMemcpyAsync(f.data(), fst.p, sizeof(int64_t) * (nch + 1), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipMemcpyAsync(mq.data(), mst.p, sizeof(int32_t) * (nch + 1), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    const int ebits = bits_for((uint64_t)n - 1);
    for (int32_t c = 0; c < nch; ++c)
      if (f[c + 1] - f[c] >= kSortLimit)
        throw Error{BFC_ERR_TOO_LARGE, "a start has so many wedges that its chunk holds 2^32 pairs or more"};
    for (int32_t c = 0; c < nch; ++c) {
      const int32_t r0 = b[c], r1 = b[c + 1];
      const int64_t np = f[c + 1] - f[c];
      const int32_t nq = mq[c + 1] - mq[c];
      if (r1 <= r0 || np == 0) continue;
      if ((size_t)np > key_cap) {
        keys.alloc(sizeof(uint64_t) * (size_t)np, s);
        ktmp.alloc(sizeof(uint64_t) * (size_t)np, s);
        key_cap = (size_t)np;
      }
      if ((size_t)nq + 1 > q_cap) {
        qlen.alloc(sizeof(int64_t) * ((size_t)nq + 1), s);
        qbeg.alloc(sizeof(int32_t) * ((size_t)nq + 1), s);
        qsrc.alloc(sizeof(int32_t) * ((size_t)nq + 1), s);
        q_cap = (size_t)nq + 1;
      }
      const int64_t fg = ((int64_t)(r1 - r0) + 3) / 4;
      const unsigned fill_grid = (unsigned)(fg < 65536 ? fg : 65536);
      if (plus)
        mid_fill_kernel<true><<<fill_grid, 256, 0, s>>>(
            S.off.as<int32_t>(), S.adj.as<int32_t>(), S.rev.as<int32_t>(), S.lo.as<int32_t>(), O.off.as<int32_t>(),
            O.lo.as<int32_t>(), moff, r0, r1, qlen.as<int64_t>(), qbeg.as<int32_t>(), qsrc.as<int32_t>());
      else
        mid_fill_kernel<false><<<fill_grid, 256, 0, s>>>(
            S.off.as<int32_t>(), S.adj.as<int32_t>(), S.rev.as<int32_t>(), S.lo.as<int32_t>(), O.off.as<int32_t>(),
            O.lo.as<int32_t>(), moff, r0, r1, qlen.as<int64_t>(), qbeg.as<int32_t>(), qsrc.as<int32_t>());
      BFC_LAUNCH_CHECK();
      exclusive_scan_i64(qlen.as<int64_t>(), qlen.as<int64_t>(), nq, nullptr, s);
      pair_emit_kernel<<<grid_for(np, kEmitTile), kEmitNT, 0, s>>>(qlen.as<int64_t>(), qbeg.as<int32_t>(),
                                                                   qsrc.as<int32_t>(), nq, np, O.adj.as<int32_t>(),
                                                                   ebits, keys.as<uint64_t>());
      BFC_LAUNCH_CHECK();
      const bool in_tmp = radix_sort_u64_keys_any(keys.as<uint64_t>(), ktmp.as<uint64_t>(), np, 0, ebits, s);
      const uint64_t* sorted = in_tmp ? ktmp.as<uint64_t>() : keys.as<uint64_t>();
      run_count_kernel<<<grid_for(np, kRunTile), kRunNT, 0, s>>>(sorted, np,
                                                                  reinterpret_cast<unsigned long long*>(tot.p));
      BFC_LAUNCH_CHECK();
      ++chunks;
    }
  }
  int64_t v = 0;
  BFC_HIP(hipMemcpyAsync(&v, tot.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BFC_HIP(hipStreamSynchronize(s));
  *total_host = v;
  if (pairs_host) *pairs_host = all_pairs;
  if (chunks_host) *chunks_host = chunks;
}

}  // namespace bfc
