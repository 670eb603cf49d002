// Device-wide exclusive scan and stable LSD radix sort (8-bit digits).
//
// Scan: reduce-then-scan.  Each workgroup of 256 threads owns a tile of 4096
// values; tile sums are scanned (recursively when there are more than one
// tile) and each tile is then scanned locally with its offset.
//
// Radix sort: per 8-bit digit, (1) a digit histogram per 4096-key tile,
// (2) an exclusive scan of the histograms laid out digit-major, so that
// counts[d * tiles + t] becomes the output position of tile t's first key
// with digit d, and (3) a stable scatter.  In the scatter each wavefront
// owns 512 consecutive keys of the tile and ranks them 64 at a time: lanes
// with equal digits are found with eight ballots (one per digit bit), and a
// per-wavefront running count per digit in LDS orders successive rounds, so
// no workgroup barrier is needed inside the ranking loop.  Keys are then
// staged in LDS in sorted order and written out so that consecutive threads
// write consecutive addresses of one digit's run.
#include "device.hpp"
#include "internal.hpp"
#include "sort.hpp"

namespace bfc {

namespace {

constexpr int kScanNT = 256;
constexpr int kScanVT = 16;
constexpr int kScanTile = kScanNT * kScanVT;

template <typename T>
__global__ __launch_bounds__(kScanNT) void scan_reduce_kernel(const T* __restrict__ in, int64_t n,
                                                              T* __restrict__ partials) {
  __shared__ T smem[kScanNT / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanVT; ++j) {
    int64_t i = base + j * kScanNT + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = block_sum<T, kScanNT>(s, smem);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kScanNT) void scan_tile_kernel(const T* in, T* out, int64_t n,
                                                            const T* __restrict__ offsets,
                                                            T* __restrict__ total) {
  __shared__ T tile[kScanTile];
  __shared__ T smem[kScanNT / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kScanVT; ++j) {
    int64_t i = base + j * kScanNT + t;
    tile[j * kScanNT + t] = i < n ? in[i] : T(0);
  }
  __syncthreads();
  T loc[kScanVT];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanVT; ++j) {
    loc[j] = s;
    s += tile[t * kScanVT + j];
  }
  T all;
  T pre = block_exclusive_scan<T, kScanNT>(s, smem, &all);
  T off = offsets ? offsets[blockIdx.x] : T(0);
#pragma unroll
  for (int j = 0; j < kScanVT; ++j) tile[t * kScanVT + j] = loc[j] + pre + off;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanVT; ++j) {
    int64_t i = base + j * kScanNT + t;
    if (i < n) out[i] = tile[j * kScanNT + t];
  }
  if (total && t == 0 && blockIdx.x == gridDim.x - 1) total[0] = off + all;
}

template <typename T>
void exclusive_scan_impl(const T* in, T* out, int64_t n, T* total, hipStream_t s) {
  if (n <= 0) {
    if (total) BFC_HIP(hipMemsetAsync(total, 0, sizeof(T), s));
    return;
  }
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    scan_tile_kernel<T><<<1, kScanNT, 0, s>>>(in, out, n, nullptr, total);
    BFC_LAUNCH_CHECK();
    return;
  }
  T* partials = nullptr;
  partials = static_cast<T*>(cache_alloc(sizeof(T) * (size_t)tiles, s));
  scan_reduce_kernel<T><<<(unsigned)tiles, kScanNT, 0, s>>>(in, n, partials);
  BFC_LAUNCH_CHECK();
  exclusive_scan_impl<T>(partials, partials, tiles, nullptr, s);
  scan_tile_kernel<T><<<(unsigned)tiles, kScanNT, 0, s>>>(in, out, n, partials, total);
  BFC_LAUNCH_CHECK();
  cache_free(partials, s);
}

// ------------------------------------------------------------------ sort
// 4096 keys per workgroup (512 threads): each tile writes 256 digit runs
// of 16 keys on average.  The tile's 36 KB of LDS (64-bit keys) lets four
// workgroups share a CU; measured against 2,048- to 12,288-key tiles and
// 256 or 1,024 threads, this shape sorted fastest.
constexpr int kSortNT = 512;
constexpr int kSortVT = 8;
constexpr int kSortTile = kSortNT * kSortVT;   // 4096 keys per workgroup
static_assert(kSortTile == kSortTileKeys, "the tile that sort.hpp announces");
constexpr int kSortWaves = kSortNT / 64;
constexpr int kPerWave = kSortTile / kSortWaves;  // 512

template <typename K>
__global__ __launch_bounds__(kSortNT) void sort_hist_kernel(const K* __restrict__ keys, int64_t n, int shift,
                                                            uint32_t* __restrict__ counts, int64_t tiles) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int j = 0; j < kSortVT; ++j) {
    int64_t i = base + j * kSortNT + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 256) counts[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// kVals false: keys only (vin and vout unused).
template <typename K, bool kVals>
__global__ __launch_bounds__(kSortNT) void sort_scatter_kernel(const K* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               int64_t n, int shift,
                                                               const uint32_t* __restrict__ offs, int64_t tiles) {
  __shared__ uint32_t wcnt[kSortWaves][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t red[kSortWaves + 1];
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kVals ? kSortTile : 1];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  for (int i = t; i < kSortWaves * 256; i += kSortNT) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  K k[kSortVT];
  uint32_t v[kSortVT];
  uint32_t r[kSortVT];
  const uint64_t lt = __lanemask_lt();
#pragma unroll
  for (int j = 0; j < kSortVT; ++j) {
    const int64_t idx = tile0 + (int64_t)w * kPerWave + j * 64 + lane;
    const bool valid = idx < n;
    k[j] = valid ? kin[idx] : K(0);
    v[j] = (kVals && valid) ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    uint32_t base = 0;
    if (valid) base = wcnt[w][d];
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    if (valid && below == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    r[j] = base + below;
  }
  __syncthreads();
  {
    // thread t < 256 handles digit t
    uint32_t tot = 0;
    if (t < 256) {
      uint32_t c[kSortWaves];
#pragma unroll
      for (int q = 0; q < kSortWaves; ++q) { c[q] = wcnt[q][t]; }
#pragma unroll
      for (int q = 0; q < kSortWaves; ++q) { wcnt[q][t] = tot; tot += c[q]; }
    }
    uint32_t all;
    const uint32_t ds = block_exclusive_scan<uint32_t, kSortNT>(tot, red, &all);
    if (t < 256) {
      dstart[t] = ds;
      goff[t] = offs[(int64_t)t * tiles + blockIdx.x];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortVT; ++j) {
    const int64_t idx = tile0 + (int64_t)w * kPerWave + j * 64 + lane;
    if (idx < n) {
      const uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
      const uint32_t pos = dstart[d] + wcnt[w][d] + r[j];
      skey[pos] = k[j];
      if (kVals) sval[pos] = v[j];
    }
  }
  __syncthreads();
  const int64_t rem = n - tile0;
  const int tile_n = rem < kSortTile ? (int)rem : kSortTile;
  for (int p = t; p < tile_n; p += kSortNT) {
    const K kk = skey[p];
    const uint32_t d = (uint32_t)(kk >> shift) & 255u;
    const int64_t dst = (int64_t)goff[d] + (p - (int64_t)dstart[d]);
    kout[dst] = kk;
    if (kVals) vout[dst] = sval[p];
  }
}

// Sorts on key bits [lo_bit, lo_bit + bits); vals may be null (keys only).
// Returns true when the sorted data ends in (ktmp, vtmp) (copy_back false).
// first_counts: the first pass's tile histograms, already counted (or null).
template <typename K>
bool radix_sort_impl(K* keys, uint32_t* vals, K* ktmp, uint32_t* vtmp, int64_t n, int bits, hipStream_t s,
                     bool copy_back = true, int lo_bit = 0, uint32_t* first_counts = nullptr) {
  if (n <= 1 || bits <= 0) return false;
  const int64_t tiles = (n + kSortTile - 1) / kSortTile;
  uint32_t* counts = nullptr;
  counts = static_cast<uint32_t*>(cache_alloc(sizeof(uint32_t) * 256 * (size_t)tiles, s));
  K* ks = keys;
  K* kd = ktmp;
  uint32_t* vs = vals;
  uint32_t* vd = vtmp;
  for (int shift = lo_bit; shift < lo_bit + bits; shift += 8) {
    uint32_t* c = counts;
    if (shift == lo_bit && first_counts) {
      c = first_counts;
    } else {
      sort_hist_kernel<K><<<(unsigned)tiles, kSortNT, 0, s>>>(ks, n, shift, counts, tiles);
      BFC_LAUNCH_CHECK();
    }
    exclusive_scan_impl<uint32_t>(c, c, 256 * tiles, nullptr, s);
    if (vals)
      sort_scatter_kernel<K, true><<<(unsigned)tiles, kSortNT, 0, s>>>(ks, vs, kd, vd, n, shift, c, tiles);
    else
      sort_scatter_kernel<K, false><<<(unsigned)tiles, kSortNT, 0, s>>>(ks, vs, kd, vd, n, shift, c, tiles);
    BFC_LAUNCH_CHECK();
    K* tk = ks; ks = kd; kd = tk;
    uint32_t* tv = vs; vs = vd; vd = tv;
  }
  const bool in_tmp = ks != keys;
  if (in_tmp && copy_back) {
    BFC_HIP(hipMemcpyAsync(keys, ks, sizeof(K) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (vals) BFC_HIP(hipMemcpyAsync(vals, vs, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
  }
  cache_free(counts, s);
  return in_tmp && !copy_back;
}

}  // namespace

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, hipStream_t s) {
  exclusive_scan_impl<int32_t>(in, out, n, total, s);
}
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, hipStream_t s) {
  exclusive_scan_impl<int64_t>(in, out, n, total, s);
}
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  exclusive_scan_impl<uint32_t>(in, out, n, nullptr, s);
}
void radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                    hipStream_t s) {
  radix_sort_impl<uint32_t>(keys, vals, ktmp, vtmp, n, bits, s);
}
void radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                    hipStream_t s) {
  radix_sort_impl<uint64_t>(keys, vals, ktmp, vtmp, n, bits, s);
}
bool radix_sort_u64_any(uint64_t* keys, uint32_t* vals, uint64_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                        hipStream_t s) {
  return radix_sort_impl<uint64_t>(keys, vals, ktmp, vtmp, n, bits, s, false);
}
bool radix_sort_u64_keys_any(uint64_t* keys, uint64_t* ktmp, int64_t n, int lo_bit, int bits, hipStream_t s) {
  return radix_sort_impl<uint64_t>(keys, nullptr, ktmp, nullptr, n, bits, s, false, lo_bit);
}
bool radix_sort_u64_keys_counted(uint64_t* keys, uint64_t* ktmp, int64_t n, int lo_bit, int bits,
                                 uint32_t* first_counts, hipStream_t s) {
  return radix_sort_impl<uint64_t>(keys, nullptr, ktmp, nullptr, n, bits, s, false, lo_bit, first_counts);
}
bool radix_sort_u64_counted(uint64_t* keys, uint32_t* vals, uint64_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                            uint32_t* first_counts, hipStream_t s) {
  return radix_sort_impl<uint64_t>(keys, vals, ktmp, vtmp, n, bits, s, false, 0, first_counts);
}

}  // namespace bfc
