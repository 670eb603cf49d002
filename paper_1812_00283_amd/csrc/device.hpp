// Wavefront (64 lanes) and workgroup helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfc {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Exclusive scan across a workgroup of NT threads (NT multiple of 64,
// NT <= 4096).  `smem` needs NT/64 + 1 elements.  Returns the exclusive
// prefix; *total receives the workgroup sum.  Contains barriers: every
// thread of the workgroup must call it.
template <typename T, int NT>
__device__ __forceinline__ T block_exclusive_scan(T v, T* smem, T* total) {
  constexpr int NW = NT / 64;
  const int lane = __lane_id();
  const int wid = threadIdx.x / 64;
  T inc = wave_inclusive_scan(v);
  if (lane == 63) smem[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    T w = lane < NW ? smem[lane] : T(0);
    T wi = wave_inclusive_scan(w);
    if (lane < NW) smem[lane] = wi - w;
    if (lane == NW - 1) smem[NW] = wi;
  }
  __syncthreads();
  T res = inc - v + smem[wid];
  *total = smem[NW];
  __syncthreads();
  return res;
}

template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T* smem) {
  constexpr int NW = NT / 64;
  const int lane = __lane_id();
  const int wid = threadIdx.x / 64;
  v = wave_sum(v);
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  T r = 0;
  if (wid == 0) {
    T w = lane < NW ? smem[lane] : T(0);
    r = wave_sum(w);
    if (lane == 0) smem[NW] = r;
  }
  __syncthreads();
  r = smem[NW];
  __syncthreads();
  return r;
}

}  // namespace bfc
