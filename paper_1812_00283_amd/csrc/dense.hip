// Dense block of top-priority vertices counted with int8 MFMA.
//
// S_U = the KU highest-priority upper vertices (ranks [nU-KU, nU)), S_L the
// KL highest lower ones.  A[i][j] = 1 when upper nU-KU+i and lower nL-KL+j
// are adjacent; P[i][j] = [p(lower j) < p(upper i)] = [deg_L <= deg_U].
// For starts u, w in S_U with w below u, the wedges through middles in S_L
// number
//     CU[i][i'] = sum_j (A[i][j] P[i][j]) A[i'][j]          (i' < i)
// and for starts v, x in S_L, through middles in S_U,
//     CL[j][j'] = sum_i (A[i][j] (1 - P[i][j])) A[i][j']    (j' < j).
// These are int8 0/1 Gram products with int32 accumulation (exact: every
// sum is at most min(KU, KL) < 2^31).  The heavy kernel seeds each S start's
// counters for ends in S with its row of CU / CL and skips exactly the
// wedges whose start, middle and end all lie in S; every butterfly is still
// counted once from its top-priority vertex (Theorem 1's argument applies to
// any split of the wedges of one start).
//
// Layout: four row-major int8 matrices padded to multiples of 32 with zeros,
// each row holding the contraction index contiguously:
//   XU = A o P       [PU][PL]   YU = A      [PU][PL]   ->  CU = XU YU^T  [PU][PU]
//   XL = (A o !P)^T  [PL][PU]   YL = A^T    [PL][PU]   ->  CL = XL YL^T  [PL][PL]
// One wavefront computes a 32x32 tile of C with v_mfma_i32_32x32x32_i8:
// lane l feeds row (l mod 32) of the X tile and row (l mod 32) of the Y tile
// (= column of Y^T), 16 contraction bytes each, the same 16 bytes of the
// contraction index for both operands, so the pairing of A- and B-operand
// bytes is the same whatever the hardware's order inside a lane.  Only tiles
// on or below the diagonal are computed.
#include "device.hpp"
#include "internal.hpp"

namespace bfc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__global__ void dense_pack_kernel(const int32_t* __restrict__ offU, const int32_t* __restrict__ adjU,
                                  const int32_t* __restrict__ offL, int32_t nU, int32_t nL, int32_t KU, int32_t KL,
                                  int32_t PU, int32_t PL, int8_t* __restrict__ XU, int8_t* __restrict__ YU,
                                  int8_t* __restrict__ XL, int8_t* __restrict__ YL) {
  const int32_t topU = nU - KU, topL = nL - KL;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < KU; i += gridDim.x * blockDim.x) {
    const int32_t r = topU + i;
    const int32_t b = offU[r], e = offU[r + 1];
    const int32_t degu = e - b;
    // first neighbour in the top lower block (lists ascend)
    int32_t lo = b, hi = e;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (adjU[mid] < topL) lo = mid + 1; else hi = mid;
    }
    for (int32_t k = lo; k < e; ++k) {
      const int32_t v = adjU[k];
      const int32_t j = v - topL;
      const bool below = (offL[v + 1] - offL[v]) <= degu;  // p(v) < p(u)
      YU[(int64_t)i * PL + j] = 1;
      YL[(int64_t)j * PU + i] = 1;
      if (below) XU[(int64_t)i * PL + j] = 1;
      else XL[(int64_t)j * PU + i] = 1;
    }
  }
}

// C[row][col] for tiles with tile_row >= tile_col; C is [P][P] int32, X and Y
// are [P][Kd] int8 (Kd multiple of 32).
__global__ __launch_bounds__(256) void dense_gram_kernel(const int8_t* __restrict__ X, const int8_t* __restrict__ Y,
                                                         int32_t P, int32_t Kd, int32_t* __restrict__ C) {
  const int lane = __lane_id();
  const int64_t tiles_1d = P / 32;
  const int64_t ntiles = tiles_1d * (tiles_1d + 1) / 2;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    // t -> (ti, tj) with tj <= ti, row-major over the lower triangle
    int64_t ti = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > t) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    const int64_t tj = t - ti * (ti + 1) / 2;
    const int r = lane & 31;
    const int h = lane >> 5;
    const int8_t* xrow = X + (ti * 32 + r) * (int64_t)Kd + 16 * h;
    const int8_t* yrow = Y + (tj * 32 + r) * (int64_t)Kd + 16 * h;
    v16i acc = {};
    for (int32_t k = 0; k < Kd; k += 32) {
      const v4i a = *reinterpret_cast<const v4i*>(xrow + k);
      const v4i b = *reinterpret_cast<const v4i*>(yrow + k);
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t row = ti * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
      const int64_t col = tj * 32 + (lane & 31);
      C[row * P + col] = acc[q];
    }
  }
}

int32_t pad32(int32_t x) { return (x + 31) / 32 * 32; }

}  // namespace

void prepare_dense(bfc_graph_s* g, hipStream_t s) {
  DenseBlock& d = g->dense;
  const int32_t K = g->tune.dense_block;
  d.KU = K > 0 ? (K < g->n_upper ? K : g->n_upper) : 0;
  d.KL = K > 0 ? (K < g->n_lower ? K : g->n_lower) : 0;
  if (d.KU <= 0 || d.KL <= 0) {
    d.KU = d.KL = 0;
    return;
  }
  d.PU = pad32(d.KU);
  d.PL = pad32(d.KL);
  const size_t bx = (size_t)d.PU * (size_t)d.PL;
  const size_t need = 4 * bx + sizeof(int32_t) * ((size_t)d.PU * d.PU + (size_t)d.PL * d.PL);
  if (d.buf.bytes < need) d.buf.alloc(need, s);
}

void dense_block(bfc_graph_s* g, hipStream_t s) {
  DenseBlock& d = g->dense;
  if (d.KU <= 0) return;
  const size_t bx = (size_t)d.PU * (size_t)d.PL;
  int8_t* XU = d.buf.as<int8_t>();
  int8_t* YU = XU + bx;
  int8_t* XL = YU + bx;
  int8_t* YL = XL + bx;
  zero_u64(XU, (int64_t)(4 * bx / 8), s);
  dense_pack_kernel<<<grid_for(d.KU, 256), 256, 0, s>>>(
      g->side[0].off.as<int32_t>(), g->side[0].adj.as<int32_t>(), g->side[1].off.as<int32_t>(), g->n_upper,
      g->n_lower, d.KU, d.KL, d.PU, d.PL, XU, YU, XL, YL);
  BFC_LAUNCH_CHECK();
  const int64_t tu = (int64_t)(d.PU / 32) * (d.PU / 32 + 1) / 2;
  const int64_t tl = (int64_t)(d.PL / 32) * (d.PL / 32 + 1) / 2;
  dense_gram_kernel<<<grid_for(tu, 4), 256, 0, s>>>(XU, YU, d.PU, d.PL, d.CU());
  BFC_LAUNCH_CHECK();
  dense_gram_kernel<<<grid_for(tl, 4), 256, 0, s>>>(XL, YL, d.PL, d.PU, d.CL());
  BFC_LAUNCH_CHECK();
}

}  // namespace bfc
