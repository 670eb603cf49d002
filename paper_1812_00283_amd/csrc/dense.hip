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
// bytes is the same whatever the hardware's order inside a lane.  Only
// blocks on or below the diagonal are computed.
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

// C = X Y^T on the blocks on or below the diagonal of a grid of
// kGB x kGB blocks; C is [P][P] int32, X and Y are [P][Kd] int8 (P and Kd
// multiples of 32).  A workgroup of eight wavefronts owns one block: per
// stage it copies a kGB x kGK slab of X and of Y into LDS (rows padded to
// kLdsRow bytes against bank conflicts; the next stage's slabs are loaded
// into registers while the current one is multiplied), and each wavefront
// multiplies a 64 x 128 part as 2 x 4 tiles of 32 x 32 with the fragment
// layout described above.  Each stage reads 2 kGB kGK bytes for 2 kGB^2 kGK
// operations (kGB operations per byte).  Workgroups are dispatched to the
// eight XCDs in turn; block indices are renumbered so that each XCD works
// through a contiguous run of the triangle, whose blocks share X panels in
// that XCD's L2.  Entries above the diagonal inside a diagonal block are
// written too (they are products like the others).
constexpr int kGB = 256;                 // block rows and columns
constexpr int kGK = 64;                  // contraction bytes per stage
constexpr int kLdsRow = kGK + 16;        // padded LDS row
constexpr int kGNT = 512;
constexpr int kChunks = kGB * kGK / 16 / kGNT;  // 16-byte loads per thread per operand and stage
constexpr int kXcds = 8;

__global__ __launch_bounds__(kGNT) void dense_gram_kernel(const int8_t* __restrict__ X, const int8_t* __restrict__ Y,
                                                          int32_t P, int32_t Kd, int32_t* __restrict__ C) {
  __shared__ __attribute__((aligned(16))) int8_t xs[2][kGB * kLdsRow];
  __shared__ __attribute__((aligned(16))) int8_t ys[2][kGB * kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;  // rows wm * 64, columns wn * 128 of the block
  // XCD-contiguous renumbering: dispatch index b runs on XCD b mod 8
  const int64_t nblk = gridDim.x, b = blockIdx.x;
  const int64_t per = nblk / kXcds, rem = nblk % kXcds, x = b % kXcds;
  const int64_t t = x * per + (x < rem ? x : rem) + b / kXcds;
  // block index -> (bi, bj), bj <= bi, row-major over the lower triangle
  int64_t bi = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (bi * (bi + 1) / 2 > t) --bi;
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  const int64_t bj = t - bi * (bi + 1) / 2;
  const int64_t row0 = bi * kGB, col0 = bj * kGB;

  v4i rx[kChunks], ry[kChunks];
  auto load = [&](int32_t k0) {
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
      const int c = tid + kGNT * i;
      const int r = c / (kGK / 16), o = (c % (kGK / 16)) * 16;
      const bool kin = k0 + o < Kd;
      const int64_t xr = row0 + r, yr = col0 + r;
      rx[i] = (kin && xr < P) ? *reinterpret_cast<const v4i*>(X + xr * Kd + k0 + o) : v4i{0, 0, 0, 0};
      ry[i] = (kin && yr < P) ? *reinterpret_cast<const v4i*>(Y + yr * Kd + k0 + o) : v4i{0, 0, 0, 0};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
      const int c = tid + kGNT * i;
      const int r = c / (kGK / 16), o = (c % (kGK / 16)) * 16;
      *reinterpret_cast<v4i*>(&xs[buf][r * kLdsRow + o]) = rx[i];
      *reinterpret_cast<v4i*>(&ys[buf][r * kLdsRow + o]) = ry[i];
    }
  };
  v16i acc[2][4] = {};
  const int r32 = lane & 31, h = lane >> 5;
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int32_t k0 = 0; k0 < Kd; k0 += kGK) {
    const bool more = k0 + kGK < Kd;
    if (more) load(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 32) {
      v4i a[2], bb[4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const v4i*>(&xs[buf][(wm * 64 + i * 32 + r32) * kLdsRow + kk + 16 * h]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bb[j] = *reinterpret_cast<const v4i*>(&ys[buf][(wn * 128 + j * 32 + r32) * kLdsRow + kk + 16 * h]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t row = row0 + wm * 64 + i * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
        const int64_t col = col0 + wn * 128 + j * 32 + r32;
        if (row < P && col < P) C[row * P + col] = acc[i][j][q];
      }
}

int32_t pad32(int32_t x) { return (x + 31) / 32 * 32; }

}  // namespace

void prepare_dense(bfc_graph_s* g, hipStream_t s) {
  DenseBlock& d = g->dense;
  // the block seeds the windows of Algorithm 2's starts over whole layers only
  const int32_t K = (g->tune.vpp || g->sched.band) ? 0 : g->tune.dense_block;
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
  const int64_t bu = (d.PU + kGB - 1) / kGB, bl = (d.PL + kGB - 1) / kGB;
  dense_gram_kernel<<<(unsigned)(bu * (bu + 1) / 2), kGNT, 0, s>>>(XU, YU, d.PU, d.PL, d.CU());
  BFC_LAUNCH_CHECK();
  dense_gram_kernel<<<(unsigned)(bl * (bl + 1) / 2), kGNT, 0, s>>>(XL, YL, d.PL, d.PU, d.CL());
  BFC_LAUNCH_CHECK();
}

}  // namespace bfc
