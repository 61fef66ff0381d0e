// gfx950 (CDNA4) kernels for multiplicative-update Euclidean NMF.
//
// The two V-streaming products of one iteration of Algorithm 1 (NNMF),
// V H^T (W update numerator) and W^T V (H update numerator), run on the
// matrix cores (v_mfma_f32_16x16x4_f32, or v_mfma_f32_16x16x32_bf16 in the
// BF16 tier) with operands staged through LDS and split along the long
// reduction dimension into partial tiles that are summed in a fixed order
// by the update kernels (no floating-point atomics anywhere).
//
// MFMA lane layout (16x16 output blocks, 64 lanes, c = lane % 16,
// g = lane / 16):  operand A supplies row i = c at reduction slot g (f32) or
// slots 8g..8g+7 (bf16); operand B supplies column j = c at the same slots;
// result register v of a lane holds D[4g + v][c].
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>


#include "nmf_device.h"
#include "nmf_internal.h"

namespace nmfk {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));  // a 32 x 32 MFMA accumulator

// 4 consecutive floats of row `row`, columns col..col+3, zero outside
// [0, rows) x [0, cols).  The vector path needs ld % 4 == 0 and a 16-byte
// aligned base, which every caller guarantees.
__device__ __forceinline__ float4 load4(const float* __restrict__ p, int64_t ld,
                                        int64_t row, int64_t rows, int64_t col,
                                        int64_t cols) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= rows) return v;
  const float* q = p + row * ld + col;
  if (col + 3 < cols) return *reinterpret_cast<const float4*>(q);
  if (col + 0 < cols) v.x = q[0];
  if (col + 1 < cols) v.y = q[1];
  if (col + 2 < cols) v.z = q[2];
  return v;
}

// 8 consecutive bf16 (as a uint4), zero outside [0, rows) x [0, cols);
// vector path needs ld % 8 == 0 and a 16-byte aligned base.
__device__ __forceinline__ uint4 load8h(const uint16_t* __restrict__ p,
                                        int64_t ld, int64_t row, int64_t rows,
                                        int64_t col, int64_t cols) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row >= rows) return v;
  const uint16_t* q = p + row * ld + col;
  if (col + 7 < cols) return *reinterpret_cast<const uint4*>(q);
  uint16_t h[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = (col + e < cols) ? q[e] : (uint16_t)0;
  v.x = h[0] | ((uint32_t)h[1] << 16);
  v.y = h[2] | ((uint32_t)h[3] << 16);
  v.z = h[4] | ((uint32_t)h[5] << 16);
  v.w = h[6] | ((uint32_t)h[7] << 16);
  return v;
}

// ---------------------------------------------------------------------------
// Distributed Gram reduction carried by a product kernel: G[e] = sum_q
// part[q][e] over the `count` per-workgroup Gram partials written by the
// previous update kernel, in one of two fixed orders (chosen by the host
// per padded rank, so every kernel that carries a given Gram gives the same
// bits; neither depends on the product's grid or workgroup size):
//  - wide: workgroups take chunks of 32 consecutive elements round-robin,
//    so every load instruction of a wave reads whole 128-byte lines.  The
//    partial range is cut into kGramSlots fixed slots; slot k of element e
//    is summed by one thread in ascending q (32 loads in flight), and the
//    slot sums are added in slot order through LDS;
//  - otherwise (small Grams, too few chunks to spread): workgroups take
//    elements round-robin; 32 lanes share an element, each summing partials
//    q = lane, lane + 32, ... in order, then a fixed xor butterfly combines
//    the 32 lane sums (commutative at each level, so every lane holds the
//    same bits).
// ---------------------------------------------------------------------------
constexpr int kGramSlots = 8;
__device__ __forceinline__ void gram_reduce_slice(const GramRed& g) {
  if (!g.part) return;
  __shared__ float slot_sum[kGramSlots][32];
  const int64_t nwg = (int64_t)gridDim.x * gridDim.y * gridDim.z;
  const int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int groups = (int)(blockDim.x >> 5), grp = threadIdx.x >> 5, l32 = threadIdx.x & 31;
  if (g.wide) {
    const int per = (g.count + kGramSlots - 1) / kGramSlots;
    for (int64_t e0 = b * 32; e0 < g.elems; e0 += nwg * 32) {
      const int64_t e = e0 + l32;
      for (int k = grp; k < kGramSlots; k += groups) {
        const int q0 = k * per, q1 = q0 + per < g.count ? q0 + per : g.count;
        float s = 0.f;
        for (int q = q0; q < q1; q += 32) {
          float v[32];
#pragma unroll
          for (int u = 0; u < 32; ++u)
            v[u] = (e < g.elems && q + u < q1) ? g.part[(int64_t)(q + u) * g.elems + e] : 0.f;
#pragma unroll
          for (int u = 0; u < 32; ++u) s += v[u];
        }
        slot_sum[k][l32] = s;
      }
      lds_barrier();
      if (grp == 0 && e < g.elems) {
        float t = slot_sum[0][l32];
#pragma unroll
        for (int k = 1; k < kGramSlots; ++k) t += slot_sum[k][l32];
        g.G[e] = t;
      }
      lds_barrier();  // slot_sum is reused by the next chunk
    }
    return;
  }
  for (int64_t e0 = b * groups; e0 < g.elems; e0 += nwg * groups) {
    const int64_t e = e0 + grp;
    float s = 0.f;
    if (e < g.elems) {
      int q = l32;
      // 16 loads in flight (one round trip for up to 512 partials), added
      // in ascending q
      for (; q < g.count; q += 16 * 32) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          v[u] = (q + 32 * u < g.count) ? g.part[(int64_t)(q + 32 * u) * g.elems + e] : 0.f;
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
      }
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
    if (e < g.elems && l32 == 0) g.G[e] = s;
  }
}

// ---------------------------------------------------------------------------
// NT product, FP32:  part[s][m][c] = sum_{k in split s} X[m][k] * Y[c][k].
// Workgroup tile BM x BN, BK reduction slots per LDS stage, WM x WN
// waves each owning (16 MB) x (16 NB) outputs.  Each lane reads 4
// consecutive k of a row with one 128-bit LDS load and feeds them to four
// MFMAs (slot g of MFMA t is k = 4g + t), so A and B see the same k order.
// Grid: x = N tiles, y = M tiles, z = splits.
// ---------------------------------------------------------------------------
template <int MB, int NB, int WM, int WN, int BK>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt(
    const float* __restrict__ X, int64_t ldx, int64_t M,
    const float* __restrict__ Y, int64_t ldy, int64_t N, int64_t K,
    int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp, GramRed gr) {
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN, PITCH = BK + 4;
  constexpr int T = 64 * WM * WN;
  constexpr int XQ = BM * (BK / 4), YQ = BN * (BK / 4);
  constexpr int XL = (XQ + T - 1) / T, YL = (YQ + T - 1) / T;
  __shared__ __attribute__((aligned(16))) float Xs[BM * PITCH];
  __shared__ __attribute__((aligned(16))) float Ys[BN * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int c = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (K < kb + kchunk) ? K : kb + kchunk;
  gram_reduce_slice(gr);

  v4f acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  float4 xr[XL], yr[YL];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int idx = tid + q * T;
      if (XQ % T == 0 || idx < XQ)
        xr[q] = load4(X, ldx, m0 + idx / (BK / 4), M, k0 + 4 * (idx % (BK / 4)), ke);
    }
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      const int idx = tid + q * T;
      if (YQ % T == 0 || idx < YQ)
        yr[q] = load4(Y, ldy, n0 + idx / (BK / 4), N, k0 + 4 * (idx % (BK / 4)), ke);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int idx = tid + q * T;
      if (XQ % T == 0 || idx < XQ)
        *reinterpret_cast<float4*>(&Xs[(idx / (BK / 4)) * PITCH + 4 * (idx % (BK / 4))]) = xr[q];
    }
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      const int idx = tid + q * T;
      if (YQ % T == 0 || idx < YQ)
        *reinterpret_cast<float4*>(&Ys[(idx / (BK / 4)) * PITCH + 4 * (idx % (BK / 4))]) = yr[q];
    }
  };

  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    lstore();
    __syncthreads();
    if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      v4f a[MB], b[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i)
        a[i] = *reinterpret_cast<const v4f*>(&Xs[(wm * 16 * MB + 16 * i + c) * PITCH + kk + 4 * g]);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        b[j] = *reinterpret_cast<const v4f*>(&Ys[(wn * 16 * NB + 16 * j + c) * PITCH + kk + 4 * g]);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = mfma_f32(a[i][t], b[j][t], acc[i][j]);
    }
    __syncthreads();
  }

  float* P = part + (int64_t)blockIdx.z * sp;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 16 * MB + 16 * i + 4 * g + v;
        const int64_t col = n0 + wn * 16 * NB + 16 * j + c;
        P[row * ldp + col] = acc[i][j][v];
      }
}

// ---------------------------------------------------------------------------
// NT product, BF16 operands (RNE copies), FP32 accumulation, 16x16x32 MFMA.
// BK bf16 per stage (a multiple of 32); a lane reads 8 consecutive k (one
// 128-bit LDS load) per operand per MFMA.
// ---------------------------------------------------------------------------
template <int MB, int NB, int WM, int WN, int BK>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt_bf16(
    const uint16_t* __restrict__ X, int64_t ldx, int64_t M,
    const uint16_t* __restrict__ Y, int64_t ldy, int64_t N, int64_t K,
    int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp, GramRed gr) {
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN, PITCH = BK + 8;
  constexpr int T = 64 * WM * WN;
  constexpr int XQ = BM * (BK / 8), YQ = BN * (BK / 8);
  constexpr int XL = (XQ + T - 1) / T, YL = (YQ + T - 1) / T;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[BM * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Ys[BN * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int c = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (K < kb + kchunk) ? K : kb + kchunk;
  gram_reduce_slice(gr);

  v4f acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  uint4 xr[XL], yr[YL];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int idx = tid + q * T;
      if (XQ % T == 0 || idx < XQ)
        xr[q] = load8h(X, ldx, m0 + idx / (BK / 8), M, k0 + 8 * (idx % (BK / 8)), ke);
    }
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      const int idx = tid + q * T;
      if (YQ % T == 0 || idx < YQ)
        yr[q] = load8h(Y, ldy, n0 + idx / (BK / 8), N, k0 + 8 * (idx % (BK / 8)), ke);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int idx = tid + q * T;
      if (XQ % T == 0 || idx < XQ)
        *reinterpret_cast<uint4*>(&Xs[(idx / (BK / 8)) * PITCH + 8 * (idx % (BK / 8))]) = xr[q];
    }
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      const int idx = tid + q * T;
      if (YQ % T == 0 || idx < YQ)
        *reinterpret_cast<uint4*>(&Ys[(idx / (BK / 8)) * PITCH + 8 * (idx % (BK / 8))]) = yr[q];
    }
  };

  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    lstore();
    __syncthreads();
    if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      v8bf a[MB], b[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i)
        a[i] = *reinterpret_cast<const v8bf*>(&Xs[(wm * 16 * MB + 16 * i + c) * PITCH + kk + 8 * g]);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        b[j] = *reinterpret_cast<const v8bf*>(&Ys[(wn * 16 * NB + 16 * j + c) * PITCH + kk + 8 * g]);
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

  float* P = part + (int64_t)blockIdx.z * sp;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 16 * MB + 16 * i + 4 * g + v;
        const int64_t col = n0 + wn * 16 * NB + 16 * j + c;
        P[row * ldp + col] = acc[i][j][v];
      }
}

// ---------------------------------------------------------------------------
// TN product, FP32:  part[s][m][c] = sum_{k in split s} A[k][m] * B[k][c].
// Both operands are read as rows (k) of contiguous floats, which is how
// V (p x n) and W (p x r) are stored for the H update numerator W^T V.
// A wave owns (16 MB) x 64 outputs.  Block a of the wave covers the rows
// m = base + MB*i + a and block b the columns base + 4*j + b, so one lane
// fetches the A values of all MB blocks (and the B values of all 4 blocks)
// with a single vector LDS load, and stores 4 adjacent columns at once.
// ---------------------------------------------------------------------------
template <int MB>
struct VecT;
template <>
struct VecT<1> {
  typedef float type;
};
template <>
struct VecT<2> {
  typedef v2f type;
};
template <>
struct VecT<4> {
  typedef v4f type;
};
template <int MB>
__device__ __forceinline__ float vget(const typename VecT<MB>::type& v, int i);
template <>
__device__ __forceinline__ float vget<1>(const float& v, int) {
  return v;
}
template <>
__device__ __forceinline__ float vget<2>(const v2f& v, int i) {
  return v[i];
}
template <>
__device__ __forceinline__ float vget<4>(const v4f& v, int i) {
  return v[i];
}

template <int MB, int WM, int WN, int BK>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_tn(
    const float* __restrict__ A, int64_t lda, int64_t M,
    const float* __restrict__ B, int64_t ldb, int64_t N, int64_t K,
    int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp, GramRed gr) {
  constexpr int NB = 4;
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN;
  constexpr int PA = BM + 4, PB = BN + 4;
  constexpr int T = 64 * WM * WN;
  constexpr int AQ = BK * (BM / 4), BQ = BK * (BN / 4);
  constexpr int AL = (AQ + T - 1) / T, BL = (BQ + T - 1) / T;
  __shared__ __attribute__((aligned(16))) float As[BK * PA];
  __shared__ __attribute__((aligned(16))) float Bs[BK * PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int c = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (K < kb + kchunk) ? K : kb + kchunk;
  gram_reduce_slice(gr);

  v4f acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  float4 ar[AL], br[BL];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < AL; ++q) {
      const int idx = tid + q * T;
      if (AQ % T == 0 || idx < AQ)
        ar[q] = load4(A, lda, k0 + idx / (BM / 4), ke, m0 + 4 * (idx % (BM / 4)), M);
    }
#pragma unroll
    for (int q = 0; q < BL; ++q) {
      const int idx = tid + q * T;
      if (BQ % T == 0 || idx < BQ)
        br[q] = load4(B, ldb, k0 + idx / (BN / 4), ke, n0 + 4 * (idx % (BN / 4)), N);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int q = 0; q < AL; ++q) {
      const int idx = tid + q * T;
      if (AQ % T == 0 || idx < AQ)
        *reinterpret_cast<float4*>(&As[(idx / (BM / 4)) * PA + 4 * (idx % (BM / 4))]) = ar[q];
    }
#pragma unroll
    for (int q = 0; q < BL; ++q) {
      const int idx = tid + q * T;
      if (BQ % T == 0 || idx < BQ)
        *reinterpret_cast<float4*>(&Bs[(idx / (BN / 4)) * PB + 4 * (idx % (BN / 4))]) = br[q];
    }
  };

  typedef typename VecT<MB>::type AV;
  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    lstore();
    __syncthreads();
    if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
    for (int t = 0; t < BK / 4; ++t) {
      const int k = 4 * t + g;
      const AV a = *reinterpret_cast<const AV*>(&As[k * PA + wm * 16 * MB + MB * c]);
      const v4f b = *reinterpret_cast<const v4f*>(&Bs[k * PB + wn * 64 + 4 * c]);
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = mfma_f32(vget<MB>(a, i), b[j], acc[i][j]);
    }
    __syncthreads();
  }

  float* P = part + (int64_t)blockIdx.z * sp;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t m = m0 + wm * 16 * MB + MB * (4 * g + v) + i;
      const int64_t col = n0 + wn * 64 + 4 * c;
      *reinterpret_cast<float4*>(&P[m * ldp + col]) =
          make_float4(acc[i][0][v], acc[i][1][v], acc[i][2][v], acc[i][3][v]);
    }
}

// ---------------------------------------------------------------------------
// V-streaming product through an asynchronous LDS ring:
//   part[s][m][c] = sum_{k in split s} X[m][k] * Y[c][k]
// with X and Y contiguous along k and padded with zeros so that every tile
// is in bounds (rows to a multiple of the tile, k to a multiple of 256).
// A stage is BM + BN rows of 128 bytes (32 floats or 64 bf16 of k).  It is
// copied global -> LDS by global_load_lds_dwordx4 (the data never passes
// through registers) and S stages are in flight at once, so the load
// latency is covered by S - 1 stages of MFMA work.  Inside a row, 16-byte
// chunk q is stored at slot q ^ (row % 8): the 16 lanes of an MFMA fragment
// (rows c = 0..15, same chunk) then hit distinct LDS banks.
// SH = 16, FP32: a chunk is 4 k-values, fed to 4 v_mfma_f32_16x16x4_f32
// (slot g of MFMA t is k = 16 kk + 4 g + t).  BF16: a chunk is the 8
// k-values a lane supplies to one v_mfma_f32_16x16x32_bf16.
// SH = 32 (the 32 x 32 matrix-core shapes, which sustain more flops on this
// chip: v_mfma_f32_32x32x2f32 and v_mfma_f32_32x32x16_bf16): a wave owns
// (32 MB) x (32 NB) outputs; lane (c, h) = (lane % 32, lane / 32) reads
// chunk 2 j + h of row c for k-group j of the stage, so in FP32 slot h of
// MFMA t of group j is k = 8 j + 4 h + t, and in BF16 the lane supplies the
// chunk's 8 k to one MFMA.  The accumulator of a 32 x 32 block holds
// D[8 (v / 4) + 4 h + v % 4][c] in element v (an in-bounds layout probe on
// the GPU confirmed it for both shapes).  MB and NB count 16- or 32-blocks.
// ---------------------------------------------------------------------------
template <int MB, int NB, int WM, int WN, int S, bool BF, int SH>
__global__ __launch_bounds__(64 * WM * WN) void k_nt_dma(
    const void* __restrict__ Xv, int64_t ldx, const void* __restrict__ Yv, int64_t ldy,
    int64_t K, int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp, GramRed gr) {
  static_assert(SH == 16 || SH == 32, "MFMA shape");
  constexpr int ES = BF ? 2 : 4;
  constexpr int BKE = 128 / ES;
  constexpr int BM = SH * MB * WM, BN = SH * NB * WN, ROWS = BM + BN;
  constexpr int W = WM * WN;
  static_assert(ROWS % (8 * W) == 0, "stage rows must split evenly over the waves");
  constexpr int L = ROWS / (8 * W);  // DMA instructions per wave per stage
  constexpr int STAGE = ROWS * 128;  // bytes
  __shared__ __attribute__((aligned(1024))) char lds[S * STAGE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int c = lane & 15, g = lane >> 4;
  // grid: x = split (fastest, so the workgroups sharing a k-chunk of the
  // small operand are dispatched together and land on the same XCD and
  // its L2), y = M tile, z = N tile
  const int64_t n0 = (int64_t)blockIdx.z * BN;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t kb = (int64_t)blockIdx.x * kchunk;
  const int64_t ke = (K < kb + kchunk) ? K : kb + kchunk;
  const int nst = (int)((ke - kb) / BKE);

  // source of this lane in each of the wave's L copy instructions: row
  // rr = 8 (wave L + j) + lane / 8 of the stage, slot lane % 8, which holds
  // chunk (lane % 8) ^ (rr % 8) = (lane % 8) ^ (lane / 8)
  const char* X = static_cast<const char*>(Xv);
  const char* Y = static_cast<const char*>(Yv);
  const int chunk = (lane & 7) ^ (lane >> 3);
  const char* src[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int rr = 8 * (wave * L + j) + (lane >> 3);
    src[j] = rr < BM ? X + ((m0 + rr) * ldx + kb) * ES + 16 * chunk
                     : Y + ((n0 + rr - BM) * ldy + kb) * ES + 16 * chunk;
  }
  auto issue = [&](int st) {
    char* dst = lds + (st % S) * STAGE;
#pragma unroll
    for (int j = 0; j < L; ++j)
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(src[j] + (int64_t)st * 128),
                                       (lds_ptr_t)(dst + (wave * L + j) * 1024), 16, 0, 0);
  };

  // accumulator of one SH x SH block
  using acc_t = typename std::conditional<SH == 32, v16f, v4f>::type;
  constexpr int AE = SH * SH / 64;  // accumulator elements per lane and block
  acc_t acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int e = 0; e < AE; ++e) acc[i][j][e] = 0.f;

  // A stage holds KG k-groups of 16-byte fragments per row (SH = 16: two
  // halves kk, lane group g reading chunk 4 kk + g; SH = 32: four groups j,
  // lane half h reading chunk 2 j + h).  All fragment reads of a stage are
  // issued first, then the stage's copies for later, then the MFMAs: the
  // later groups' reads and the copy instructions complete under the first
  // group's MFMAs, so a wave stalls on LDS once per stage, not per group.
  using frag_t = typename std::conditional<BF, v8bf, v4f>::type;
  constexpr int KG = SH == 32 ? 4 : 2;
  const int fr = SH == 32 ? (lane & 31) : c;            // fragment row of this lane
  const int fq = SH == 32 ? (lane >> 5) : g;            // chunk within a k-group
  frag_t fa[KG][MB], fb[KG][NB];
  auto read_frags = [&](const char* buf) {
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const int off = 16 * (((8 / KG) * kk + fq) ^ (fr & 7));
#pragma unroll
      for (int i = 0; i < MB; ++i)
        fa[kk][i] = *reinterpret_cast<const frag_t*>(buf + (wm * SH * MB + SH * i + fr) * 128 + off);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        fb[kk][j] =
            *reinterpret_cast<const frag_t*>(buf + (BM + wn * SH * NB + SH * j + fr) * 128 + off);
    }
  };
  auto mfmas = [&]() {
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      if constexpr (BF) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            if constexpr (SH == 32)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[kk][i], fb[kk][j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = mfma_bf16(fa[kk][i], fb[kk][j], acc[i][j]);
          }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              if constexpr (SH == 32)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[kk][i][t], fb[kk][j][t], acc[i][j], 0, 0, 0);
              else
                acc[i][j] = mfma_f32(fa[kk][i][t], fb[kk][j][t], acc[i][j]);
            }
      }
    }
  };

  // Stage st lives in buffer st % S.  At the top of iteration st, stages
  // st .. st + S - 2 have been issued; once this wave's copies of stage st
  // have landed, one barrier certifies both that every wave's copies of
  // stage st are in LDS and that every wave has finished reading stage
  // st - 1, whose buffer is then refilled with stage st + S - 1.
  const int pre = nst < S - 1 ? nst : S - 1;
  for (int st = 0; st < pre; ++st) issue(st);
  // Gram of the previous update, reduced by this kernel so the next one can
  // use it: here, under the latency of the first copies (its loads and
  // stores only make the ring's vmcnt waits below stricter), or with at_end
  // after the loop, where it delays no stage (the default: measured faster).
  if (!gr.at_end) gram_reduce_slice(gr);
  for (int st = 0; st < nst; ++st) {
    const int later = nst - 1 - st;
    wait_stage<L, S>(later < S - 2 ? later : S - 2);
    lds_barrier();
    read_frags(lds + (st % S) * STAGE);
    if (st + S - 1 < nst) issue(st + S - 1);
    mfmas();
  }

  if (gr.at_end) gram_reduce_slice(gr);
  float* P = part + (int64_t)blockIdx.x * sp;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < AE; ++v) {
        const int rr = SH == 32 ? 8 * (v / 4) + 4 * fq + (v % 4) : 4 * g + v;
        const int64_t row = m0 + wm * SH * MB + SH * i + rr;
        const int64_t col = n0 + wn * SH * NB + SH * j + fr;
        P[row * ldp + col] = acc[i][j][v];
      }
}

// ---------------------------------------------------------------------------
// Split-K sums.  The partial tiles are summed in ascending split order; the
// loads of 8 splits are issued together before the (ordered) adds so the
// loop is not a chain of dependent memory round trips.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 sum_splits4(const float* __restrict__ part, int64_t off,
                                              int64_t sp, int splits) {
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  int q = 0;
  for (; q + 8 <= splits; q += 8) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const float4*>(part + (q + u) * sp + off);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s.x += v[u].x; s.y += v[u].y; s.z += v[u].z; s.w += v[u].w;
    }
  }
  for (; q < splits; ++q) {
    const float4 v = *reinterpret_cast<const float4*>(part + q * sp + off);
    s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
  }
  return s;
}

__device__ __forceinline__ void add4(float4& s, const float4& v) {
  s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
}
__device__ __forceinline__ void add4(float& s, float v) { s += v; }

// Split-K sums of NI items at once (each a float4 or a float at part + off,
// split pitch sp), every item summed in ascending split order.  The loads
// of B splits of all NI items are issued before any of them is added, so a
// tile's items cost one memory round trip per B splits.
template <int NI, int B, typename T>
__device__ __forceinline__ void sum_splits_batch(const float* __restrict__ part,
                                                 const int64_t (&off)[NI], const bool (&ok)[NI],
                                                 int64_t sp, int splits, T (&s)[NI]) {
#pragma unroll
  for (int e = 0; e < NI; ++e) s[e] = T{};
  for (int q = 0; q < splits; q += B) {
    T v[NI][B];
#pragma unroll
    for (int e = 0; e < NI; ++e)
#pragma unroll
      for (int u = 0; u < B; ++u) {
        v[e][u] = T{};
        if (ok[e] && q + u < splits) v[e][u] = *reinterpret_cast<const T*>(part + (q + u) * sp + off[e]);
      }
#pragma unroll
    for (int e = 0; e < NI; ++e)
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (q + u < splits) add4(s[e], v[e][u]);
  }
}

// Gram reduction: G[m][c] = sum_s part[s][m][c], s ascending; 4 columns per
// thread (rp is a multiple of 16, the partial pitch a multiple of 4).
__global__ void k_reduce_gram(const float* __restrict__ part, int64_t ldp,
                              int64_t sp, int splits, int rp,
                              float* __restrict__ G, uint16_t* __restrict__ Gbf) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rp * rp / 4) return;
  const int64_t m = idx / (rp / 4), cc = 4 * (idx % (rp / 4));
  const float4 s = sum_splits4(part, m * ldp + cc, sp, splits);
  *reinterpret_cast<float4*>(&G[m * rp + cc]) = s;
  if (Gbf) {
    Gbf[m * rp + cc + 0] = to_bf16(s.x);
    Gbf[m * rp + cc + 1] = to_bf16(s.y);
    Gbf[m * rp + cc + 2] = to_bf16(s.z);
    Gbf[m * rp + cc + 3] = to_bf16(s.w);
  }
}

// ---------------------------------------------------------------------------
// W half-step epilogue (eq. nnmf_v_update):
//   a_ik = sum_s part[s][i][k]                 (numerator (V H^T)_ik)
//   b_ik = sum_l w_il G_lk                     (denominator (W (H H^T))_ik)
//   w_ik <- w_ik * (a_ik / b_ik)  if b_ik > 0, else unchanged.
// A workgroup takes ROWS rows of W at a time (grid-stride) with all RP
// ranks; it snapshots the rows in LDS (rounded to bf16 in the BF16 tier,
// where the product takes bf16 operands) and streams G through LDS in chunks
// of KC columns.  Each thread produces KPT adjacent ranks of one row per
// chunk (ROWS * KC / KPT == 256): KPT = 4, or 1 when p is too small for the
// 4-rank blocks to number 256.  Both forms add in the same order.
// With gout != nullptr (RP <= 64) the workgroup also accumulates the Gram
// W_new^T W_new of the rows it updated (bf16-rounded in the BF16 tier) and
// writes it to gout[blockIdx.x]; the next product kernel reduces these.
// gram_only skips the update and only forms the Gram of the current W.
// ---------------------------------------------------------------------------
template <int RP, int KPT>
__global__ __launch_bounds__(256) void k_update_w(
    int64_t p, int r, const float* __restrict__ part, int64_t ldp, int64_t sp,
    int splits, const float* __restrict__ G, float* __restrict__ Wp,
    float* __restrict__ Wc, float* __restrict__ WT, uint16_t* __restrict__ WbT, int64_t ldwt,
    int bf16, float* __restrict__ gout, int gram_only) {
  constexpr int KC = RP < 64 ? RP : 64;
  constexpr int ROWS = 256 * KPT / KC;    // KPT rank entries per thread (4, or 1 for small p)
  constexpr bool FUSE = RP <= 64;         // Gram partial fits one thread tile
  constexpr int TB = RP / 16;             // Gram tile per thread: TB x TB
  constexpr int WSP = RP + 4;             // padded row pitch: the 4 rows a wave reads sit in distinct banks
  __shared__ __attribute__((aligned(16))) float Ws[ROWS * WSP];
  __shared__ __attribute__((aligned(16))) float Gs[RP * KC];
  __shared__ __attribute__((aligned(16))) float Wn[FUSE ? ROWS * RP : 4];
  const int tid = threadIdx.x;
  const int i = tid / (KC / KPT), k4 = KPT * (tid % (KC / KPT));
  const bool gram = FUSE && gout != nullptr;
  const int gk = (tid / 16) * TB, gl = (tid % 16) * TB;
  float ga[TB][TB];
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) ga[a][b] = 0.f;

  for (int64_t blk = blockIdx.x; blk * ROWS < p; blk += gridDim.x) {
    const int64_t i0 = blk * ROWS;
    const int64_t row = i0 + i;
    if (FUSE && !gram_only) {
      // All global loads of the row block are issued before the first wait:
      // the rows (one float4 per thread), this thread's split sums and, on
      // the first block, G.  KC == RP here, and for KPT == 4 the float4 a
      // thread loads is the one it updates.
      constexpr int NQ = ROWS * RP / 4;
      constexpr int NG = (RP * RP / 4 + 255) / 256;
      const bool tq = NQ % 256 == 0 || tid < NQ;
      const int ti = tid / (RP / 4), tl4 = 4 * (tid % (RP / 4));
      const bool first = blk == blockIdx.x;
      float4 wt = make_float4(0.f, 0.f, 0.f, 0.f);
      if (tq && i0 + ti < p) wt = *reinterpret_cast<const float4*>(&Wp[(i0 + ti) * RP + tl4]);
      float4 gq[NG];
#pragma unroll
      for (int e = 0; e < NG; ++e) {
        const int idx = tid + 256 * e;
        gq[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (first && idx < RP * RP / 4) gq[e] = *reinterpret_cast<const float4*>(&G[4 * idx]);
      }
      const int64_t off[1] = {row * ldp + k4};
      const bool ok[1] = {row < p};
      float4 a4[1];
      float a1[1];
      float w1 = 0.f;
      if constexpr (KPT == 4) {
        sum_splits_batch<1, 16>(part, off, ok, sp, splits, a4);
      } else {
        if (row < p) w1 = Wp[row * RP + k4];
        sum_splits_batch<1, 16>(part, off, ok, sp, splits, a1);
      }
      __syncthreads();
      if (tq) {
        float4 w = wt;
        if (bf16) {
          w.x = bf16_val(w.x); w.y = bf16_val(w.y); w.z = bf16_val(w.z); w.w = bf16_val(w.w);
        }
        *reinterpret_cast<float4*>(&Ws[ti * WSP + tl4]) = w;
      }
      if (first) {
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          const int idx = tid + 256 * e;
          float4 gv = gq[e];
          if (bf16) {
            gv.x = bf16_val(gv.x); gv.y = bf16_val(gv.y); gv.z = bf16_val(gv.z); gv.w = bf16_val(gv.w);
          }
          if (idx < RP * RP / 4) *reinterpret_cast<float4*>(&Gs[4 * idx]) = gv;
        }
      }
      __syncthreads();
      const int k = k4;
      if constexpr (KPT == 1) {
        float wn = 0.f;
        if (row < p) {
          float b = 0.f;
#pragma unroll 8
          for (int l = 0; l < RP; ++l) b = fmaf(Ws[i * WSP + l], Gs[l * KC + k4], b);
          wn = (b > 0.f) ? w1 * (a1[0] / b) : w1;
          Wp[row * RP + k] = wn;
          if (k < r) Wc[row * r + k] = wn;
          if (WT) WT[(int64_t)k * ldwt + row] = wn;
          if (WbT) WbT[(int64_t)k * ldwt + row] = to_bf16(wn);
        }
        Wn[i * RP + k] = bf16 ? bf16_val(wn) : wn;
      } else {
        float4 wn = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < p) {
          const float4 a = a4[0];
          float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;
#pragma unroll 8
          for (int l = 0; l < RP; ++l) {
            const float wl = Ws[i * WSP + l];
            const float4 g4 = *reinterpret_cast<const float4*>(&Gs[l * KC + k4]);
            b0 = fmaf(wl, g4.x, b0);
            b1 = fmaf(wl, g4.y, b1);
            b2 = fmaf(wl, g4.z, b2);
            b3 = fmaf(wl, g4.w, b3);
          }
          const float4 w = wt;
          wn.x = (b0 > 0.f) ? w.x * (a.x / b0) : w.x;
          wn.y = (b1 > 0.f) ? w.y * (a.y / b1) : w.y;
          wn.z = (b2 > 0.f) ? w.z * (a.z / b2) : w.z;
          wn.w = (b3 > 0.f) ? w.w * (a.w / b3) : w.w;
          *reinterpret_cast<float4*>(&Wp[row * RP + k]) = wn;
          const float wv[4] = {wn.x, wn.y, wn.z, wn.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (k + e < r) Wc[row * r + k + e] = wv[e];
            if (WT) WT[(int64_t)(k + e) * ldwt + row] = wv[e];
            if (WbT) WbT[(int64_t)(k + e) * ldwt + row] = to_bf16(wv[e]);
          }
        }
        if (bf16) {
          wn.x = bf16_val(wn.x); wn.y = bf16_val(wn.y); wn.z = bf16_val(wn.z); wn.w = bf16_val(wn.w);
        }
        *reinterpret_cast<float4*>(&Wn[i * RP + k]) = wn;
      }
    } else {
    __syncthreads();
    for (int idx = tid; idx < ROWS * RP / 4; idx += 256) {
      const int ii = idx / (RP / 4), l4 = 4 * (idx % (RP / 4));
      float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i0 + ii < p) w = *reinterpret_cast<const float4*>(&Wp[(i0 + ii) * RP + l4]);
      if (bf16) {
        w.x = bf16_val(w.x); w.y = bf16_val(w.y); w.z = bf16_val(w.z); w.w = bf16_val(w.w);
      }
      *reinterpret_cast<float4*>(&Ws[ii * WSP + l4]) = w;
      if (FUSE && gram_only) *reinterpret_cast<float4*>(&Wn[ii * RP + l4]) = w;
    }
    if (!gram_only) {
      for (int kc0 = 0; kc0 < RP; kc0 += KC) {
        if (!FUSE || kc0 > 0 || blk == blockIdx.x) {  // G chunk (once when RP <= 64)
          __syncthreads();
          for (int idx = tid; idx < RP * KC / 4; idx += 256) {
            const int l = idx / (KC / 4), kk = 4 * (idx % (KC / 4));
            float4 gv = *reinterpret_cast<const float4*>(&G[l * RP + kc0 + kk]);
            if (bf16) {
              gv.x = bf16_val(gv.x); gv.y = bf16_val(gv.y); gv.z = bf16_val(gv.z); gv.w = bf16_val(gv.w);
            }
            *reinterpret_cast<float4*>(&Gs[l * KC + kk]) = gv;
          }
        }
        __syncthreads();
        const int k = kc0 + k4;
        if constexpr (KPT == 1) {
          float wn = 0.f;
          if (row < p) {
            float a = 0.f;
            int q = 0;
            for (; q + 8 <= splits; q += 8) {
              float v[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) v[u] = part[(q + u) * sp + row * ldp + k];
#pragma unroll
              for (int u = 0; u < 8; ++u) a += v[u];
            }
            for (; q < splits; ++q) a += part[q * sp + row * ldp + k];
            float b = 0.f;
#pragma unroll 8
            for (int l = 0; l < RP; ++l) b = fmaf(Ws[i * WSP + l], Gs[l * KC + k4], b);
            const float w = Wp[row * RP + k];
            wn = (b > 0.f) ? w * (a / b) : w;
            Wp[row * RP + k] = wn;
            if (k < r) Wc[row * r + k] = wn;
            if (WT) WT[(int64_t)k * ldwt + row] = wn;
            if (WbT) WbT[(int64_t)k * ldwt + row] = to_bf16(wn);
          }
          if (FUSE) Wn[i * RP + k] = bf16 ? bf16_val(wn) : wn;
          continue;
        }
        float4 wn = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < p) {
          const float4 a = sum_splits4(part, row * ldp + k, sp, splits);
          float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;
#pragma unroll 8
          for (int l = 0; l < RP; ++l) {
            const float wl = Ws[i * WSP + l];
            const float4 g4 = *reinterpret_cast<const float4*>(&Gs[l * KC + k4]);
            b0 = fmaf(wl, g4.x, b0);
            b1 = fmaf(wl, g4.y, b1);
            b2 = fmaf(wl, g4.z, b2);
            b3 = fmaf(wl, g4.w, b3);
          }
          const float4 w = *reinterpret_cast<const float4*>(&Wp[row * RP + k]);
          wn.x = (b0 > 0.f) ? w.x * (a.x / b0) : w.x;
          wn.y = (b1 > 0.f) ? w.y * (a.y / b1) : w.y;
          wn.z = (b2 > 0.f) ? w.z * (a.z / b2) : w.z;
          wn.w = (b3 > 0.f) ? w.w * (a.w / b3) : w.w;
          *reinterpret_cast<float4*>(&Wp[row * RP + k]) = wn;
          const float wv[4] = {wn.x, wn.y, wn.z, wn.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (k + e < r) Wc[row * r + k + e] = wv[e];
            if (WT) WT[(int64_t)(k + e) * ldwt + row] = wv[e];
            if (WbT) WbT[(int64_t)(k + e) * ldwt + row] = to_bf16(wv[e]);
          }
        }
        if (FUSE) {
          if (bf16) {
            wn.x = bf16_val(wn.x); wn.y = bf16_val(wn.y); wn.z = bf16_val(wn.z); wn.w = bf16_val(wn.w);
          }
          *reinterpret_cast<float4*>(&Wn[i * RP + k]) = wn;
        }
      }
    }
    }
    if (gram) {
      __syncthreads();
#pragma unroll 4
      for (int ii = 0; ii < ROWS; ++ii) {
        float x[TB], y[TB];
#pragma unroll
        for (int a = 0; a < TB; ++a) {
          x[a] = Wn[ii * RP + gk + a];
          y[a] = Wn[ii * RP + gl + a];
        }
#pragma unroll
        for (int a = 0; a < TB; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) ga[a][b] = fmaf(x[a], y[b], ga[a][b]);
      }
    }
  }
  if (gram) {
    float* out = gout + (int64_t)blockIdx.x * RP * RP;
#pragma unroll
    for (int a = 0; a < TB; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) out[(gk + a) * RP + gl + b] = ga[a][b];
  }
}

// ---------------------------------------------------------------------------
// H half-step epilogue (eq. nnmf_w_update), with the new W:
//   s_kj = sum_s part[s][k][j]                 (numerator (W^T V)_kj)
//   d_kj = sum_l G_kl h_lj                     (denominator ((W^T W) H)_kj)
//   h_kj <- h_kj * (s_kj / d_kj)  if d_kj > 0, else unchanged.
// A workgroup takes COLS columns of H at a time (grid-stride) with all RP
// ranks: 64, or 32 / 16 when n is too small for 64-column blocks to number
// 256; each thread produces 4 adjacent columns of one rank at a time.
// With gout != nullptr (RP <= 64) it also accumulates the Gram H_new H_new^T
// of its columns into gout[blockIdx.x]; gram_only skips the update.
// ---------------------------------------------------------------------------
template <int RP, int COLS>
__global__ __launch_bounds__(256) void k_update_h(
    int64_t n, int r, const float* __restrict__ part, int64_t ldp, int64_t sp,
    int splits, const float* __restrict__ G, float* __restrict__ Hp,
    int64_t ldh, float* __restrict__ Hc, uint16_t* __restrict__ Hb, int bf16,
    float* __restrict__ gout, int gram_only) {
  constexpr int KC = RP < 64 ? RP : 64;
  constexpr bool FUSE = RP <= 64;
  constexpr int TB = RP / 16;
  __shared__ __attribute__((aligned(16))) float Hs[RP * COLS];
  __shared__ __attribute__((aligned(16))) float Gs[KC * RP];
  constexpr int HP = RP + 1;  // padded pitch: conflict-free column writes
  __shared__ float HnT[FUSE ? COLS * HP : 4];  // [j][k]
  const int tid = threadIdx.x;
  const bool gram = FUSE && gout != nullptr;
  const int gk = (tid / 16) * TB, gl = (tid % 16) * TB;
  float ga[TB][TB];
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) ga[a][b] = 0.f;

  for (int64_t blk = blockIdx.x; blk * COLS < n; blk += gridDim.x) {
    const int64_t j0 = blk * COLS;
    if (FUSE && !gram_only) {
      // All global loads of the column block are issued before the first
      // wait: the block of H (NI float4 per thread; KC == RP, so entry e of
      // a thread is also the item it updates), its split sums and, on the
      // first block, G.
      constexpr int NQ = RP * COLS / 4;
      constexpr int NI = (NQ + 255) / 256;
      constexpr int NG = (RP * RP / 4 + 255) / 256;
      constexpr int B = NI >= 4 ? 4 : 16 / NI;
      const bool first = blk == blockIdx.x;
      float4 hr[NI], sv[NI], gq[NG];
      int64_t off[NI];
      bool ok[NI];
#pragma unroll
      for (int e = 0; e < NI; ++e) {
        const int idx = tid + 256 * e;
        const int kk = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
        ok[e] = (NQ % 256 == 0 || idx < NQ) && j0 + j4 < n;
        off[e] = (int64_t)kk * ldp + j0 + j4;
        hr[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok[e]) hr[e] = *reinterpret_cast<const float4*>(&Hp[(int64_t)kk * ldh + j0 + j4]);
      }
#pragma unroll
      for (int e = 0; e < NG; ++e) {
        const int idx = tid + 256 * e;
        gq[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (first && idx < RP * RP / 4) gq[e] = *reinterpret_cast<const float4*>(&G[4 * idx]);
      }
      sum_splits_batch<NI, B>(part, off, ok, sp, splits, sv);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < NI; ++e) {
        const int idx = tid + 256 * e;
        if (NQ % 256 == 0 || idx < NQ) {
          const int kk = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
          float4 h = hr[e];
          if (bf16) {
            h.x = bf16_val(h.x); h.y = bf16_val(h.y); h.z = bf16_val(h.z); h.w = bf16_val(h.w);
          }
          *reinterpret_cast<float4*>(&Hs[kk * COLS + j4]) = h;
        }
      }
      if (first) {
        // G transposed (Gs[l][k] = G[k][l]): the items of a wave then read
        // consecutive words of one row
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          const int idx = tid + 256 * e;
          float4 gv = gq[e];
          if (bf16) {
            gv.x = bf16_val(gv.x); gv.y = bf16_val(gv.y); gv.z = bf16_val(gv.z); gv.w = bf16_val(gv.w);
          }
          if (idx < RP * RP / 4) {
            const int gk_ = (4 * idx) / RP, gl0 = (4 * idx) % RP;
            Gs[(gl0 + 0) * RP + gk_] = gv.x;
            Gs[(gl0 + 1) * RP + gk_] = gv.y;
            Gs[(gl0 + 2) * RP + gk_] = gv.z;
            Gs[(gl0 + 3) * RP + gk_] = gv.w;
          }
        }
      }
      __syncthreads();
      // denominators of all NI items of this thread at once: they share the
      // column group j4 (ranks tid / (COLS / 4) + e * 1024 / COLS), so one
      // read of H serves all of them; each sum still runs over l ascending
      const int j4t = 4 * (tid % (COLS / 4));
      float dd[NI][4];
#pragma unroll
      for (int e = 0; e < NI; ++e) dd[e][0] = dd[e][1] = dd[e][2] = dd[e][3] = 0.f;
#pragma unroll 4
      for (int l = 0; l < RP; ++l) {
        const float4 h4 = *reinterpret_cast<const float4*>(&Hs[l * COLS + j4t]);
#pragma unroll
        for (int e = 0; e < NI; ++e) {
          const int kk = (tid + 256 * e) / (COLS / 4);
          const float gl_ = Gs[l * RP + (kk < RP ? kk : 0)];
          dd[e][0] = fmaf(gl_, h4.x, dd[e][0]);
          dd[e][1] = fmaf(gl_, h4.y, dd[e][1]);
          dd[e][2] = fmaf(gl_, h4.z, dd[e][2]);
          dd[e][3] = fmaf(gl_, h4.w, dd[e][3]);
        }
      }
#pragma unroll
      for (int e = 0; e < NI; ++e) {
        const int idx = tid + 256 * e;
        if (NQ % 256 != 0 && idx >= NQ) continue;
        const int kk = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
        const int64_t j = j0 + j4;
        const int k = kk;
        float4 hn = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok[e]) {
          const float d0 = dd[e][0], d1 = dd[e][1], d2 = dd[e][2], d3 = dd[e][3];
          const float4 sum = sv[e], h = hr[e];
          hn.x = (d0 > 0.f) ? h.x * (sum.x / d0) : h.x;
          hn.y = (d1 > 0.f) ? h.y * (sum.y / d1) : h.y;
          hn.z = (d2 > 0.f) ? h.z * (sum.z / d2) : h.z;
          hn.w = (d3 > 0.f) ? h.w * (sum.w / d3) : h.w;
          *reinterpret_cast<float4*>(&Hp[(int64_t)k * ldh + j]) = hn;
          const float hv[4] = {hn.x, hn.y, hn.z, hn.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (j + u < n) {
              if (k < r) Hc[(int64_t)k * n + j + u] = hv[u];
              if (Hb) Hb[(int64_t)k * ldh + j + u] = to_bf16(hv[u]);
            }
          }
        }
        if (bf16) {
          hn.x = bf16_val(hn.x); hn.y = bf16_val(hn.y); hn.z = bf16_val(hn.z); hn.w = bf16_val(hn.w);
        }
        HnT[(j4 + 0) * HP + k] = hn.x;
        HnT[(j4 + 1) * HP + k] = hn.y;
        HnT[(j4 + 2) * HP + k] = hn.z;
        HnT[(j4 + 3) * HP + k] = hn.w;
      }
    } else {
    __syncthreads();
    for (int idx = tid; idx < RP * COLS / 4; idx += 256) {
      const int l = idx / (COLS / 4), jj = 4 * (idx % (COLS / 4));
      float4 h = *reinterpret_cast<const float4*>(&Hp[(int64_t)l * ldh + j0 + jj]);
      if (bf16) {
        h.x = bf16_val(h.x); h.y = bf16_val(h.y); h.z = bf16_val(h.z); h.w = bf16_val(h.w);
      }
      *reinterpret_cast<float4*>(&Hs[l * COLS + jj]) = h;
      if (FUSE && gram_only) {
        HnT[(jj + 0) * HP + l] = h.x;
        HnT[(jj + 1) * HP + l] = h.y;
        HnT[(jj + 2) * HP + l] = h.z;
        HnT[(jj + 3) * HP + l] = h.w;
      }
    }
    if (!gram_only) {
      for (int kc0 = 0; kc0 < RP; kc0 += KC) {
        if (!FUSE || kc0 > 0 || blk == blockIdx.x) {
          __syncthreads();
          for (int idx = tid; idx < KC * RP / 4; idx += 256) {
            float4 gv = *reinterpret_cast<const float4*>(&G[(int64_t)kc0 * RP + 4 * idx]);
            if (bf16) {
              gv.x = bf16_val(gv.x); gv.y = bf16_val(gv.y); gv.z = bf16_val(gv.z); gv.w = bf16_val(gv.w);
            }
            *reinterpret_cast<float4*>(&Gs[4 * idx]) = gv;
          }
        }
        __syncthreads();
        for (int idx = tid; idx < KC * COLS / 4; idx += 256) {
          const int kk = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
          const int64_t j = j0 + j4;
          const int k = kc0 + kk;
          float4 hn = make_float4(0.f, 0.f, 0.f, 0.f);
          if (j < n) {
            float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
#pragma unroll 8
            for (int l = 0; l < RP; ++l) {
              const float gl_ = Gs[kk * RP + l];
              const float4 h4 = *reinterpret_cast<const float4*>(&Hs[l * COLS + j4]);
              d0 = fmaf(gl_, h4.x, d0);
              d1 = fmaf(gl_, h4.y, d1);
              d2 = fmaf(gl_, h4.z, d2);
              d3 = fmaf(gl_, h4.w, d3);
            }
            const float4 sv = sum_splits4(part, (int64_t)k * ldp + j, sp, splits);
            const float4 h = *reinterpret_cast<const float4*>(&Hp[(int64_t)k * ldh + j]);
            hn.x = (d0 > 0.f) ? h.x * (sv.x / d0) : h.x;
            hn.y = (d1 > 0.f) ? h.y * (sv.y / d1) : h.y;
            hn.z = (d2 > 0.f) ? h.z * (sv.z / d2) : h.z;
            hn.w = (d3 > 0.f) ? h.w * (sv.w / d3) : h.w;
            *reinterpret_cast<float4*>(&Hp[(int64_t)k * ldh + j]) = hn;
            const float hv[4] = {hn.x, hn.y, hn.z, hn.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              if (j + e < n) {
                if (k < r) Hc[(int64_t)k * n + j + e] = hv[e];
                if (Hb) Hb[(int64_t)k * ldh + j + e] = to_bf16(hv[e]);
              }
            }
          }
          if (FUSE) {
            if (bf16) {
              hn.x = bf16_val(hn.x); hn.y = bf16_val(hn.y); hn.z = bf16_val(hn.z); hn.w = bf16_val(hn.w);
            }
            HnT[(j4 + 0) * HP + k] = hn.x;
            HnT[(j4 + 1) * HP + k] = hn.y;
            HnT[(j4 + 2) * HP + k] = hn.z;
            HnT[(j4 + 3) * HP + k] = hn.w;
          }
        }
      }
    }
    }
    if (gram) {
      __syncthreads();
#pragma unroll 4
      for (int jj = 0; jj < COLS; ++jj) {
        float x[TB], y[TB];
#pragma unroll
        for (int a = 0; a < TB; ++a) {
          x[a] = HnT[jj * HP + gk + a];
          y[a] = HnT[jj * HP + gl + a];
        }
#pragma unroll
        for (int a = 0; a < TB; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) ga[a][b] = fmaf(x[a], y[b], ga[a][b]);
      }
    }
  }
  if (gram) {
    float* out = gout + (int64_t)blockIdx.x * RP * RP;
#pragma unroll
    for (int a = 0; a < TB; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) out[(gk + a) * RP + gl + b] = ga[a][b];
  }
}

// ---------------------------------------------------------------------------
// Update epilogues with the denominators on the matrix cores: the H update
// at padded ranks 128 and 256, the W update at 256 (at 128 the vector-unit
// W update above measured faster).  At these ranks W (H H^T) and (W^T W) H
// are dense products (K = rp), so they are formed by MFMA from LDS-staged
// operands in chunks of 128 bytes of K:
//   D (M x N) = A (M x K) * B (K x N), A staged row-major, B transposed
// (one 128-byte row per output column), 16-byte chunk q of row t stored at
// slot q ^ (t % 8) as in the V passes.  FP32: v_mfma_f32_16x16x4_f32 on the
// float32 operands; BF16 tier: v_mfma_f32_16x16x32_bf16 on their bfloat16
// roundings (the operands the tier's products use), float32 accumulation.
// ---------------------------------------------------------------------------

// 16-byte chunk slot of element e (of ES bytes) in staged row t
template <int ES>
__device__ __forceinline__ int stage_off(int t, int e) {
  constexpr int PER = 16 / ES;  // elements per chunk
  const int q = e / PER;
  return t * 128 + 16 * (q ^ (t & 7)) + (e % PER) * ES;
}

template <bool BF>
__device__ __forceinline__ void stage_put(char* lds, int t, int e, float v) {
  if constexpr (BF) {
    *reinterpret_cast<uint16_t*>(lds + stage_off<2>(t, e)) = to_bf16(v);
  } else {
    *reinterpret_cast<float*>(lds + stage_off<4>(t, e)) = v;
  }
}

// elements e4 .. e4 + 3 (e4 a multiple of 4) of staged row t in one store:
// 16 bytes (float32) or 8 bytes (bfloat16), at the offsets of stage_off
template <bool BF>
__device__ __forceinline__ void stage_put4(char* lds, int t, int e4, float4 v) {
  if constexpr (BF) {
    const uint2 h = make_uint2((uint32_t)to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16),
                               (uint32_t)to_bf16(v.z) | ((uint32_t)to_bf16(v.w) << 16));
    *reinterpret_cast<uint2*>(lds + stage_off<2>(t, e4)) = h;
  } else {
    *reinterpret_cast<float4*>(lds + stage_off<4>(t, e4)) = v;
  }
}

// acc[i][j] += A rows (a0 + 16 i + c) x B^T rows (b0 + 16 j + c) over one
// staged chunk (KE = 128 / ES elements of K).
template <int MI, int NJ, bool BF>
__device__ __forceinline__ void mma_chunk(const char* A, int a0, const char* Bt, int b0,
                                          v4f (&acc)[MI][NJ]) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int q = 4 * kk + g;
    const int off = 16 * (q ^ (c & 7));
    if constexpr (BF) {
      v8bf a[MI], b[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = *reinterpret_cast<const v8bf*>(A + (a0 + 16 * i + c) * 128 + off);
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = *reinterpret_cast<const v8bf*>(Bt + (b0 + 16 * j + c) * 128 + off);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    } else {
      v4f a[MI], b[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = *reinterpret_cast<const v4f*>(A + (a0 + 16 * i + c) * 128 + off);
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = *reinterpret_cast<const v4f*>(Bt + (b0 + 16 * j + c) * 128 + off);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc[i][j] = mfma_f32(a[i][t], b[j][t], acc[i][j]);
    }
  }
}

// W half-step, rp in {128, 256}: a block of 64 WR threads x 4 waves along
// the ranks takes ROWS = 32 WR rows of W (grid-stride);
// D = W_rows (ROWS x rp) * G (rp x rp).  Wave (wr, wc) ends with
// D[i0 + 32 wr + 16 ib + 4 g + v][wc rp/4 + 16 kb + c].
template <int RP, int WR, bool BF>
__global__ __launch_bounds__(256 * WR) void k_update_w_mma(
    int64_t p, int r, const float* __restrict__ part, int64_t ldp, int64_t sp, int splits,
    const float* __restrict__ G, float* __restrict__ Wp, float* __restrict__ Wc,
    float* __restrict__ WT, uint16_t* __restrict__ WbT, int64_t ldwt) {
  constexpr int ES = BF ? 2 : 4, KE = 128 / ES, T = 256 * WR;
  constexpr int ROWS = 32 * WR, MI = 2, NJ = RP / 64;
  __shared__ __attribute__((aligned(1024))) char As[ROWS * 128];
  __shared__ __attribute__((aligned(1024))) char Bs[RP * 128];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int wc = wave & 3, wr = wave >> 2;
  const int kb = wc * (RP / 4), ib = 32 * wr;
  for (int64_t blk = blockIdx.x; blk * ROWS < p; blk += gridDim.x) {
    const int64_t i0 = blk * ROWS;
    v4f acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int l0 = 0; l0 < RP; l0 += KE) {
      __syncthreads();
      // A: rows i0 .. i0 + ROWS of W (ppad rows, zero beyond p), columns l0 ..
      for (int idx = tid; idx < ROWS * KE / 4; idx += T) {
        const int t = idx / (KE / 4), e4 = 4 * (idx % (KE / 4));
        stage_put4<BF>(As, t, e4, *reinterpret_cast<const float4*>(&Wp[(i0 + t) * RP + l0 + e4]));
      }
      // B^T: row k holds G[l0 .. l0 + KE][k], which is row k of G (a Gram
      // matrix is symmetric), so it is staged like A
      for (int idx = tid; idx < RP * KE / 4; idx += T) {
        const int t = idx / (KE / 4), e4 = 4 * (idx % (KE / 4));
        stage_put4<BF>(Bs, t, e4, *reinterpret_cast<const float4*>(&G[(int64_t)t * RP + l0 + e4]));
      }
      __syncthreads();
      mma_chunk<MI, NJ, BF>(As, ib, Bs, kb, acc);
    }
    // ratio update; the numerators are summed over the splits in ascending
    // order, all of this lane's entries of one split loaded together
    float na[MI][NJ][4];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) na[i][j][v] = 0.f;
    for (int q = 0; q < splits; ++q) {
      float x[MI][NJ][4];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t row = i0 + ib + 16 * i + 4 * g + v;
            x[i][j][v] = 0.f;
            if (row < p) x[i][j][v] = part[q * sp + row * ldp + kb + 16 * j + c];
          }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) na[i][j][v] += x[i][j][v];
    }
    // every W value of this lane first (its own entries), so the loads share
    // one memory round trip instead of waiting one by one behind the stores
    float wo[MI][NJ][4];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = i0 + ib + 16 * i + 4 * g + v;
          wo[i][j][v] = row < p ? Wp[row * RP + kb + 16 * j + c] : 0.f;
        }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int k = kb + 16 * j + c;
        float wv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = i0 + ib + 16 * i + 4 * g + v;
          wv[v] = 0.f;
          if (row >= p) continue;
          const float a = na[i][j][v];
          const float b = acc[i][j][v];
          const float w = wo[i][j][v];
          const float wn = (b > 0.f) ? w * (a / b) : w;
          Wp[row * RP + k] = wn;
          if (k < r) Wc[row * r + k] = wn;
          wv[v] = wn;
        }
        const int64_t rb = i0 + ib + 16 * i + 4 * g;  // 4 consecutive rows: one store
        if (rb + 3 < p) {
          if (WT) *reinterpret_cast<float4*>(&WT[(int64_t)k * ldwt + rb]) = make_float4(wv[0], wv[1], wv[2], wv[3]);
          if (WbT) {
            const uint2 h = make_uint2((uint32_t)to_bf16(wv[0]) | ((uint32_t)to_bf16(wv[1]) << 16),
                                       (uint32_t)to_bf16(wv[2]) | ((uint32_t)to_bf16(wv[3]) << 16));
            *reinterpret_cast<uint2*>(&WbT[(int64_t)k * ldwt + rb]) = h;
          }
        } else {
          for (int v = 0; v < 4; ++v)
            if (rb + v < p) {
              if (WT) WT[(int64_t)k * ldwt + rb + v] = wv[v];
              if (WbT) WbT[(int64_t)k * ldwt + rb + v] = to_bf16(wv[v]);
            }
        }
      }
  }
}

// H half-step, rp in {128, 256}: a block of 4 waves along the ranks x WC
// along the columns takes COLS = 64 WC columns of H (grid-stride);
// D = G (rp x rp) * H_cols (rp x COLS).  Wave (wr, wc) ends with
// D[wr rp/4 + 16 kb + 4 g + v][j0 + 64 wc + 16 jb + c].
template <int RP, int WC, bool BF>
__global__ __launch_bounds__(256 * WC) void k_update_h_mma(
    int64_t n, int r, const float* __restrict__ part, int64_t ldp, int64_t sp, int splits,
    const float* __restrict__ G, float* __restrict__ Hp, int64_t ldh, float* __restrict__ Hc,
    uint16_t* __restrict__ Hb) {
  constexpr int ES = BF ? 2 : 4, KE = 128 / ES, T = 256 * WC;
  constexpr int COLS = 64 * WC, MI = RP / 64, NJ = 4;
  __shared__ __attribute__((aligned(1024))) char As[RP * 128];
  __shared__ __attribute__((aligned(1024))) char Bs[COLS * 128];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int wr = wave & 3, wc = wave >> 2;
  const int kb = wr * (RP / 4), jb0 = 64 * wc;
  for (int64_t blk = blockIdx.x; blk * COLS < n; blk += gridDim.x) {
    const int64_t j0 = blk * COLS;
    v4f acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int l0 = 0; l0 < RP; l0 += KE) {
      __syncthreads();
      // A: rows of G, columns l0 ..
      for (int idx = tid; idx < RP * KE / 4; idx += T) {
        const int t = idx / (KE / 4), e4 = 4 * (idx % (KE / 4));
        stage_put4<BF>(As, t, e4, *reinterpret_cast<const float4*>(&G[(int64_t)t * RP + l0 + e4]));
      }
      // B^T: row jj holds H[l0 .. l0 + KE][j0 + jj] (H is rp x ldh, zero-padded)
      for (int idx = tid; idx < KE * COLS / 4; idx += T) {
        const int e = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
        const float4 h = *reinterpret_cast<const float4*>(&Hp[(int64_t)(l0 + e) * ldh + j0 + j4]);
        stage_put<BF>(Bs, j4 + 0, e, h.x);
        stage_put<BF>(Bs, j4 + 1, e, h.y);
        stage_put<BF>(Bs, j4 + 2, e, h.z);
        stage_put<BF>(Bs, j4 + 3, e, h.w);
      }
      __syncthreads();
      mma_chunk<MI, NJ, BF>(As, kb, Bs, jb0, acc);
    }
    // per 16-rank tile i of this lane: the numerators summed over the splits
    // in ascending order (the tile's entries of one split loaded together),
    // then its H values, then the updates.  A tile at a time keeps the live
    // registers few (all tiles at once spilled at rank 256), and a lane's
    // H values are loaded before its stores (its own entries only) so they
    // do not wait one by one behind them.
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      float ns[NJ][4];
#pragma unroll
      for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) ns[jb][v] = 0.f;
      for (int q = 0; q < splits; ++q) {
        float x[NJ][4];
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t j = j0 + jb0 + 16 * jb + c;
            x[jb][v] = 0.f;
            if (j < n) x[jb][v] = part[q * sp + (int64_t)(kb + 16 * i + 4 * g + v) * ldp + j];
          }
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
          for (int v = 0; v < 4; ++v) ns[jb][v] += x[jb][v];
      }
      float hv[NJ][4];
#pragma unroll
      for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = j0 + jb0 + 16 * jb + c;
          hv[jb][v] = 0.f;
          if (j < n) hv[jb][v] = Hp[(int64_t)(kb + 16 * i + 4 * g + v) * ldh + j];
        }
#pragma unroll
      for (int jb = 0; jb < NJ; ++jb) {
        const int64_t j = j0 + jb0 + 16 * jb + c;
        if (j >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = kb + 16 * i + 4 * g + v;
          const float s = ns[jb][v];
          const float d = acc[i][jb][v];
          const float h = hv[jb][v];
          const float hn = (d > 0.f) ? h * (s / d) : h;
          Hp[(int64_t)k * ldh + j] = hn;
          if (k < r) Hc[(int64_t)k * n + j] = hn;
          if (Hb) Hb[(int64_t)k * ldh + j] = to_bf16(hn);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Objective partials (eq. nnmf-objfn), direct residual in float64:
// each 64 x 64 tile accumulates sum (v_ij - sum_k w_ik h_kj)^2 with the
// inner products formed by float64 FMAs of the float32 factors (exactly
// converted).  The W block is staged in LDS row-major with a padded pitch
// (conflict-free stores), H rank-major; a thread owns a 4 x 4 block and
// loads its V entries first, so their latency overlaps the staging and the
// products.  The tile total is reduced in a fixed order.  Wp == nullptr
// means W = 0 (gives ||V||_F^2).
// ---------------------------------------------------------------------------
template <int RP>
__global__ __launch_bounds__(256) void k_objective(
    const float* __restrict__ V, int64_t ldv, int64_t p, int64_t n,
    const float* __restrict__ Wp, const float* __restrict__ Hp, int64_t ldh,
    double* __restrict__ part) {
  constexpr int KC = RP < 64 ? RP : 64;
  constexpr int WP = KC + 4;  // W row pitch (16-byte aligned rows)
  __shared__ __attribute__((aligned(16))) float Ws[64 * WP];
  __shared__ __attribute__((aligned(16))) float Hs[KC * 64];
  __shared__ double red[4];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;

  float4 vq[4];  // this thread's 4 x 4 block of V
#pragma unroll
  for (int a = 0; a < 4; ++a) vq[a] = load4(V, ldv, i0 + 4 * ty + a, p, j0 + 4 * tx, n);

  double s[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) s[a][b] = 0.0;

  if (Wp) {
    for (int kc0 = 0; kc0 < RP; kc0 += KC) {
      __syncthreads();
      for (int idx = tid; idx < 64 * KC / 4; idx += 256) {
        const int ii = idx / (KC / 4), k4 = 4 * (idx % (KC / 4));
        const float4 w = *reinterpret_cast<const float4*>(&Wp[(i0 + ii) * RP + kc0 + k4]);
        float* d = &Ws[ii * WP + k4];
        d[0] = w.x; d[1] = w.y; d[2] = w.z; d[3] = w.w;
      }
      for (int idx = tid; idx < KC * 64 / 4; idx += 256) {
        const int kk = idx / 16, j4 = 4 * (idx % 16);
        const float4 h = *reinterpret_cast<const float4*>(&Hp[(int64_t)(kc0 + kk) * ldh + j0 + j4]);
        float* d = &Hs[kk * 64 + j4];
        d[0] = h.x; d[1] = h.y; d[2] = h.z; d[3] = h.w;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < KC; ++kk) {
        double wd[4], hd[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) wd[a] = Ws[(4 * ty + a) * WP + kk];
#pragma unroll
        for (int b = 0; b < 4; ++b) hd[b] = Hs[kk * 64 + 4 * tx + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) s[a][b] = fma(wd[a], hd[b], s[a][b]);
      }
    }
  }

  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t row = i0 + 4 * ty + a;
    const int64_t col = j0 + 4 * tx;
    const float vv[4] = {vq[a].x, vq[a].y, vq[a].z, vq[a].w};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (row < p && col + b < n) {
        const double e = (double)vv[b] - s[a][b];
        acc = fma(e, e, acc);
      }
    }
  }
  // fixed-order reduction: butterfly within the wave, then waves 0..3
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0)
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_reduce_f64(const double* __restrict__ part,
                                                    int64_t count, double* __restrict__ out) {
  // thread t sums part[t], part[t + 256], ... in ascending order (8 loads in
  // flight), then a fixed tree combines the 256 thread sums
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  int64_t q = tid;
  for (; q + 7 * 256 < count; q += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[q + 256 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < count; q += 256) s += part[q];
  sh[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[0] = sh[0];
}

// ---------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------
__global__ void k_copy_pad(const float* __restrict__ src, int64_t lds, int64_t rows,
                           int64_t cols, float* __restrict__ dst, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / cols, j = idx % cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

__global__ void k_fill_f32(float* __restrict__ dst, int64_t count, float v) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * blockDim.x)
    dst[idx] = v;
}

__global__ void k_fill_u32(uint32_t* __restrict__ dst, int64_t count, uint32_t v) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * blockDim.x)
    dst[idx] = v;
}

// Copy (float32, or bfloat16 RNE) through a 32 x 32 LDS tile; with
// `transpose` the tile is written out transposed so both reads and writes
// stay coalesced.
template <typename OutT>
__device__ __forceinline__ OutT convert_out(float x);
template <>
__device__ __forceinline__ float convert_out<float>(float x) {
  return x;
}
template <>
__device__ __forceinline__ uint16_t convert_out<uint16_t>(float x) {
  return to_bf16(x);
}

template <typename OutT>
__global__ __launch_bounds__(256) void k_convert(const float* __restrict__ src, int64_t lds,
                                                 int64_t rows, int64_t cols,
                                                 OutT* __restrict__ dst, int64_t ldd,
                                                 int transpose) {
  __shared__ OutT t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int q = 0; q < 4; ++q) {
    const int64_t i = r0 + ty + 8 * q, j = c0 + tx;
    OutT h = OutT(0);
    if (i < rows && j < cols) h = convert_out<OutT>(src[i * lds + j]);
    if (!transpose) {
      if (i < rows && j < cols) dst[i * ldd + j] = h;
    } else {
      t[ty + 8 * q][tx] = h;
    }
  }
  if (!transpose) return;
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int64_t jo = c0 + ty + 8 * q, io = r0 + tx;  // dst row = source column
    if (jo < cols && io < rows) dst[jo * ldd + io] = t[tx][ty + 8 * q];
  }
}

__global__ void k_validate(const float* __restrict__ V, int64_t ldv, int64_t p, int64_t n,
                           uint32_t* __restrict__ flag) {
  const int64_t total = p * n;
  uint32_t bad = 0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const float v = V[(idx / n) * ldv + idx % n];
    if (!(v >= 0.f) || !__builtin_isfinite(v)) bad = 1;
  }
  if (bad) atomicOr(flag, 1u);
}

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): 10 rounds of the
// multiply-xor bijection with key schedule bumped by the Weyl constants.
__device__ __forceinline__ uint32_t philox_first(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  return c0;
}

__global__ void k_uniform(float* __restrict__ dst, int64_t rows, int64_t cols, int64_t ldd,
                          uint32_t k0, uint32_t k1, uint32_t stream_id) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = philox_first((uint32_t)idx, (uint32_t)(idx >> 32), stream_id, 0u, k0, k1);
    // 23 random bits + 1/2, scaled by 2^-23: exactly representable, in (0, 1)
    const float u = ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f);
    dst[(idx / cols) * ldd + idx % cols] = u;
  }
}

// Gauge fixing of a factorization (W H is unchanged): w_k <- w_k / |w_k|,
// h_k <- h_k |w_k| for every column k of W with a nonzero norm.  One
// workgroup per column sums the squares in float64 in a fixed order.
__global__ __launch_bounds__(256) void k_col_norms(const float* __restrict__ W, int64_t p, int r,
                                                   float* __restrict__ norms) {
  __shared__ double sh[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < p; i += 256) {
    const double w = W[i * r + k];
    s += w * w;
  }
  sh[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  if (tid == 0) norms[k] = (float)sqrt(sh[0]);
}

__global__ void k_apply_gauge(float* __restrict__ W, int64_t p, int r, float* __restrict__ H,
                              int64_t n, const float* __restrict__ norms) {
  const int64_t tw = p * r, total = tw + (int64_t)r * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < tw) {
      const float nk = norms[idx % r];
      if (nk > 0.f) W[idx] = W[idx] / nk;
    } else {
      const int64_t j = idx - tw;
      const float nk = norms[j / n];
      if (nk > 0.f) H[j] = H[j] * nk;
    }
  }
}

// ---------------------------------------------------------------------------
// Least-squares dictionary for a warm start (r <= 64):
//   W = max(A (G + delta I)^{-1}, floor),  A = V H^T,  G = H H^T,
//   delta = 1e-6 tr(G) / r,  floor = floor_rel * max(W)  (at least FLT_MIN)
// A comes from the pass-1 partials, G from the Gram reduction of that pass.
// ---------------------------------------------------------------------------
// One workgroup: Cholesky factor G + delta I = L L^T in float64, L^{-1} by
// forward substitution (one column per thread), Ginv = L^{-T} L^{-1}.
__global__ __launch_bounds__(256) void k_ls_inverse(const float* __restrict__ G, int rp, int r,
                                                    double* __restrict__ Ginv) {
  __shared__ double L[64 * 64];
  __shared__ double Li[64 * 64];
  __shared__ double s_delta;
  const int tid = threadIdx.x;
  for (int e = tid; e < r * r; e += 256) L[e] = (double)G[(e / r) * rp + e % r];
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < r; ++i) t += L[i * r + i];
    s_delta = t > 0.0 ? 1e-6 * t / r : 1e-300;
  }
  __syncthreads();
  for (int i = tid; i < r; i += 256) L[i * r + i] += s_delta;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    if (tid == 0) L[k * r + k] = sqrt(fmax(L[k * r + k], s_delta));
    __syncthreads();
    const double dk = L[k * r + k];
    for (int i = k + 1 + tid; i < r; i += 256) L[i * r + k] /= dk;
    __syncthreads();
    const int m = r - k - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) L[i * r + j] -= L[i * r + k] * L[j * r + k];
    }
    __syncthreads();
  }
  for (int j = tid; j < r; j += 256) {
    for (int i = 0; i < r; ++i) {
      if (i < j) {
        Li[i * r + j] = 0.0;
        continue;
      }
      double x = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) x -= L[i * r + k] * Li[k * r + j];
      Li[i * r + j] = x / L[i * r + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < rp * rp; e += 256) {
    const int i = e / rp, j = e % rp;
    double x = 0.0;
    if (i < r && j < r)
      for (int k = (i > j ? i : j); k < r; ++k) x += Li[k * r + i] * Li[k * r + j];
    Ginv[e] = x;
  }
}

// 64 rows per workgroup: a_i = sum_s part[s][i] (splits in order), w_i =
// a_i Ginv with float64 accumulation, written to Wp; the largest entry is
// folded into maxbits (bits of a nonnegative float order like the values).
__global__ __launch_bounds__(256) void k_ls_apply(const float* __restrict__ part, int64_t ldp,
                                                  int64_t sp, int splits,
                                                  const double* __restrict__ Ginv, int rp, int r,
                                                  int64_t p, float* __restrict__ Wp,
                                                  uint32_t* __restrict__ maxbits) {
  __shared__ float As[64 * 65];
  __shared__ double Gs[64 * 64];
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < rp * rp; e += 256) Gs[e] = Ginv[e];
  for (int e = tid; e < 64 * rp; e += 256) {
    const int ii = e / rp, k = e % rp;
    float a = 0.f;
    if (i0 + ii < p)
      for (int q = 0; q < splits; ++q) a += part[(int64_t)q * sp + (i0 + ii) * ldp + k];
    As[ii * 65 + k] = a;
  }
  __syncthreads();
  float mx = 0.f;
  for (int e = tid; e < 64 * rp; e += 256) {
    const int ii = e / rp, k = e % rp;
    if (i0 + ii >= p) continue;
    double w = 0.0;
    if (k < r)
      for (int j = 0; j < r; ++j) w += (double)As[ii * 65 + j] * Gs[j * rp + k];
    const float wf = (float)w;
    Wp[(i0 + ii) * rp + k] = wf;
    mx = fmaxf(mx, wf);
  }
  red[tid] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmaxf(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) atomicMax(maxbits, __float_as_uint(red[0]));
}

// W <- max(W, floor) on the r live columns; also the caller's W (p x r).
__global__ void k_ls_clip(float* __restrict__ Wp, int rp, int r, int64_t p,
                          const uint32_t* __restrict__ maxbits, float floor_rel,
                          float* __restrict__ Wcaller) {
  const float fl = fmaxf(floor_rel * __uint_as_float(*maxbits), 1.17549435e-38f);
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < p * r;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / r;
    const int k = (int)(idx % r);
    const float w = fmaxf(Wp[i * rp + k], fl);
    Wp[i * rp + k] = w;
    Wcaller[idx] = w;
  }
}

inline unsigned grid1d(int64_t total, int threads, int64_t cap = 65536) {
  int64_t b = (total + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Configurations and launchers
// ---------------------------------------------------------------------------
typedef hipError_t (*NtLaunch)(const void*, int64_t, int64_t, const void*, int64_t, int64_t,
                               int64_t, int64_t, float*, int64_t, int64_t, const GramRed&, dim3,
                               hipStream_t);

template <int MB, int NB, int WM, int WN, int BK>
hipError_t nt_f32(const void* X, int64_t ldx, int64_t M, const void* Y, int64_t ldy, int64_t N,
                  int64_t K, int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                  const GramRed& gr, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_gemm_nt<MB, NB, WM, WN, BK>), grid, dim3(64 * WM * WN), 0, st,
                     static_cast<const float*>(X), ldx, M, static_cast<const float*>(Y), ldy, N,
                     K, kchunk, part, ldp, sp, gr);
  return hipGetLastError();
}

template <int MB, int NB, int WM, int WN, int BK>
hipError_t nt_bf16(const void* X, int64_t ldx, int64_t M, const void* Y, int64_t ldy, int64_t N,
                   int64_t K, int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                   const GramRed& gr, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_gemm_nt_bf16<MB, NB, WM, WN, BK>), grid, dim3(64 * WM * WN), 0, st,
                     static_cast<const uint16_t*>(X), ldx, M, static_cast<const uint16_t*>(Y),
                     ldy, N, K, kchunk, part, ldp, sp, gr);
  return hipGetLastError();
}

template <int MB, int WM, int WN, int BK>
hipError_t tn_f32(const void* A, int64_t lda, int64_t M, const void* B, int64_t ldb, int64_t N,
                  int64_t K, int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                  const GramRed& gr, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_gemm_tn<MB, WM, WN, BK>), grid, dim3(64 * WM * WN), 0, st,
                     static_cast<const float*>(A), lda, M, static_cast<const float*>(B), ldb, N,
                     K, kchunk, part, ldp, sp, gr);
  return hipGetLastError();
}

struct NtEntry {
  int mb, nb, wm, wn, bk;
  NtLaunch f32, bf16;
};
#define NTE(MB, NB, WM, WN, BK, BKH) \
  {MB, NB, WM, WN, BK, &nt_f32<MB, NB, WM, WN, BK>, &nt_bf16<MB, NB, WM, WN, BKH>}
// id: (MB, NB, WM, WN, BK fp32 / BK bf16); tile (16 MB WM) x (16 NB WN)
static const NtEntry kNt[] = {
    NTE(2, 1, 4, 1, 32, 64),  //  0: 128 x 16
    NTE(2, 2, 4, 1, 32, 64),  //  1: 128 x 32
    NTE(2, 4, 4, 1, 32, 64),  //  2: 128 x 64
    NTE(4, 4, 2, 2, 32, 64),  //  3: 128 x 128
    NTE(1, 1, 1, 1, 32, 64),  //  4: 16 x 16
    NTE(2, 2, 1, 1, 32, 64),  //  5: 32 x 32
    NTE(2, 2, 2, 2, 32, 64),  //  6: 64 x 64
    NTE(1, 4, 1, 4, 32, 64),  //  7: 16 x 256
    NTE(2, 4, 1, 4, 32, 64),  //  8: 32 x 256
    NTE(4, 4, 1, 4, 32, 64),  //  9: 64 x 256
    NTE(2, 2, 4, 2, 32, 64),  // 10: 128 x 64, 8 waves
};
#undef NTE
static const int kNtCount = sizeof(kNt) / sizeof(kNt[0]);

struct TnEntry {
  int mb, wm, wn, bk;
  NtLaunch f32;
};
#define TNE(MB, WM, WN, BK) {MB, WM, WN, BK, &tn_f32<MB, WM, WN, BK>}
// id: (MB, WM, WN, BK); tile (16 MB WM) x (64 WN)
static const TnEntry kTn[] = {
    TNE(1, 1, 4, 32),  //  0: 16 x 256
    TNE(2, 1, 4, 32),  //  1: 32 x 256
    TNE(4, 1, 4, 32),  //  2: 64 x 256
    TNE(4, 2, 2, 32),  //  3: 128 x 128
    TNE(1, 1, 1, 32),  //  4: 16 x 64
    TNE(2, 1, 1, 32),  //  5: 32 x 64
    TNE(4, 1, 1, 32),  //  6: 64 x 64
    TNE(2, 2, 4, 32),  //  7: 64 x 256, 8 waves
};
#undef TNE
static const int kTnCount = sizeof(kTn) / sizeof(kTn[0]);

static NtCfg make_nt(int id) {
  NtCfg c;
  c.id = id;
  c.bm = 16 * kNt[id].mb * kNt[id].wm;
  c.bn = 16 * kNt[id].nb * kNt[id].wn;
  c.threads = 64 * kNt[id].wm * kNt[id].wn;
  c.bk = kNt[id].bk;
  c.bk_bf16 = 2 * kNt[id].bk;
  return c;
}

static TnCfg make_tn(int id) {
  TnCfg c;
  c.id = id;
  c.bm = 16 * kTn[id].mb * kTn[id].wm;
  c.bn = 64 * kTn[id].wn;
  c.threads = 64 * kTn[id].wm * kTn[id].wn;
  c.bk = kTn[id].bk;
  return c;
}

int nt_config_count() { return kNtCount; }
int tn_config_count() { return kTnCount; }
NtCfg nt_config_by_id(int id) { return make_nt(id < 0 || id >= kNtCount ? 2 : id); }
TnCfg tn_config_by_id(int id) { return make_tn(id < 0 || id >= kTnCount ? 2 : id); }

NtCfg nt_config(int rp, bool gram) {
  if (gram) {
    switch (rp) {
      case 16: return make_nt(4);
      case 32: return make_nt(5);
      case 64: return make_nt(6);
      default: return make_nt(3);
    }
  }
  switch (rp) {  // M = p (long), N = rank
    case 16: return make_nt(0);
    case 32: return make_nt(1);
    case 64: return make_nt(2);
    default: return make_nt(3);
  }
}

// BF16: pass 1 uses the same shapes as FP32 (M = p, N = rank); pass 2 runs
// as an NT product with M = rank and N = n (transposed bf16 copy of V).
NtCfg nt_bf16_config(int rp, bool gram) {
  if (gram) return nt_config(rp, true);
  switch (rp) {
    case 16: return make_nt(7);
    case 32: return make_nt(8);
    case 64: return make_nt(9);
    default: return make_nt(3);
  }
}

TnCfg tn_config(int rp, bool gram) {
  if (gram) {
    switch (rp) {
      case 16: return make_tn(4);
      case 32: return make_tn(5);
      case 64: return make_tn(6);
      default: return make_tn(3);
    }
  }
  switch (rp) {  // M = rank, N = n (long)
    case 16: return make_tn(0);
    case 32: return make_tn(1);
    case 64: return make_tn(2);
    default: return make_tn(3);
  }
}

static dim3 tiles3(int64_t M, int64_t N, int bm, int bn, int splits) {
  return dim3((unsigned)((N + bn - 1) / bn), (unsigned)((M + bm - 1) / bm), (unsigned)splits);
}

hipError_t launch_gemm_nt(const NtCfg& cfg, const float* X, int64_t ldx, int64_t M,
                          const float* Y, int64_t ldy, int64_t N, int64_t K, int splits,
                          int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                          const GramRed& gr, hipStream_t st) {
  if (cfg.id < 0 || cfg.id >= kNtCount) return hipErrorInvalidValue;
  return kNt[cfg.id].f32(X, ldx, M, Y, ldy, N, K, kchunk, part, ldp, sp, gr,
                         tiles3(M, N, cfg.bm, cfg.bn, splits), st);
}

hipError_t launch_gemm_nt_bf16(const NtCfg& cfg, const uint16_t* X, int64_t ldx, int64_t M,
                               const uint16_t* Y, int64_t ldy, int64_t N, int64_t K,
                               int splits, int64_t kchunk, float* part, int64_t ldp,
                               int64_t sp, const GramRed& gr, hipStream_t st) {
  if (cfg.id < 0 || cfg.id >= kNtCount) return hipErrorInvalidValue;
  return kNt[cfg.id].bf16(X, ldx, M, Y, ldy, N, K, kchunk, part, ldp, sp, gr,
                          tiles3(M, N, cfg.bm, cfg.bn, splits), st);
}

typedef hipError_t (*DmaLaunch)(const void*, int64_t, const void*, int64_t, int64_t, int64_t,
                                float*, int64_t, int64_t, const GramRed&, dim3, hipStream_t);

template <int MB, int NB, int WM, int WN, int S, bool BF, int SH>
hipError_t dma_inst(const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t K,
                    int64_t kchunk, float* part, int64_t ldp, int64_t sp, const GramRed& gr,
                    dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_nt_dma<MB, NB, WM, WN, S, BF, SH>), grid, dim3(64 * WM * WN), 0, st, X,
                     ldx, Y, ldy, K, kchunk, part, ldp, sp, gr);
  return hipGetLastError();
}

struct DmaEntry {
  int sh, mb, nb, wm, wn, s;
  DmaLaunch f32, bf16;
};
#define DME(MB, NB, WM, WN, S)                                              \
  {16, MB, NB, WM, WN, S, &dma_inst<MB, NB, WM, WN, S, false, 16>,          \
   &dma_inst<MB, NB, WM, WN, S, true, 16>}
#define DME32(MB, NB, WM, WN, S)                                            \
  {32, MB, NB, WM, WN, S, &dma_inst<MB, NB, WM, WN, S, false, 32>,          \
   &dma_inst<MB, NB, WM, WN, S, true, 32>}
// id: (MB, NB, WM, WN, stages); tile (SH MB WM) x (SH NB WN), SH = 16 for
// DME and 32 for DME32
static const DmaEntry kDma[] = {
    DME(4, 1, 2, 1, 3),  // 0: 128 x 16   pass 1, r <= 16
    DME(2, 2, 4, 1, 3),  // 1: 128 x 32   pass 1, r <= 32
    DME(2, 4, 4, 1, 3),  // 2: 128 x 64   pass 1, r <= 64
    DME(4, 4, 2, 2, 2),  // 3: 128 x 128  r > 64
    DME(1, 4, 1, 2, 3),  // 4: 16 x 128   pass 2, r <= 16
    DME(1, 4, 2, 2, 3),  // 5: 32 x 128   pass 2, r <= 32
    DME(2, 4, 2, 2, 3),  // 6: 64 x 128   pass 2, r <= 64
    DME(2, 4, 4, 1, 4),  // 7: 128 x 64, 4 stages
    DME(2, 4, 2, 2, 4),  // 8: 64 x 128, 4 stages
    // narrow tiles for problems whose default tiling leaves fewer than 256
    // workgroups (1024 waves: one per SIMD)
    DME(1, 4, 4, 1, 3),  // 9:  64 x 64    pass 1, r <= 64
    DME(2, 2, 2, 2, 3),  // 10: 64 x 64    pass 2, r <= 64
    DME(1, 2, 4, 1, 3),  // 11: 64 x 32    pass 1, r <= 32
    DME(1, 2, 2, 2, 3),  // 12: 32 x 64    pass 2, r <= 32
    DME(2, 1, 2, 1, 3),  // 13: 64 x 16    pass 1, r <= 16
    DME(1, 2, 1, 2, 3),  // 14: 16 x 64    pass 2, r <= 16
    // all 256 ranks in one workgroup, so V^T is read once (BF16 pass 2)
    DME(8, 4, 2, 2, 3),  // 15: 256 x 128  pass 2, r = 256, 3 stages
    // rank 256, BF16: all ranks in one workgroup of 8 waves (two per SIMD)
    DME(4, 4, 4, 2, 3),  // 16: 256 x 128  pass 2, 3 stages (144 KB)
    DME(4, 4, 2, 4, 3),  // 17: 128 x 256  pass 1, 3 stages
    // 64 x 64 per wave at rank 64 (16 accumulators, 8 fragment reads per
    // 4 k): two-wave tiles (two workgroups per CU) and four-wave tiles
    DME(4, 4, 2, 1, 3),  // 18: 128 x 64   pass 1, 72 KB
    DME(4, 4, 1, 2, 3),  // 19: 64 x 128   pass 2, 72 KB
    DME(4, 4, 4, 1, 3),  // 20: 256 x 64   pass 1, 120 KB
    DME(4, 4, 1, 4, 3),  // 21: 64 x 256   pass 2, 120 KB
    DME(4, 4, 4, 1, 2),  // 22: 256 x 64   pass 1, 80 KB
    DME(4, 4, 1, 4, 2),  // 23: 64 x 256   pass 2, 80 KB
    // rank 64, 2 stages (48 KB): three workgroups per CU
    DME(2, 4, 4, 1, 2),  // 24: 128 x 64   pass 1
    DME(2, 4, 2, 2, 2),  // 25: 64 x 128   pass 2
    // the same tiles on the 32 x 32 matrix-core shapes
    DME32(1, 2, 4, 1, 3),  // 26: 128 x 64   pass 1, r <= 64 (as 2)
    DME32(1, 2, 2, 2, 3),  // 27: 64 x 128   pass 2, r <= 64 (as 6)
    DME32(1, 1, 4, 1, 3),  // 28: 128 x 32   pass 1, r <= 32 (as 1)
    DME32(1, 1, 1, 4, 3),  // 29: 32 x 128   pass 2, r <= 32 (as 5)
    DME32(2, 2, 2, 2, 2),  // 30: 128 x 128  r > 64 (as 3)
    DME32(2, 2, 4, 2, 3),  // 31: 256 x 128  pass 2, 8 waves (as 16)
    DME32(2, 2, 2, 4, 3),  // 32: 128 x 256  pass 1, 8 waves (as 17)
    DME32(1, 1, 2, 2, 3),  // 33: 64 x 64    pass 1, r <= 64 narrow (as 9)
    DME32(1, 1, 2, 2, 3),  // 34: 64 x 64    pass 2, r <= 64 narrow (as 10)
    DME32(1, 1, 2, 1, 3),  // 35: 64 x 32    pass 1, r <= 32 narrow (as 11)
    DME32(1, 1, 1, 2, 3),  // 36: 32 x 64    pass 2, r <= 32 narrow (as 12)
};
#undef DME
#undef DME32
static const int kDmaCount = sizeof(kDma) / sizeof(kDma[0]);

DmaCfg dma_config_by_id(int id) {
  if (id < 0 || id >= kDmaCount) id = 2;
  DmaCfg c;
  c.id = id;
  c.bm = kDma[id].sh * kDma[id].mb * kDma[id].wm;
  c.bn = kDma[id].sh * kDma[id].nb * kDma[id].wn;
  c.threads = 64 * kDma[id].wm * kDma[id].wn;
  return c;
}

DmaCfg dma_config(int rp, bool pass1, bool narrow, bool bf16) {
  // BF16 at rank 256: one workgroup of 8 waves for all 256 ranks, so V
  // (pass 1) or V^T (pass 2) is read once (8192 x 32768: pass 2 186 -> 158
  // us, pass 1 165 -> 160 us against 128 x 128 tiles; in FP32, bound by the
  // matrix cores, the 128 x 128 tiles are as fast)
  if (rp == 256 && bf16) return dma_config_by_id(pass1 ? 17 : 16);
  // BF16 at rank 128: 256 x 128 / 128 x 256 tiles of 8 waves, 3 stages (with
  // about 256 workgroups: 8192 x 32768, 126.8 -> 121.5 and 128.5 -> 118.7 us
  // against 128 x 128 tiles with 2 stages)
  if (rp == 128 && bf16) return dma_config_by_id(pass1 ? 16 : 17);
  // FP32 from rank 64 up: the 32 x 32 matrix-core shape (8192 x 32768, rank
  // 128: 553.8 -> 512.9 us per pass; 4096 x 16384, rank 64: 179.8 -> 177.2
  // us per iteration); at lower ranks, on the narrow tiles and in BF16 the
  // 16 x 16 shapes measured as fast or faster
  if (rp > 64) return dma_config_by_id(bf16 ? 3 : 30);
  if (narrow) {
    if (pass1) return dma_config_by_id(rp == 16 ? 13 : rp == 32 ? 11 : 9);
    return dma_config_by_id(rp == 16 ? 14 : rp == 32 ? 12 : 10);
  }
  if (rp == 64 && !bf16) return dma_config_by_id(pass1 ? 26 : 27);
  if (pass1) return dma_config_by_id(rp == 16 ? 0 : rp == 32 ? 1 : 2);
  return dma_config_by_id(rp == 16 ? 4 : rp == 32 ? 5 : 6);
}

hipError_t launch_nt_dma(const DmaCfg& cfg, bool bf16, const void* X, int64_t ldx, int64_t M,
                         const void* Y, int64_t ldy, int64_t N, int64_t K, int splits,
                         int64_t kchunk, float* part, int64_t ldp, int64_t sp, const GramRed& gr,
                         hipStream_t st) {
  if (cfg.id < 0 || cfg.id >= kDmaCount) return hipErrorInvalidValue;
  const dim3 grid((unsigned)splits, (unsigned)((M + cfg.bm - 1) / cfg.bm),
                  (unsigned)((N + cfg.bn - 1) / cfg.bn));
  return bf16 ? kDma[cfg.id].bf16(X, ldx, Y, ldy, K, kchunk, part, ldp, sp, gr, grid, st)
              : kDma[cfg.id].f32(X, ldx, Y, ldy, K, kchunk, part, ldp, sp, gr, grid, st);
}

hipError_t launch_gemm_tn(const TnCfg& cfg, const float* A, int64_t lda, int64_t M,
                          const float* B, int64_t ldb, int64_t N, int64_t K, int splits,
                          int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                          const GramRed& gr, hipStream_t st) {
  if (cfg.id < 0 || cfg.id >= kTnCount) return hipErrorInvalidValue;
  return kTn[cfg.id].f32(A, lda, M, B, ldb, N, K, kchunk, part, ldp, sp, gr,
                         tiles3(M, N, cfg.bm, cfg.bn, splits), st);
}

hipError_t launch_reduce_gram(const float* part, int64_t ldp, int64_t sp, int splits, int rp,
                              float* G, uint16_t* Gbf, hipStream_t st) {
  const int64_t total = (int64_t)rp * rp / 4;
  hipLaunchKernelGGL(k_reduce_gram, dim3(grid1d(total, 64)), dim3(64), 0, st, part, ldp, sp,
                     splits, rp, G, Gbf);
  return hipGetLastError();
}

#define RP_SWITCH(RPV, CALL) \
  switch (RPV) {             \
    case 16: CALL(16); break; \
    case 32: CALL(32); break; \
    case 64: CALL(64); break; \
    case 128: CALL(128); break; \
    case 256: CALL(256); break; \
    default: return hipErrorInvalidValue; \
  }

// Rank entries per thread of k_update_w: 4 (1024 / KC rows per block), or 1
// (a quarter of the rows per block) when 4 would leave fewer than 256 blocks.
int update_w_kpt(int rp, int64_t p) {
  const int64_t per4 = 1024 / (rp < 64 ? rp : 64);
  return (p + per4 - 1) / per4 >= 256 ? 4 : 1;
}

int update_grid(int rp, int64_t extent, int cap, int kpt) {
  const int64_t per = kpt * 256 / (rp < 64 ? rp : 64);  // rows per block
  int64_t blocks = (extent + per - 1) / per;
  if (cap > 0 && blocks > cap) blocks = cap;
  return (int)(blocks < 1 ? 1 : blocks);
}

// Columns per block of k_update_h: 64, or 32 / 16 when that leaves fewer
// than 256 blocks (a small problem would otherwise occupy few CUs).
int update_h_cols(int64_t n) {
  if ((n + 63) / 64 >= 256) return 64;
  if ((n + 31) / 32 >= 256) return 32;
  return 16;
}

int update_h_grid(int64_t n, int cap, int cols) {
  int64_t blocks = (n + cols - 1) / cols;
  if (cap > 0 && blocks > cap) blocks = cap;
  return (int)(blocks < 1 ? 1 : blocks);
}

hipError_t launch_update_w(int rp, int64_t p, int r, const float* part, int64_t ldp, int64_t sp,
                           int splits, const float* G, float* Wp, float* Wcaller, float* WT,
                           uint16_t* WbT, int64_t ldwt, bool bf16, float* gout, int grid,
                           int kpt, bool gram_only, hipStream_t st) {
  if (rp == 256) {
    // matrix-core denominators (no Gram partials at this rank); rank 128
    // measured faster on the vector units below
    // 64-row blocks of 8 waves, or 32-row blocks of 4 when p is small
    const int wr = (p + 63) / 64 >= 256 ? 2 : 1;
    const dim3 g((unsigned)((p + 32 * wr - 1) / (32 * wr)));
#define UWM(R, WR)                                                                              \
  do {                                                                                          \
    if (bf16)                                                                                   \
      hipLaunchKernelGGL((k_update_w_mma<R, WR, true>), g, dim3(256 * WR), 0, st, p, r, part,    \
                         ldp, sp, splits, G, Wp, Wcaller, WT, WbT, ldwt);                       \
    else                                                                                        \
      hipLaunchKernelGGL((k_update_w_mma<R, WR, false>), g, dim3(256 * WR), 0, st, p, r, part,   \
                         ldp, sp, splits, G, Wp, Wcaller, WT, WbT, ldwt);                       \
  } while (0)
    if (wr == 2) UWM(256, 2);
    else UWM(256, 1);
#undef UWM
    return hipGetLastError();
  }
#define UW(R)                                                                                  \
  do {                                                                                          \
    if (kpt == 4)                                                                               \
      hipLaunchKernelGGL((k_update_w<R, 4>), dim3(grid), dim3(256), 0, st, p, r, part, ldp, sp,   \
                         splits, G, Wp, Wcaller, WT, WbT, ldwt, (int)bf16, gout, (int)gram_only); \
    else                                                                                        \
      hipLaunchKernelGGL((k_update_w<R, 1>), dim3(grid), dim3(256), 0, st, p, r, part, ldp, sp,   \
                         splits, G, Wp, Wcaller, WT, WbT, ldwt, (int)bf16, gout, (int)gram_only); \
  } while (0)
  switch (rp) {
    case 16: UW(16); break;
    case 32: UW(32); break;
    case 64: UW(64); break;
    case 128: UW(128); break;
    default: return hipErrorInvalidValue;
  }
#undef UW
  return hipGetLastError();
}

hipError_t launch_update_h(int rp, int64_t n, int r, const float* part, int64_t ldp, int64_t sp,
                           int splits, const float* G, float* Hp, int64_t ldh, float* Hcaller,
                           uint16_t* Hb, bool bf16, float* gout, int grid, int cols,
                           bool gram_only, hipStream_t st) {
  if (rp > 64) {
    // matrix-core denominators (no Gram partials at these ranks);
    // 128-column blocks of 8 waves, or 64-column blocks of 4 when n is small
    const int wc = (n + 127) / 128 >= 256 ? 2 : 1;
    const dim3 g((unsigned)((n + 64 * wc - 1) / (64 * wc)));
#define UHM(R, WC)                                                                               \
  do {                                                                                           \
    if (bf16)                                                                                    \
      hipLaunchKernelGGL((k_update_h_mma<R, WC, true>), g, dim3(256 * WC), 0, st, n, r, part,    \
                         ldp, sp, splits, G, Hp, ldh, Hcaller, Hb);                              \
    else                                                                                         \
      hipLaunchKernelGGL((k_update_h_mma<R, WC, false>), g, dim3(256 * WC), 0, st, n, r, part,   \
                         ldp, sp, splits, G, Hp, ldh, Hcaller, Hb);                              \
  } while (0)
    if (rp == 128 && wc == 2) UHM(128, 2);
    else if (rp == 128) UHM(128, 1);
    else if (rp == 256 && wc == 2) UHM(256, 2);
    else if (rp == 256) UHM(256, 1);
    else return hipErrorInvalidValue;
#undef UHM
    return hipGetLastError();
  }
#define UH(R)                                                                                  \
  do {                                                                                          \
    if (cols == 64)                                                                             \
      hipLaunchKernelGGL((k_update_h<R, 64>), dim3(grid), dim3(256), 0, st, n, r, part, ldp, sp, \
                         splits, G, Hp, ldh, Hcaller, Hb, (int)bf16, gout, (int)gram_only);     \
    else if (cols == 32)                                                                        \
      hipLaunchKernelGGL((k_update_h<R, 32>), dim3(grid), dim3(256), 0, st, n, r, part, ldp, sp, \
                         splits, G, Hp, ldh, Hcaller, Hb, (int)bf16, gout, (int)gram_only);     \
    else                                                                                        \
      hipLaunchKernelGGL((k_update_h<R, 16>), dim3(grid), dim3(256), 0, st, n, r, part, ldp, sp, \
                         splits, G, Hp, ldh, Hcaller, Hb, (int)bf16, gout, (int)gram_only);     \
  } while (0)
  switch (rp) {
    case 16: UH(16); break;
    case 32: UH(32); break;
    case 64: UH(64); break;
    default: return hipErrorInvalidValue;
  }
#undef UH
  return hipGetLastError();
}

int64_t objective_parts(int64_t p, int64_t n) { return ((p + 63) / 64) * ((n + 63) / 64); }

hipError_t launch_objective(int rp, const float* V, int64_t ldv, int64_t p, int64_t n,
                            const float* Wp, const float* Hp, int64_t ldh, double* part,
                            hipStream_t st) {
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((p + 63) / 64));
#define OBJ(R) \
  hipLaunchKernelGGL(k_objective<R>, grid, dim3(256), 0, st, V, ldv, p, n, Wp, Hp, ldh, part)
  RP_SWITCH(rp, OBJ)
#undef OBJ
  return hipGetLastError();
}

hipError_t launch_reduce_f64(const double* part, int64_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, st, part, count, out);
  return hipGetLastError();
}

hipError_t launch_copy_pad(const float* src, int64_t lds, int64_t rows, int64_t cols, float* dst,
                           int64_t ldd, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_pad, dim3(grid1d(rows * cols, 256)), dim3(256), 0, st, src, lds, rows,
                     cols, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* dst, int64_t count, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid1d(count, 256)), dim3(256), 0, st, dst, count, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* dst, int64_t count, uint32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid1d(count, 256)), dim3(256), 0, st, dst, count, v);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* src, int64_t lds, int64_t rows, int64_t cols,
                            uint16_t* dst, int64_t ldd, bool transpose, hipStream_t st) {
  const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_convert<uint16_t>, grid, dim3(256), 0, st, src, lds, rows, cols, dst, ldd,
                     (int)transpose);
  return hipGetLastError();
}

hipError_t launch_transpose_f32(const float* src, int64_t lds, int64_t rows, int64_t cols,
                                float* dst, int64_t ldd, hipStream_t st) {
  const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_convert<float>, grid, dim3(256), 0, st, src, lds, rows, cols, dst, ldd, 1);
  return hipGetLastError();
}

hipError_t launch_validate(const float* V, int64_t ldv, int64_t p, int64_t n, uint32_t* flag,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(grid1d(p * n, 256, 16384)), dim3(256), 0, st, V, ldv, p, n,
                     flag);
  return hipGetLastError();
}

hipError_t launch_gauge(float* W, int64_t p, int r, float* H, int64_t n, float* norms,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)r), dim3(256), 0, st, W, p, r, norms);
  hipLaunchKernelGGL(k_apply_gauge, dim3(grid1d(p * r + (int64_t)r * n, 256)), dim3(256), 0, st, W,
                     p, r, H, n, norms);
  return hipGetLastError();
}

hipError_t launch_ls_refit(const float* G, int rp, int r, int64_t p, const float* part, int64_t ldp,
                           int64_t sp, int splits, double* ginv, uint32_t* maxbits,
                           float floor_rel, float* Wp, float* Wcaller, hipStream_t st) {
  if (rp > 64 || r > rp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, maxbits, (int64_t)1, 0u);
  hipLaunchKernelGGL(k_ls_inverse, dim3(1), dim3(256), 0, st, G, rp, r, ginv);
  hipLaunchKernelGGL(k_ls_apply, dim3((unsigned)((p + 63) / 64)), dim3(256), 0, st, part, ldp, sp,
                     splits, ginv, rp, r, p, Wp, maxbits);
  hipLaunchKernelGGL(k_ls_clip, dim3(grid1d(p * r, 256)), dim3(256), 0, st, Wp, rp, r, p, maxbits,
                     floor_rel, Wcaller);
  return hipGetLastError();
}

hipError_t launch_uniform(float* dst, int64_t rows, int64_t cols, int64_t ldd, uint64_t seed,
                          uint32_t stream_id, hipStream_t st) {
  hipLaunchKernelGGL(k_uniform, dim3(grid1d(rows * cols, 256)), dim3(256), 0, st, dst, rows, cols,
                     ldd, (uint32_t)seed, (uint32_t)(seed >> 32), stream_id);
  return hipGetLastError();
}

}  // namespace nmfk
