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
#include <stdint.h>

#include "nmf_internal.h"

namespace nmfk {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even float -> bfloat16 bits (hardware conversion).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  __bf16 b = (__bf16)x;
  return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf16_val(float x) {
  return __builtin_bit_cast(float, (uint32_t)to_bf16(x) << 16);
}

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
// NT product, FP32:  part[s][m][c] = sum_{k in split s} X[m][k] * Y[c][k].
// Workgroup tile BM x BN, BK = 32 reduction slots per LDS stage, WM x WN
// waves each owning (16 MB) x (16 NB) outputs.  Each lane reads 4
// consecutive k of a row with one 128-bit LDS load and feeds them to four
// MFMAs (slot g of MFMA t is k = 4g + t), so A and B see the same k order.
// Grid: x = N tiles, y = M tiles, z = splits.
// ---------------------------------------------------------------------------
template <int MB, int NB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt(
    const float* __restrict__ X, int64_t ldx, int64_t M,
    const float* __restrict__ Y, int64_t ldy, int64_t N, int64_t K,
    int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp) {
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN, BK = 32, PITCH = BK + 4;
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
// BK = 64 bf16 per stage; a lane reads 8 consecutive k (one 128-bit LDS
// load) per operand per MFMA.
// ---------------------------------------------------------------------------
template <int MB, int NB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt_bf16(
    const uint16_t* __restrict__ X, int64_t ldx, int64_t M,
    const uint16_t* __restrict__ Y, int64_t ldy, int64_t N, int64_t K,
    int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp) {
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN, BK = 64, PITCH = BK + 8;
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

template <int MB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_tn(
    const float* __restrict__ A, int64_t lda, int64_t M,
    const float* __restrict__ B, int64_t ldb, int64_t N, int64_t K,
    int64_t kchunk, float* __restrict__ part, int64_t ldp, int64_t sp) {
  constexpr int NB = 4;
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN, BK = 32;
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
// Gram reduction: G[m][c] = sum_s part[s][m][c], s ascending.
// ---------------------------------------------------------------------------
__global__ void k_reduce_gram(const float* __restrict__ part, int64_t ldp,
                              int64_t sp, int splits, int rp,
                              float* __restrict__ G, uint16_t* __restrict__ Gbf) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rp * rp) return;
  const int64_t m = idx / rp, cc = idx % rp;
  float s = 0.f;
  for (int q = 0; q < splits; ++q) s += part[q * sp + m * ldp + cc];
  G[idx] = s;
  if (Gbf) Gbf[idx] = to_bf16(s);
}

// ---------------------------------------------------------------------------
// W half-step epilogue (eq. nnmf_v_update):
//   a_ik = sum_s part[s][i][k]                 (numerator (V H^T)_ik)
//   b_ik = sum_l w_il G_lk                     (denominator (W (H H^T))_ik)
//   w_ik <- w_ik * (a_ik / b_ik)  if b_ik > 0, else unchanged.
// A workgroup owns ROWS rows of W and all RP ranks; it snapshots its rows in
// LDS (rounded to bf16 in the BF16 tier, where the product takes bf16
// operands) and streams G through LDS in chunks of KC columns.
// ---------------------------------------------------------------------------
template <int RP>
__global__ __launch_bounds__(256) void k_update_w(
    int64_t p, int r, const float* __restrict__ part, int64_t ldp, int64_t sp,
    int splits, const float* __restrict__ G, float* __restrict__ Wp,
    float* __restrict__ Wc, uint16_t* __restrict__ WbT, int64_t ldwt,
    int bf16) {
  constexpr int ROWS = 32, KC = RP < 64 ? RP : 64;
  __shared__ float Ws[ROWS * RP];
  __shared__ float Gs[RP * KC];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * ROWS;

  for (int idx = tid; idx < ROWS * RP; idx += 256) {
    const int i = idx / RP, l = idx % RP;
    float w = (i0 + i < p) ? Wp[(i0 + i) * RP + l] : 0.f;
    Ws[idx] = bf16 ? bf16_val(w) : w;
  }
  for (int kc0 = 0; kc0 < RP; kc0 += KC) {
    __syncthreads();
    for (int idx = tid; idx < RP * KC; idx += 256) {
      const int l = idx / KC, kk = idx % KC;
      const float gv = G[l * RP + kc0 + kk];
      Gs[idx] = bf16 ? bf16_val(gv) : gv;
    }
    __syncthreads();
    for (int idx = tid; idx < ROWS * KC; idx += 256) {
      const int i = idx / KC, kk = idx % KC;
      const int64_t row = i0 + i;
      if (row >= p) continue;
      const int k = kc0 + kk;
      float b = 0.f;
#pragma unroll 8
      for (int l = 0; l < RP; ++l) b = fmaf(Ws[i * RP + l], Gs[l * KC + kk], b);
      float a = 0.f;
      for (int q = 0; q < splits; ++q) a += part[q * sp + row * ldp + k];
      const float w = Wp[row * RP + k];
      const float wn = (b > 0.f) ? w * (a / b) : w;
      Wp[row * RP + k] = wn;
      if (k < r) Wc[row * r + k] = wn;
      if (WbT) WbT[(int64_t)k * ldwt + row] = to_bf16(wn);
    }
  }
}

// ---------------------------------------------------------------------------
// H half-step epilogue (eq. nnmf_w_update), with the new W:
//   s_kj = sum_s part[s][k][j]                 (numerator (W^T V)_kj)
//   d_kj = sum_l G_kl h_lj                     (denominator ((W^T W) H)_kj)
//   h_kj <- h_kj * (s_kj / d_kj)  if d_kj > 0, else unchanged.
// A workgroup owns COLS columns of H and all RP ranks.
// ---------------------------------------------------------------------------
template <int RP>
__global__ __launch_bounds__(256) void k_update_h(
    int64_t n, int r, const float* __restrict__ part, int64_t ldp, int64_t sp,
    int splits, const float* __restrict__ G, float* __restrict__ Hp,
    int64_t ldh, float* __restrict__ Hc, uint16_t* __restrict__ Hb, int bf16) {
  constexpr int COLS = 64, KC = RP < 64 ? RP : 64;
  __shared__ float Hs[RP * COLS];
  __shared__ float Gs[KC * RP];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * COLS;

  for (int idx = tid; idx < RP * COLS; idx += 256) {
    const int l = idx / COLS, jj = idx % COLS;
    const float h = Hp[(int64_t)l * ldh + j0 + jj];
    Hs[idx] = bf16 ? bf16_val(h) : h;
  }
  for (int kc0 = 0; kc0 < RP; kc0 += KC) {
    __syncthreads();
    for (int idx = tid; idx < KC * RP; idx += 256) {
      const float gv = G[(int64_t)kc0 * RP + idx];
      Gs[idx] = bf16 ? bf16_val(gv) : gv;
    }
    __syncthreads();
    for (int idx = tid; idx < KC * COLS; idx += 256) {
      const int kk = idx / COLS, jj = idx % COLS;
      const int64_t j = j0 + jj;
      if (j >= n) continue;
      const int k = kc0 + kk;
      float d = 0.f;
#pragma unroll 8
      for (int l = 0; l < RP; ++l) d = fmaf(Gs[kk * RP + l], Hs[l * COLS + jj], d);
      float s = 0.f;
      for (int q = 0; q < splits; ++q) s += part[q * sp + (int64_t)k * ldp + j];
      const float h = Hp[(int64_t)k * ldh + j];
      const float hn = (d > 0.f) ? h * (s / d) : h;
      Hp[(int64_t)k * ldh + j] = hn;
      if (k < r) Hc[(int64_t)k * n + j] = hn;
      if (Hb) Hb[(int64_t)k * ldh + j] = to_bf16(hn);
    }
  }
}

// ---------------------------------------------------------------------------
// Objective partials (eq. nnmf-objfn), direct residual in float64:
// each 64 x 64 tile accumulates sum (v_ij - sum_k w_ik h_kj)^2 with the
// inner products formed by float64 FMAs of the float32 factors.  A thread
// owns a 4 x 4 block; the tile total is reduced in a fixed order.
// Wp == nullptr means W = 0 (gives ||V||_F^2).
// ---------------------------------------------------------------------------
template <int RP>
__global__ __launch_bounds__(256) void k_objective(
    const float* __restrict__ V, int64_t ldv, int64_t p, int64_t n,
    const float* __restrict__ Wp, const float* __restrict__ Hp, int64_t ldh,
    double* __restrict__ part) {
  constexpr int KC = RP < 64 ? RP : 64;
  __shared__ __attribute__((aligned(16))) float WsT[KC * 64];
  __shared__ __attribute__((aligned(16))) float Hs[KC * 64];
  __shared__ double red[4];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;

  double s[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) s[a][b] = 0.0;

  if (Wp) {
    for (int kc0 = 0; kc0 < RP; kc0 += KC) {
      __syncthreads();
      for (int idx = tid; idx < 64 * KC; idx += 256) {
        const int ii = idx / KC, kk = idx % KC;
        WsT[kk * 64 + ii] = Wp[(i0 + ii) * RP + kc0 + kk];
      }
      for (int idx = tid; idx < KC * 64; idx += 256) {
        const int kk = idx / 64, jj = idx % 64;
        Hs[idx] = Hp[(int64_t)(kc0 + kk) * ldh + j0 + jj];
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < KC; ++kk) {
        const float4 w = *reinterpret_cast<const float4*>(&WsT[kk * 64 + 4 * ty]);
        const float4 h = *reinterpret_cast<const float4*>(&Hs[kk * 64 + 4 * tx]);
        const double wd[4] = {(double)w.x, (double)w.y, (double)w.z, (double)w.w};
        const double hd[4] = {(double)h.x, (double)h.y, (double)h.z, (double)h.w};
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
    const float4 v = load4(V, ldv, row, p, col, n);
    const float vv[4] = {v.x, v.y, v.z, v.w};
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
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t q = tid; q < count; q += 256) s += part[q];
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

// Cast to bf16 through a 32 x 32 LDS tile; with `transpose` the tile is
// written out transposed so both reads and writes stay coalesced.
__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src,
                                                   int64_t lds, int64_t rows,
                                                   int64_t cols, uint16_t* __restrict__ dst,
                                                   int64_t ldd, int transpose) {
  __shared__ uint16_t t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int q = 0; q < 4; ++q) {
    const int64_t i = r0 + ty + 8 * q, j = c0 + tx;
    uint16_t h = 0;
    if (i < rows && j < cols) h = to_bf16(src[i * lds + j]);
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
// NT instances: id -> (MB, NB, WM, WN)
//  0: 2,1,4,1 (128 x 16)   1: 2,2,4,1 (128 x 32)   2: 2,4,4,1 (128 x 64)
//  3: 4,4,2,2 (128 x 128)  4: 1,1,1,1 (16 x 16)    5: 2,2,1,1 (32 x 32)
//  6: 2,2,2,2 (64 x 64)    7: 1,4,1,4 (16 x 256)   8: 2,4,1,4 (32 x 256)
//  9: 4,4,1,4 (64 x 256)
static const int kNt[10][4] = {{2, 1, 4, 1}, {2, 2, 4, 1}, {2, 4, 4, 1}, {4, 4, 2, 2},
                               {1, 1, 1, 1}, {2, 2, 1, 1}, {2, 2, 2, 2}, {1, 4, 1, 4},
                               {2, 4, 1, 4}, {4, 4, 1, 4}};

static NtCfg make_nt(int id) {
  NtCfg c;
  c.id = id;
  c.bm = 16 * kNt[id][0] * kNt[id][2];
  c.bn = 16 * kNt[id][1] * kNt[id][3];
  c.threads = 64 * kNt[id][2] * kNt[id][3];
  return c;
}

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

// TN instances: id -> (MB, WM, WN); tile (16 MB WM) x (64 WN)
//  0: 1,1,4 (16 x 256)  1: 2,1,4 (32 x 256)  2: 4,1,4 (64 x 256)
//  3: 4,2,2 (128 x 128) 4: 1,1,1 (16 x 64)   5: 2,1,1 (32 x 64)
//  6: 4,1,1 (64 x 64)
static const int kTn[7][3] = {{1, 1, 4}, {2, 1, 4}, {4, 1, 4}, {4, 2, 2},
                              {1, 1, 1}, {2, 1, 1}, {4, 1, 1}};

static TnCfg make_tn(int id) {
  TnCfg c;
  c.id = id;
  c.bm = 16 * kTn[id][0] * kTn[id][1];
  c.bn = 64 * kTn[id][2];
  c.threads = 64 * kTn[id][1] * kTn[id][2];
  return c;
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

#define NT_CASE(ID, KERN, T)                                                          \
  case ID:                                                                           \
    hipLaunchKernelGGL((KERN<kNtArgs##ID>), grid, dim3(cfg.threads), 0, st, X, ldx, M, \
                       Y, ldy, N, K, kchunk, part, ldp, sp);                          \
    break;

#define kNtArgs0 2, 1, 4, 1
#define kNtArgs1 2, 2, 4, 1
#define kNtArgs2 2, 4, 4, 1
#define kNtArgs3 4, 4, 2, 2
#define kNtArgs4 1, 1, 1, 1
#define kNtArgs5 2, 2, 1, 1
#define kNtArgs6 2, 2, 2, 2
#define kNtArgs7 1, 4, 1, 4
#define kNtArgs8 2, 4, 1, 4
#define kNtArgs9 4, 4, 1, 4

hipError_t launch_gemm_nt(const NtCfg& cfg, const float* X, int64_t ldx, int64_t M,
                          const float* Y, int64_t ldy, int64_t N, int64_t K, int splits,
                          int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                          hipStream_t st) {
  const dim3 grid = tiles3(M, N, cfg.bm, cfg.bn, splits);
  switch (cfg.id) {
    NT_CASE(0, k_gemm_nt, float)
    NT_CASE(1, k_gemm_nt, float)
    NT_CASE(2, k_gemm_nt, float)
    NT_CASE(3, k_gemm_nt, float)
    NT_CASE(4, k_gemm_nt, float)
    NT_CASE(5, k_gemm_nt, float)
    NT_CASE(6, k_gemm_nt, float)
    NT_CASE(7, k_gemm_nt, float)
    NT_CASE(8, k_gemm_nt, float)
    NT_CASE(9, k_gemm_nt, float)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_nt_bf16(const NtCfg& cfg, const uint16_t* X, int64_t ldx, int64_t M,
                               const uint16_t* Y, int64_t ldy, int64_t N, int64_t K,
                               int splits, int64_t kchunk, float* part, int64_t ldp,
                               int64_t sp, hipStream_t st) {
  const dim3 grid = tiles3(M, N, cfg.bm, cfg.bn, splits);
  switch (cfg.id) {
    NT_CASE(0, k_gemm_nt_bf16, uint16_t)
    NT_CASE(1, k_gemm_nt_bf16, uint16_t)
    NT_CASE(2, k_gemm_nt_bf16, uint16_t)
    NT_CASE(3, k_gemm_nt_bf16, uint16_t)
    NT_CASE(4, k_gemm_nt_bf16, uint16_t)
    NT_CASE(5, k_gemm_nt_bf16, uint16_t)
    NT_CASE(6, k_gemm_nt_bf16, uint16_t)
    NT_CASE(7, k_gemm_nt_bf16, uint16_t)
    NT_CASE(8, k_gemm_nt_bf16, uint16_t)
    NT_CASE(9, k_gemm_nt_bf16, uint16_t)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define TN_CASE(ID, MB, WM, WN)                                                         \
  case ID:                                                                             \
    hipLaunchKernelGGL((k_gemm_tn<MB, WM, WN>), grid, dim3(cfg.threads), 0, st, A, lda, \
                       M, B, ldb, N, K, kchunk, part, ldp, sp);                         \
    break;

hipError_t launch_gemm_tn(const TnCfg& cfg, const float* A, int64_t lda, int64_t M,
                          const float* B, int64_t ldb, int64_t N, int64_t K, int splits,
                          int64_t kchunk, float* part, int64_t ldp, int64_t sp,
                          hipStream_t st) {
  const dim3 grid = tiles3(M, N, cfg.bm, cfg.bn, splits);
  switch (cfg.id) {
    TN_CASE(0, 1, 1, 4)
    TN_CASE(1, 2, 1, 4)
    TN_CASE(2, 4, 1, 4)
    TN_CASE(3, 4, 2, 2)
    TN_CASE(4, 1, 1, 1)
    TN_CASE(5, 2, 1, 1)
    TN_CASE(6, 4, 1, 1)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_gram(const float* part, int64_t ldp, int64_t sp, int splits, int rp,
                              float* G, uint16_t* Gbf, hipStream_t st) {
  const int64_t total = (int64_t)rp * rp;
  hipLaunchKernelGGL(k_reduce_gram, dim3(grid1d(total, 256)), dim3(256), 0, st, part, ldp, sp,
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

hipError_t launch_update_w(int rp, int64_t p, int r, const float* part, int64_t ldp, int64_t sp,
                           int splits, const float* G, float* Wp, float* Wcaller,
                           uint16_t* WbT, int64_t ldwt, bool bf16, hipStream_t st) {
  const dim3 grid((unsigned)((p + 31) / 32));
#define UW(R)                                                                                 \
  hipLaunchKernelGGL(k_update_w<R>, grid, dim3(256), 0, st, p, r, part, ldp, sp, splits, G, Wp, \
                     Wcaller, WbT, ldwt, (int)bf16)
  RP_SWITCH(rp, UW)
#undef UW
  return hipGetLastError();
}

hipError_t launch_update_h(int rp, int64_t n, int r, const float* part, int64_t ldp, int64_t sp,
                           int splits, bool transposed, const float* G, float* Hp, int64_t ldh,
                           float* Hcaller, uint16_t* Hb, bool bf16, hipStream_t st) {
  if (transposed) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 63) / 64));
#define UH(R)                                                                                 \
  hipLaunchKernelGGL(k_update_h<R>, grid, dim3(256), 0, st, n, r, part, ldp, sp, splits, G, Hp, \
                     ldh, Hcaller, Hb, (int)bf16)
  RP_SWITCH(rp, UH)
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
  hipLaunchKernelGGL(k_cast_bf16, grid, dim3(256), 0, st, src, lds, rows, cols, dst, ldd,
                     (int)transpose);
  return hipGetLastError();
}

hipError_t launch_validate(const float* V, int64_t ldv, int64_t p, int64_t n, uint32_t* flag,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(grid1d(p * n, 256, 16384)), dim3(256), 0, st, V, ldv, p, n,
                     flag);
  return hipGetLastError();
}

hipError_t launch_uniform(float* dst, int64_t rows, int64_t cols, int64_t ldd, uint64_t seed,
                          uint32_t stream_id, hipStream_t st) {
  hipLaunchKernelGGL(k_uniform, dim3(grid1d(rows * cols, 256)), dim3(256), 0, st, dst, rows, cols,
                     ldd, (uint32_t)seed, (uint32_t)(seed >> 32), stream_id);
  return hipGetLastError();
}

}  // namespace nmfk
