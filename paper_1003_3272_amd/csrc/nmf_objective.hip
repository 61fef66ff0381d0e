// gfx950 float64 objective of the Euclidean update (eq. nnmf-objfn):
// partials of ||V - W H||_F^2, one double per 64 x 64 tile, the inner
// products formed on the float64 matrix cores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmf_device.h"
#include "nmf_internal.h"

namespace nmfk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// The same objective partials with W H formed on the float64 matrix cores
// (v_mfma_f64_16x16x4f64; the float64 vector and matrix peaks are equal,
// but one MFMA does 1024 multiply-adds per wave from one operand register
// pair per lane, so the issue and LDS overheads of the scalar form vanish).
// A workgroup covers a 64 x 64 tile with 4 waves of 32 x 32 (2 x 2 blocks of
// 16 x 16).  Lane (c, g) supplies row c of the A block and column c of the
// B block for k-slot g, and holds D[g + 4 v][c] of each block (the float64
// layout; the float32 16x16 MFMAs hold rows 4 g + v).  Within a
// group of 4 k-steps lane g takes k = 4 g + s at step s, so its W values
// are one 16-byte LDS read per group (the k order inside a dot product
// differs from the scalar form only in float64 rounding).  Each lane's 16
// V values are loaded before the products; the tile total is reduced in a
// fixed order.  Wp == nullptr means W = 0 (gives ||V||_F^2).
template <int RP>
__global__ __launch_bounds__(256) void k_objective_mma(
    const float* __restrict__ V, int64_t ldv, int64_t p, int64_t n,
    const float* __restrict__ Wp, const float* __restrict__ Hp, int64_t ldh,
    double* __restrict__ part) {
  constexpr int KC = RP < 64 ? RP : 64;
  constexpr int WP = KC + 4;  // W row pitch (16-byte aligned rows)
  constexpr int HP = 64 + 4;  // H row pitch
  __shared__ __attribute__((aligned(16))) float Ws[64 * WP];
  __shared__ __attribute__((aligned(16))) float Hs[KC * HP];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int wr = wave & 1, wc = wave >> 1;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;

  float vv[2][2][4];  // V at this lane's 16 outputs
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = i0 + 32 * wr + 16 * bi + g + 4 * v;
        const int64_t col = j0 + 32 * wc + 16 * bj + c;
        vv[bi][bj][v] = (row < p && col < n) ? V[row * ldv + col] : 0.f;
      }

  v4d acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};

  if (Wp) {
    for (int kc0 = 0; kc0 < RP; kc0 += KC) {
      __syncthreads();
      for (int idx = tid; idx < 64 * KC / 4; idx += 256) {
        const int ii = idx / (KC / 4), k4 = 4 * (idx % (KC / 4));
        *reinterpret_cast<float4*>(&Ws[ii * WP + k4]) =
            *reinterpret_cast<const float4*>(&Wp[(i0 + ii) * RP + kc0 + k4]);
      }
      for (int idx = tid; idx < KC * 64 / 4; idx += 256) {
        const int kk = idx / 16, j4 = 4 * (idx % 16);
        *reinterpret_cast<float4*>(&Hs[kk * HP + j4]) =
            *reinterpret_cast<const float4*>(&Hp[(int64_t)(kc0 + kk) * ldh + j0 + j4]);
      }
      __syncthreads();
#pragma unroll 2
      for (int k0 = 0; k0 < KC; k0 += 16) {
        float4 wa[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
          wa[bi] = *reinterpret_cast<const float4*>(&Ws[(32 * wr + 16 * bi + c) * WP + k0 + 4 * g]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int kk = k0 + 4 * g + s;
          double hb[2];
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) hb[bj] = Hs[kk * HP + 32 * wc + 16 * bj + c];
#pragma unroll
          for (int bi = 0; bi < 2; ++bi) {
            const double a = (double)(s == 0 ? wa[bi].x : s == 1 ? wa[bi].y : s == 2 ? wa[bi].z
                                                                                   : wa[bi].w);
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
              acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, hb[bj], acc[bi][bj], 0, 0, 0);
          }
        }
      }
    }
  }

  double sum = 0.0;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double e = (double)vv[bi][bj][v] - acc[bi][bj][v];
        sum = fma(e, e, sum);  // padded entries have v = 0 and W H = 0
      }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (lane == 0) red[wave] = sum;
  __syncthreads();
  if (tid == 0)
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

hipError_t launch_objective_mma(int rp, const float* V, int64_t ldv, int64_t p, int64_t n,
                                const float* Wp, const float* Hp, int64_t ldh, double* part,
                                hipStream_t st) {
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((p + 63) / 64));
#define OBJ(R)                                                                                 \
  case R:                                                                                      \
    hipLaunchKernelGGL(k_objective_mma<R>, grid, dim3(256), 0, st, V, ldv, p, n, Wp, Hp, ldh, \
                       part);                                                                  \
    break;
  switch (rp) {
    OBJ(16)
    OBJ(32)
    OBJ(64)
    OBJ(128)
    OBJ(256)
    default:
      return hipErrorInvalidValue;
  }
#undef OBJ
  return hipGetLastError();
}

}  // namespace nmfk
