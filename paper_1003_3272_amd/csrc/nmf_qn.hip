// gfx950 kernels of the quasi-Newton acceleration QN(q) (Zhou, Alexander &
// Lange 2011, cited in the Discussion of the paper) of the multiplicative
// NMF map F (one iteration of Algorithm 1).
//
// The state vector x is the context's padded factor pair [Wp | Hp] (ppad x
// rp, then rp x npad, contiguous; padding is zero in every vector).  One QN
// iteration, entirely on the device so that it can be replayed as a graph:
//   x0 = x;  x1 = F(x0);  x2 = F(x1)                  (the MM kernels)
//   u_s = x1 - x0, v_s = x2 - x1 in slot s of rings U, V (float64)
//   the new row/column of U^T U and U^T V (3q dot products, float64)
//   c = (U^T U - U^T V)^-1 U^T u_s  (q x q, float64, partial pivoting)
//   xq = max(x1 + V c, kappa x1)      (the projected quasi-Newton point)
//   f(x2), f(xq) by the objective kernels; take xq iff the system was
//   regular, xq feasible and f(xq) <= f(x2); else keep x2
//   commit: the chosen point's derived copies (caller's W, H, W^T, bf16)
// Every decision is read from device memory by the kernels that depend on
// it, so the sequence of launches never changes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmf_device.h"
#include "nmf_internal.h"

namespace nmfk {
namespace {

constexpr int kQnMax = 16;      // largest q
constexpr int kDotBlocks = 256;  // partial-sum blocks of the dot products

// st[0]: QN iterations done; st[1]: accepted; st[2]: regular system;
// st[3]: infeasible point seen; st[4]: take.
__global__ void k_qn_pairs(const float* __restrict__ x0, const float* __restrict__ x1,
                           const float* __restrict__ x2, double* __restrict__ U,
                           double* __restrict__ V, int64_t D, int q,
                           const int32_t* __restrict__ st) {
  const int s = st[0] % q;
  double* u = U + (int64_t)s * D;
  double* v = V + (int64_t)s * D;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * 256) {
    const double a = x0[i], b = x1[i], c = x2[i];
    u[i] = b - a;  // differences of two floats: exact in float64
    v[i] = c - b;
  }
}

// Partial sums (per block, fixed order) of u_s . u_j, u_s . v_j and
// u_j . v_s for every slot j < q: dpart[block][3 q].  Each wave reduces its
// 3q sums with lane shuffles; thread k < 3q then adds the four waves' sums
// in wave order.
__global__ __launch_bounds__(256) void k_qn_dots(const double* __restrict__ U,
                                                 const double* __restrict__ V, int64_t D, int q,
                                                 const int32_t* __restrict__ st,
                                                 double* __restrict__ dpart) {
  __shared__ double sh[4][3 * kQnMax];
  const int s = st[0] % q;
  const double* us = U + (int64_t)s * D;
  const double* vs = V + (int64_t)s * D;
  double acc[3 * kQnMax];
#pragma unroll
  for (int k = 0; k < 3 * kQnMax; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * 256) {
    const double a = us[i], b = vs[i];
#pragma unroll
    for (int j = 0; j < kQnMax; ++j) {
      if (j < q) {
        const double uj = U[(int64_t)j * D + i], vj = V[(int64_t)j * D + i];
        acc[3 * j + 0] = fma(a, uj, acc[3 * j + 0]);
        acc[3 * j + 1] = fma(a, vj, acc[3 * j + 1]);
        acc[3 * j + 2] = fma(uj, b, acc[3 * j + 2]);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3 * kQnMax; ++k) {
    if (k < 3 * q) {
      double v = acc[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) sh[wave][k] = v;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 3 * q)
    dpart[(int64_t)blockIdx.x * 3 * q + t] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
}

// One wave: thread t < 3q finishes dot product t (blocks in order); the
// slot's row and column of U^T U (symmetric) and U^T V are updated; then
// (U^T U - U^T V) c = U^T u_s is solved over the filled slots by Gaussian
// elimination with partial pivoting, the matrix in LDS and each elimination
// step spread over the lanes.  A pivot below 1e-12 of the largest |entry|
// marks the system singular (c = 0, st[2] = 0).  Clears st[3] for the
// combine.
__global__ __launch_bounds__(64) void k_qn_solve(const double* __restrict__ dpart, int nblocks,
                                                 int q, int32_t* __restrict__ st,
                                                 double* __restrict__ GUU,
                                                 double* __restrict__ GUV,
                                                 double* __restrict__ coef) {
  __shared__ double dots[3 * kQnMax];
  __shared__ double A[kQnMax][kQnMax + 1];
  __shared__ double fct[kQnMax];
  __shared__ double x[kQnMax];
  __shared__ int piv_s, ok_s;
  if (blockIdx.x != 0) return;
  const int t = threadIdx.x;
  const int s = st[0] % q;
  const int m = st[0] + 1 < q ? st[0] + 1 : q;  // filled slots: 0 .. m - 1
  if (t < 3 * q) {
    double a = 0.0;
    for (int k = 0; k < nblocks; ++k) a += dpart[(int64_t)k * 3 * q + t];
    dots[t] = a;
  }
  __syncthreads();
  if (t < q) {
    const double a = dots[3 * t + 0], b = dots[3 * t + 1], c = dots[3 * t + 2];
    GUU[s * kQnMax + t] = a;
    GUU[t * kQnMax + s] = a;
    GUV[s * kQnMax + t] = b;
    GUV[t * kQnMax + s] = c;
  }
  // the system, with row and column s taken from the fresh dot products
  // (the entries stored above are read by later launches only)
  double amax = 0.0;
  for (int idx = t; idx < m * (m + 1); idx += 64) {
    const int i = idx / (m + 1), j = idx % (m + 1);
    double v;
    if (j == m) {
      v = dots[3 * i + 0];  // (U^T u_s)_i = u_i . u_s
    } else {
      if (i == s)
        v = dots[3 * j + 0] - dots[3 * j + 1];  // u_s . u_j - u_s . v_j
      else if (j == s)
        v = dots[3 * i + 0] - dots[3 * i + 2];  // u_i . u_s - u_i . v_s
      else
        v = GUU[i * kQnMax + j] - GUV[i * kQnMax + j];
      amax = fmax(amax, fabs(v));
    }
    A[i][j] = v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  if (t == 0) ok_s = amax > 0.0 && isfinite(amax);
  __syncthreads();
  for (int col = 0; col < m; ++col) {
    if (!ok_s) break;  // uniform: read after a barrier
    if (t == 0) {
      int piv = col;
      for (int i = col + 1; i < m; ++i)
        if (fabs(A[i][col]) > fabs(A[piv][col])) piv = i;
      piv_s = piv;
      if (!(fabs(A[piv][col]) > 1e-12 * amax)) ok_s = 0;
    }
    __syncthreads();
    if (!ok_s) break;
    const int piv = piv_s;
    if (piv != col && t >= col && t <= m) {
      const double tmp = A[col][t];
      A[col][t] = A[piv][t];
      A[piv][t] = tmp;
    }
    __syncthreads();
    if (t > col && t < m) fct[t] = A[t][col] / A[col][col];
    __syncthreads();
    for (int idx = t; idx < (m - col - 1) * (m - col); idx += 64) {
      const int i = col + 1 + idx / (m - col), j = col + 1 + idx % (m - col);
      A[i][j] -= fct[i] * A[col][j];
    }
    __syncthreads();
  }
  if (t == 0) {
    int ok = ok_s;
    for (int i = 0; i < kQnMax; ++i) x[i] = 0.0;
    if (ok) {
      for (int i = m - 1; i >= 0; --i) {
        double v = A[i][m];
        for (int j = i + 1; j < m; ++j) v -= A[i][j] * x[j];
        x[i] = v / A[i][i];
      }
      for (int i = 0; i < m; ++i) ok = ok && isfinite(x[i]);
    }
    for (int j = 0; j < kQnMax; ++j) coef[j] = ok ? x[j] : 0.0;
    st[2] = ok;
    st[3] = 0;
  }
}

// xq = max(x1 + sum_j c_j v_j, kappa x1) in float64, rounded to float32 (x1
// itself when the system was singular); st[3] = 1 if xq is infeasible
// (negative, or zero where x1 is positive).
__global__ void k_qn_combine(const float* __restrict__ x1, const double* __restrict__ V,
                             const double* __restrict__ coef, int64_t D, int q, float kappa,
                             int32_t* __restrict__ st, float* __restrict__ xq) {
  const bool ok = st[2] != 0;
  double c[kQnMax];
#pragma unroll
  for (int j = 0; j < kQnMax; ++j) c[j] = coef[j];
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * 256) {
    const double b = x1[i];
    double y = b;
    if (ok) {
#pragma unroll
      for (int j = 0; j < kQnMax; ++j)
        if (j < q) y = fma(c[j], V[(int64_t)j * D + i], y);
      y = fmax(y, (double)kappa * b);
    }
    const float yf = (float)y;
    xq[i] = yf;
    bad |= (yf < 0.f) || (yf == 0.f && b > 0.0) || !(yf == yf);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st[3], 1);
}

// Decision: take xq iff the system was regular, xq feasible and f(xq) <=
// f(x2).  Records the accepted objective for iteration st[0] in fout
// (host-visible, cap entries), then advances the counters.
__global__ void k_qn_select(const double* __restrict__ fvals, int32_t* __restrict__ st,
                            double* __restrict__ fout, int32_t cap) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double f2 = fvals[0], fq = fvals[1];
  const int take = st[2] != 0 && st[3] == 0 && fq <= f2;
  st[4] = take;
  if (st[0] < cap) fout[st[0]] = take ? fq : f2;
  st[0] += 1;
  st[1] += take;
}

// If xq was taken: x = xq, and its derived copies: the caller's W (p x r)
// and H (r x n), and W^T (float32, pitch ldwt) or bf16(W^T) and bf16(H).
__global__ void k_qn_commit(const int32_t* __restrict__ st, const float* __restrict__ xq,
                            float* __restrict__ Wp, int64_t ppad, int rp, int64_t npad,
                            int64_t p, int r, int64_t n, float* __restrict__ Wc,
                            float* __restrict__ Hc, float* __restrict__ WT,
                            uint16_t* __restrict__ WbT, int64_t ldwt, uint16_t* __restrict__ Hb) {
  if (st[4] == 0) return;
  const int64_t dw = ppad * rp, D = dw + (int64_t)rp * npad;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * 256) {
    const float y = xq[i];
    Wp[i] = y;  // Hp follows Wp contiguously
    if (i < dw) {
      const int64_t row = i / rp;
      const int k = (int)(i % rp);
      if (row < p && k < r) Wc[row * r + k] = y;
      if (WT) WT[(int64_t)k * ldwt + row] = y;
      if (WbT) WbT[(int64_t)k * ldwt + row] = to_bf16(y);
    } else {
      const int64_t j2 = i - dw;
      const int k = (int)(j2 / npad);
      const int64_t j = j2 % npad;
      if (k < r && j < n) Hc[(int64_t)k * n + j] = y;
      if (Hb) Hb[j2] = to_bf16(y);
    }
  }
}

__global__ void k_qn_copy(const float* __restrict__ src, float* __restrict__ dst, int64_t D4) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < D4;
       i += (int64_t)gridDim.x * 256)
    reinterpret_cast<float4*>(dst)[i] = reinterpret_cast<const float4*>(src)[i];
}

unsigned qblocks(int64_t total, int64_t cap = 1024) {
  const int64_t b = (total + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

int qn_max_q() { return kQnMax; }
int qn_dot_blocks() { return kDotBlocks; }

hipError_t launch_qn_copy(const float* src, float* dst, int64_t D, hipStream_t st) {
  if (D % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qn_copy, dim3(qblocks(D / 4)), dim3(256), 0, st, src, dst, D / 4);
  return hipGetLastError();
}

hipError_t launch_qn_pairs(const float* x0, const float* x1, const float* x2, double* U,
                           double* V, int64_t D, int q, const int32_t* state, hipStream_t st) {
  hipLaunchKernelGGL(k_qn_pairs, dim3(qblocks(D)), dim3(256), 0, st, x0, x1, x2, U, V, D, q,
                     state);
  return hipGetLastError();
}

hipError_t launch_qn_dots_solve(const double* U, const double* V, int64_t D, int q,
                                int32_t* state, double* dpart, double* GUU, double* GUV,
                                double* coef, hipStream_t st) {
  if (q < 1 || q > kQnMax) return hipErrorInvalidValue;
  const unsigned blocks = qblocks(D, kDotBlocks);  // at most kDotBlocks rows of dpart
  hipLaunchKernelGGL(k_qn_dots, dim3(blocks), dim3(256), 0, st, U, V, D, q, state, dpart);
  hipLaunchKernelGGL(k_qn_solve, dim3(1), dim3(64), 0, st, dpart, (int)blocks, q, state, GUU,
                     GUV, coef);
  return hipGetLastError();
}

hipError_t launch_qn_combine(const float* x1, const double* V, const double* coef, int64_t D,
                             int q, float kappa, int32_t* state, float* xq, hipStream_t st) {
  hipLaunchKernelGGL(k_qn_combine, dim3(qblocks(D)), dim3(256), 0, st, x1, V, coef, D, q, kappa,
                     state, xq);
  return hipGetLastError();
}

hipError_t launch_qn_select(const double* fvals, int32_t* state, double* fout, int32_t cap,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_qn_select, dim3(1), dim3(64), 0, st, fvals, state, fout, cap);
  return hipGetLastError();
}

hipError_t launch_qn_commit(const int32_t* state, const float* xq, float* Wp, int64_t ppad, int rp,
                            int64_t npad, int64_t p, int r, int64_t n, float* Wc, float* Hc,
                            float* WT, uint16_t* WbT, int64_t ldwt, uint16_t* Hb,
                            hipStream_t st) {
  const int64_t D = ppad * rp + (int64_t)rp * npad;
  hipLaunchKernelGGL(k_qn_commit, dim3(qblocks(D)), dim3(256), 0, st, state, xq, Wp, ppad, rp,
                     npad, p, r, n, Wc, Hc, WT, WbT, ldwt, Hb);
  return hipGetLastError();
}

}  // namespace nmfk
