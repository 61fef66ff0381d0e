// gfx950 kernels of the Poisson (Kullback-Leibler) multiplicative update,
// Sec. 3.1, last display.  With B = W H the objective to be maximized is
//   L(W, H) = sum_ij [v_ij ln b_ij - b_ij]
// and one iteration updates W and H simultaneously, both from iteration n:
//   w_ik <- w_ik sqrt( sum_j r_ij h_kj / sum_j h_kj )
//   h_kj <- h_kj sqrt( sum_i r_ij w_ik / sum_i w_ik ),   r_ij = v_ij / b_ij
// (r_ij = 0 where v_ij = 0; a zero denominator keeps the entry).
//
// The two numerators are V-streaming products like the Euclidean ones, on
// the same LDS copy ring, with V replaced by R = V / B: pass 1 forms
// R H^T over V's rows, pass 2 W^T R over V^T's rows.  R is never stored.
// Each workgroup holds all padded ranks of the factor it streams (H in pass
// 1, W^T in pass 2), so every wave recomputes the B values of its own data
// rows on the matrix cores from the staged factor rows and from the other
// factor's rows for those data rows, kept in registers.  The B block comes
// out of the MFMA in exactly the lane layout of the data fragment it divides
// (lane (c, g), register v: data row c, k = 16 kk + 4 g + v), so R is formed
// in registers and fed straight to the numerator MFMAs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmf_device.h"
#include "nmf_internal.h"

namespace nmfk {
namespace {

// part[s][m][c] = sum_{k in split s} X'[m][k] Y'[c][k] where the data
// operand (X for DX, else Y) is replaced by data / B.  The factor operand
// (Y for DX, else X) has all RP padded ranks in the tile.  G holds the
// other factor: DX: W (row-major, pitch ldg: G[datarow * ldg + l]); !DX:
// H (rank-major, pitch ldg: G[l * ldg + datacol]).
template <int MB, int NB, int WM, int WN, int S, bool DX>
__global__ __launch_bounds__(64 * WM * WN) void k_kl_pass(
    const float* __restrict__ Xf, int64_t ldx, const float* __restrict__ Yf, int64_t ldy,
    int64_t K, int64_t kchunk, const float* __restrict__ G, int64_t ldg,
    float* __restrict__ part, int64_t ldp, int64_t sp) {
  constexpr int BM = 16 * MB * WM, BN = 16 * NB * WN, ROWS = BM + BN;
  constexpr int W = WM * WN;
  constexpr int RP = DX ? BN : BM;   // factor rows in the tile: every rank
  constexpr int ND = DX ? MB : NB;   // data blocks of 16 rows per wave
  constexpr int FR0 = DX ? BM : 0;   // first factor row of a stage
  static_assert(ROWS % (8 * W) == 0, "stage rows must split evenly over the waves");
  constexpr int L = ROWS / (8 * W);
  constexpr int STAGE = ROWS * 128;
  __shared__ __attribute__((aligned(1024))) char lds[S * STAGE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int c = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)blockIdx.z * BN;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t kb = (int64_t)blockIdx.x * kchunk;
  const int64_t ke = (K < kb + kchunk) ? K : kb + kchunk;
  const int nst = (int)((ke - kb) / 32);

  const char* X = reinterpret_cast<const char*>(Xf);
  const char* Y = reinterpret_cast<const char*>(Yf);
  const int chunk = (lane & 7) ^ (lane >> 3);
  const char* src[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int rr = 8 * (wave * L + j) + (lane >> 3);
    src[j] = rr < BM ? X + ((m0 + rr) * ldx + kb) * 4 + 16 * chunk
                     : Y + ((n0 + rr - BM) * ldy + kb) * 4 + 16 * chunk;
  }
  auto issue = [&](int st) {
    char* dst = lds + (st % S) * STAGE;
#pragma unroll
    for (int j = 0; j < L; ++j)
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(src[j] + (int64_t)st * 128),
                                       (lds_ptr_t)(dst + (wave * L + j) * 1024), 16, 0, 0);
  };

  // the other factor for this wave's data rows: lane (c, g) holds rank
  // 4 s + g of data row 16 d + c (the B operand of the B-recompute MFMAs)
  float gf[ND][RP / 4];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int s = 0; s < RP / 4; ++s) {
      if constexpr (DX)
        gf[d][s] = G[(m0 + wm * 16 * MB + 16 * d + c) * ldg + 4 * s + g];
      else
        gf[d][s] = G[(int64_t)(4 * s + g) * ldg + n0 + wn * 16 * NB + 16 * d + c];
    }

  v4f acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](const char* buf) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int q = 4 * kk + g;
      const int off = 16 * (q ^ (c & 7));
      v4f a[MB], b[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i)
        a[i] = *reinterpret_cast<const v4f*>(buf + (wm * 16 * MB + 16 * i + c) * 128 + off);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        b[j] = *reinterpret_cast<const v4f*>(buf + (BM + wn * 16 * NB + 16 * j + c) * 128 + off);
      // B^T blocks (k x data row) over all ranks: A operand = factor
      // F[l][k] at row k = 16 kk + c, slot l = 4 s + g (one float per lane
      // from the staged factor rows); B operand = the register copy gf
      v4f bt[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) bt[d] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < RP / 4; ++s) {
        const int fr = FR0 + 4 * s + g;
        const float fv =
            *reinterpret_cast<const float*>(buf + fr * 128 + 16 * ((4 * kk + (c >> 2)) ^ (fr & 7)) +
                                            4 * (c & 3));
#pragma unroll
        for (int d = 0; d < ND; ++d) bt[d] = mfma_f32(fv, gf[d][s], bt[d]);
      }
      // R = V / B in the data fragments (zero where v = 0)
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if constexpr (DX) a[d][t] = a[d][t] > 0.f ? a[d][t] / bt[d][t] : 0.f;
          else b[d][t] = b[d][t] > 0.f ? b[d][t] / bt[d][t] : 0.f;
        }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = mfma_f32(a[i][t], b[j][t], acc[i][j]);
    }
  };

  const int pre = nst < S - 1 ? nst : S - 1;
  for (int st = 0; st < pre; ++st) issue(st);
  for (int st = 0; st < nst; ++st) {
    const int later = nst - 1 - st;
    wait_stage<L, S>(later < S - 2 ? later : S - 2);
    lds_barrier();
    if (st + S - 1 < nst) issue(st + S - 1);
    compute(lds + (st % S) * STAGE);
  }

  float* P = part + (int64_t)blockIdx.x * sp;
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

// Denominators of both updates from the current factors, float64 sums in a
// fixed order: den[k] = sum_j H[k][j] (j < n), den[rp + k] = sum_i W[i][k]
// (i < p).  Grid (rp, 2).  Thread t sums a contiguous segment of the row
// (column) in ascending order with 16 loads in flight (float4 items of H,
// single floats of the strided W column), then the 256 segment sums meet in
// a fixed tree.
__global__ __launch_bounds__(256) void k_kl_sums(const float* __restrict__ Wp, int rp, int64_t p,
                                                 const float* __restrict__ Hp, int64_t ldh,
                                                 int64_t n, float* __restrict__ den) {
  __shared__ double sh[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  if (blockIdx.y == 0) {
    // segments of a multiple of 4 columns (rows of H start 16-byte aligned)
    const int64_t seg = 4 * (((n + 255) / 256 + 3) / 4);
    const int64_t j0 = tid * seg, j1 = j0 + seg < n ? j0 + seg : n;
    const float* row = Hp + (int64_t)k * ldh;
    for (int64_t j = j0; j < j1; j += 64) {
      float4 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t jj = j + 4 * u;
        if (jj + 3 < j1) {
          v[u] = *reinterpret_cast<const float4*>(row + jj);
        } else {
          v[u].x = jj < j1 ? row[jj] : 0.f;
          v[u].y = jj + 1 < j1 ? row[jj + 1] : 0.f;
          v[u].z = jj + 2 < j1 ? row[jj + 2] : 0.f;
          v[u].w = 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        s += (double)v[u].x;
        s += (double)v[u].y;
        s += (double)v[u].z;
        s += (double)v[u].w;
      }
    }
  } else {
    const int64_t seg = (p + 255) / 256;
    const int64_t i0 = tid * seg, i1 = i0 + seg < p ? i0 + seg : p;
    for (int64_t i = i0; i < i1; i += 16) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = i + u < i1 ? Wp[(i + u) * rp + k] : 0.f;
#pragma unroll
      for (int u = 0; u < 16; ++u) s += (double)v[u];
    }
  }
  sh[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  if (tid == 0) den[blockIdx.y * rp + k] = (float)sh[0];
}

// sum_s x[s sp] for s < splits, added in ascending s; the loads of 8 splits
// are issued before they are added, so the sum costs one memory round trip
// per 8 splits
__device__ __forceinline__ float split_sum(const float* __restrict__ x, int64_t sp, int splits) {
  float num = 0.f;
  for (int s0 = 0; s0 < splits; s0 += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s0 + u < splits ? x[(int64_t)(s0 + u) * sp] : 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s0 + u < splits) num += v[u];
  }
  return num;
}

// w_ik <- w_ik sqrt(num_ik / den_k) for i < p, k < rp, with num = the split
// sums of pass 1 (in ascending split order) and den = den[k]; den_k <= 0
// keeps w_ik (padded ranks have den_k = 0 and stay zero, padded rows are not
// touched).  Writes Wp, W^T (pitch ldwt) and the caller's W (p x r).
__global__ __launch_bounds__(256) void k_kl_update_w(
    const float* __restrict__ part, int64_t ldp, int64_t sp, int splits,
    const float* __restrict__ den, float* __restrict__ Wp, int rp, int64_t p, int r,
    float* __restrict__ WT, int64_t ldwt, float* __restrict__ Wc) {
  const int64_t total = p * rp;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / rp;
    const int k = (int)(idx % rp);
    const float num = split_sum(part + i * ldp + k, sp, splits);
    const float dk = den[k];
    float w = Wp[idx];
    if (dk > 0.f) w = w * sqrtf(num / dk);
    Wp[idx] = w;
    WT[(int64_t)k * ldwt + i] = w;
    if (k < r) Wc[i * r + k] = w;
  }
}

// h_kj <- h_kj sqrt(num_kj / den_k) for k < rp, j < n, num from the pass-2
// split sums, den = den[rp + k]; writes Hp (pitch ldh) and the caller's H.
__global__ __launch_bounds__(256) void k_kl_update_h(
    const float* __restrict__ part, int64_t ldp, int64_t sp, int splits,
    const float* __restrict__ den, float* __restrict__ Hp, int64_t ldh, int rp, int64_t n, int r,
    float* __restrict__ Hc) {
  const int64_t total = (int64_t)rp * n;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int k = (int)(idx / n);
    const int64_t j = idx % n;
    const float num = split_sum(part + (int64_t)k * ldp + j, sp, splits);
    const float dk = den[rp + k];
    float h = Hp[(int64_t)k * ldh + j];
    if (dk > 0.f) h = h * sqrtf(num / dk);
    Hp[(int64_t)k * ldh + j] = h;
    if (k < r) Hc[(int64_t)k * n + j] = h;
  }
}

// Objective partials: one double per 64 x 64 tile of
//   sum_ij [v_ij ln b_ij - b_ij],  b_ij = sum_k w_ik h_kj
// with b formed by float64 FMAs of the float32 factors and 0 ln 0 = 0.
template <int RP>
__global__ __launch_bounds__(256) void k_kl_objective(
    const float* __restrict__ V, int64_t ldv, int64_t p, int64_t n,
    const float* __restrict__ Wp, const float* __restrict__ Hp, int64_t ldh,
    double* __restrict__ part) {
  constexpr int WPITCH = RP + 4;
  __shared__ __attribute__((aligned(16))) float Ws[64 * WPITCH];
  __shared__ __attribute__((aligned(16))) float Hs[RP * 64];
  __shared__ double red[4];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  for (int idx = tid; idx < 64 * RP; idx += 256) {
    const int ii = idx / RP, kk = idx % RP;
    Ws[ii * WPITCH + kk] = Wp[(i0 + ii) * RP + kk];
  }
  for (int idx = tid; idx < RP * 64; idx += 256) {
    const int kk = idx / 64, jj = idx % 64;
    Hs[idx] = Hp[(int64_t)kk * ldh + j0 + jj];
  }
  __syncthreads();
  double s[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) s[a][b] = 0.0;
#pragma unroll 4
  for (int kk = 0; kk < RP; ++kk) {
    double wd[4], hd[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) wd[a] = Ws[(4 * ty + a) * WPITCH + kk];
#pragma unroll
    for (int b = 0; b < 4; ++b) hd[b] = Hs[kk * 64 + 4 * tx + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) s[a][b] = fma(wd[a], hd[b], s[a][b]);
  }
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t row = i0 + 4 * ty + a;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t col = j0 + 4 * tx + b;
      if (row < p && col < n) {
        const double v = (double)V[row * ldv + col];
        acc += (v > 0.0 ? v * log(s[a][b]) : 0.0) - s[a][b];
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0)
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

unsigned blocks(int64_t total, int64_t cap = 2048) {
  const int64_t b = (total + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

void kl_tiles(int rp, int* bm1, int* bn1, int* bm2, int* bn2) {
  // pass 1: 128 data rows x all rp ranks; pass 2: rp ranks x 128 data columns
  *bm1 = 128;
  *bn1 = rp;
  *bm2 = rp;
  *bn2 = 128;
}

hipError_t launch_kl_pass(int rp, bool pass1, const float* X, int64_t ldx, int64_t M,
                          const float* Y, int64_t ldy, int64_t N, int64_t K, int splits,
                          int64_t kchunk, const float* G, int64_t ldg, float* part, int64_t ldp,
                          int64_t sp, hipStream_t st) {
  int bm1, bn1, bm2, bn2;
  kl_tiles(rp, &bm1, &bn1, &bm2, &bn2);
  const int bm = pass1 ? bm1 : bm2, bn = pass1 ? bn1 : bn2;
  const dim3 grid((unsigned)splits, (unsigned)((M + bm - 1) / bm), (unsigned)((N + bn - 1) / bn));
#define KLP(MB, NB, WM, WN, DX)                                                                \
  hipLaunchKernelGGL((k_kl_pass<MB, NB, WM, WN, 3, DX>), grid, dim3(64 * WM * WN), 0, st, X, ldx, \
                     Y, ldy, K, kchunk, G, ldg, part, ldp, sp)
  if (pass1) {
    switch (rp) {
      case 16: KLP(4, 1, 2, 1, true); break;
      case 32: KLP(2, 2, 4, 1, true); break;
      case 64: KLP(2, 4, 4, 1, true); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (rp) {
      case 16: KLP(1, 4, 1, 2, false); break;
      case 32: KLP(2, 2, 1, 4, false); break;
      case 64: KLP(4, 2, 1, 4, false); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef KLP
  return hipGetLastError();
}

hipError_t launch_kl_sums(const float* Wp, int rp, int64_t p, const float* Hp, int64_t ldh,
                          int64_t n, float* den, hipStream_t st) {
  hipLaunchKernelGGL(k_kl_sums, dim3((unsigned)rp, 2), dim3(256), 0, st, Wp, rp, p, Hp, ldh, n,
                     den);
  return hipGetLastError();
}

hipError_t launch_kl_update_w(const float* part, int64_t ldp, int64_t sp, int splits,
                              const float* den, float* Wp, int rp, int64_t p, int r, float* WT,
                              int64_t ldwt, float* Wc, hipStream_t st) {
  hipLaunchKernelGGL(k_kl_update_w, dim3(blocks(p * rp)), dim3(256), 0, st, part, ldp, sp, splits,
                     den, Wp, rp, p, r, WT, ldwt, Wc);
  return hipGetLastError();
}

hipError_t launch_kl_update_h(const float* part, int64_t ldp, int64_t sp, int splits,
                              const float* den, float* Hp, int64_t ldh, int rp, int64_t n, int r,
                              float* Hc, hipStream_t st) {
  hipLaunchKernelGGL(k_kl_update_h, dim3(blocks((int64_t)rp * n)), dim3(256), 0, st, part, ldp,
                     sp, splits, den, Hp, ldh, rp, n, r, Hc);
  return hipGetLastError();
}

hipError_t launch_kl_objective(int rp, const float* V, int64_t ldv, int64_t p, int64_t n,
                               const float* Wp, const float* Hp, int64_t ldh, double* part,
                               hipStream_t st) {
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((p + 63) / 64));
  switch (rp) {
    case 16:
      hipLaunchKernelGGL(k_kl_objective<16>, grid, dim3(256), 0, st, V, ldv, p, n, Wp, Hp, ldh,
                         part);
      break;
    case 32:
      hipLaunchKernelGGL(k_kl_objective<32>, grid, dim3(256), 0, st, V, ldv, p, n, Wp, Hp, ldh,
                         part);
      break;
    case 64:
      hipLaunchKernelGGL(k_kl_objective<64>, grid, dim3(256), 0, st, V, ldv, p, n, Wp, Hp, ldh,
                         part);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nmfk
