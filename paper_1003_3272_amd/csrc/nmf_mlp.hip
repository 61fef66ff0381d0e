// Warm-start network on gfx950: h0 = softplus(M2 relu(M1 v + b1) + b2)
// maps a column v of V (p values) to a starting column of H (r values).
//
// Every product runs on the bf16 LDS copy ring (launch_nt_dma, float32
// accumulation) as an NT product of two operands contiguous along the
// reduction dimension.  To make that true for the forward pass, the input
// gradient and both weight gradients, activations are kept in both layouts
// (batch-major and feature-major):
//
//   Z1  = X M1^T        X   = bf16(V^T)  (B x P),  M1b  (D x P)     K = P
//   Z2  = A1 M2^T       A1  (B x D),               M2b  (R x D)     K = D
//   dA1 = dZ2 M2        dZ2 (B x R),               M2Tb (D x R)     K = R
//   gM1 = dZ1^T X       dZ1T (D x B),              XT = bf16(V) (P x B)  K = B
//   gM2 = dZ2^T A1      dZ2T (R x B),              A1T  (D x B)     K = B
//
// (B = batch = columns of V, P = p, D = hidden, R = r padded to 64, every
// dimension zero-padded to the tile.)  Fused epilogues add biases,
// apply ReLU / softplus, form the loss and its error, write both layouts,
// and emit per-workgroup bias-gradient partials; Adam (Kingma & Ba 2015)
// updates float32 master weights and refreshes their bf16 copies.  Padded
// examples get a zero error, so they contribute nothing to any gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/nmf.h"
#include "nmf_internal.h"

using namespace nmfk;

namespace {

inline int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  __bf16 b = (__bf16)x;
  return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf16_float(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// Sum of the split-K partials of one element, splits in ascending order.
__device__ __forceinline__ float sum_parts(const float* __restrict__ part, int64_t off, int64_t sp,
                                           int splits) {
  float s = 0.f;
  for (int q = 0; q < splits; ++q) s += part[q * sp + off];
  return s;
}

__device__ __forceinline__ float softplus_f(float z) {
  return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
}
__device__ __forceinline__ float sigmoid_f(float z) {
  if (z >= 0.f) return 1.f / (1.f + expf(-z));
  const float e = expf(z);
  return e / (1.f + e);
}

// Forward epilogue of layer 1 on a 64 (examples) x 64 (hidden) tile:
// A1 = relu(Z1 + b1) in both layouts.
__global__ __launch_bounds__(256) void k_fwd1_epi(const float* __restrict__ part, int64_t ldp,
                                                  int64_t sp, int splits,
                                                  const float* __restrict__ b1,
                                                  uint16_t* __restrict__ A1, int64_t D,
                                                  uint16_t* __restrict__ A1T, int64_t Bp) {
  __shared__ uint16_t t[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  const int64_t b0 = (int64_t)blockIdx.y * 64, h0 = (int64_t)blockIdx.x * 64;
  for (int q = 0; q < 16; ++q) {
    const int bb = ty + 4 * q;
    const int64_t b = b0 + bb, h = h0 + tx;
    const float z = sum_parts(part, b * ldp + h, sp, splits) + b1[h];
    const uint16_t a = bf16_bits(fmaxf(z, 0.f));
    A1[b * D + h] = a;
    t[bb][tx] = a;
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int hh = ty + 4 * q;
    A1T[(h0 + hh) * Bp + b0 + tx] = t[tx][hh];
  }
}

// Forward epilogue of layer 2 on a 64 (examples) x R tile.
//   predict (T == nullptr): H0[o][b] = softplus(Z2 + b2) for o < r, b < n.
//   train: error dZ2 = 2 (y - t) / (n r) * sigmoid(z) (zero outside the data)
//          in both layouts, the tile's squared-error sum (loss partial) and
//          its column sums of dZ2 (bias-gradient partial).
template <int R>
__global__ __launch_bounds__(256) void k_fwd2_epi(const float* __restrict__ part, int64_t ldp,
                                                  int64_t sp, int splits,
                                                  const float* __restrict__ b2, int r, int64_t n,
                                                  float* __restrict__ H0, int64_t ldh,
                                                  const float* __restrict__ T, int64_t ldt,
                                                  uint16_t* __restrict__ dZ2,
                                                  uint16_t* __restrict__ dZ2T, int64_t Bp,
                                                  double* __restrict__ loss_part,
                                                  float* __restrict__ gb2_part) {
  __shared__ float e[64][R + 1];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  const double scale = 2.0 / ((double)n * (double)r);
  double sq = 0.0;
  for (int idx = tid; idx < 64 * R; idx += 256) {
    const int bb = idx / R, o = idx % R;
    const int64_t b = b0 + bb;
    const float z = sum_parts(part, b * ldp + o, sp, splits) + b2[o];
    const float y = softplus_f(z);
    const bool in = (o < r) && (b < n);
    float err = 0.f;
    if (T) {
      if (in) {
        const float d = y - T[(int64_t)o * ldt + b];
        sq += (double)d * (double)d;
        err = (float)(scale * (double)d) * sigmoid_f(z);
      }
      dZ2[b * R + o] = bf16_bits(err);
    }
    e[bb][o] = T ? err : y;
  }
  __syncthreads();
  if (T) {
    for (int idx = tid; idx < R * 64; idx += 256) {
      const int o = idx / 64, bb = idx % 64;
      dZ2T[(int64_t)o * Bp + b0 + bb] = bf16_bits(e[bb][o]);
    }
    for (int o = tid; o < R; o += 256) {
      float s = 0.f;
      for (int bb = 0; bb < 64; ++bb) s += e[bb][o];
      gb2_part[(int64_t)blockIdx.x * R + o] = s;
    }
    red[tid] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) loss_part[blockIdx.x] = red[0];
  } else {
    for (int idx = tid; idx < R * 64; idx += 256) {
      const int o = idx / 64, bb = idx % 64;
      const int64_t b = b0 + bb;
      if (o < r && b < n) H0[(int64_t)o * ldh + b] = e[bb][o];
    }
  }
}

// Backward epilogue of layer 1 on a 64 x 64 tile: dZ1 = dA1 * [A1 > 0],
// written feature-major, plus the tile's column sums (bias-gradient partial).
__global__ __launch_bounds__(256) void k_bwd1_epi(const float* __restrict__ part, int64_t ldp,
                                                  int64_t sp, int splits,
                                                  const uint16_t* __restrict__ A1, int64_t D,
                                                  uint16_t* __restrict__ dZ1T, int64_t Bp,
                                                  float* __restrict__ gb1_part) {
  __shared__ float t[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blockIdx.y * 64, h0 = (int64_t)blockIdx.x * 64;
  for (int q = 0; q < 16; ++q) {
    const int bb = ty + 4 * q;
    const int64_t b = b0 + bb, h = h0 + tx;
    const float g = sum_parts(part, b * ldp + h, sp, splits);
    t[bb][tx] = (bf16_float(A1[b * D + h]) > 0.f) ? g : 0.f;
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int hh = ty + 4 * q;
    dZ1T[(h0 + hh) * Bp + b0 + tx] = bf16_bits(t[tx][hh]);
  }
  if (threadIdx.x < 64) {
    float s = 0.f;
    for (int bb = 0; bb < 64; ++bb) s += t[bb][threadIdx.x];
    gb1_part[(int64_t)blockIdx.y * D + h0 + threadIdx.x] = s;
  }
}

// g = sum over `count` partial arrays (stride `stride`), ascending.
__device__ __forceinline__ float grad_of(const float* __restrict__ part, int64_t stride,
                                         int count, int64_t i) {
  float s = 0.f;
  for (int q = 0; q < count; ++q) s += part[q * stride + i];
  return s;
}

// Adam on one parameter array of `count` elements whose gradient is the sum
// of `parts` partial arrays.  With grad_out != nullptr only the gradient is
// written (no update).  Refreshes the bf16 copy (pitch-preserving) and, for
// M2, its transpose (rows x cols -> cols x rows).
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ part, int64_t stride, int parts, int64_t count,
                       int64_t cols, float lr, float beta1, float beta2, float eps, float c1,
                       float c2, uint16_t* __restrict__ wb, uint16_t* __restrict__ wbT,
                       float* __restrict__ grad_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float g = grad_of(part, stride, parts, i);
    if (grad_out) {
      grad_out[i] = g;
      continue;
    }
    const float mi = beta1 * m[i] + (1.f - beta1) * g;
    const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = bf16_bits(wi);
    if (wbT) {
      const int64_t rr = i / cols, cc = i % cols;
      wbT[cc * (count / cols) + rr] = bf16_bits(wi);
    }
  }
}

// dst (rows x ldd) = src (rows x cols, pitch lds) zero-padded, as bf16 or
// float32 and optionally transposed.
// acc[0] += loss[0] * scale: the minibatch loss (a float64 sum of squared
// errors) added to the epoch's running total on the device, so a training
// loop needs no host round trip per step.
__global__ void k_loss_accum(const double* __restrict__ loss, double scale,
                             double* __restrict__ acc) {
  if (blockIdx.x == 0 && threadIdx.x == 0) acc[0] += loss[0] * scale;
}

__global__ void k_pack(const float* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                       float* __restrict__ dstf, uint16_t* __restrict__ dstb, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / cols, j = idx % cols;
    const float x = src[i * lds + j];
    if (dstf) dstf[i * ldd + j] = x;
    if (dstb) dstb[i * ldd + j] = bf16_bits(x);
  }
}

unsigned blocks_for(int64_t total, int threads) {
  int64_t b = (total + threads - 1) / threads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

}  // namespace

struct nmf_mlp {
  hipStream_t st = nullptr;
  int p = 0, d = 0, r = 0;
  int64_t P = 0, D = 0, R = 0;  // padded dims
  int64_t nmax = 0, Bp = 0;     // largest batch and its padded size
  void* ws = nullptr;
  // float32 masters and Adam moments (padded shapes)
  float *M1 = nullptr, *b1 = nullptr, *M2 = nullptr, *b2 = nullptr;
  float *mM1 = nullptr, *mb1 = nullptr, *mM2 = nullptr, *mb2 = nullptr;
  float *vM1 = nullptr, *vb1 = nullptr, *vM2 = nullptr, *vb2 = nullptr;
  // bf16 weights
  uint16_t *M1b = nullptr, *M2b = nullptr, *M2Tb = nullptr;
  // activations (bf16) for a batch of up to Bp examples
  uint16_t *X = nullptr, *XT = nullptr, *A1 = nullptr, *A1T = nullptr;
  uint16_t *dZ2 = nullptr, *dZ2T = nullptr, *dZ1T = nullptr;
  // partials
  float *pz1 = nullptr, *pz2 = nullptr, *pda = nullptr, *pg1 = nullptr, *pg2 = nullptr;
  float *gb1p = nullptr, *gb2p = nullptr;
  float* gtmp = nullptr;  // padded gradient staging for nmf_mlp_grads
  double *lossp = nullptr, *lossd = nullptr, *hostbuf = nullptr;
  DmaCfg cf1{}, cf2{}, cba{}, cg1{}, cg2{};
  int64_t step = 0;
  // warm start: the mean dictionary W-bar (p x r) that nmf_ws_predict hands
  // out as W0, and the device accumulator of nmf_ws_train's epoch loss
  float* Wbar = nullptr;
  double* lossacc = nullptr;
};

namespace {

#define MTRY_HIP(expr)                        \
  do {                                        \
    if ((expr) != hipSuccess) return NMF_EDEVICE; \
  } while (0)

struct Plan {
  int splits;
  int64_t kchunk, ldp, rows, sp;
};

Plan mlp_plan(int64_t M, int64_t N, int64_t K, const DmaCfg& c, int64_t target) {
  Plan pl;
  const int64_t tiles = (M / c.bm) * (N / c.bn);
  const int64_t steps = K / 256;
  int64_t want = std::max<int64_t>(1, target / std::max<int64_t>(1, tiles));
  want = std::min<int64_t>(want, std::max<int64_t>(1, steps));
  want = std::min<int64_t>(want, 32);
  const int64_t per = (steps + want - 1) / want;
  pl.kchunk = std::max<int64_t>(256, per * 256);
  pl.splits = (int)std::max<int64_t>(1, (K + pl.kchunk - 1) / pl.kchunk);
  pl.rows = M;
  pl.ldp = N;
  pl.sp = M * N;
  return pl;
}

// Cast the batch V (p x n, pitch ldv) into X = bf16(V^T) (Bp x P) and
// XT = bf16(V) (P x Bp); padding stays zero.
nmf_status load_batch(nmf_mlp* m, const float* V, int64_t n, int64_t ldv) {
  MTRY_HIP(launch_cast_bf16(V, ldv, m->p, n, m->XT, m->Bp, false, m->st));
  MTRY_HIP(launch_cast_bf16(V, ldv, m->p, n, m->X, m->P, true, m->st));
  return NMF_OK;
}

nmf_status zero_batch(nmf_mlp* m) {
  // clear the activation buffers that padded examples / features read
  MTRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(m->X), m->Bp * m->P / 2, 0u, m->st));
  MTRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(m->XT), m->Bp * m->P / 2, 0u, m->st));
  return NMF_OK;
}

// Forward pass over the batch already in X; layer-2 epilogue in predict or
// train mode (T = targets r x n pitch ldt).
nmf_status forward(nmf_mlp* m, int64_t n, float* H0, int64_t ldh, const float* T, int64_t ldt) {
  const GramRed none = {nullptr, 0, 0, nullptr};
  const Plan p1 = mlp_plan(m->Bp, m->D, m->P, m->cf1, 512);
  MTRY_HIP(launch_nt_dma(m->cf1, true, m->X, m->P, m->Bp, m->M1b, m->P, m->D, m->P, p1.splits,
                         p1.kchunk, m->pz1, p1.ldp, p1.sp, none, m->st));
  hipLaunchKernelGGL(k_fwd1_epi, dim3((unsigned)(m->D / 64), (unsigned)(m->Bp / 64)), dim3(256), 0,
                     m->st, m->pz1, p1.ldp, p1.sp, p1.splits, m->b1, m->A1, m->D, m->A1T, m->Bp);
  MTRY_HIP(hipGetLastError());
  const Plan p2 = mlp_plan(m->Bp, m->R, m->D, m->cf2, 512);
  MTRY_HIP(launch_nt_dma(m->cf2, true, m->A1, m->D, m->Bp, m->M2b, m->D, m->R, m->D, p2.splits,
                         p2.kchunk, m->pz2, p2.ldp, p2.sp, none, m->st));
  const dim3 g2((unsigned)(m->Bp / 64));
#define FWD2(RR)                                                                                \
  hipLaunchKernelGGL(k_fwd2_epi<RR>, g2, dim3(256), 0, m->st, m->pz2, p2.ldp, p2.sp, p2.splits, \
                     m->b2, m->r, n, H0, ldh, T, ldt, m->dZ2, m->dZ2T, m->Bp, m->lossp, m->gb2p)
  switch (m->R) {
    case 64: FWD2(64); break;
    default: return NMF_EUNSUPPORTED;
  }
#undef FWD2
  MTRY_HIP(hipGetLastError());
  return NMF_OK;
}

// Backward pass (after a train-mode forward): weight-gradient partials in
// pg1 / pg2 and bias-gradient partials in gb1p / gb2p.
nmf_status backward(nmf_mlp* m, Plan* pg1, Plan* pg2) {
  const GramRed none = {nullptr, 0, 0, nullptr};
  const Plan pa = mlp_plan(m->Bp, m->D, m->R, m->cba, 512);
  MTRY_HIP(launch_nt_dma(m->cba, true, m->dZ2, m->R, m->Bp, m->M2Tb, m->R, m->D, m->R, pa.splits,
                         pa.kchunk, m->pda, pa.ldp, pa.sp, none, m->st));
  hipLaunchKernelGGL(k_bwd1_epi, dim3((unsigned)(m->D / 64), (unsigned)(m->Bp / 64)), dim3(256), 0,
                     m->st, m->pda, pa.ldp, pa.sp, pa.splits, m->A1, m->D, m->dZ1T, m->Bp,
                     m->gb1p);
  MTRY_HIP(hipGetLastError());
  *pg1 = mlp_plan(m->D, m->P, m->Bp, m->cg1, 512);
  MTRY_HIP(launch_nt_dma(m->cg1, true, m->dZ1T, m->Bp, m->D, m->XT, m->Bp, m->P, m->Bp,
                         pg1->splits, pg1->kchunk, m->pg1, pg1->ldp, pg1->sp, none, m->st));
  *pg2 = mlp_plan(m->R, m->D, m->Bp, m->cg2, 512);
  MTRY_HIP(launch_nt_dma(m->cg2, true, m->dZ2T, m->Bp, m->R, m->A1T, m->Bp, m->D, m->Bp,
                         pg2->splits, pg2->kchunk, m->pg2, pg2->ldp, pg2->sp, none, m->st));
  return NMF_OK;
}

// Adam over the four parameter arrays, or (grads != nullptr) export the
// gradients [gM1 (d x p), gb1 (d), gM2 (r x d), gb2 (r)] instead.
nmf_status adam_all(nmf_mlp* m, const Plan& pg1, const Plan& pg2, float lr, float* const* grads,
                    float* gtmp) {
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const int64_t t = m->step + 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  const int nbt = (int)(m->Bp / 64);
  struct Job {
    float *w, *mo, *vo;
    const float* part;
    int64_t stride;
    int parts;
    int64_t count, cols;
    uint16_t *wb, *wbT;
  } jobs[4] = {
      {m->M1, m->mM1, m->vM1, m->pg1, pg1.sp, pg1.splits, m->D * m->P, m->P, m->M1b, nullptr},
      {m->b1, m->mb1, m->vb1, m->gb1p, m->D, nbt, m->D, m->D, nullptr, nullptr},
      {m->M2, m->mM2, m->vM2, m->pg2, pg2.sp, pg2.splits, m->R * m->D, m->D, m->M2b, m->M2Tb},
      {m->b2, m->mb2, m->vb2, m->gb2p, m->R, nbt, m->R, m->R, nullptr, nullptr},
  };
  for (int j = 0; j < 4; ++j) {
    const Job& J = jobs[j];
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(J.count, 256)), dim3(256), 0, m->st, J.w, J.mo,
                       J.vo, J.part, J.stride, J.parts, J.count, J.cols, lr, beta1, beta2, eps, c1,
                       c2, J.wb, J.wbT, grads ? gtmp : nullptr);
    MTRY_HIP(hipGetLastError());
    if (grads) {
      // unpad into the caller's array
      const int64_t rows = (j == 0) ? m->d : (j == 2) ? m->r : 1;
      const int64_t cols = (j == 0) ? m->p : (j == 1) ? m->d : (j == 2) ? m->d : m->r;
      const int64_t ld = (j == 0) ? m->P : (j == 2) ? m->D : 0;
      MTRY_HIP(launch_copy_pad(gtmp, ld ? ld : cols, rows, cols, grads[j], cols, m->st));
    }
  }
  if (!grads) m->step = t;
  return NMF_OK;
}

nmf_status check_batch(nmf_mlp* m, const float* V, int64_t n, int64_t ldv) {
  if (!m || !V || n < 1 || n > m->nmax || ldv < n) return NMF_EINVAL;
  if (reinterpret_cast<uintptr_t>(V) % 4 != 0) return NMF_EINVAL;
  return NMF_OK;
}

}  // namespace

extern "C" {

nmf_status nmf_mlp_create(nmf_mlp** out, int32_t p, int32_t hidden, int32_t r, int64_t max_batch,
                          const float* M1, const float* b1, const float* M2, const float* b2,
                          void* stream) {
  if (!out) return NMF_EINVAL;
  *out = nullptr;
  if (p < 1 || hidden < 1 || r < 1 || max_batch < 1 || !M1 || !b1 || !M2 || !b2)
    return NMF_EINVAL;
  if (r > 64 || hidden % 128 != 0 || p > 65536 || max_batch > (int64_t)1 << 24)
    return NMF_EUNSUPPORTED;
  nmf_mlp* m = new (std::nothrow) nmf_mlp();
  if (!m) return NMF_ENOMEM;
  m->st = static_cast<hipStream_t>(stream);
  m->p = p;
  m->d = hidden;
  m->r = r;
  m->P = rup(p, 256);
  m->D = hidden;
  m->R = 64;  // output rows padded to one 64-deep bf16 stage (K of dA1)
  m->nmax = max_batch;
  m->Bp = rup(max_batch, 256);
  m->cf1 = dma_config_by_id(3);   // 128 x 128
  m->cf2 = dma_config(m->R, true);  // 128 x R
  m->cba = dma_config_by_id(3);
  m->cg1 = dma_config_by_id(3);
  m->cg2 = dma_config(m->R, false);  // R x 128
  const Plan p1 = mlp_plan(m->Bp, m->D, m->P, m->cf1, 512);
  const Plan p2 = mlp_plan(m->Bp, m->R, m->D, m->cf2, 512);
  const Plan pa = mlp_plan(m->Bp, m->D, m->R, m->cba, 512);
  const Plan g1 = mlp_plan(m->D, m->P, m->Bp, m->cg1, 512);
  const Plan g2 = mlp_plan(m->R, m->D, m->Bp, m->cg2, 512);
  const int64_t P = m->P, D = m->D, R = m->R, Bp = m->Bp;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  size_t o_f[12];
  const int64_t fsz[4] = {D * P, D, R * D, R};
  for (int j = 0; j < 12; ++j) o_f[j] = take(4 * (size_t)fsz[j % 4]);
  const size_t oM1b = take(2 * (size_t)D * P), oM2b = take(2 * (size_t)R * D),
               oM2Tb = take(2 * (size_t)D * R);
  const size_t oX = take(2 * (size_t)Bp * P), oXT = take(2 * (size_t)P * Bp),
               oA1 = take(2 * (size_t)Bp * D), oA1T = take(2 * (size_t)D * Bp),
               odZ2 = take(2 * (size_t)Bp * R), odZ2T = take(2 * (size_t)R * Bp),
               odZ1T = take(2 * (size_t)D * Bp);
  const size_t opz1 = take(4 * (size_t)p1.splits * p1.sp), opz2 = take(4 * (size_t)p2.splits * p2.sp),
               opda = take(4 * (size_t)pa.splits * pa.sp), opg1 = take(4 * (size_t)g1.splits * g1.sp),
               opg2 = take(4 * (size_t)g2.splits * g2.sp);
  const size_t ogb1 = take(4 * (size_t)(Bp / 64) * D), ogb2 = take(4 * (size_t)(Bp / 64) * R);
  const size_t olp = take(8 * (size_t)(Bp / 64)), old = take(16);
  const size_t ogt = take(4 * (size_t)D * P);
  if (hipMalloc(&m->ws, off) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&m->hostbuf), 16, 0) != hipSuccess) {
    (void)hipGetLastError();
    if (m->ws) (void)hipFree(m->ws);
    delete m;
    return NMF_ENOMEM;
  }
  char* base = static_cast<char*>(m->ws);
  float** fp[12] = {&m->M1, &m->b1, &m->M2, &m->b2, &m->mM1, &m->mb1,
                    &m->mM2, &m->mb2, &m->vM1, &m->vb1, &m->vM2, &m->vb2};
  for (int j = 0; j < 12; ++j) *fp[j] = reinterpret_cast<float*>(base + o_f[j]);
  m->M1b = reinterpret_cast<uint16_t*>(base + oM1b);
  m->M2b = reinterpret_cast<uint16_t*>(base + oM2b);
  m->M2Tb = reinterpret_cast<uint16_t*>(base + oM2Tb);
  m->X = reinterpret_cast<uint16_t*>(base + oX);
  m->XT = reinterpret_cast<uint16_t*>(base + oXT);
  m->A1 = reinterpret_cast<uint16_t*>(base + oA1);
  m->A1T = reinterpret_cast<uint16_t*>(base + oA1T);
  m->dZ2 = reinterpret_cast<uint16_t*>(base + odZ2);
  m->dZ2T = reinterpret_cast<uint16_t*>(base + odZ2T);
  m->dZ1T = reinterpret_cast<uint16_t*>(base + odZ1T);
  m->pz1 = reinterpret_cast<float*>(base + opz1);
  m->pz2 = reinterpret_cast<float*>(base + opz2);
  m->pda = reinterpret_cast<float*>(base + opda);
  m->pg1 = reinterpret_cast<float*>(base + opg1);
  m->pg2 = reinterpret_cast<float*>(base + opg2);
  m->gb1p = reinterpret_cast<float*>(base + ogb1);
  m->gb2p = reinterpret_cast<float*>(base + ogb2);
  m->lossp = reinterpret_cast<double*>(base + olp);
  m->lossd = reinterpret_cast<double*>(base + old);
  m->gtmp = reinterpret_cast<float*>(base + ogt);
  nmf_status s = NMF_OK;
  if (launch_fill_u32(static_cast<uint32_t*>(m->ws), (int64_t)(off / 4), 0u, m->st) != hipSuccess)
    s = NMF_EDEVICE;
  // masters (padded) and their bf16 copies
  auto pack = [&](const float* src, int64_t rows, int64_t cols, float* dstf, uint16_t* dstb,
                  int64_t ldd) {
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(rows * cols, 256)), dim3(256), 0, m->st, src, cols,
                       rows, cols, dstf, dstb, ldd);
    return hipGetLastError() == hipSuccess;
  };
  if (s == NMF_OK &&
      !(pack(M1, hidden, p, m->M1, m->M1b, P) && pack(b1, 1, hidden, m->b1, nullptr, D) &&
        pack(M2, r, hidden, m->M2, m->M2b, D) && pack(b2, 1, r, m->b2, nullptr, R)))
    s = NMF_EDEVICE;
  if (s == NMF_OK && launch_cast_bf16(m->M2, D, R, D, m->M2Tb, R, true, m->st) != hipSuccess)
    s = NMF_EDEVICE;
  if (s == NMF_OK && hipStreamSynchronize(m->st) != hipSuccess) s = NMF_EDEVICE;
  if (s != NMF_OK) {
    nmf_mlp_destroy(m);
    return s;
  }
  *out = m;
  return NMF_OK;
}

nmf_status nmf_mlp_predict(nmf_mlp* m, const float* V, int64_t n, int64_t ldv, float* H0) {
  if (!m || n < 1 || ldv < n) return NMF_EINVAL;
  if (!H0 || reinterpret_cast<uintptr_t>(H0) % 4 != 0) return NMF_EINVAL;
  // column chunks of at most max_batch examples; H0 keeps row stride n
  for (int64_t a = 0; a < n; a += m->nmax) {
    const int64_t nb = std::min<int64_t>(m->nmax, n - a);
    nmf_status s = check_batch(m, V + a, nb, ldv);
    if (s != NMF_OK) return s;
    if (nb != m->Bp) {
      s = zero_batch(m);
      if (s != NMF_OK) return s;
    }
    s = load_batch(m, V + a, nb, ldv);
    if (s == NMF_OK) s = forward(m, nb, H0 + a, n, nullptr, 0);
    if (s != NMF_OK) return s;
  }
  return NMF_OK;
}

}  // extern "C"

namespace {

// One minibatch: forward with targets T, backward, then Adam (grads ==
// nullptr) or the gradients exported to grads.  The loss partials are left
// in m->lossp.
nmf_status train_core(nmf_mlp* m, const float* V, int64_t n, int64_t ldv, const float* T,
                      int64_t ldt, float lr, float* const* grads) {
  nmf_status s = check_batch(m, V, n, ldv);
  if (s != NMF_OK) return s;
  if (!T || reinterpret_cast<uintptr_t>(T) % 4 != 0 || ldt < n) return NMF_EINVAL;
  if (n != m->Bp) {
    s = zero_batch(m);
    if (s != NMF_OK) return s;
  }
  s = load_batch(m, V, n, ldv);
  if (s == NMF_OK) s = forward(m, n, nullptr, 0, T, ldt);
  Plan pg1{}, pg2{};
  if (s == NMF_OK) s = backward(m, &pg1, &pg2);
  if (s == NMF_OK) s = adam_all(m, pg1, pg2, lr, grads, m->gtmp);
  return s;
}

// splitmix64 (Steele, Lea & Flood 2014): the seeded order of nmf_ws_train.
uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

static nmf_status train_or_grad(nmf_mlp* m, const float* V, int64_t n, int64_t ldv,
                                const float* T, int64_t ldt, float lr, double* loss_host,
                                float* const* grads) {
  nmf_status s = train_core(m, V, n, ldv, T, ldt, lr, grads);
  if (s != NMF_OK) return s;
  if (loss_host) {
    MTRY_HIP(launch_reduce_f64(m->lossp, m->Bp / 64, m->lossd, m->st));
    MTRY_HIP(hipMemcpyAsync(m->hostbuf, m->lossd, 8, hipMemcpyDeviceToHost, m->st));
    MTRY_HIP(hipStreamSynchronize(m->st));
    *loss_host = m->hostbuf[0] / ((double)n * (double)m->r);
  }
  return NMF_OK;
}

nmf_status nmf_mlp_train_step(nmf_mlp* m, const float* V, int64_t n, int64_t ldv, const float* H,
                              int64_t ldh, float lr, double* loss_host) {
  if (!(lr > 0.f) || !std::isfinite(lr)) return NMF_EINVAL;
  return train_or_grad(m, V, n, ldv, H, ldh, lr, loss_host, nullptr);
}

nmf_status nmf_mlp_grads(nmf_mlp* m, const float* V, int64_t n, int64_t ldv, const float* H,
                         int64_t ldh, float* gM1, float* gb1, float* gM2, float* gb2,
                         double* loss_host) {
  if (!gM1 || !gb1 || !gM2 || !gb2) return NMF_EINVAL;
  float* const grads[4] = {gM1, gb1, gM2, gb2};
  return train_or_grad(m, V, n, ldv, H, ldh, 0.f, loss_host, grads);
}

nmf_status nmf_mlp_get_params(nmf_mlp* m, float* M1, float* b1, float* M2, float* b2) {
  if (!m || !M1 || !b1 || !M2 || !b2) return NMF_EINVAL;
  MTRY_HIP(launch_copy_pad(m->M1, m->P, m->d, m->p, M1, m->p, m->st));
  MTRY_HIP(launch_copy_pad(m->b1, m->d, 1, m->d, b1, m->d, m->st));
  MTRY_HIP(launch_copy_pad(m->M2, m->D, m->r, m->d, M2, m->d, m->st));
  MTRY_HIP(launch_copy_pad(m->b2, m->r, 1, m->r, b2, m->r, m->st));
  return NMF_OK;
}

nmf_status nmf_ws_set_dictionary(nmf_mlp* m, const float* Wbar) {
  if (!m || !Wbar || reinterpret_cast<uintptr_t>(Wbar) % 4 != 0) return NMF_EINVAL;
  const size_t bytes = sizeof(float) * (size_t)m->p * m->r;
  if (!m->Wbar && hipMalloc(reinterpret_cast<void**>(&m->Wbar), bytes) != hipSuccess) {
    m->Wbar = nullptr;
    (void)hipGetLastError();
    return NMF_ENOMEM;
  }
  MTRY_HIP(hipMemcpyAsync(m->Wbar, Wbar, bytes, hipMemcpyDeviceToDevice, m->st));
  return NMF_OK;
}

nmf_status nmf_ws_predict(nmf_mlp* m, const float* V, int64_t p, int64_t n, int64_t ldv,
                          float* W0, float* H0) {
  if (!m || !W0 || reinterpret_cast<uintptr_t>(W0) % 4 != 0) return NMF_EINVAL;
  if (p != m->p || !m->Wbar) return NMF_EINVAL;
  if (!V || n < 1 || ldv < n || !H0 || reinterpret_cast<uintptr_t>(H0) % 4 != 0)
    return NMF_EINVAL;
  MTRY_HIP(hipMemcpyAsync(W0, m->Wbar, sizeof(float) * (size_t)m->p * m->r,
                          hipMemcpyDeviceToDevice, m->st));
  return nmf_mlp_predict(m, V, n, ldv, H0);
}

nmf_status nmf_ws_train(nmf_mlp* m, const float* const* V, const float* const* H, int32_t count,
                        int64_t n, int64_t ldv, int64_t ldh, int32_t epochs, int32_t batch,
                        float lr, float decay, uint64_t seed, double* loss_host) {
  if (!m || !V || !H || count < 1 || n < 1 || ldv < n || ldh < n || epochs < 1) return NMF_EINVAL;
  if (batch < 1 || batch > m->nmax) return NMF_EINVAL;
  if (!(lr > 0.f) || !std::isfinite(lr) || !(decay > 0.f && decay <= 1.f)) return NMF_EINVAL;
  for (int32_t i = 0; i < count; ++i)
    if (!V[i] || !H[i] || reinterpret_cast<uintptr_t>(V[i]) % 4 != 0 ||
        reinterpret_cast<uintptr_t>(H[i]) % 4 != 0)
      return NMF_EINVAL;
  if (!m->lossacc && hipMalloc(reinterpret_cast<void**>(&m->lossacc), 256) != hipSuccess) {
    m->lossacc = nullptr;
    (void)hipGetLastError();
    return NMF_ENOMEM;
  }
  std::vector<int32_t> order(count);
  for (int32_t i = 0; i < count; ++i) order[i] = i;
  uint64_t rng = seed;
  float rate = lr;
  for (int32_t ep = 0; ep < epochs; ++ep) {
    // matrices in a seeded random order (Fisher-Yates), minibatches of
    // `batch` consecutive columns (column slices, no copies)
    for (int32_t i = count - 1; i > 0; --i) {
      const int32_t j = (int32_t)(splitmix64(rng) % (uint64_t)(i + 1));
      std::swap(order[i], order[j]);
    }
    MTRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(m->lossacc), 2, 0u, m->st));
    int64_t steps = 0;
    for (int32_t q = 0; q < count; ++q) {
      const float* Vm = V[order[q]];
      const float* Hm = H[order[q]];
      for (int64_t a = 0; a < n; a += batch) {
        const int64_t nb = std::min<int64_t>(batch, n - a);
        nmf_status s = train_core(m, Vm + a, nb, ldv, Hm + a, ldh, rate, nullptr);
        if (s != NMF_OK) return s;
        MTRY_HIP(launch_reduce_f64(m->lossp, m->Bp / 64, m->lossd, m->st));
        hipLaunchKernelGGL(k_loss_accum, dim3(1), dim3(64), 0, m->st, m->lossd,
                           1.0 / ((double)nb * (double)m->r), m->lossacc);
        MTRY_HIP(hipGetLastError());
        ++steps;
      }
    }
    if (loss_host) {
      MTRY_HIP(hipMemcpyAsync(m->hostbuf, m->lossacc, 8, hipMemcpyDeviceToHost, m->st));
      MTRY_HIP(hipStreamSynchronize(m->st));
      loss_host[ep] = m->hostbuf[0] / (double)steps;
    }
    rate *= decay;
  }
  return NMF_OK;
}

void nmf_mlp_destroy(nmf_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->st);
  if (m->Wbar) (void)hipFree(m->Wbar);
  if (m->lossacc) (void)hipFree(m->lossacc);
  if (m->ws) (void)hipFree(m->ws);
  if (m->hostbuf) (void)hipHostFree(m->hostbuf);
  delete m;
}

}  // extern "C"
