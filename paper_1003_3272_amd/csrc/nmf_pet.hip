// gfx950 kernels and C ABI of the penalized PET reconstruction MM algorithm,
// Sec. 3.2 (Algorithm 2).  Intensities lambda (p pixels on a rows x cols
// grid), geometry E (d lines x p pixels, dense), counts y (d).  Every
// iteration, for all pixels in parallel:
//   ratio_i  = y_i / (E_s lambda)_i                  (0 where y_i = 0)
//   c_j      = lambda_j sum_i e_ij ratio_i           (= sum_i z_ij)
//   b_j      = mu (|N_j| lambda_j + sum_{k in N_j} lambda_k) - 1
//   a_j      = -2 mu |N_j|
//   lambda_j <- the positive root of a x^2 + b x + c = 0
// with E_s = E scaled to unit column sums (Algorithm 2, first step) and N
// the 4-neighbour system of the grid.  The root is evaluated as
// 2 c / (-b + sqrt(b^2 - 4 a c)) when b <= 0, algebraically equal to the
// printed (-b - sqrt(b^2 - 4 a c)) / (2 a) and free of its cancellation when
// mu is small (in float32 the printed form loses all digits near mu = 1e-7),
// and in the printed form when b > 0, where it does not cancel; at mu = 0
// the update is c, the EM update (eq. PET_algorithm).
//
// Layout: E_s (d x p) and its transpose (p x dpad), row-major, float32, so
// that both products are row dot products read with coalesced 16-byte loads
// (one wave per line, then one wave per pixel); partial sums combine in a
// fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>

#include "../../include/nmf.h"
#include "nmf_internal.h"

using namespace nmfk;

namespace {

inline int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

__device__ __forceinline__ float wave_sum(float s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}
__device__ __forceinline__ double wave_sum_d(double s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// Column sums of E (d x p), float64 in a fixed order: one wave per column.
__global__ __launch_bounds__(256) void k_pet_colsum(const float* __restrict__ E, int64_t d,
                                                    int64_t p, double* __restrict__ colsum) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= p) return;
  double s = 0.0;
  for (int64_t i = lane; i < d; i += 64) s += (double)E[i * p + j];
  s = wave_sum_d(s);
  if (lane == 0) colsum[j] = s;
}

// E_s = E / colsum (zero columns stay zero) into Es (d x p) and EsT
// (p x dpad, padding zero).
__global__ void k_pet_scale(const float* __restrict__ E, int64_t d, int64_t p,
                            const double* __restrict__ colsum, float* __restrict__ Es,
                            float* __restrict__ EsT, int64_t dpad) {
  const int64_t total = d * p;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / p, j = idx % p;
    const double cs = colsum[j];
    const float v = cs > 0.0 ? (float)((double)E[idx] / cs) : 0.f;
    Es[idx] = v;
    EsT[j * dpad + i] = v;
  }
}

// ratio_i = y_i / (E_s lambda)_i (0 where y_i = 0): one wave per line.
__global__ __launch_bounds__(256) void k_pet_forward(const float* __restrict__ Es, int64_t d,
                                                     int64_t p, const float* __restrict__ lam,
                                                     const float* __restrict__ y,
                                                     float* __restrict__ ratio) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= d) return;
  const float* row = Es + i * p;
  float s = 0.f;
  for (int64_t j = 4 * lane; j < p; j += 256) {
    const float4 e = *reinterpret_cast<const float4*>(row + j);
    const float4 l = *reinterpret_cast<const float4*>(lam + j);
    s = fmaf(e.x, l.x, s);
    s = fmaf(e.y, l.y, s);
    s = fmaf(e.z, l.z, s);
    s = fmaf(e.w, l.w, s);
  }
  s = wave_sum(s);
  if (lane == 0) ratio[i] = y[i] > 0.f ? y[i] / s : 0.f;
}

// c_j = lambda_j (E_s^T ratio)_j and the positive root: one wave per pixel.
__global__ __launch_bounds__(256) void k_pet_backward(const float* __restrict__ EsT, int64_t dpad,
                                                      int64_t p, const float* __restrict__ ratio,
                                                      const float* __restrict__ lam, int rows,
                                                      int cols, float mu,
                                                      float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= p) return;
  const float* row = EsT + j * dpad;
  float t = 0.f;
  for (int64_t i = 4 * lane; i < dpad; i += 256) {
    const float4 e = *reinterpret_cast<const float4*>(row + i);
    const float4 q = *reinterpret_cast<const float4*>(ratio + i);
    t = fmaf(e.x, q.x, t);
    t = fmaf(e.y, q.y, t);
    t = fmaf(e.z, q.z, t);
    t = fmaf(e.w, q.w, t);
  }
  t = wave_sum(t);
  if (lane != 0) return;
  const float lj = lam[j];
  const float c = lj * t;
  const int r = (int)(j / cols), cc = (int)(j % cols);
  float cnt = 0.f, nsum = 0.f;
  if (r > 0) { cnt += 1.f; nsum += lam[j - cols]; }
  if (r + 1 < rows) { cnt += 1.f; nsum += lam[j + cols]; }
  if (cc > 0) { cnt += 1.f; nsum += lam[j - 1]; }
  if (cc + 1 < cols) { cnt += 1.f; nsum += lam[j + 1]; }
  const float b = mu * (cnt * lj + nsum) - 1.f;
  const float a = -2.f * mu * cnt;
  float v = c;
  if (a != 0.f) {
    // a < 0 and c >= 0: the roots have opposite signs (or one is 0), and
    // the positive one is (b + s) / (-2a) = 2c / (s - b), s = sqrt(b^2 - 4ac);
    // take the form whose sum does not cancel
    const float s = sqrtf(fmaxf(b * b - 4.f * a * c, 0.f));
    if (b > 0.f)
      v = (b + s) / (-2.f * a);
    else
      v = s - b > 0.f ? 2.f * c / (s - b) : 0.f;
  }
  out[j] = v;
}

__global__ void k_pet_copy(const float* __restrict__ src, float* __restrict__ dst, int64_t p) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256)
    dst[j] = src[j];
}

// Objective partials (float64): part[i] = y_i ln B_i - B_i for the lines,
// B_i from float64 products; part[d + j] = -(mu / 2) [(lambda_j -
// lambda_right)^2 + (lambda_j - lambda_below)^2] for the pixels.
__global__ __launch_bounds__(256) void k_pet_objective(const float* __restrict__ Es, int64_t d,
                                                       int64_t p, const float* __restrict__ lam,
                                                       const float* __restrict__ y, int rows,
                                                       int cols, double mu,
                                                       double* __restrict__ part) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w < d) {
    const float* row = Es + w * p;
    double s = 0.0;
    for (int64_t j = lane; j < p; j += 64) s = fma((double)row[j], (double)lam[j], s);
    s = wave_sum_d(s);
    if (lane == 0) part[w] = (y[w] > 0.f ? (double)y[w] * log(s) : 0.0) - s;
  } else if (w < d + (p + 63) / 64) {
    const int64_t j = (w - d) * 64 + lane;
    if (j < p) {
      const int r = (int)(j / cols), cc = (int)(j % cols);
      const double lj = lam[j];
      double pen = 0.0;
      if (cc + 1 < cols) pen += (lj - lam[j + 1]) * (lj - lam[j + 1]);
      if (r + 1 < rows) pen += (lj - lam[j + cols]) * (lj - lam[j + cols]);
      part[d + j] = -0.5 * mu * pen;
    }
  }
}

unsigned pblocks(int64_t total, int64_t cap = 65535) {
  const int64_t b = (total + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

constexpr int kPetGraphs = 5;  // graphs of 1, 2, 4, 8 and 16 iterations

}  // namespace

struct nmf_pet {
  hipStream_t st = nullptr;
  int64_t d = 0, p = 0, dpad = 0;
  int rows = 0, cols = 0;
  float mu = 0.f;
  double mu_d = 0.0;
  float* lam = nullptr;  // caller's intensities, updated in place
  void* ws = nullptr;
  float *Es = nullptr, *EsT = nullptr, *y = nullptr, *ratio = nullptr, *tmp = nullptr;
  double *colsum = nullptr, *part = nullptr;
  double* hostbuf = nullptr;      // pinned, coherent
  double* hostbuf_dev = nullptr;  // the same memory as the device addresses it
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gp[kPetGraphs] = {};
};

namespace {

#define PTRY_HIP(expr)                              \
  do {                                              \
    if ((expr) != hipSuccess) return NMF_EDEVICE;   \
  } while (0)

nmf_status pet_iter(nmf_pet* m) {
  hipLaunchKernelGGL(k_pet_forward, dim3((unsigned)((m->d + 3) / 4)), dim3(256), 0, m->st, m->Es,
                     m->d, m->p, m->lam, m->y, m->ratio);
  PTRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pet_backward, dim3((unsigned)((m->p + 3) / 4)), dim3(256), 0, m->st,
                     m->EsT, m->dpad, m->p, m->ratio, m->lam, m->rows, m->cols, m->mu, m->tmp);
  PTRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pet_copy, dim3(pblocks(m->p, 1024)), dim3(256), 0, m->st, m->tmp, m->lam,
                     m->p);
  PTRY_HIP(hipGetLastError());
  return NMF_OK;
}

nmf_status pet_capture(nmf_pet* m, int iters, hipGraphExec_t* out) {
  if (!m->cap_stream) PTRY_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
  hipStream_t user = m->st;
  m->st = m->cap_stream;
  hipGraph_t graph = nullptr;
  nmf_status s = NMF_OK;
  if (hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    s = NMF_EDEVICE;
  if (s == NMF_OK) {
    for (int it = 0; it < iters && s == NMF_OK; ++it) s = pet_iter(m);
    const hipError_t e = hipStreamEndCapture(m->cap_stream, &graph);
    if (s == NMF_OK && (e != hipSuccess || !graph)) s = NMF_EDEVICE;
  }
  m->st = user;
  if (s == NMF_OK && (hipGraphInstantiate(out, graph, nullptr, nullptr, 0) != hipSuccess ||
                      hipGraphUpload(*out, m->st) != hipSuccess))
    s = NMF_EDEVICE;
  if (graph) (void)hipGraphDestroy(graph);
  return s;
}

nmf_status pet_objective_sync(nmf_pet* m, double* f) {
  const int64_t waves = m->d + (m->p + 63) / 64;
  hipLaunchKernelGGL(k_pet_objective, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, m->st,
                     m->Es, m->d, m->p, m->lam, m->y, m->rows, m->cols, m->mu_d, m->part);
  PTRY_HIP(hipGetLastError());
  PTRY_HIP(launch_reduce_f64(m->part, m->d + m->p, m->hostbuf_dev, m->st));
  PTRY_HIP(hipStreamSynchronize(m->st));
  *f = m->hostbuf[0];
  return NMF_OK;
}

void pet_free(nmf_pet* m) {
  if (!m) return;
  for (hipGraphExec_t g : m->gp)
    if (g) (void)hipGraphExecDestroy(g);
  if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
  if (m->ws) (void)hipFree(m->ws);
  if (m->hostbuf) (void)hipHostFree(m->hostbuf);
  delete m;
}

}  // namespace

extern "C" {

nmf_status nmf_pet_create(nmf_pet** out, const float* E, int64_t d, int64_t p, const float* y,
                          int32_t rows, int32_t cols, double mu, float* lambda, void* stream) {
  if (!out) return NMF_EINVAL;
  *out = nullptr;
  if (!E || !y || !lambda || d < 1 || p < 1 || rows < 1 || cols < 1) return NMF_EINVAL;
  if ((int64_t)rows * cols != p || !(mu >= 0.0) || !std::isfinite(mu)) return NMF_EINVAL;
  for (const void* q : {static_cast<const void*>(E), static_cast<const void*>(y),
                        static_cast<const void*>(lambda)})
    if (reinterpret_cast<uintptr_t>(q) % 16 != 0) return NMF_EINVAL;
  if (p % 4 != 0 || d > (int64_t)1 << 30 || p > (int64_t)1 << 30) return NMF_EUNSUPPORTED;
  nmf_pet* m = new (std::nothrow) nmf_pet();
  if (!m) return NMF_ENOMEM;
  m->st = static_cast<hipStream_t>(stream);
  m->d = d;
  m->p = p;
  m->dpad = rup(d, 64);
  m->rows = rows;
  m->cols = cols;
  m->mu = (float)mu;
  m->mu_d = mu;
  m->lam = lambda;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t oEs = take(4 * (size_t)d * p), oEsT = take(4 * (size_t)p * m->dpad);
  const size_t oy = take(4 * (size_t)m->dpad), orat = take(4 * (size_t)m->dpad);
  const size_t otmp = take(4 * (size_t)p), ocs = take(8 * (size_t)p);
  const size_t opart = take(8 * (size_t)(d + p));
  if (hipMalloc(&m->ws, off) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&m->hostbuf), 4 * sizeof(double),
                    hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    pet_free(m);
    return NMF_ENOMEM;
  }
  nmf_status s = NMF_OK;
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&m->hostbuf_dev), m->hostbuf, 0) !=
      hipSuccess)
    s = NMF_EDEVICE;
  char* b = static_cast<char*>(m->ws);
  m->Es = reinterpret_cast<float*>(b + oEs);
  m->EsT = reinterpret_cast<float*>(b + oEsT);
  m->y = reinterpret_cast<float*>(b + oy);
  m->ratio = reinterpret_cast<float*>(b + orat);
  m->tmp = reinterpret_cast<float*>(b + otmp);
  m->colsum = reinterpret_cast<double*>(b + ocs);
  m->part = reinterpret_cast<double*>(b + opart);
  // zero everything (the transposed copy's padding and the counts' tail
  // must read as zero), then scale E and copy y
  if (s == NMF_OK &&
      launch_fill_u32(static_cast<uint32_t*>(m->ws), (int64_t)(off / 4), 0u, m->st) != hipSuccess)
    s = NMF_EDEVICE;
  if (s == NMF_OK) {
    hipLaunchKernelGGL(k_pet_colsum, dim3((unsigned)((p + 3) / 4)), dim3(256), 0, m->st, E, d, p,
                       m->colsum);
    hipLaunchKernelGGL(k_pet_scale, dim3(pblocks(d * p)), dim3(256), 0, m->st, E, d, p, m->colsum,
                       m->Es, m->EsT, m->dpad);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(m->y, y, 4 * (size_t)d, hipMemcpyDeviceToDevice, m->st) != hipSuccess ||
        hipStreamSynchronize(m->st) != hipSuccess)
      s = NMF_EDEVICE;
  }
  if (s != NMF_OK) {
    pet_free(m);
    return s;
  }
  *out = m;
  return NMF_OK;
}

nmf_status nmf_pet_step(nmf_pet* m, int32_t iters) {
  if (!m || iters < 0) return NMF_EINVAL;
  constexpr int top = kPetGraphs - 1;
  int32_t left = iters;
  for (int j = top; j >= 0; --j) {
    const int32_t n = 1 << j;
    while (left >= n) {
      if (!m->gp[j]) {
        nmf_status s = pet_capture(m, n, &m->gp[j]);
        if (s != NMF_OK) return s;
      }
      PTRY_HIP(hipGraphLaunch(m->gp[j], m->st));
      left -= n;
      if (j < top) break;
    }
  }
  return NMF_OK;
}

nmf_status nmf_pet_objective(nmf_pet* m, double* f_host) {
  if (!m || !f_host) return NMF_EINVAL;
  double f;
  nmf_status s = pet_objective_sync(m, &f);
  if (s != NMF_OK) return s;
  *f_host = f;
  return std::isfinite(f) ? NMF_OK : NMF_ENONFINITE;
}

nmf_status nmf_pet_solve(nmf_pet* m, int32_t max_iters, double tol, int32_t check_every,
                         int32_t* iters_done, double* f_host) {
  if (!m || !iters_done || !f_host || max_iters < 0 || check_every < 1 || !(tol >= 0.0))
    return NMF_EINVAL;
  *iters_done = 0;
  double f_prev;
  nmf_status s = nmf_pet_objective(m, &f_prev);
  *f_host = f_prev;
  if (s != NMF_OK) return s;
  int32_t k = 0;
  while (k < max_iters) {
    const int32_t todo = std::min(check_every, max_iters - k);
    s = nmf_pet_step(m, todo);
    if (s != NMF_OK) return s;
    k += todo;
    double f;
    s = nmf_pet_objective(m, &f);
    *iters_done = k;
    *f_host = f;
    if (s != NMF_OK) return s;
    const bool done = std::fabs(f - f_prev) / (std::fabs(f_prev) + 1.0) < tol;
    f_prev = f;
    if (done) return NMF_OK;
  }
  return NMF_ENOTCONVERGED;
}

void nmf_pet_destroy(nmf_pet* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->st);
  pet_free(m);
}

}  // extern "C"
