// gfx950 kernels and C ABI of the penalized PET reconstruction MM algorithm,
// Sec. 3.2 (Algorithm 2).  Intensities lambda (p pixels on a rows x cols
// grid), geometry E (d lines x p pixels), counts y (d).  Every iteration,
// for all pixels in parallel:
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
// Two layouts of E_s, chosen at creation.  Dense: E_s (d x p) and its
// transpose (p x dpad), row-major float32, so that both products are row
// dot products read with coalesced 16-byte loads (one wave per line, then
// one wave per pixel).  Sparse (a line of flight crosses O(sqrt p) pixels,
// so E_s of a ring scanner is about 2% dense): E_s by lines and by pixels in
// padded rows (ELL) of (value, index) pairs in increasing index order, a
// wave per line and a group of 16, 32 or 64 lanes per pixel, lambda and the
// ratios gathered from L2.  An iteration reads src intensities and writes
// dst (ping-pong between the caller's buffer and a workspace copy, so the
// neighbour sums never see a half-updated image); partial sums combine in a
// fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "../../include/nmf.h"
#include "nmf_internal.h"

using namespace nmfk;

namespace {

inline int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

template <int G>
__device__ __forceinline__ float group_sum(float s) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}
__device__ __forceinline__ double wave_sum_d(double s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}
__device__ __forceinline__ int wave_sum_i(int s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// ---- set-up ----------------------------------------------------------------

// Column sums of E (float64, fixed order) and nonzeros per column: one wave
// per column.
__global__ __launch_bounds__(256) void k_pet_colsum(const float* __restrict__ E, int64_t d,
                                                    int64_t p, double* __restrict__ colsum,
                                                    int32_t* __restrict__ colcnt) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= p) return;
  double s = 0.0;
  int cnt = 0;
  for (int64_t i = lane; i < d; i += 64) {
    const float v = E[i * p + j];
    s += (double)v;
    cnt += v != 0.f;
  }
  s = wave_sum_d(s);
  cnt = wave_sum_i(cnt);
  if (lane == 0) {
    colsum[j] = s;
    colcnt[j] = cnt;
  }
}

// Nonzeros per line: one wave per line.
__global__ __launch_bounds__(256) void k_pet_rowcnt(const float* __restrict__ E, int64_t d,
                                                    int64_t p, int32_t* __restrict__ rowcnt) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= d) return;
  int cnt = 0;
  for (int64_t j = lane; j < p; j += 64) cnt += E[i * p + j] != 0.f;
  cnt = wave_sum_i(cnt);
  if (lane == 0) rowcnt[i] = cnt;
}

// out[0] = largest line count, out[1] = largest pixel count (one block).
__global__ void k_pet_maxcnt(const int32_t* __restrict__ rowcnt, int64_t d,
                             const int32_t* __restrict__ colcnt, int64_t p,
                             double* __restrict__ out) {
  __shared__ int sm[2][256];
  int a = 0, b = 0;
  for (int64_t i = threadIdx.x; i < d; i += 256) a = max(a, rowcnt[i]);
  for (int64_t j = threadIdx.x; j < p; j += 256) b = max(b, colcnt[j]);
  sm[0][threadIdx.x] = a;
  sm[1][threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[0][threadIdx.x] = max(sm[0][threadIdx.x], sm[0][threadIdx.x + s]);
      sm[1][threadIdx.x] = max(sm[1][threadIdx.x], sm[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (double)sm[0][0];
    out[1] = (double)sm[1][0];
  }
}

__device__ __forceinline__ float scaled(float e, double cs) {
  return cs > 0.0 ? (float)((double)e / cs) : 0.f;
}

// Dense: E_s = E / colsum (zero columns stay zero) into Es (d x p) and EsT
// (p x dpad, padding zero).
__global__ void k_pet_scale(const float* __restrict__ E, int64_t d, int64_t p,
                            const double* __restrict__ colsum, float* __restrict__ Es,
                            float* __restrict__ EsT, int64_t dpad) {
  const int64_t total = d * p;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / p, j = idx % p;
    const float v = scaled(E[idx], colsum[j]);
    Es[idx] = v;
    EsT[j * dpad + i] = v;
  }
}

// Sparse, by lines: the nonzeros of line i in increasing pixel order, packed
// by a wave-wide ballot.  One wave per line.
__global__ __launch_bounds__(256) void k_pet_fill_rows(const float* __restrict__ E, int64_t d,
                                                       int64_t p, const double* __restrict__ colsum,
                                                       int64_t wr, float* __restrict__ val,
                                                       int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= d) return;
  const uint64_t below = (1ull << lane) - 1ull;
  int64_t base = 0;
  for (int64_t j0 = 0; j0 < p; j0 += 64) {
    const int64_t j = j0 + lane;
    const float v = j < p ? E[i * p + j] : 0.f;
    const uint64_t mask = __ballot(v != 0.f);
    if (v != 0.f) {
      const int64_t at = i * wr + base + __popcll(mask & below);
      val[at] = scaled(v, colsum[j]);
      idx[at] = (int32_t)j;
    }
    base += __popcll(mask);
  }
}

// Sparse, by pixels: the nonzeros of column j in increasing line order.  One
// wave per pixel (column reads are strided; this runs once).
__global__ __launch_bounds__(256) void k_pet_fill_cols(const float* __restrict__ E, int64_t d,
                                                       int64_t p, const double* __restrict__ colsum,
                                                       int64_t wc, float* __restrict__ val,
                                                       int32_t* __restrict__ idx) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= p) return;
  const uint64_t below = (1ull << lane) - 1ull;
  const double cs = colsum[j];
  int64_t base = 0;
  for (int64_t i0 = 0; i0 < d; i0 += 64) {
    const int64_t i = i0 + lane;
    const float v = i < d ? E[i * p + j] : 0.f;
    const uint64_t mask = __ballot(v != 0.f);
    if (v != 0.f) {
      const int64_t at = j * wc + base + __popcll(mask & below);
      val[at] = scaled(v, cs);
      idx[at] = (int32_t)i;
    }
    base += __popcll(mask);
  }
}

// ---- one iteration ---------------------------------------------------------

__device__ __forceinline__ float ratio_of(float y, float s) { return y > 0.f ? y / s : 0.f; }

// The positive root for pixel j from t = (E_s^T ratio)_j and the source
// image.
__device__ __forceinline__ float pet_root(float t, const float* __restrict__ lam, int64_t j,
                                          int rows, int cols, float mu) {
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
  if (a == 0.f) return c;
  // a < 0 and c >= 0: the roots have opposite signs (or one is 0), and the
  // positive one is (b + s) / (-2a) = 2c / (s - b), s = sqrt(b^2 - 4ac);
  // take the form whose sum does not cancel
  const float s = sqrtf(fmaxf(b * b - 4.f * a * c, 0.f));
  if (b > 0.f) return (b + s) / (-2.f * a);
  return s - b > 0.f ? 2.f * c / (s - b) : 0.f;
}

// Dense ratio_i: one wave per line.
__global__ __launch_bounds__(256) void k_pet_forward(const float* __restrict__ Es, int64_t d,
                                                     int64_t p, const float* __restrict__ lam,
                                                     const float* __restrict__ y,
                                                     float* __restrict__ ratio,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
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
  s = group_sum<64>(s);
  if (lane == 0) ratio[i] = ratio_of(y[i], s);
}

// Dense update: one wave per pixel.
__global__ __launch_bounds__(256) void k_pet_backward(const float* __restrict__ EsT, int64_t dpad,
                                                      int64_t p, const float* __restrict__ ratio,
                                                      const float* __restrict__ lam, int rows,
                                                      int cols, float mu,
                                                      float* __restrict__ out,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
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
  t = group_sum<64>(t);
  if (lane == 0) out[j] = pet_root(t, lam, j, rows, cols, mu);
}

// Sparse ratio_i: one wave per line, lane k takes the entries k, k + 64, ...
__global__ __launch_bounds__(256) void k_pet_forward_ell(const float* __restrict__ val,
                                                         const int32_t* __restrict__ idx,
                                                         const int32_t* __restrict__ cnt,
                                                         int64_t wr, int64_t d,
                                                         const float* __restrict__ lam,
                                                         const float* __restrict__ y,
                                                         float* __restrict__ ratio,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= d) return;
  const int n = cnt[i];
  const float* v = val + i * wr;
  const int32_t* ix = idx + i * wr;
  float s = 0.f;
  for (int k = lane; k < n; k += 64) s = fmaf(v[k], lam[ix[k]], s);
  s = group_sum<64>(s);
  if (lane == 0) ratio[i] = ratio_of(y[i], s);
}

// Sparse update: a group of G lanes per pixel (G divides 64).
template <int G>
__global__ __launch_bounds__(256) void k_pet_backward_ell(const float* __restrict__ val,
                                                          const int32_t* __restrict__ idx,
                                                          const int32_t* __restrict__ cnt,
                                                          int64_t wc, int64_t p,
                                                          const float* __restrict__ ratio,
                                                          const float* __restrict__ lam, int rows,
                                                          int cols, float mu,
                                                          float* __restrict__ out,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
  const int64_t j = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int g = threadIdx.x % G;
  if (j >= p) return;  // whole groups leave together
  const int n = cnt[j];
  const float* v = val + j * wc;
  const int32_t* ix = idx + j * wc;
  float t = 0.f;
  for (int k = g; k < n; k += G) t = fmaf(v[k], ratio[ix[k]], t);
  t = group_sum<G>(t);
  if (g == 0) out[j] = pet_root(t, lam, j, rows, cols, mu);
}

__global__ void k_pet_copy(const float* __restrict__ src, float* __restrict__ dst, int64_t p,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256)
    dst[j] = src[j];
}

// ---- objective (float64) -----------------------------------------------------

// -(mu / 2) [(lambda_j - lambda_right)^2 + (lambda_j - lambda_below)^2]:
// every neighbour pair once.
__device__ __forceinline__ double pet_penalty_part(const float* __restrict__ lam, int64_t j,
                                                   int rows, int cols, double mu) {
  const int r = (int)(j / cols), cc = (int)(j % cols);
  const double lj = lam[j];
  double pen = 0.0;
  if (cc + 1 < cols) pen += (lj - lam[j + 1]) * (lj - lam[j + 1]);
  if (r + 1 < rows) pen += (lj - lam[j + cols]) * (lj - lam[j + cols]);
  return -0.5 * mu * pen;
}

__device__ __forceinline__ double line_term(float y, double b) {
  return (y > 0.f ? (double)y * log(b) : 0.0) - b;
}

// part[i] = y_i ln B_i - B_i (B_i in float64) for the lines, then the
// penalty parts, each times sign (+1, or -1 for the quasi-Newton test, which
// minimizes); one wave per line, then one wave per 64 pixels.
__global__ __launch_bounds__(256) void k_pet_objective(const float* __restrict__ Es, int64_t d,
                                                       int64_t p, const float* __restrict__ lam,
                                                       const float* __restrict__ y, int rows,
                                                       int cols, double mu, double sign,
                                                       double* __restrict__ part,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w < d) {
    const float* row = Es + w * p;
    double s = 0.0;
    for (int64_t j = lane; j < p; j += 64) s = fma((double)row[j], (double)lam[j], s);
    s = wave_sum_d(s);
    if (lane == 0) part[w] = sign * line_term(y[w], s);
  } else if (w < d + (p + 63) / 64) {
    const int64_t j = (w - d) * 64 + lane;
    if (j < p) part[d + j] = sign * pet_penalty_part(lam, j, rows, cols, mu);
  }
}

__global__ __launch_bounds__(256) void k_pet_objective_ell(
    const float* __restrict__ val, const int32_t* __restrict__ idx, const int32_t* __restrict__ cnt,
    int64_t wr, int64_t d, int64_t p, const float* __restrict__ lam, const float* __restrict__ y,
    int rows, int cols, double mu, double sign, double* __restrict__ part,
    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // the solve has stopped
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w < d) {
    const int n = cnt[w];
    const float* v = val + w * wr;
    const int32_t* ix = idx + w * wr;
    double s = 0.0;
    for (int k = lane; k < n; k += 64) s = fma((double)v[k], (double)lam[ix[k]], s);
    s = wave_sum_d(s);
    if (lane == 0) part[w] = sign * line_term(y[w], s);
  } else if (w < d + (p + 63) / 64) {
    const int64_t j = (w - d) * 64 + lane;
    if (j < p) part[d + j] = sign * pet_penalty_part(lam, j, rows, cols, mu);
  }
}

// The quasi-Newton decision taken (st[4]): lambda = xq.
__global__ void k_pet_qn_commit(const int32_t* __restrict__ st, const float* __restrict__ xq,
                                float* __restrict__ lam, int64_t p) {
  if (st[4] == 0) return;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256)
    lam[j] = xq[j];
}

// The stopping rule on the device, after a block of check_every iterations
// and the objective of its result (f in sd[1]): st = {stop, iterations done,
// iteration cap, check_every}, sd = {f at the previous check, f, tol}.
// stop: 1 the rule held, 2 another block would pass the cap, 3 f is not
// finite.  Once stop is set, every gated kernel of later blocks returns at
// once.
__global__ void k_pet_test(int32_t* __restrict__ st, double* __restrict__ sd) {
  if (blockIdx.x != 0 || threadIdx.x != 0 || st[0] != 0) return;
  const int32_t it = st[1] + st[3];
  st[1] = it;
  const double f = sd[1], fp = sd[0];
  if (!isfinite(f)) {
    st[0] = 3;
    return;
  }
  sd[0] = f;
  if (fabs(f - fp) / (fabs(fp) + 1.0) < sd[2])
    st[0] = 1;
  else if (it + st[3] > st[2])
    st[0] = 2;
}

__global__ void k_pet_solve_init(int32_t* __restrict__ st, double* __restrict__ sd, int32_t cap,
                                 int32_t check_every, double f0, double tol) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  st[0] = 0;
  st[1] = 0;
  st[2] = cap;
  st[3] = check_every;
  sd[0] = f0;
  sd[1] = f0;
  sd[2] = tol;
}

unsigned pblocks(int64_t total, int64_t cap = 65535) {
  const int64_t b = (total + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

constexpr int kPetGraphs = 5;  // graphs of 1, 2, 4, 8 and 16 iterations
constexpr int32_t kPetQnCap = 65536;  // QN iterations recorded per solve
constexpr int kPetSolveBlocks = 8;    // check blocks per replay of the solve graph
constexpr float kPetQnKappa = 0.5f;   // projection lambda >= kappa F(lambda)

}  // namespace

struct nmf_pet {
  hipStream_t st = nullptr;
  int64_t d = 0, p = 0, dpad = 0;
  int rows = 0, cols = 0;
  float mu = 0.f;
  double mu_d = 0.0;
  bool sparse = false;
  int64_t wr = 0, wc = 0;  // ELL widths (sparse)
  int group = 64;          // lanes per pixel in the sparse update
  float* lam = nullptr;    // caller's intensities, updated in place
  void* ws = nullptr;      // fixed-size part
  void* ws_e = nullptr;    // the layout of E_s
  float *y = nullptr, *ratio = nullptr, *lam2 = nullptr;
  double *colsum = nullptr, *part = nullptr;
  int32_t *rowcnt = nullptr, *colcnt = nullptr;
  uint32_t* flag = nullptr;
  float *Es = nullptr, *EsT = nullptr;       // dense
  float *rval = nullptr, *cval = nullptr;    // sparse values
  int32_t *ridx = nullptr, *cidx = nullptr;  // sparse indices
  double* hostbuf = nullptr;      // pinned, coherent
  double* hostbuf_dev = nullptr;  // the same memory as the device addresses it
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gp[kPetGraphs] = {};
  // device-side stopping rule of nmf_pet_solve
  const int32_t* gate = nullptr;  // the stop flag while a solve graph is captured
  int32_t* sst = nullptr;         // {stop, iterations, cap, check_every}
  double* ssd = nullptr;          // {f_prev, f, tol}
  hipGraphExec_t solve_graph = nullptr;
  int32_t solve_check = 0;  // check_every of solve_graph
  // QN(q)
  int qn_q = 0;
  void* qn_ws = nullptr;
  size_t qn_bytes = 0;
  float *qx0 = nullptr, *qxq = nullptr;
  double *qU = nullptr, *qV = nullptr, *qdpart = nullptr, *qGUU = nullptr, *qGUV = nullptr;
  double *qcoef = nullptr, *qf = nullptr;
  int32_t* qst = nullptr;
  double* qfout = nullptr;      // pinned, coherent: -f after every QN iteration
  double* qfout_dev = nullptr;  // its device-side address
  hipGraphExec_t qn_graph = nullptr;
};

namespace {

#define PTRY_HIP(expr)                              \
  do {                                              \
    if ((expr) != hipSuccess) return NMF_EDEVICE;   \
  } while (0)

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  }
};

nmf_status pet_iter(nmf_pet* m, const float* src, float* dst) {
  const unsigned lines = (unsigned)((m->d + 3) / 4);
  if (!m->sparse) {
    hipLaunchKernelGGL(k_pet_forward, dim3(lines), dim3(256), 0, m->st, m->Es, m->d, m->p, src,
                       m->y, m->ratio, m->gate);
    PTRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pet_backward, dim3((unsigned)((m->p + 3) / 4)), dim3(256), 0, m->st,
                       m->EsT, m->dpad, m->p, m->ratio, src, m->rows, m->cols, m->mu, dst,
                       m->gate);
    PTRY_HIP(hipGetLastError());
    return NMF_OK;
  }
  hipLaunchKernelGGL(k_pet_forward_ell, dim3(lines), dim3(256), 0, m->st, m->rval, m->ridx,
                     m->rowcnt, m->wr, m->d, src, m->y, m->ratio, m->gate);
  PTRY_HIP(hipGetLastError());
  const int g = m->group;
  const unsigned blocks = (unsigned)((m->p + 256 / g - 1) / (256 / g));
  if (g == 16)
    hipLaunchKernelGGL(k_pet_backward_ell<16>, dim3(blocks), dim3(256), 0, m->st, m->cval,
                       m->cidx, m->colcnt, m->wc, m->p, m->ratio, src, m->rows, m->cols, m->mu,
                       dst, m->gate);
  else if (g == 32)
    hipLaunchKernelGGL(k_pet_backward_ell<32>, dim3(blocks), dim3(256), 0, m->st, m->cval,
                       m->cidx, m->colcnt, m->wc, m->p, m->ratio, src, m->rows, m->cols, m->mu,
                       dst, m->gate);
  else
    hipLaunchKernelGGL(k_pet_backward_ell<64>, dim3(blocks), dim3(256), 0, m->st, m->cval,
                       m->cidx, m->colcnt, m->wc, m->p, m->ratio, src, m->rows, m->cols, m->mu,
                       dst, m->gate);
  PTRY_HIP(hipGetLastError());
  return NMF_OK;
}

// `iters` iterations from and back into the caller's buffer: they alternate
// caller -> copy -> caller, and an odd count ends with a copy back.
nmf_status pet_iters(nmf_pet* m, int iters) {
  for (int it = 0; it < iters; ++it) {
    const bool even = (it & 1) == 0;
    nmf_status s = pet_iter(m, even ? m->lam : m->lam2, even ? m->lam2 : m->lam);
    if (s != NMF_OK) return s;
  }
  if (iters & 1) {
    hipLaunchKernelGGL(k_pet_copy, dim3(pblocks(m->p, 1024)), dim3(256), 0, m->st, m->lam2,
                       m->lam, m->p, m->gate);
    PTRY_HIP(hipGetLastError());
  }
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
    s = pet_iters(m, iters);
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

// sign * f(lam) into out (device-visible address), in a fixed order.
nmf_status pet_objective_enqueue(nmf_pet* m, const float* lam, double sign, double* out) {
  const int64_t waves = m->d + (m->p + 63) / 64;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  if (m->sparse)
    hipLaunchKernelGGL(k_pet_objective_ell, dim3(blocks), dim3(256), 0, m->st, m->rval, m->ridx,
                       m->rowcnt, m->wr, m->d, m->p, lam, m->y, m->rows, m->cols, m->mu_d, sign,
                       m->part, m->gate);
  else
    hipLaunchKernelGGL(k_pet_objective, dim3(blocks), dim3(256), 0, m->st, m->Es, m->d, m->p, lam,
                       m->y, m->rows, m->cols, m->mu_d, sign, m->part, m->gate);
  PTRY_HIP(hipGetLastError());
  PTRY_HIP(launch_reduce_f64(m->part, m->d + m->p, out, m->st));
  return NMF_OK;
}

nmf_status pet_objective_sync(nmf_pet* m, double* f) {
  nmf_status s = pet_objective_enqueue(m, m->lam, 1.0, m->hostbuf_dev);
  if (s != NMF_OK) return s;
  PTRY_HIP(hipStreamSynchronize(m->st));
  *f = m->hostbuf[0];
  return NMF_OK;
}

// One QN iteration (Zhou, Alexander & Lange), every decision on the device:
// x0 = lambda; x1 = F(x0) (in lam2); x2 = F(x1) (in lambda); the secant pair
// (x1 - x0, x2 - x1) enters the float64 rings; xq = max(x1 + V c, kappa x1);
// -f(x2) and -f(xq) are compared (the shared selection minimizes); lambda =
// xq when taken.
nmf_status pet_qn_enqueue(nmf_pet* m) {
  const int64_t D = m->p;
  const int q = m->qn_q;
  PTRY_HIP(launch_qn_copy(m->lam, m->qx0, D, m->st));
  nmf_status s = pet_iter(m, m->lam, m->lam2);
  if (s == NMF_OK) s = pet_iter(m, m->lam2, m->lam);
  if (s != NMF_OK) return s;
  PTRY_HIP(launch_qn_pairs(m->qx0, m->lam2, m->lam, m->qU, m->qV, D, q, m->qst, m->st));
  PTRY_HIP(launch_qn_dots_solve(m->qU, m->qV, D, q, m->qst, m->qdpart, m->qGUU, m->qGUV, m->qcoef,
                                m->st));
  PTRY_HIP(launch_qn_combine(m->lam2, m->qV, m->qcoef, D, q, kPetQnKappa, m->qst, m->qxq, m->st));
  s = pet_objective_enqueue(m, m->lam, -1.0, m->qf + 0);
  if (s == NMF_OK) s = pet_objective_enqueue(m, m->qxq, -1.0, m->qf + 1);
  if (s != NMF_OK) return s;
  PTRY_HIP(launch_qn_select(m->qf, m->qst, m->qfout_dev, kPetQnCap, m->st));
  hipLaunchKernelGGL(k_pet_qn_commit, dim3(pblocks(D, 1024)), dim3(256), 0, m->st, m->qst, m->qxq,
                     m->lam, D);
  PTRY_HIP(hipGetLastError());
  return NMF_OK;
}

// QN workspace (kept while q is unchanged) and its graph; the history is
// cleared on every call.
nmf_status pet_qn_prepare(nmf_pet* m, int q) {
  const int64_t D = m->p;
  const int qm = qn_max_q();
  if (m->qn_q != q || !m->qn_ws) {
    if (m->qn_graph) (void)hipGraphExecDestroy(m->qn_graph);
  if (m->solve_graph) (void)hipGraphExecDestroy(m->solve_graph);
    m->qn_graph = nullptr;
    if (m->qn_ws) (void)hipFree(m->qn_ws);
    m->qn_ws = nullptr;
    Carver a;
    const size_t ox0 = a.take(4 * (size_t)D), oxq = a.take(4 * (size_t)D);
    const size_t oU = a.take(8 * (size_t)q * D), oV = a.take(8 * (size_t)q * D);
    const size_t odp = a.take(8 * (size_t)qn_dot_blocks() * 3 * q);
    const size_t oguu = a.take(8 * (size_t)qm * qm), oguv = a.take(8 * (size_t)qm * qm);
    const size_t oc = a.take(8 * (size_t)qm), of = a.take(8 * 2), ost = a.take(4 * 8);
    if (hipMalloc(&m->qn_ws, a.off) != hipSuccess) {
      m->qn_ws = nullptr;
      (void)hipGetLastError();
      return NMF_ENOMEM;
    }
    m->qn_bytes = a.off;
    char* b = static_cast<char*>(m->qn_ws);
    m->qx0 = reinterpret_cast<float*>(b + ox0);
    m->qxq = reinterpret_cast<float*>(b + oxq);
    m->qU = reinterpret_cast<double*>(b + oU);
    m->qV = reinterpret_cast<double*>(b + oV);
    m->qdpart = reinterpret_cast<double*>(b + odp);
    m->qGUU = reinterpret_cast<double*>(b + oguu);
    m->qGUV = reinterpret_cast<double*>(b + oguv);
    m->qcoef = reinterpret_cast<double*>(b + oc);
    m->qf = reinterpret_cast<double*>(b + of);
    m->qst = reinterpret_cast<int32_t*>(b + ost);
    m->qn_q = q;
    if (!m->qfout) {
      if (hipHostMalloc(reinterpret_cast<void**>(&m->qfout), sizeof(double) * kPetQnCap,
                        hipHostMallocCoherent) != hipSuccess) {
        m->qfout = nullptr;
        (void)hipGetLastError();
        return NMF_ENOMEM;
      }
      PTRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&m->qfout_dev), m->qfout, 0));
    }
  }
  PTRY_HIP(launch_fill_u32(static_cast<uint32_t*>(m->qn_ws), (int64_t)(m->qn_bytes / 4), 0u,
                           m->st));
  if (!m->qn_graph) {
    if (!m->cap_stream) PTRY_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    PTRY_HIP(hipStreamSynchronize(m->st));
    hipStream_t user = m->st;
    m->st = m->cap_stream;
    hipGraph_t graph = nullptr;
    nmf_status s = NMF_OK;
    if (hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      s = NMF_EDEVICE;
    if (s == NMF_OK) {
      s = pet_qn_enqueue(m);
      const hipError_t e = hipStreamEndCapture(m->cap_stream, &graph);
      if (s == NMF_OK && (e != hipSuccess || !graph)) s = NMF_EDEVICE;
    }
    m->st = user;
    if (s == NMF_OK && (hipGraphInstantiate(&m->qn_graph, graph, nullptr, nullptr, 0) !=
                            hipSuccess ||
                        hipGraphUpload(m->qn_graph, m->st) != hipSuccess))
      s = NMF_EDEVICE;
    if (graph) (void)hipGraphDestroy(graph);
    if (s != NMF_OK) return s;
  }
  return NMF_OK;
}

// kPetSolveBlocks check blocks, each check_every gated iterations, the gated
// objective into ssd[1] and the test, captured as one graph.
nmf_status pet_solve_capture(nmf_pet* m, int32_t check_every) {
  if (m->solve_graph && m->solve_check == check_every) return NMF_OK;
  if (m->solve_graph) (void)hipGraphExecDestroy(m->solve_graph);
  m->solve_graph = nullptr;
  if (!m->cap_stream) PTRY_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
  PTRY_HIP(hipStreamSynchronize(m->st));
  hipStream_t user = m->st;
  m->st = m->cap_stream;
  m->gate = m->sst;
  hipGraph_t graph = nullptr;
  nmf_status s = NMF_OK;
  if (hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    s = NMF_EDEVICE;
  if (s == NMF_OK) {
    for (int b = 0; b < kPetSolveBlocks && s == NMF_OK; ++b) {
      s = pet_iters(m, check_every);
      if (s == NMF_OK) s = pet_objective_enqueue(m, m->lam, 1.0, m->ssd + 1);
      if (s == NMF_OK) {
        hipLaunchKernelGGL(k_pet_test, dim3(1), dim3(64), 0, m->st, m->sst, m->ssd);
        if (hipGetLastError() != hipSuccess) s = NMF_EDEVICE;
      }
    }
    const hipError_t e = hipStreamEndCapture(m->cap_stream, &graph);
    if (s == NMF_OK && (e != hipSuccess || !graph)) s = NMF_EDEVICE;
  }
  m->gate = nullptr;
  m->st = user;
  if (s == NMF_OK && (hipGraphInstantiate(&m->solve_graph, graph, nullptr, nullptr, 0) !=
                          hipSuccess ||
                      hipGraphUpload(m->solve_graph, m->st) != hipSuccess))
    s = NMF_EDEVICE;
  if (graph) (void)hipGraphDestroy(graph);
  if (s == NMF_OK) m->solve_check = check_every;
  return s;
}

void pet_free(nmf_pet* m) {
  if (!m) return;
  for (hipGraphExec_t g : m->gp)
    if (g) (void)hipGraphExecDestroy(g);
  if (m->qn_graph) (void)hipGraphExecDestroy(m->qn_graph);
  if (m->qn_ws) (void)hipFree(m->qn_ws);
  if (m->qfout) (void)hipHostFree(m->qfout);
  if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
  if (m->ws_e) (void)hipFree(m->ws_e);
  if (m->ws) (void)hipFree(m->ws);
  if (m->hostbuf) (void)hipHostFree(m->hostbuf);
  delete m;
}

// Workspace, validation, counts and the layout of E_s.  Synchronizes.
nmf_status pet_setup(nmf_pet* m, const float* E, const float* y, int32_t layout) {
  const int64_t d = m->d, p = m->p;
  Carver a;
  const size_t oy = a.take(4 * (size_t)m->dpad), orat = a.take(4 * (size_t)m->dpad);
  const size_t olam2 = a.take(4 * (size_t)p), ocs = a.take(8 * (size_t)p);
  const size_t opart = a.take(8 * (size_t)(d + p)), orc = a.take(4 * (size_t)d);
  const size_t occ = a.take(4 * (size_t)p), ofl = a.take(4);
  const size_t osst = a.take(4 * 4), ossd = a.take(8 * 4);
  if (hipMalloc(&m->ws, a.off) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&m->hostbuf), 4 * sizeof(double),
                    hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return NMF_ENOMEM;
  }
  PTRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&m->hostbuf_dev), m->hostbuf, 0));
  char* b = static_cast<char*>(m->ws);
  m->y = reinterpret_cast<float*>(b + oy);
  m->ratio = reinterpret_cast<float*>(b + orat);
  m->lam2 = reinterpret_cast<float*>(b + olam2);
  m->colsum = reinterpret_cast<double*>(b + ocs);
  m->part = reinterpret_cast<double*>(b + opart);
  m->rowcnt = reinterpret_cast<int32_t*>(b + orc);
  m->colcnt = reinterpret_cast<int32_t*>(b + occ);
  m->flag = reinterpret_cast<uint32_t*>(b + ofl);
  m->sst = reinterpret_cast<int32_t*>(b + osst);
  m->ssd = reinterpret_cast<double*>(b + ossd);
  // zero everything (the ratios' padding must read as zero)
  PTRY_HIP(launch_fill_u32(static_cast<uint32_t*>(m->ws), (int64_t)(a.off / 4), 0u, m->st));
  // E, y and the start must be finite and nonnegative
  PTRY_HIP(launch_validate(E, p, d, p, m->flag, m->st));
  PTRY_HIP(launch_validate(y, d, 1, d, m->flag, m->st));
  PTRY_HIP(launch_validate(m->lam, p, 1, p, m->flag, m->st));
  hipLaunchKernelGGL(k_pet_colsum, dim3((unsigned)((p + 3) / 4)), dim3(256), 0, m->st, E, d, p,
                     m->colsum, m->colcnt);
  hipLaunchKernelGGL(k_pet_rowcnt, dim3((unsigned)((d + 3) / 4)), dim3(256), 0, m->st, E, d, p,
                     m->rowcnt);
  hipLaunchKernelGGL(k_pet_maxcnt, dim3(1), dim3(256), 0, m->st, m->rowcnt, d, m->colcnt, p,
                     m->hostbuf_dev);
  PTRY_HIP(hipGetLastError());
  PTRY_HIP(hipMemcpyAsync(m->y, y, 4 * (size_t)d, hipMemcpyDeviceToDevice, m->st));
  PTRY_HIP(hipMemcpyAsync(m->hostbuf + 2, m->flag, sizeof(uint32_t), hipMemcpyDeviceToHost,
                          m->st));
  PTRY_HIP(hipStreamSynchronize(m->st));
  uint32_t bad;
  std::memcpy(&bad, m->hostbuf + 2, sizeof(bad));
  if (bad) return NMF_EINVAL;
  const int64_t maxrow = (int64_t)m->hostbuf[0], maxcol = (int64_t)m->hostbuf[1];
  // the padded rows pay when each is at most a quarter of a dense one
  m->sparse = layout == NMF_PET_SPARSE ||
              (layout == NMF_PET_AUTO && 4 * maxrow <= p && 4 * maxcol <= d);
  Carver e;
  if (!m->sparse) {
    const size_t oEs = e.take(4 * (size_t)d * p), oEsT = e.take(4 * (size_t)p * m->dpad);
    if (hipMalloc(&m->ws_e, e.off) != hipSuccess) {
      (void)hipGetLastError();
      return NMF_ENOMEM;
    }
    char* q = static_cast<char*>(m->ws_e);
    m->Es = reinterpret_cast<float*>(q + oEs);
    m->EsT = reinterpret_cast<float*>(q + oEsT);
    PTRY_HIP(launch_fill_u32(static_cast<uint32_t*>(m->ws_e), (int64_t)(e.off / 4), 0u, m->st));
    hipLaunchKernelGGL(k_pet_scale, dim3(pblocks(d * p)), dim3(256), 0, m->st, E, d, p, m->colsum,
                       m->Es, m->EsT, m->dpad);
  } else {
    m->wr = std::max<int64_t>(rup(maxrow, 4), 4);
    m->wc = std::max<int64_t>(rup(maxcol, 4), 4);
    m->group = maxcol > 32 ? 64 : (maxcol > 16 ? 32 : 16);
    const size_t orv = e.take(4 * (size_t)d * m->wr), ori = e.take(4 * (size_t)d * m->wr);
    const size_t ocv = e.take(4 * (size_t)p * m->wc), oci = e.take(4 * (size_t)p * m->wc);
    if (hipMalloc(&m->ws_e, e.off) != hipSuccess) {
      (void)hipGetLastError();
      return NMF_ENOMEM;
    }
    char* q = static_cast<char*>(m->ws_e);
    m->rval = reinterpret_cast<float*>(q + orv);
    m->ridx = reinterpret_cast<int32_t*>(q + ori);
    m->cval = reinterpret_cast<float*>(q + ocv);
    m->cidx = reinterpret_cast<int32_t*>(q + oci);
    PTRY_HIP(launch_fill_u32(static_cast<uint32_t*>(m->ws_e), (int64_t)(e.off / 4), 0u, m->st));
    hipLaunchKernelGGL(k_pet_fill_rows, dim3((unsigned)((d + 3) / 4)), dim3(256), 0, m->st, E, d,
                       p, m->colsum, m->wr, m->rval, m->ridx);
    hipLaunchKernelGGL(k_pet_fill_cols, dim3((unsigned)((p + 3) / 4)), dim3(256), 0, m->st, E, d,
                       p, m->colsum, m->wc, m->cval, m->cidx);
  }
  PTRY_HIP(hipGetLastError());
  PTRY_HIP(hipStreamSynchronize(m->st));
  return NMF_OK;
}

}  // namespace

extern "C" {

nmf_status nmf_pet_create(nmf_pet** out, const float* E, int64_t d, int64_t p, const float* y,
                          int32_t rows, int32_t cols, double mu, float* lambda, int32_t layout,
                          void* stream) {
  if (!out) return NMF_EINVAL;
  *out = nullptr;
  if (!E || !y || !lambda || d < 1 || p < 1 || rows < 1 || cols < 1) return NMF_EINVAL;
  if ((int64_t)rows * cols != p || !(mu >= 0.0) || !std::isfinite(mu)) return NMF_EINVAL;
  if (layout < NMF_PET_AUTO || layout > NMF_PET_SPARSE) return NMF_EINVAL;
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
  const nmf_status s = pet_setup(m, E, y, layout);
  if (s != NMF_OK) {
    (void)hipStreamSynchronize(m->st);
    pet_free(m);
    return s;
  }
  *out = m;
  return NMF_OK;
}

nmf_status nmf_pet_layout(const nmf_pet* m, int32_t* layout) {
  if (!m || !layout) return NMF_EINVAL;
  *layout = m->sparse ? NMF_PET_SPARSE : NMF_PET_DENSE;
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
  if (max_iters >= check_every) {
    // whole check blocks on the device: the rule is tested there after each
    // block and stops the blocks after it; the host reads the state once per
    // replay of kPetSolveBlocks blocks
    s = pet_solve_capture(m, check_every);
    if (s != NMF_OK) return s;
    hipLaunchKernelGGL(k_pet_solve_init, dim3(1), dim3(64), 0, m->st, m->sst, m->ssd, max_iters,
                       check_every, f_prev, tol);
    PTRY_HIP(hipGetLastError());
    int32_t* hs = reinterpret_cast<int32_t*>(m->hostbuf);  // pinned
    const int64_t blocks = max_iters / check_every;
    for (int64_t r = 0; r <= blocks / kPetSolveBlocks; ++r) {
      PTRY_HIP(hipGraphLaunch(m->solve_graph, m->st));
      PTRY_HIP(hipMemcpyAsync(hs, m->sst, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, m->st));
      PTRY_HIP(hipStreamSynchronize(m->st));
      if (hs[0] != 0) break;
    }
    const int32_t stop = hs[0];
    k = hs[1];
    PTRY_HIP(hipMemcpyAsync(m->hostbuf, m->ssd, 2 * sizeof(double), hipMemcpyDeviceToHost, m->st));
    PTRY_HIP(hipStreamSynchronize(m->st));
    *iters_done = k;
    *f_host = m->hostbuf[1];
    f_prev = m->hostbuf[0];
    if (stop == 1) return NMF_OK;
    if (stop == 3) return NMF_ENONFINITE;
    // stop == 2: fewer than check_every iterations remain
  }
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

nmf_status nmf_pet_solve_qn(nmf_pet* m, int32_t q, int32_t max_evals, double tol,
                            int32_t check_every, int32_t* evals_done, int32_t* accepted,
                            double* f_host, double* trace, int32_t trace_len) {
  if (!m || !evals_done || !f_host || q < 1 || max_evals < 0 || check_every < 1 ||
      !(tol >= 0.0) || (trace && trace_len < 0))
    return NMF_EINVAL;
  if (q > qn_max_q() || max_evals / 2 > kPetQnCap) return NMF_EINVAL;
  *evals_done = 0;
  if (accepted) *accepted = 0;
  double f_prev;
  nmf_status s = nmf_pet_objective(m, &f_prev);
  *f_host = f_prev;
  if (s != NMF_OK) return s;
  int32_t nt = 0;
  if (trace && nt < trace_len) trace[nt++] = f_prev;
  s = pet_qn_prepare(m, q);
  if (s != NMF_OK) return s;
  // chunks of check_every map evaluations (check_every / 2 QN iterations,
  // at least one); the rule is tested on the accepted objective at the end
  // of each chunk
  const int32_t chunk = std::max<int32_t>(1, check_every / 2);
  const int32_t total = max_evals / 2;
  int32_t it = 0;
  bool done = false;
  double f = f_prev;
  while (!done && it < total) {
    const int32_t todo = std::min(chunk, total - it);
    for (int32_t k = 0; k < todo; ++k) PTRY_HIP(hipGraphLaunch(m->qn_graph, m->st));
    PTRY_HIP(hipStreamSynchronize(m->st));
    for (int32_t k = it; k < it + todo; ++k)
      if (trace && nt < trace_len) trace[nt++] = -m->qfout[k];
    it += todo;
    f = -m->qfout[it - 1];
    if (!std::isfinite(f)) {
      s = NMF_ENONFINITE;
      break;
    }
    done = std::fabs(f - f_prev) / (std::fabs(f_prev) + 1.0) < tol;
    f_prev = f;
  }
  *evals_done = 2 * it;
  *f_host = f;
  if (accepted) {
    int32_t* st = reinterpret_cast<int32_t*>(m->hostbuf);  // pinned
    PTRY_HIP(hipMemcpyAsync(st, m->qst, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, m->st));
    PTRY_HIP(hipStreamSynchronize(m->st));
    *accepted = st[1];
  }
  if (s != NMF_OK) return s;
  return done ? NMF_OK : NMF_ENOTCONVERGED;
}

void nmf_pet_destroy(nmf_pet* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->st);
  pet_free(m);
}

}  // extern "C"
