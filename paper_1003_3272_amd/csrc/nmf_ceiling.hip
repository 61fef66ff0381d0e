// Measured rate ceilings of the device the library runs on: an HBM read
// stream and the dense throughput of the matrix and vector instructions the
// kernels use.  A measurement aid beside the published peaks (which assume
// a clock and an issue rate the chip need not sustain); not a step of the
// method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmf_ceiling.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kGrid = 2048;                    // workgroups of the compute kinds
constexpr int kThreads = 256;
constexpr int64_t kSinkBytes = 4 << 20;        // >= kGrid * kThreads * 8
constexpr int64_t kMinBytes = 64ll << 20;
constexpr int kReadGrid = 4096;

// Streams count float4 items, each once, and writes one sum per workgroup
// (so the loads are not dead); sink holds kReadGrid floats.
__global__ __launch_bounds__(kThreads) void k_read(const float4* __restrict__ x, int64_t count,
                                                   float* __restrict__ sink) {
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kThreads) {
    const float4 v = x[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ float red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// CH independent accumulator chains per wave, iters rounds; every lane
// writes one value of its chains to sink[global thread id].
template <int CH>
__global__ __launch_bounds__(kThreads) void k_mfma_f64(double* __restrict__ sink, int iters,
                                                      double a0) {
  v4d acc[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const double a = a0 + threadIdx.x * 1e-9, b = a0 * 0.5;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < CH; ++i) s += (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(kThreads) void k_mfma_f32(double* __restrict__ sink, int iters,
                                                      float a0) {
  v4f acc[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  const float a = a0 + threadIdx.x * 1e-7f, b = a0 * 0.5f;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CH; ++i) s += (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(kThreads) void k_mfma_bf16(double* __restrict__ sink, int iters,
                                                       float a0) {
  v4f acc[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  v8bf a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(a0 + threadIdx.x * 1e-3f);
    b[e] = (__bf16)(a0 * 0.5f);
  }
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CH; ++i) s += (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// the 32 x 32 shapes: v_mfma_f32_32x32x2f32 (BF false) or
// v_mfma_f32_32x32x16_bf16 (BF true)
template <int CH, bool BF>
__global__ __launch_bounds__(kThreads) void k_mfma32(double* __restrict__ sink, int iters,
                                                    float a0) {
  v16f acc[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[i][e] = 0.f;
  const float af = a0 + threadIdx.x * 1e-7f, bfv = a0 * 0.5f;
  v8bf a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(a0 + threadIdx.x * 1e-3f);
    b[e] = (__bf16)(a0 * 0.5f);
  }
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if constexpr (BF)
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i], 0, 0, 0);
      else
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(af, bfv, acc[i], 0, 0, 0);
    }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CH; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[i][e];
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(kThreads) void k_fma_f64(double* __restrict__ sink, int iters,
                                                     double a0) {
  double acc[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) acc[i] = a0 * (double)(threadIdx.x + i);
  const double a = a0 * 0.999, b = a0 * 1e-3;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = fma(acc[i], a, b);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < CH; ++i) s += acc[i];
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// One launch of the kind; its work (bytes or flops) goes to *work.
hipError_t launch_kind(int32_t kind, void* buf, int64_t bytes, hipStream_t st, double* work) {
  double* sink = static_cast<double*>(buf);
  const dim3 g(kGrid), b(kThreads);
  const double waves = (double)kGrid * (kThreads / 64);
  switch (kind) {
    case NMF_CEIL_HBM_READ: {
      // reads [0, bytes - sink), the per-workgroup sums go to the tail
      const int64_t count = (bytes - kSinkBytes) / 16;
      float* rsink = reinterpret_cast<float*>(static_cast<char*>(buf) + (bytes - kSinkBytes));
      hipLaunchKernelGGL(k_read, dim3(kReadGrid), b, 0, st,
                         static_cast<const float4*>(buf), count, rsink);
      *work = (double)count * 16.0;
      break;
    }
    case NMF_CEIL_MFMA_F32:
      hipLaunchKernelGGL(k_mfma_f32<8>, g, b, 0, st, sink, 2048, 1.f);
      *work = waves * 2048 * 8 * 2.0 * 16 * 16 * 4;
      break;
    case NMF_CEIL_MFMA_BF16:
      hipLaunchKernelGGL(k_mfma_bf16<8>, g, b, 0, st, sink, 1024, 1.f);
      *work = waves * 1024 * 8 * 2.0 * 16 * 16 * 32;
      break;
    case NMF_CEIL_MFMA_F64:
      hipLaunchKernelGGL(k_mfma_f64<4>, g, b, 0, st, sink, 1024, 1.0);
      *work = waves * 1024 * 4 * 2.0 * 16 * 16 * 4;
      break;
    case NMF_CEIL_FMA_F64:
      hipLaunchKernelGGL(k_fma_f64<16>, g, b, 0, st, sink, 4096, 1.0);
      *work = (double)kGrid * kThreads * 4096 * 16 * 2.0;
      break;
    case NMF_CEIL_MFMA_F32_32:
      hipLaunchKernelGGL((k_mfma32<4, false>), g, b, 0, st, sink, 1024, 1.f);
      *work = waves * 1024 * 4 * 2.0 * 32 * 32 * 2;
      break;
    case NMF_CEIL_MFMA_BF16_32:
      hipLaunchKernelGGL((k_mfma32<4, true>), g, b, 0, st, sink, 512, 1.f);
      *work = waves * 512 * 4 * 2.0 * 32 * 32 * 16;
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" int32_t nmf_ceiling(int32_t kind, void* buf, int64_t bytes, int32_t reps,
                               double* rate_host, void* stream) {
  if (kind < NMF_CEIL_HBM_READ || kind > NMF_CEIL_MFMA_BF16_32 || !buf || !rate_host ||
      bytes < kMinBytes || bytes % 256 != 0 || reps < 1 || reps > 1000)
    return -1;
  if (reinterpret_cast<uintptr_t>(buf) % 256 != 0) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double work = 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return -3;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -3;
  }
  int32_t rc = -3;
  float ms = 0.f;
  do {
    if (launch_kind(kind, buf, bytes, st, &work) != hipSuccess) break;  // warm-up
    if (hipEventRecord(e0, st) != hipSuccess) break;
    bool ok = true;
    for (int32_t i = 0; i < reps && ok; ++i) ok = launch_kind(kind, buf, bytes, st, &work) == hipSuccess;
    if (!ok || hipEventRecord(e1, st) != hipSuccess) break;
    if (hipEventSynchronize(e1) != hipSuccess) break;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) break;
    *rate_host = work * reps / (ms * 1e-3);
    rc = 0;
  } while (false);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
