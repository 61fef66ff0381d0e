// Batched tier: many independent multiplicative-update NMF problems of
// uneven p, n and r (r <= 64) advanced together by ONE persistent kernel
// launch per call (replayed from a hipGraph).
//
// One iteration of a problem (Algorithm 1, W update then H update) is two
// phases of tiles:
//   phase W, tile t: rows [t*MB, t*MB+MB) of V.  A = V_rows H^T (K = n) on
//     the matrix cores, then the fused epilogue B = W_rows G_H,
//     W_rows <- W_rows * A / B (entry kept where B <= 0), and the tile's
//     partial Gram W_rows^T W_rows;
//   phase H, tile t: columns [t*NB, t*NB+NB) of V.  S^T = V_cols^T W (K = p),
//     then D^T = H_cols^T G_W, H_cols <- H_cols * S / D (same guard), and the
//     tile's partial Gram H_cols H_cols^T.
// The last tile of a phase to finish (an arrival counter per problem) sums
// the partial Grams in tile order, so G_W and G_H are deterministic, and then
// publishes the phase as done.  A phase-W tile of iteration i waits until
// phase H of iteration i-1 of its problem is done; a phase-H tile waits for
// phase W of the same iteration (which also orders every read of W and H
// before the next overwrite).
//
// Workgroups of the persistent grid take tiles from one queue in the order
// (iteration, phase, problem, tile); a tile only waits for tiles earlier in
// that order, which running workgroups hold, so the schedule cannot
// deadlock.  Every wait is bounded in time as well: past the bound the
// kernel raises an error flag, every other wait returns at once and all
// workgroups leave, so the launch always ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/nmf.h"
#include "nmf_internal.h"

namespace nmfb {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kThreads = 256;
constexpr int kMaxNB = 128;
constexpr int kMaxMB = 128;
constexpr int kStageBytes = (kMaxMB + 64) * 128;  // largest copy-ring stage
// Copy-ring depth: 3 stages (72 KB of LDS) with two workgroups per CU, 5
// stages (120 KB) with one.
constexpr int kLdsBytes3 = 3 * kStageBytes, kLdsBytes5 = 5 * kStageBytes;
static_assert((kMaxMB * 68 + 64 * 68) * 4 <= kLdsBytes3, "phase W epilogue fits");
static_assert((64 * (kMaxNB + 16) + 64 * 80) * 4 <= kLdsBytes3, "phase H epilogue fits");

// The persistent kernels' LDS: the copy ring during a tile's product, then
// the tile's epilogue.  At namespace scope so that the out-of-line tile
// functions address it directly (as LDS, not through generic pointers); each
// kernel allocates only the array its tile functions use.
__shared__ __attribute__((aligned(1024))) char g_lds3[kLdsBytes3];
__shared__ __attribute__((aligned(1024))) char g_lds5[kLdsBytes5];
template <int S>
__device__ __forceinline__ char* lds_base() {
  static_assert(S == 3 || S == 5, "ring depth");
  if constexpr (S == 3) return g_lds3;
  else return g_lds5;
}

// A wait longer than this many ticks of the 100 MHz constant clock (2 s)
// means the schedule is broken: raise the error flag and leave.
constexpr uint64_t kWaitTicks = 200000000ull;

}  // namespace

// Per-problem descriptor (device copy; see the host builder for meaning).
struct Prob {
  float* V;      // padded copy of V: rows round_up(p, 128), k to round_up(n, 32)
  float* VT;     // padded V^T: rows round_up(n, 128), k to round_up(p, 32)
  const float* Vsrc;  // caller's V (read once, at creation)
  float* Wp;     // p x rp, pitch rp (working W, padded columns zero)
  float* WT;     // W^T: rpy rows, k to round_up(p, 32), padding zero
  float* Hp;     // rpy rows, k to round_up(n, 32), padded rows and columns zero
  float* GH;     // rp x rp
  float* GW;     // rp x rp
  float* gpart;  // max(tilesW, tilesH) x rp x rp partial Grams
  float* W;      // caller's W (p x r)
  float* H;      // caller's H (r x n)
  int64_t ldv, ldvt, ldsrc, ldh, ldwt;  // row pitches (floats), see spread()
  int32_t p, n, r, rp;  // rp = r rounded up to 16; rpy = rp rounded up to 32
  int32_t msw, msh;     // phase W tile rows = 64 msw; phase H tile columns = 64 msh
  int32_t tilesW, tilesH;
  int32_t kw, kh;       // 32-float stages along n (phase W) and along p (phase H)
};

// Counter block, cleared before every launch: [0] error flag of this launch;
// for each queue q, [kHeadBase + 32 q] its head and [kHeadBase + 32 q + 1]
// its completed tiles; then 4 per problem from kCtrBase: W arrivals, W
// phases done, H arrivals, H phases done.  One more word after the block
// keeps the error flag across launches until the host reads and clears it.
constexpr int kMaxQueues = 16;
constexpr int kCtrErr = 0;
constexpr int kHeadBase = 32;
constexpr int kCtrBase = kHeadBase + 32 * kMaxQueues;

// One tile queue: its schedule starts at sched[off] and holds per_iter
// tiles per iteration.
struct QInfo {
  uint32_t off, per_iter;
};

namespace {

// s_waitcnt vmcnt(VM) (gfx9 encoding, vmcnt split over bits 3:0 and
// 15:14), leaving expcnt and lgkmcnt unconstrained.
template <int VM>
__device__ __forceinline__ void wait_vm() {
  static_assert(VM >= 0 && VM < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((VM & 0xF) | (0x7 << 4) | (0xF << 8) | (((VM >> 4) & 0x3) << 14));
}

// Coherence of the data tiles pass to each other (factors, W^T, Grams,
// partial Grams).  Every access to it is device-scope: loads and stores are
// relaxed agent-scope atomics (sc1: served at the device's coherence point,
// not from a compute unit's L1 or a non-coherent L2 line), and the copy ring
// reads these operands with the same cache policy.  A producer's stores are
// therefore visible device-wide once its vmcnt has drained, which every wave
// waits for before thread 0 advances the counter that publishes the tile; a
// consumer issues its loads only after it has seen that counter.  V and V^T,
// which no tile writes, are read through the caches as usual, and no
// whole-cache write-back or invalidation is needed anywhere.
__device__ __forceinline__ uint32_t ld_counter(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float2 ld2_dev(const float* p) {  // 8-byte aligned
  const uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}
__device__ __forceinline__ float4 ld4_dev(const float* p) {  // 8-byte aligned
  const float2 a = ld2_dev(p), b = ld2_dev(p + 2);
  return make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ float ld1_dev(const float* p) {
  return __uint_as_float(__hip_atomic_load(reinterpret_cast<const uint32_t*>(p), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st2_dev(float* p, float a, float b) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p),
                     (uint64_t)__float_as_uint(a) | ((uint64_t)__float_as_uint(b) << 32),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st4_dev(float* p, float4 v) {
  st2_dev(p, v.x, v.y);
  st2_dev(p + 2, v.z, v.w);
}
__device__ __forceinline__ void st1_dev(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// 4 consecutive floats of row `row`, columns col..col+3 (device scope), zero
// outside [0, rows) x [0, cols); ld and col multiples of 2.
__device__ __forceinline__ float4 ld4m_dev(const float* p, int64_t ld, int64_t row, int64_t rows,
                                           int64_t col, int64_t cols) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= rows) return v;
  const float* q = p + row * ld + col;
  if (col + 3 < cols) return ld4_dev(q);
  if (col + 0 < cols) v.x = ld1_dev(q);
  if (col + 1 < cols) v.y = ld1_dev(q + 1);
  if (col + 2 < cols) v.z = ld1_dev(q + 2);
  return v;
}

// Thread 0 waits until *c >= target (bounded); the barrier orders every
// wave's later loads after that observation.  The workgroup learns whether
// the wait succeeded.
__device__ bool wait_geq(const uint32_t* c, uint32_t target, uint32_t* ctr, uint32_t* sticky,
                         int* s_flag) {
  if (threadIdx.x == 0) {
    int ok = 1;
    if (ld_counter(c) < target) {
      const uint64_t t0 = wall_clock64();
      while (ld_counter(c) < target) {
        if (ld_counter(ctr + kCtrErr)) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > kWaitTicks) {
          __hip_atomic_fetch_or(ctr + kCtrErr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_or(sticky, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

// Publish the tile and count its arrival; the last arrival of the phase sums
// the partial Grams (device-scope loads, ascending tile order) and marks the
// phase done.  Every wave first waits for its own device-scope stores to
// complete; after the barrier thread 0 advances the arrival counter.
__device__ void finish_tile(const Prob& P, int tiles, uint32_t iter, uint32_t* arr,
                            uint32_t* done, float* G, int* s_flag) {
  wait_vm<0>();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = __hip_atomic_fetch_add(arr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = (old + 1 == (iter + 1) * (uint32_t)tiles);
  }
  __syncthreads();
  if (!*s_flag) return;
  // G[e] = sum_q part[q][e]: each thread owns up to 8 float pairs of G and
  // reads 4 partials per round (32 independent 8-byte loads)
  const int rp = P.rp, e2n = rp * rp / 2;
  float2 acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = make_float2(0.f, 0.f);
  int q = 0;
  for (; q + 3 < tiles; q += 4) {
    float2 v[4][8];
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e2 = threadIdx.x + kThreads * u;
        v[qq][u] = e2 < e2n ? ld2_dev(P.gpart + ((int64_t)(q + qq) * e2n + e2) * 2)
                            : make_float2(0.f, 0.f);
      }
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc[u].x += v[qq][u].x;
        acc[u].y += v[qq][u].y;
      }
  }
  for (; q < tiles; ++q)
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e2 = threadIdx.x + kThreads * u;
      if (e2 < e2n) {
        const float2 v = ld2_dev(P.gpart + ((int64_t)q * e2n + e2) * 2);
        acc[u].x += v.x;
        acc[u].y += v.y;
      }
    }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e2 = threadIdx.x + kThreads * u;
    if (e2 < e2n) st2_dev(G + 2 * e2, acc[u].x, acc[u].y);
  }
  wait_vm<0>();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(done, iter + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 4 consecutive floats of row `row`, columns col..col+3, zero outside
// [0, rows) x [0, cols) (ld % 4 == 0 and a 16-byte aligned base).
__device__ __forceinline__ float4 ld4(const float* __restrict__ p, int64_t ld, int64_t row,
                                      int64_t rows, int64_t col, int64_t cols) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= rows) return v;
  const float* q = p + row * ld + col;
  if (col + 3 < cols) return *reinterpret_cast<const float4*>(q);
  if (col + 0 < cols) v.x = q[0];
  if (col + 1 < cols) v.y = q[1];
  if (col + 2 < cols) v.z = q[2];
  return v;
}

__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
__device__ __forceinline__ float4 lds4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}


// ---------------------------------------------------------------------------
// The product of a tile, C[m][c] = sum_k X[m][k] Y[c][k] (m < MB = 64 MS,
// c < RPY = 32 or 64 rows of Y), both operands contiguous along k and zero
// beyond the data, through an asynchronous global -> LDS copy ring: a stage
// is MB + RPY rows of 128 bytes (32 floats of k) copied by
// global_load_lds_dwordx4 (no register staging) with 3 stages in flight.
// Inside a row, 16-byte chunk q sits at slot q ^ (row % 8), so the 16 rows
// of an MFMA fragment read distinct banks.  Wave w owns rows
// [16 MS w, 16 MS (w+1)); a lane's 128-bit read holds 4 consecutive k that
// feed four MFMAs (slot g of MFMA e is k = 4g + e within the 16-k group),
// for A and B alike.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Barrier for the ring: a __syncthreads() would also wait for every
// outstanding copy (they are counted by vmcnt); this one retires the wave's
// own LDS reads and meets at a bare s_barrier.  The asm statements keep the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void ring_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int S, int MS, int NT>
__device__ __forceinline__ void ring_nt(const float* __restrict__ X, int64_t ldx,
                                        const float* __restrict__ Y, int64_t ldy, int nst,
                                        char* lds, v4f (&acc)[MS][NT]) {
  constexpr int MB = 64 * MS, RPY = (NT <= 2) ? 32 : 64, ROWS = MB + RPY;
  constexpr int L = ROWS / 32;  // copy instructions per wave per stage
  constexpr int STAGE = ROWS * 128;
  static_assert(ROWS % 32 == 0 && STAGE <= kStageBytes, "stage layout");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c = lane & 15, g = lane >> 4;
  // lane's source in copy j: stage row rr = 8 (wave L + j) + lane / 8, slot
  // lane % 8, holding chunk (lane % 8) ^ (rr % 8) = (lane % 8) ^ (lane / 8)
  const int chunk = (lane & 7) ^ (lane >> 3);
  const char* src[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int rr = 8 * (wave * L + j) + (lane >> 3);
    src[j] = rr < MB ? reinterpret_cast<const char*>(X + rr * ldx) + 16 * chunk
                     : reinterpret_cast<const char*>(Y + (rr - MB) * ldy) + 16 * chunk;
  }
  // copy j of this wave carries 8 rows of X (cached) or of Y (device-scope
  // reads: the Y operands are written by other tiles)
  auto issue = [&](int st) {
    char* dst = lds + (st % S) * STAGE;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const void* sp = static_cast<const void*>(src[j] + (int64_t)st * 128);
      lds_ptr_t dp = (lds_ptr_t)(dst + (wave * L + j) * 1024);
      if (8 * (wave * L + j) < MB) __builtin_amdgcn_global_load_lds(sp, dp, 16, 0, 0);
      else __builtin_amdgcn_global_load_lds(sp, dp, 16, 0, 16);
    }
  };
#pragma unroll
  for (int a = 0; a < MS; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  const int wrow = 16 * MS * wave;
  auto compute = [&](const char* buf) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int off = 16 * ((4 * kk + g) ^ (c & 7));
      v4f a[MS], b[NT];
#pragma unroll
      for (int ms = 0; ms < MS; ++ms)
        a[ms] = *reinterpret_cast<const v4f*>(buf + (wrow + 16 * ms + c) * 128 + off);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = *reinterpret_cast<const v4f*>(buf + (MB + 16 * nt + c) * 128 + off);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[ms][nt] = mfma(a[ms][e], b[nt][e], acc[ms][nt]);
    }
  };
  // Stage st lives in buffer st % S.  At the top of iteration st, stages st
  // .. min(st + S - 2, nst - 1) have been issued; once this wave's copies of
  // stage st have landed (at most L copies per later stage outstanding), one
  // barrier certifies that every wave's copies of stage st are in LDS and
  // that every wave has finished computing stage st - 1, whose buffer is
  // then refilled with stage st + S - 1.
  const int pre = nst < S - 1 ? nst : S - 1;
  for (int st = 0; st < pre; ++st) issue(st);
  for (int st = 0; st < nst; ++st) {
    const int later = nst - 1 - st;
    if (S >= 5 && later >= 3) wait_vm<(S >= 5 ? 3 * L : 0)>();
    else if (S >= 4 && later >= 2) wait_vm<(S >= 4 ? 2 * L : 0)>();
    else if (later >= 1) wait_vm<L>();
    else wait_vm<0>();
    ring_barrier();
    if (st + S - 1 < nst) issue(st + S - 1);
    compute(lds + (st % S) * STAGE);
  }
  __syncthreads();  // every wave is done with the ring before the epilogue reuses it
}

// ---------------------------------------------------------------------------
// Phase W tile t: rows [t MB, t MB + MB) of V, K = n.
// ---------------------------------------------------------------------------
template <int S, int MS, int NT>
__device__ __attribute__((noinline)) void tile_w(const Prob& P, int t) {
  constexpr int MB = 64 * MS, RP = 16 * NT;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, c = lane & 15, g = lane >> 4;
  const int64_t p0 = (int64_t)t * MB;
  const int64_t p = P.p;
  // the epilogue's inputs (the tile's W rows and G_H), loaded while the
  // product runs
  constexpr int NWP = MB * (RP / 4) / kThreads;
  constexpr int NGP = (RP * (RP / 4) + kThreads - 1) / kThreads;
  static_assert(MB * (RP / 4) % kThreads == 0, "W rows split evenly");
  float4 wpre[NWP], gpre[NGP];
#pragma unroll
  for (int u = 0; u < NWP; ++u) {
    const int idx = tid + kThreads * u, row = idx / (RP / 4), q = idx % (RP / 4);
    wpre[u] = (p0 + row < p) ? ld4_dev(&P.Wp[(p0 + row) * RP + 4 * q]) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int u = 0; u < NGP; ++u) {
    const int idx = tid + kThreads * u;
    gpre[u] = idx < RP * (RP / 4) ? ld4_dev(&P.GH[4 * idx]) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  v4f acc[MS][NT];
  ring_nt<S, MS, NT>(P.V + p0 * P.ldv, P.ldv, P.Hp, P.ldh, P.kw, lds_base<S>(), acc);
  float* lds = reinterpret_cast<float*>(lds_base<S>());
  const int wrow = 16 * MS * wv;

  // ---- epilogue: B = W_rows G_H, W <- W * (A / B), W^T, partial Gram -----
  constexpr int PS = RP + 4;
  float* Ws = lds;                // [MB][PS]
  float* Gs = lds + kMaxMB * 68;  // [RP][PS]
#pragma unroll
  for (int u = 0; u < NWP; ++u) {
    const int idx = tid + kThreads * u, row = idx / (RP / 4), q = idx % (RP / 4);
    st4(&Ws[row * PS + 4 * q], wpre[u]);
  }
#pragma unroll
  for (int u = 0; u < NGP; ++u) {
    const int idx = tid + kThreads * u;
    if (idx < RP * (RP / 4)) st4(&Gs[(4 * idx / RP) * PS + 4 * idx % RP], gpre[u]);
  }
  __syncthreads();
  v4f den[MS][NT];
#pragma unroll
  for (int a = 0; a < MS; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) den[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < RP; k0 += 16) {
    float4 a[MS], b[NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) a[ms] = lds4(&Ws[(wrow + 16 * ms + c) * PS + k0 + 4 * g]);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) b[nt] = lds4(&Gs[(16 * nt + c) * PS + k0 + 4 * g]);
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        den[ms][nt] = mfma(a[ms].x, b[nt].x, den[ms][nt]);
        den[ms][nt] = mfma(a[ms].y, b[nt].y, den[ms][nt]);
        den[ms][nt] = mfma(a[ms].z, b[nt].z, den[ms][nt]);
        den[ms][nt] = mfma(a[ms].w, b[nt].w, den[ms][nt]);
      }
  }
  // new W in place of the numerators
#pragma unroll
  for (int ms = 0; ms < MS; ++ms)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = wrow + 16 * ms + 4 * g + v, col = 16 * nt + c;
        const float w = Ws[lr * PS + col], d = den[ms][nt][v];
        acc[ms][nt][v] = (d > 0.f) ? w * (acc[ms][nt][v] / d) : w;
      }
  // the wave's own rows only (its reads above are done)
#pragma unroll
  for (int ms = 0; ms < MS; ++ms)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ws[(wrow + 16 * ms + 4 * g + v) * PS + 16 * nt + c] = acc[ms][nt][v];
  __syncthreads();
  for (int idx = tid; idx < MB * (RP / 4); idx += kThreads) {
    const int row = idx / (RP / 4), q = idx % (RP / 4);
    if (p0 + row < p) st4_dev(&P.Wp[(p0 + row) * RP + 4 * q], lds4(&Ws[row * PS + 4 * q]));
  }
  // W^T (RP x ldwt), the operand of the phase-H products: 4 rows of W per store
  for (int idx = tid; idx < RP * (MB / 4); idx += kThreads) {
    const int k = idx % RP, r0 = 4 * (idx / RP);  // k fastest: conflict-free LDS reads
    float* dst = P.WT + (int64_t)k * P.ldwt + p0 + r0;
    if (p0 + r0 + 3 < p) {
      st4_dev(dst, make_float4(Ws[r0 * PS + k], Ws[(r0 + 1) * PS + k], Ws[(r0 + 2) * PS + k],
                               Ws[(r0 + 3) * PS + k]));
    } else {
      for (int e = 0; e < 4; ++e)
        if (p0 + r0 + e < p) st1_dev(dst + e, Ws[(r0 + e) * PS + k]);
    }
  }
  // partial Gram C[i][j] = sum_m Wn[m][i] Wn[m][j] over the tile's rows
  float* gp = P.gpart + (int64_t)t * RP * RP;
  for (int st = wv; st < NT * NT; st += 4) {
    const int it = st / NT, jt = st % NT;
    v4f cg = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
    for (int m0 = 0; m0 < MB; m0 += 4)
      cg = mfma(Ws[(m0 + g) * PS + 16 * it + c], Ws[(m0 + g) * PS + 16 * jt + c], cg);
#pragma unroll
    for (int v = 0; v < 4; ++v) st1_dev(&gp[(16 * it + 4 * g + v) * RP + 16 * jt + c], cg[v]);
  }
}

// ---------------------------------------------------------------------------
// Phase H tile t: columns [t NB, t NB + NB) of V (rows of V^T), K = p.
// ---------------------------------------------------------------------------
template <int S, int MS, int NT>
__device__ __attribute__((noinline)) void tile_h(const Prob& P, int t) {
  constexpr int NB = 64 * MS, RP = 16 * NT;
  constexpr int PV = NB + 16;
  constexpr int PR = (RP == 48) ? 80 : RP + 16;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, c = lane & 15, g = lane >> 4;
  const int64_t j0 = (int64_t)t * NB;
  const int64_t n = P.n;
  // the epilogue's inputs (the tile's H columns), loaded while the product
  // runs; G_W is written by the phase-W tiles and read after the product
  constexpr int NHP = RP * (NB / 4) / kThreads;
  static_assert(RP * (NB / 4) % kThreads == 0, "H columns split evenly");
  float4 hpre[NHP];
#pragma unroll
  for (int u = 0; u < NHP; ++u) {
    const int idx = tid + kThreads * u, row = idx / (NB / 4), q = idx % (NB / 4);
    hpre[u] = ld4m_dev(P.Hp, P.ldh, row, RP, j0 + 4 * q, n);
  }
  v4f acc[MS][NT];
  ring_nt<S, MS, NT>(P.VT + j0 * P.ldvt, P.ldvt, P.WT, P.ldwt, P.kh, lds_base<S>(), acc);
  float* lds = reinterpret_cast<float*>(lds_base<S>());
  const int wcol = 16 * MS * wv;

  // ---- epilogue: D^T = H_cols^T G_W, H <- H * (S / D), partial Gram ------
  float* Hs = lds;                       // [RP][PV]
  float* Gs = lds + 64 * (kMaxNB + 16);  // [RP][PR]
  // all of this thread's G_W loads first, then the LDS stores (one memory
  // round trip, not one per store)
  constexpr int NGQ = (RP * (RP / 4) + kThreads - 1) / kThreads;
  float4 gq[NGQ];
#pragma unroll
  for (int u = 0; u < NGQ; ++u) {
    const int idx = tid + kThreads * u, row = idx / (RP / 4), q = idx % (RP / 4);
    gq[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (idx < RP * (RP / 4)) gq[u] = ld4_dev(&P.GW[row * RP + 4 * q]);
  }
#pragma unroll
  for (int u = 0; u < NHP; ++u) {
    const int idx = tid + kThreads * u, row = idx / (NB / 4), q = idx % (NB / 4);
    st4(&Hs[row * PV + 4 * q], hpre[u]);
  }
#pragma unroll
  for (int u = 0; u < NGQ; ++u) {
    const int idx = tid + kThreads * u, row = idx / (RP / 4), q = idx % (RP / 4);
    if (idx < RP * (RP / 4)) st4(&Gs[row * PR + 4 * q], gq[u]);
  }
  __syncthreads();
  v4f den[MS][NT];
#pragma unroll
  for (int a = 0; a < MS; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) den[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int k0 = 0; k0 < RP; k0 += 4) {
    float a[MS], b[NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) a[ms] = Hs[(k0 + g) * PV + wcol + 16 * ms + c];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) b[nt] = Gs[(k0 + g) * PR + 16 * nt + c];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) den[ms][nt] = mfma(a[ms], b[nt], den[ms][nt]);
  }
  // new H in place of the numerators
#pragma unroll
  for (int ms = 0; ms < MS; ++ms)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = wcol + 16 * ms + 4 * g + v, k = 16 * nt + c;
        const float h = Hs[k * PV + m], d = den[ms][nt][v];
        acc[ms][nt][v] = (d > 0.f) ? h * (acc[ms][nt][v] / d) : h;
      }
  // the wave's own columns only (its reads above are done)
#pragma unroll
  for (int ms = 0; ms < MS; ++ms)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) Hs[(16 * nt + c) * PV + wcol + 16 * ms + 4 * g + v] = acc[ms][nt][v];
  __syncthreads();
  // columns >= n hold zeros (masked loads, zero numerators) and rows of Hp
  // are padded to a multiple of 32 columns, so whole float4s are stored
  for (int idx = tid; idx < RP * (NB / 4); idx += kThreads) {
    const int row = idx / (NB / 4), q = idx % (NB / 4);
    if (j0 + 4 * q < n) st4_dev(&P.Hp[row * P.ldh + j0 + 4 * q], lds4(&Hs[row * PV + 4 * q]));
  }
  // partial Gram C[i][j] = sum_m Hn[i][m] Hn[j][m] over the tile's columns
  float* gp = P.gpart + (int64_t)t * RP * RP;
  for (int st = wv; st < NT * NT; st += 4) {
    const int it = st / NT, jt = st % NT;
    v4f cg = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int m0 = 0; m0 < NB; m0 += 16) {
      const float4 a = lds4(&Hs[(16 * it + c) * PV + m0 + 4 * g]);
      const float4 b = lds4(&Hs[(16 * jt + c) * PV + m0 + 4 * g]);
      cg = mfma(a.x, b.x, cg);
      cg = mfma(a.y, b.y, cg);
      cg = mfma(a.z, b.z, cg);
      cg = mfma(a.w, b.w, cg);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) st1_dev(&gp[(16 * it + 4 * g + v) * RP + 16 * jt + c], cg[v]);
  }
}

#define NMFB_CASES(X) X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 1) X(2, 2) X(2, 3) X(2, 4)

// The persistent loop.  Queue q's schedule holds one iteration's tiles, each
// coded as problem << 17 | phase << 16 | tile; entry e of iteration i is
// queue slot i * per_iter + e.  With per-XCD queues (`local`) a workgroup
// serves the queue of the XCD it runs on (hardware register XCC_ID), so a
// problem's tiles share one L2 for the operands they read through the cache;
// a workgroup on an XCD without a queue leaves at once (the host's check of
// the completed tiles reports any queue nobody served).
__device__ __forceinline__ uint32_t xcc_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 0xF;
}

template <int S>
__device__ __forceinline__ void persistent_loop(const Prob* __restrict__ probs,
                                                const uint32_t* __restrict__ sched,
                                                const QInfo* __restrict__ queues, int nq,
                                                uint32_t iters, int local,
                                                uint32_t* __restrict__ ctr,
                                                uint32_t* __restrict__ sticky) {
  __shared__ uint32_t s_slot;
  __shared__ int s_flag;
  const int q = local ? (int)xcc_id() : 0;
  if (q >= nq) return;
  const uint32_t per_iter = queues[q].per_iter, total = iters * per_iter;
  const uint32_t* qs = sched + queues[q].off;
  uint32_t* head = ctr + kHeadBase + 32 * q;
  for (;;) {
    if (threadIdx.x == 0)
      s_slot = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t slot = s_slot;
    __syncthreads();
    if (slot >= total) break;
    const uint32_t iter = slot / per_iter;
    const uint32_t code = __builtin_amdgcn_readfirstlane(qs[slot % per_iter]);
    const int b = (int)(code >> 17), phase = (int)((code >> 16) & 1), t = (int)(code & 0xffff);
    const Prob& P = probs[b];  // uniform: read with scalar loads, never copied
    uint32_t* pc = ctr + kCtrBase + 4 * b;
    if (phase == 0) {
      if (!wait_geq(pc + 3, iter, ctr, sticky, &s_flag)) break;  // H of iteration - 1
      switch (P.msw * 8 + P.rp / 16) {
#define CASE_W(MS, NT) \
  case MS * 8 + NT:    \
    tile_w<S, MS, NT>(P, t); \
    break;
        NMFB_CASES(CASE_W)
#undef CASE_W
        default: break;
      }
      finish_tile(P, P.tilesW, iter, pc + 0, pc + 1, P.GW, &s_flag);
    } else {
      if (!wait_geq(pc + 1, iter + 1, ctr, sticky, &s_flag)) break;  // W of this iteration
      switch (P.msh * 8 + P.rp / 16) {
#define CASE_H(MS, NT) \
  case MS * 8 + NT:    \
    tile_h<S, MS, NT>(P, t); \
    break;
        NMFB_CASES(CASE_H)
#undef CASE_H
        default: break;
      }
      finish_tile(P, P.tilesH, iter, pc + 2, pc + 3, P.GH, &s_flag);
    }
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(head + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
}

// Two workgroups per CU, 3-stage rings.
__global__ __launch_bounds__(kThreads, 2) void k_batch_persistent3(
    const Prob* __restrict__ probs, const uint32_t* __restrict__ sched,
    const QInfo* __restrict__ queues, int nq, uint32_t iters, int local,
    uint32_t* __restrict__ ctr, uint32_t* __restrict__ sticky) {
  persistent_loop<3>(probs, sched, queues, nq, iters, local, ctr, sticky);
}

// One workgroup per CU, 5-stage rings.
__global__ __launch_bounds__(kThreads, 1) void k_batch_persistent5(
    const Prob* __restrict__ probs, const uint32_t* __restrict__ sched,
    const QInfo* __restrict__ queues, int nq, uint32_t iters, int local,
    uint32_t* __restrict__ ctr, uint32_t* __restrict__ sticky) {
  persistent_loop<5>(probs, sched, queues, nq, iters, local, ctr, sticky);
}

// After a launch: every queue must have completed all of its tiles (a
// queue whose XCD ran none of the workgroups would not have); otherwise
// raise the error flags.
__global__ void k_batch_verify(const QInfo* __restrict__ queues, int nq, uint32_t iters,
                               uint32_t* __restrict__ ctr, uint32_t* __restrict__ sticky) {
  const int q = threadIdx.x;
  if (q < nq && ctr[kHeadBase + 32 * q + 1] != iters * queues[q].per_iter) {
    atomicOr(ctr + kCtrErr, 1u);
    atomicOr(sticky, 1u);
  }
}

// XCC_ID of every workgroup of a grid (host check of the XCD-local mode).
__global__ void k_batch_xcc_probe(uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

// Set-up and copy kernels (grid.y = problem).
// The caller's V into the padded copies V (row-major) and V^T through
// 32 x 32 LDS tiles, so both copies are written with coalesced stores.
__global__ __launch_bounds__(256) void k_batch_pad(const Prob* __restrict__ probs) {
  __shared__ float sh[32][33];
  const Prob& P = probs[blockIdx.y];
  const int ti = (P.p + 31) / 32, tj = (P.n + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int tile = blockIdx.x; tile < ti * tj; tile += gridDim.x) {
    const int64_t i0 = (int64_t)(tile / tj) * 32, j0 = (int64_t)(tile % tj) * 32;
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int64_t i = i0 + k, j = j0 + tx;
      float v = 0.f;
      if (i < P.p && j < P.n) {
        v = P.Vsrc[i * P.ldsrc + j];
        P.V[i * P.ldv + j] = v;
      }
      sh[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int64_t j = j0 + k, i = i0 + tx;
      if (i < P.p && j < P.n) P.VT[j * P.ldvt + i] = sh[tx][k];
    }
  }
}

__global__ __launch_bounds__(256) void k_batch_load(const Prob* __restrict__ probs) {
  const Prob P = probs[blockIdx.y];
  const int64_t nw = (int64_t)P.p * P.rp, nh = (int64_t)P.rp * P.ldh;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < nw + nh; e += (int64_t)gridDim.x * 256) {
    if (e < nw) {
      const int64_t i = e / P.rp;
      const int k = (int)(e % P.rp);
      P.Wp[e] = (k < P.r) ? P.W[i * P.r + k] : 0.f;
    } else {
      const int64_t f = e - nw;
      const int k = (int)(f / P.ldh);
      const int64_t j = f % P.ldh;
      P.Hp[f] = (k < P.r && j < P.n) ? P.H[(int64_t)k * P.n + j] : 0.f;
    }
  }
}

__global__ __launch_bounds__(256) void k_batch_store(const Prob* __restrict__ probs) {
  const Prob P = probs[blockIdx.y];
  const int64_t nw = (int64_t)P.p * P.r, nh = (int64_t)P.r * P.n;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < nw + nh; e += (int64_t)gridDim.x * 256) {
    if (e < nw) {
      const int64_t i = e / P.r;
      const int k = (int)(e % P.r);
      P.W[e] = P.Wp[i * P.rp + k];
    } else {
      const int64_t f = e - nw;
      const int k = (int)(f / P.n);
      const int64_t j = f % P.n;
      P.H[f] = P.Hp[(int64_t)k * P.ldh + j];
    }
  }
}

// G_H = H H^T of the loaded H (one workgroup per problem and 16 x 16 block
// of G; a lane pair of 16 x 16 threads forms each entry by a float32
// running sum over the columns in order).
__global__ __launch_bounds__(256) void k_batch_gram_h(const Prob* __restrict__ probs) {
  const Prob P = probs[blockIdx.y];
  const int nb = P.rp / 16;
  if ((int)blockIdx.x >= nb * nb) return;
  const int bi = blockIdx.x / nb, bj = blockIdx.x % nb;
  const int i = 16 * bi + (threadIdx.x >> 4), k = 16 * bj + (threadIdx.x & 15);
  const float* hi = P.Hp + (int64_t)i * P.ldh;
  const float* hk = P.Hp + (int64_t)k * P.ldh;
  float s = 0.f;
  for (int64_t j = 0; j < P.n; ++j) s = fmaf(hi[j], hk[j], s);
  P.GH[i * P.rp + k] = s;
}

// Objective tiles: 64 x 64 blocks of V - W H of every problem, float64
// accumulation of float64 products of the float32 factors; one double per
// tile, summed per problem in tile order by k_batch_obj_sum.
__global__ __launch_bounds__(256) void k_batch_objective(const Prob* __restrict__ probs,
                                                         const int4* __restrict__ tiles,
                                                         double* __restrict__ part, int zero_w) {
  __shared__ __attribute__((aligned(16))) float WsT[64 * 64];
  __shared__ __attribute__((aligned(16))) float Hs[64 * 64];
  __shared__ double red[4];
  const int4 td = tiles[blockIdx.x];
  const Prob P = probs[td.x];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t i0 = (int64_t)td.y * 64, j0 = (int64_t)td.z * 64;
  const int rp = P.rp;
  for (int idx = tid; idx < 64 * rp; idx += 256) {
    const int ii = idx / rp, kk = idx % rp;
    WsT[kk * 64 + ii] = (i0 + ii < P.p) ? P.Wp[(i0 + ii) * rp + kk] : 0.f;
  }
  for (int idx = tid; idx < rp * 64; idx += 256) {
    const int kk = idx / 64, jj = idx % 64;
    Hs[idx] = (j0 + jj < P.n) ? P.Hp[(int64_t)kk * P.ldh + j0 + jj] : 0.f;
  }
  __syncthreads();
  double s[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) s[a][b] = 0.0;
  for (int kk = 0; kk < (zero_w ? 0 : rp); ++kk) {  // zero_w: W = 0, f = ||V||^2
    const float4 w = lds4(&WsT[kk * 64 + 4 * ty]);
    const float4 h = lds4(&Hs[kk * 64 + 4 * tx]);
    const double wd[4] = {(double)w.x, (double)w.y, (double)w.z, (double)w.w};
    const double hd[4] = {(double)h.x, (double)h.y, (double)h.z, (double)h.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) s[a][b] = fma(wd[a], hd[b], s[a][b]);
  }
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t row = i0 + 4 * ty + a, col = j0 + 4 * tx;
    const float4 v = ld4(P.V, P.ldv, row, P.p, col, P.n);
    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (row < P.p && col + b < P.n) {
        const double e = (double)vv[b] - s[a][b];
        acc = fma(e, e, acc);
      }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_batch_obj_sum(const double* __restrict__ part,
                                                       const int64_t* __restrict__ first,
                                                       double* __restrict__ f) {
  __shared__ double sh[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t lo = first[b], hi = first[b + 1];
  double s = 0.0;
  for (int64_t q = lo + tid; q < hi; q += 256) s += part[q];
  sh[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  if (tid == 0) f[b] = sh[0];
}

__global__ void k_batch_fill(uint32_t* __restrict__ p, int64_t count) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
inline int64_t up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Row pitch (floats) of a streamed matrix: 64 floats (256 bytes) more when
// the pitch is a multiple of 4 KB, so that the rows of one copy-ring stage
// spread over the HBM channels (as for the single-problem copies).
inline int64_t spread(int64_t elems) { return (elems * 4) % 4096 == 0 ? elems + 64 : elems; }

}  // namespace
}  // namespace nmfb

using nmfb::Prob;

struct nmf_batch {
  int count = 0;
  hipStream_t st = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0, cus = 0;
  std::vector<nmf_problem> user;
  std::vector<Prob> host;       // descriptors (device pointers)
  char* arena = nullptr;        // factors, Grams, partials (one allocation)
  size_t factor_bytes = 0;      // leading part of the arena that tuning saves
  Prob* dprobs = nullptr;
  uint32_t* ctr = nullptr;
  int64_t nctr = 0;
  uint32_t* sched = nullptr;
  nmfb::QInfo* dq = nullptr;        // queue table (device)
  std::vector<nmfb::QInfo> queues;  // host copy
  int local = 0;                    // XCD-local queues (else one global queue)
  int nq = 1;
  int4* obj_tiles = nullptr;
  int64_t nobj = 0;
  int64_t* obj_first = nullptr;
  double* obj_part = nullptr;
  double* fdev = nullptr;
  double* hostbuf = nullptr;
  int32_t table[NMF_BATCH_TABLE_LEN] = {0};
  hipGraphExec_t graph = nullptr;
  int32_t graph_iters = 0;
  uint32_t* hosterr = nullptr;
};

namespace nmfb {
namespace {

#define BTRY_HIP(x)                                \
  do {                                             \
    if ((x) != hipSuccess) return NMF_EDEVICE;     \
  } while (0)
#define BTRY(x)                          \
  do {                                   \
    const nmf_status s_ = (x);           \
    if (s_ != NMF_OK) return s_;         \
  } while (0)

// Default tile table (rows of phase-W tiles and columns of phase-H tiles in
// units of 64, per padded-rank class 16 / 32 / 48 / 64; workgroups per CU).
void default_table(int32_t* t) {
  const int32_t d[NMF_BATCH_TABLE_LEN] = {1, 1, 1, 1, 1, 1, 1, 1, 2};
  std::memcpy(t, d, sizeof(d));
}

bool table_ok(const int32_t* t) {
  for (int q = 0; q < 8; ++q)
    if (t[q] != 1 && t[q] != 2) return false;
  return t[8] >= 1 && t[8] <= 2;
}

// Apply the table to the descriptors and rebuild the schedule.
nmf_status plan(nmf_batch* b) {
  // problems in decreasing order of work, so that large tiles start early;
  // in the XCD-local mode each problem goes to the queue with the least work
  // so far (largest first)
  std::vector<int> order(b->count);
  for (int i = 0; i < b->count; ++i) order[i] = i;
  auto work = [&](int i) {
    const Prob& a = b->host[i];
    return (int64_t)a.p * a.n * a.rp;
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  for (int i = 0; i < b->count; ++i) {
    Prob& P = b->host[i];
    const int cls = P.rp / 16 - 1;
    P.msw = b->table[2 * cls];
    P.msh = b->table[2 * cls + 1];
    P.tilesW = (int32_t)((P.p + 64 * P.msw - 1) / (64 * P.msw));
    P.tilesH = (int32_t)((P.n + 64 * P.msh - 1) / (64 * P.msh));
    if (P.tilesW > 65535 || P.tilesH > 65535) return NMF_EUNSUPPORTED;
  }
  std::vector<std::vector<int>> members(b->nq);
  std::vector<int64_t> load(b->nq, 0);
  for (int i : order) {
    const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    members[q].push_back(i);
    load[q] += work(i);
  }
  std::vector<uint32_t> all;
  b->queues.assign(b->nq, QInfo{0, 0});
  for (int q = 0; q < b->nq; ++q) {
    b->queues[q].off = (uint32_t)all.size();
    for (int i : members[q])
      for (int t = 0; t < b->host[i].tilesW; ++t) all.push_back(((uint32_t)i << 17) | (uint32_t)t);
    for (int i : members[q])
      for (int t = 0; t < b->host[i].tilesH; ++t)
        all.push_back(((uint32_t)i << 17) | (1u << 16) | (uint32_t)t);
    b->queues[q].per_iter = (uint32_t)all.size() - b->queues[q].off;
  }
  if (b->sched) (void)hipFree(b->sched);
  b->sched = nullptr;
  BTRY_HIP(hipMalloc(&b->sched, std::max<size_t>(1, all.size()) * sizeof(uint32_t)));
  BTRY_HIP(hipMemcpyAsync(b->sched, all.data(), all.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, b->st));
  BTRY_HIP(hipMemcpyAsync(b->dq, b->queues.data(), b->nq * sizeof(QInfo), hipMemcpyHostToDevice,
                          b->st));
  BTRY_HIP(hipMemcpyAsync(b->dprobs, b->host.data(), b->host.size() * sizeof(Prob),
                          hipMemcpyHostToDevice, b->st));
  BTRY_HIP(hipStreamSynchronize(b->st));
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_iters = 0;
  return NMF_OK;
}

// XCD-local mode if the XCC_ID register partitions a persistent grid into
// nq <= kMaxQueues equal groups numbered 0 .. nq - 1 (else one global queue).
// NMF_BATCH_QUEUES=1 in the environment forces the global queue.
nmf_status choose_queues(nmf_batch* b) {
  b->local = 0;
  b->nq = 1;
  const char* env = std::getenv("NMF_BATCH_QUEUES");
  if (env && std::strcmp(env, "1") == 0) return NMF_OK;
  const int grid = 2 * b->cus;
  uint32_t* d = nullptr;
  BTRY_HIP(hipMalloc(&d, grid * sizeof(uint32_t)));
  std::vector<uint32_t> h(grid, 0xffffffffu);
  hipLaunchKernelGGL(k_batch_xcc_probe, dim3(grid), dim3(64), 0, b->st, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, grid * sizeof(uint32_t), hipMemcpyDeviceToHost, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  (void)hipFree(d);
  if (e != hipSuccess) return NMF_EDEVICE;
  int cnt[kMaxQueues] = {0};
  for (uint32_t v : h) {
    if (v >= (uint32_t)kMaxQueues) return NMF_OK;
    ++cnt[v];
  }
  int nq = 0;
  while (nq < kMaxQueues && cnt[nq] > 0) ++nq;
  for (int q = nq; q < kMaxQueues; ++q)
    if (cnt[q]) return NMF_OK;  // ids not contiguous from 0
  for (int q = 0; q < nq; ++q)
    if (cnt[q] != cnt[0]) return NMF_OK;  // unequal groups
  if (nq > 1) {
    b->local = 1;
    b->nq = nq;
  }
  return NMF_OK;
}

nmf_status enqueue_steps(nmf_batch* b, int32_t iters, hipStream_t s) {
  for (const QInfo& q : b->queues)
    if ((uint64_t)iters * q.per_iter >= 0xffffffffull) return NMF_EUNSUPPORTED;
  hipLaunchKernelGGL(k_batch_fill, dim3((unsigned)std::min<int64_t>(64, (b->nctr + 255) / 256)),
                     dim3(256), 0, s, b->ctr, b->nctr);
  BTRY_HIP(hipGetLastError());
  const unsigned grid = (unsigned)(b->cus * b->table[8]);
  if (b->table[8] == 2)
    hipLaunchKernelGGL(k_batch_persistent3, dim3(grid), dim3(kThreads), 0, s, b->dprobs, b->sched,
                       b->dq, b->nq, (uint32_t)iters, b->local, b->ctr, b->ctr + b->nctr);
  else
    hipLaunchKernelGGL(k_batch_persistent5, dim3(grid), dim3(kThreads), 0, s, b->dprobs, b->sched,
                       b->dq, b->nq, (uint32_t)iters, b->local, b->ctr, b->ctr + b->nctr);
  BTRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_batch_verify, dim3(1), dim3(64), 0, s, b->dq, b->nq, (uint32_t)iters, b->ctr,
                     b->ctr + b->nctr);
  BTRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_batch_store, dim3(64, (unsigned)b->count), dim3(256), 0, s, b->dprobs);
  BTRY_HIP(hipGetLastError());
  return NMF_OK;
}

nmf_status capture(nmf_batch* b, int32_t iters) {
  if (!b->cap_stream) BTRY_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  BTRY_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  const nmf_status s = enqueue_steps(b, iters, b->cap_stream);
  const hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
  if (s != NMF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess || !graph) return NMF_EDEVICE;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  const hipError_t ei = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return NMF_EDEVICE;
  b->graph_iters = iters;
  // upload now, so that the first launch costs what every later one does
  return hipGraphUpload(b->graph, b->st) == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

// Synchronize; NMF_EDEVICE if a launch since the last check hit the wait
// bound (the flag is then cleared).
nmf_status check_error(nmf_batch* b) {
  BTRY_HIP(hipMemcpyAsync(b->hosterr, b->ctr + b->nctr, 4, hipMemcpyDeviceToHost, b->st));
  BTRY_HIP(hipStreamSynchronize(b->st));
  if (!*b->hosterr) return NMF_OK;
  hipLaunchKernelGGL(k_batch_fill, dim3(1), dim3(256), 0, b->st, b->ctr + b->nctr, (int64_t)1);
  BTRY_HIP(hipStreamSynchronize(b->st));
  return NMF_EDEVICE;
}

}  // namespace
}  // namespace nmfb

extern "C" {

nmf_status nmf_batch_create(nmf_batch** out, const nmf_problem* probs, int32_t count,
                            void* stream) {
  using namespace nmfb;
  if (!out) return NMF_EINVAL;
  *out = nullptr;
  if (!probs || count < 1 || count > 16383) return NMF_EINVAL;
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = probs[i];
    if (!q.V || !q.W || !q.H || q.p < 1 || q.n < 1 || q.r < 1 || q.ldv < q.n) return NMF_EINVAL;
    if (q.p > INT32_MAX || q.n > INT32_MAX || q.reserved != 0) return NMF_EINVAL;
    if (reinterpret_cast<uintptr_t>(q.V) % 4 || reinterpret_cast<uintptr_t>(q.W) % 4 ||
        reinterpret_cast<uintptr_t>(q.H) % 4)
      return NMF_EINVAL;
    if (q.r > 64) return NMF_EUNSUPPORTED;
  }
  nmf_batch* b = new (std::nothrow) nmf_batch();
  if (!b) return NMF_ENOMEM;
  b->count = count;
  b->st = reinterpret_cast<hipStream_t>(stream);
  b->user.assign(probs, probs + count);
  b->host.resize(count);
  default_table(b->table);
  nmf_status s = NMF_OK;
  auto fail = [&](nmf_status e) {
    nmf_batch_destroy(b);
    return e;
  };
  if (hipGetDevice(&b->device) != hipSuccess) return fail(NMF_EDEVICE);
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) !=
      hipSuccess)
    return fail(NMF_EDEVICE);
  // arena: Wp and Hp of all problems, then G_H of all problems (together
  // the state that tuning saves and restores), then G_W, partial Grams, W^T,
  // and the padded copies of V and V^T
  size_t off = 0;
  std::vector<size_t> oW(count), oH(count), oGH(count), oGW(count), oP(count), oWT(count),
      oV(count), oVT(count);
  auto rpy_of = [](int64_t rp) { return up(rp, 32); };
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = probs[i];
    const int64_t rp = up(q.r, 16);
    oW[i] = off;
    off += up(q.p * rp * 4, 256);
    oH[i] = off;
    off += up(rpy_of(rp) * spread(up(q.n, 32)) * 4, 256);
  }
  for (int i = 0; i < count; ++i) {
    const int64_t rp = up(probs[i].r, 16);
    oGH[i] = off;
    off += up(rp * rp * 4, 256);
  }
  b->factor_bytes = off;  // W, H and G_H: the state carried between calls
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = probs[i];
    const int64_t rp = up(q.r, 16);
    oGW[i] = off;
    off += up(rp * rp * 4, 256);
    // partial Grams for the smallest tiles (64 rows / columns)
    const int64_t tiles = std::max((q.p + 63) / 64, (q.n + 63) / 64);
    oP[i] = off;
    off += up(tiles * rp * rp * 4, 256);
    oWT[i] = off;
    off += up(rpy_of(rp) * spread(up(q.p, 32)) * 4, 256);
  }
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = probs[i];
    oV[i] = off;
    off += up(up(q.p, 128) * spread(up(q.n, 32)) * 4, 1024);
    oVT[i] = off;
    off += up(up(q.n, 128) * spread(up(q.p, 32)) * 4, 1024);
  }
  if (hipMalloc(&b->arena, off) != hipSuccess) return fail(NMF_ENOMEM);
  if (hipMemsetAsync(b->arena, 0, off, b->st) != hipSuccess) return fail(NMF_EDEVICE);
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = probs[i];
    Prob& P = b->host[i];
    P.Vsrc = q.V;
    P.ldsrc = q.ldv;
    P.V = reinterpret_cast<float*>(b->arena + oV[i]);
    P.ldv = spread(up(q.n, 32));
    P.VT = reinterpret_cast<float*>(b->arena + oVT[i]);
    P.ldvt = spread(up(q.p, 32));
    P.p = (int32_t)q.p;
    P.n = (int32_t)q.n;
    P.r = q.r;
    P.rp = (int32_t)up(q.r, 16);
    P.ldh = spread(up(q.n, 32));
    P.ldwt = spread(up(q.p, 32));
    P.kw = (int32_t)(up(q.n, 32) / 32);
    P.kh = (int32_t)(up(q.p, 32) / 32);
    P.Wp = reinterpret_cast<float*>(b->arena + oW[i]);
    P.Hp = reinterpret_cast<float*>(b->arena + oH[i]);
    P.WT = reinterpret_cast<float*>(b->arena + oWT[i]);
    P.GH = reinterpret_cast<float*>(b->arena + oGH[i]);
    P.GW = reinterpret_cast<float*>(b->arena + oGW[i]);
    P.gpart = reinterpret_cast<float*>(b->arena + oP[i]);
    P.W = q.W;
    P.H = q.H;
  }
  b->nctr = kCtrBase + 4 * (int64_t)count;
  if (hipMalloc(&b->dprobs, count * sizeof(Prob)) != hipSuccess) return fail(NMF_ENOMEM);
  if (hipMalloc(&b->ctr, (b->nctr + 1) * 4) != hipSuccess) return fail(NMF_ENOMEM);
  if (hipMemsetAsync(b->ctr, 0, (b->nctr + 1) * 4, b->st) != hipSuccess) return fail(NMF_EDEVICE);
  if (hipHostMalloc(&b->hostbuf, count * sizeof(double)) != hipSuccess) return fail(NMF_ENOMEM);
  if (hipHostMalloc(&b->hosterr, sizeof(uint32_t)) != hipSuccess) return fail(NMF_ENOMEM);
  // objective tiles
  std::vector<int4> ot;
  std::vector<int64_t> first(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    first[i] = (int64_t)ot.size();
    const nmf_problem& q = probs[i];
    for (int64_t a = 0; a < (q.p + 63) / 64; ++a)
      for (int64_t c = 0; c < (q.n + 63) / 64; ++c) ot.push_back(make_int4(i, (int)a, (int)c, 0));
  }
  first[count] = (int64_t)ot.size();
  b->nobj = (int64_t)ot.size();
  if (b->nobj > INT32_MAX) return fail(NMF_EUNSUPPORTED);
  if (hipMalloc(&b->obj_tiles, ot.size() * sizeof(int4)) != hipSuccess ||
      hipMalloc(&b->obj_first, first.size() * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&b->obj_part, ot.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&b->fdev, count * sizeof(double)) != hipSuccess)
    return fail(NMF_ENOMEM);
  if (hipMemcpyAsync(b->obj_tiles, ot.data(), ot.size() * sizeof(int4), hipMemcpyHostToDevice,
                     b->st) != hipSuccess ||
      hipMemcpyAsync(b->obj_first, first.data(), first.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice, b->st) != hipSuccess)
    return fail(NMF_EDEVICE);
  if (hipMalloc(&b->dq, kMaxQueues * sizeof(QInfo)) != hipSuccess) return fail(NMF_ENOMEM);
  s = choose_queues(b);
  if (s != NMF_OK) return fail(s);
  s = plan(b);
  if (s != NMF_OK) return fail(s);
  hipLaunchKernelGGL(k_batch_pad, dim3(256, (unsigned)count), dim3(256), 0, b->st, b->dprobs);
  if (hipGetLastError() != hipSuccess) return fail(NMF_EDEVICE);
  s = nmf_batch_load(b);
  if (s != NMF_OK) return fail(s);
  if (hipStreamSynchronize(b->st) != hipSuccess) return fail(NMF_EDEVICE);
  *out = b;
  return NMF_OK;
}

nmf_status nmf_batch_load(nmf_batch* b) {
  using namespace nmfb;
  if (!b) return NMF_EINVAL;
  hipLaunchKernelGGL(k_batch_load, dim3(64, (unsigned)b->count), dim3(256), 0, b->st, b->dprobs);
  BTRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_batch_gram_h, dim3(16, (unsigned)b->count), dim3(256), 0, b->st, b->dprobs);
  BTRY_HIP(hipGetLastError());
  return NMF_OK;
}

nmf_status nmf_batch_step(nmf_batch* b, int32_t iters) {
  using namespace nmfb;
  if (!b || iters < 0) return NMF_EINVAL;
  if (iters == 0) return NMF_OK;
  if (!b->graph || b->graph_iters != iters) BTRY(capture(b, iters));
  BTRY_HIP(hipGraphLaunch(b->graph, b->st));
  return NMF_OK;
}

nmf_status nmf_batch_check(nmf_batch* b) {
  if (!b) return NMF_EINVAL;
  return nmfb::check_error(b);
}

}  // extern "C"

namespace nmfb {
namespace {

// f[b] = ||V_b - W_b H_b||^2 (or ||V_b||^2 with zero_w) into the host
// buffer; synchronizes.
nmf_status batch_objectives(nmf_batch* b, int zero_w) {
  hipLaunchKernelGGL(k_batch_objective, dim3((unsigned)b->nobj), dim3(256), 0, b->st, b->dprobs,
                     b->obj_tiles, b->obj_part, zero_w);
  BTRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_batch_obj_sum, dim3((unsigned)b->count), dim3(256), 0, b->st, b->obj_part,
                     b->obj_first, b->fdev);
  BTRY_HIP(hipGetLastError());
  BTRY_HIP(hipMemcpyAsync(b->hostbuf, b->fdev, b->count * sizeof(double), hipMemcpyDeviceToHost,
                          b->st));
  return check_error(b);
}

}  // namespace
}  // namespace nmfb

extern "C" {

nmf_status nmf_batch_objective(nmf_batch* b, double* f_host) {
  using namespace nmfb;
  if (!b || !f_host) return NMF_EINVAL;
  BTRY(batch_objectives(b, 0));
  for (int i = 0; i < b->count; ++i) {
    if (!std::isfinite(b->hostbuf[i])) return NMF_ENONFINITE;
    f_host[i] = b->hostbuf[i];
  }
  return NMF_OK;
}

nmf_status nmf_batch_get_table(nmf_batch* b, int32_t* table) {
  if (!b || !table) return NMF_EINVAL;
  std::memcpy(table, b->table, sizeof(b->table));
  return NMF_OK;
}

nmf_status nmf_batch_set_table(nmf_batch* b, const int32_t* table) {
  using namespace nmfb;
  if (!b || !table || !table_ok(table)) return NMF_EINVAL;
  BTRY_HIP(hipStreamSynchronize(b->st));
  std::memcpy(b->table, table, sizeof(b->table));
  return plan(b);
}

nmf_status nmf_batch_tune(nmf_batch* b, int32_t trial_iters, double* best_ms) {
  using namespace nmfb;
  if (!b || trial_iters < 1) return NMF_EINVAL;
  BTRY_HIP(hipStreamSynchronize(b->st));
  // save the factors and G_H (restored at the end, so tuning leaves the
  // state exactly as it found it)
  char* save = nullptr;
  BTRY_HIP(hipMalloc(&save, b->factor_bytes));
  BTRY_HIP(hipMemcpyAsync(save, b->arena, b->factor_bytes, hipMemcpyDeviceToDevice, b->st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  nmf_status s = NMF_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = NMF_EDEVICE;
  auto timed = [&](const int32_t* t, float* ms) -> nmf_status {
    std::memcpy(b->table, t, sizeof(b->table));
    BTRY(plan(b));
    BTRY(enqueue_steps(b, 1, b->st));  // warm-up
    BTRY_HIP(hipEventRecord(e0, b->st));
    BTRY(enqueue_steps(b, trial_iters, b->st));
    BTRY_HIP(hipEventRecord(e1, b->st));
    BTRY_HIP(hipEventSynchronize(e1));
    BTRY_HIP(hipEventElapsedTime(ms, e0, e1));
    return check_error(b);
  };
  // which rank classes occur
  bool used[4] = {false, false, false, false};
  for (const Prob& P : b->host) used[P.rp / 16 - 1] = true;
  int32_t best[NMF_BATCH_TABLE_LEN];
  std::memcpy(best, b->table, sizeof(best));
  float tbest = 0.f;
  if (s == NMF_OK) s = timed(best, &tbest);
  // coordinate descent over the workgroups per CU, then each class's
  // (phase W rows, phase H columns)
  for (int w = 1; w <= 2 && s == NMF_OK; ++w) {
    if (w == best[8]) continue;
    int32_t cand[NMF_BATCH_TABLE_LEN];
    std::memcpy(cand, best, sizeof(cand));
    cand[8] = w;
    float tm = 0.f;
    s = timed(cand, &tm);
    if (s == NMF_OK && tm < 0.98f * tbest) {
      tbest = tm;
      std::memcpy(best, cand, sizeof(best));
    }
  }
  for (int cls = 0; cls < 4 && s == NMF_OK; ++cls) {
    if (!used[cls]) continue;
    for (int mw = 1; mw <= 2 && s == NMF_OK; ++mw)
      for (int mh = 1; mh <= 2 && s == NMF_OK; ++mh) {
        if (mw == best[2 * cls] && mh == best[2 * cls + 1]) continue;
        int32_t cand[NMF_BATCH_TABLE_LEN];
        std::memcpy(cand, best, sizeof(cand));
        cand[2 * cls] = mw;
        cand[2 * cls + 1] = mh;
        float tm = 0.f;
        s = timed(cand, &tm);
        if (s == NMF_OK && tm < 0.98f * tbest) {
          tbest = tm;
          std::memcpy(best, cand, sizeof(best));
        }
      }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  std::memcpy(b->table, best, sizeof(best));
  nmf_status s2 = plan(b);
  if (s == NMF_OK) s = s2;
  // restore the state (factors and G_H) and the caller's copies
  if (hipMemcpyAsync(b->arena, save, b->factor_bytes, hipMemcpyDeviceToDevice, b->st) !=
      hipSuccess)
    s = NMF_EDEVICE;
  hipLaunchKernelGGL(k_batch_store, dim3(64, (unsigned)b->count), dim3(256), 0, b->st, b->dprobs);
  if (hipStreamSynchronize(b->st) != hipSuccess) s = NMF_EDEVICE;
  (void)hipFree(save);
  if (best_ms) *best_ms = (double)tbest / trial_iters;
  return s;
}

void nmf_batch_destroy(nmf_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->st);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->arena) (void)hipFree(b->arena);
  if (b->dprobs) (void)hipFree(b->dprobs);
  if (b->ctr) (void)hipFree(b->ctr);
  if (b->sched) (void)hipFree(b->sched);
  if (b->dq) (void)hipFree(b->dq);
  if (b->obj_tiles) (void)hipFree(b->obj_tiles);
  if (b->obj_first) (void)hipFree(b->obj_first);
  if (b->obj_part) (void)hipFree(b->obj_part);
  if (b->fdev) (void)hipFree(b->fdev);
  if (b->hostbuf) (void)hipHostFree(b->hostbuf);
  if (b->hosterr) (void)hipHostFree(b->hosterr);
  delete b;
}

nmf_status nmf_batch_solve(const nmf_problem* probs, int32_t count, int32_t max_iters,
                           const nmf_options* opt, int32_t* iters_done, double* f_out,
                           void* stream) {
  using namespace nmfb;
  if (max_iters < 0 || !probs || count < 1) return NMF_EINVAL;
  nmf_options o;
  nmf_default_options(&o);
  if (opt) o = *opt;
  if (o.check_every < 1 || !(o.tol >= 0.0) || !std::isfinite(o.tol)) return NMF_EINVAL;
  // the batched tier runs the Euclidean update in float32
  if (o.precision != NMF_FP32 || o.loss != NMF_LOSS_EUCLIDEAN) return NMF_EUNSUPPORTED;
  if (o.tol_kind != NMF_TOL_REL_CHANGE && o.tol_kind != NMF_TOL_GAP_NORMALIZED)
    return NMF_EUNSUPPORTED;
  if (iters_done) *iters_done = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // argument checks of nmf_batch_create before any device work
  for (int32_t i = 0; i < count; ++i) {
    const nmf_problem& P = probs[i];
    if (!P.V || !P.W || !P.H || P.p < 1 || P.n < 1 || P.r < 1 || P.ldv < P.n || P.reserved != 0)
      return NMF_EINVAL;
    if (P.r > 64) return NMF_EUNSUPPORTED;
  }
  if (o.validate) {
    uint32_t* flag = nullptr;
    if (hipMalloc(&flag, sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return NMF_ENOMEM;
    }
    nmf_status s = NMF_OK;
    uint32_t bad = 0;
    if (nmfk::launch_fill_u32(flag, 1, 0u, st) != hipSuccess) s = NMF_EDEVICE;
    for (int32_t i = 0; i < count && s == NMF_OK; ++i)
      if (nmfk::launch_validate(probs[i].V, probs[i].ldv, probs[i].p, probs[i].n, flag, st) !=
          hipSuccess)
        s = NMF_EDEVICE;
    if (s == NMF_OK && (hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st) !=
                            hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
      s = NMF_EDEVICE;
    (void)hipFree(flag);
    if (s != NMF_OK) return s;
    if (bad) return NMF_EINVAL;
  }
  if (o.seed != 0) {
    // Algorithm 1's U(0,1) start on the device: problem i draws W from
    // Philox stream 2i and H from stream 2i + 1 under key seed (problem 0
    // gets the draws of nmf_init with the same seed)
    for (int32_t i = 0; i < count; ++i) {
      const nmf_problem& P = probs[i];
      if (nmfk::launch_uniform(P.W, P.p, P.r, P.r, o.seed, 2u * (uint32_t)i, st) != hipSuccess ||
          nmfk::launch_uniform(P.H, P.r, P.n, P.n, o.seed, 2u * (uint32_t)i + 1u, st) !=
              hipSuccess)
        return NMF_EDEVICE;
    }
  }
  nmf_batch* b = nullptr;
  nmf_status s = nmf_batch_create(&b, probs, count, stream);
  if (s != NMF_OK) return s;
  std::vector<double> nv2(count, 0.0), fprev(count, 0.0);
  if (o.tol_kind == NMF_TOL_GAP_NORMALIZED) {
    s = batch_objectives(b, 1);
    for (int32_t i = 0; s == NMF_OK && i < count; ++i) nv2[i] = b->hostbuf[i];
  }
  if (s == NMF_OK) s = batch_objectives(b, 0);
  for (int32_t i = 0; s == NMF_OK && i < count; ++i) {
    fprev[i] = b->hostbuf[i];
    if (!std::isfinite(fprev[i])) s = NMF_ENONFINITE;
  }
  // chunks of check_every iterations (one persistent launch each), then the
  // objectives of every problem; stop once every problem meets the rule
  int32_t done_iters = 0;
  bool all = false;
  while (s == NMF_OK && done_iters < max_iters && !all) {
    const int32_t todo = std::min(o.check_every, max_iters - done_iters);
    s = nmf_batch_step(b, todo);
    if (s == NMF_OK) s = batch_objectives(b, 0);
    if (s != NMF_OK) break;
    done_iters += todo;
    all = true;
    for (int32_t i = 0; i < count; ++i) {
      const double f = b->hostbuf[i];
      if (!std::isfinite(f)) {
        s = NMF_ENONFINITE;
        break;
      }
      const bool ok = (o.tol_kind == NMF_TOL_REL_CHANGE)
                          ? std::fabs(f - fprev[i]) / (std::fabs(fprev[i]) + 1.0) < o.tol
                          : (nv2[i] > 0.0 ? f / nv2[i] : 0.0) <= o.tol;
      all = all && ok;
      fprev[i] = f;
    }
  }
  if (iters_done) *iters_done = done_iters;
  if (f_out)
    for (int32_t i = 0; i < count; ++i) f_out[i] = fprev[i];
  nmf_batch_destroy(b);
  if (s != NMF_OK) return s;
  return all ? NMF_OK : NMF_ENOTCONVERGED;
}

}  // extern "C"
