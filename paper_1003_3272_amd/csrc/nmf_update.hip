// gfx950 H half-step epilogue (eq. nnmf_w_update) for padded ranks up to 64
// with both of its small products on the matrix cores:
//   s_kj = sum_s part[s][k][j]               (numerator (W^T V)_kj, split order)
//   d_kj = sum_l G_kl h_lj                   (denominator ((W^T W) H)_kj)
//   h_kj <- h_kj * (s_kj / d_kj)  if d_kj > 0, else unchanged
// and, for the next W half-step, this workgroup's partial Gram
//   sum over its columns j of h_kj h_lj      (H_new H_new^T)
// accumulated over the column blocks it takes (grid-stride) into
// gout[blockIdx.x] (gram_only: the partial Gram of the current H alone, in
// the same order, so a context that starts from an H reproduces the Grams
// of one that reached it).  The vector-unit form does both products with scalar
// FMAs from LDS; here each is a (RP x K) (K x N) product of
// v_mfma_f32_16x16x4_f32 from LDS-staged operands.  In the BF16 tier G, H
// and the new H enter the products rounded to bfloat16 (the tier's operand
// rounding; the products of two bf16 values are exact in float32), and the
// ratio uses the float32 master H.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmf_device.h"
#include "nmf_internal.h"

namespace nmfk {
namespace {

// Split sums of NI float4 items at part + off[e] (split pitch sp), each in
// ascending split order; the loads of B splits of all items are issued
// before any is added.
template <int NI, int B>
__device__ __forceinline__ void split_sums(const float* __restrict__ part,
                                           const int64_t (&off)[NI], const bool (&ok)[NI],
                                           int64_t sp, int splits, float4 (&s)[NI]) {
#pragma unroll
  for (int e = 0; e < NI; ++e) s[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int q = 0; q < splits; q += B) {
    float4 v[NI][B];
#pragma unroll
    for (int e = 0; e < NI; ++e)
#pragma unroll
      for (int u = 0; u < B; ++u) {
        v[e][u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok[e] && q + u < splits)
          v[e][u] = *reinterpret_cast<const float4*>(part + (q + u) * sp + off[e]);
      }
#pragma unroll
    for (int e = 0; e < NI; ++e)
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (q + u < splits) {
          s[e].x += v[e][u].x;
          s[e].y += v[e][u].y;
          s[e].z += v[e][u].z;
          s[e].w += v[e][u].w;
        }
  }
}

// A workgroup of 4 waves takes COLS columns with all RP ranks.  Its loads,
// the ratio update and the stores use float4 items (a thread's items: rank
// kk, 4 adjacent columns); the products meet them through LDS.  Denominator:
// wave w owns the 16-column strip w (of COLS / 16) and every 16-rank tile;
// lane (c, g) supplies A = G[16 mt + c][l] and B = H[l][16 w + c] for k-slot
// g, and at step s of a group of 16 l it takes l = 4 g + s, so that its G
// values are one 16-byte LDS read per group.  It ends with
// D[16 mt + 4 g + v][16 w + c].  Gram: wave w owns the 16-rank row tile w
// (of RP / 16) and every column tile, over K = the block's columns, in the
// same way.
template <int RP, int COLS, bool EG>
__global__ __launch_bounds__(256) void k_update_h_mf(
    int64_t n, int r, const float* __restrict__ part, int64_t ldp, int64_t sp, int splits,
    const float* __restrict__ G, float* __restrict__ Hp, int64_t ldh, float* __restrict__ Hc,
    uint16_t* __restrict__ Hb, int bf16, float* __restrict__ gout, int gram_only) {
  static_assert(RP % 16 == 0 && RP <= 64 && COLS % 16 == 0 && COLS <= 64, "tile shape");
  constexpr int MT = RP / 16, JT = COLS / 16;
  constexpr int GP = RP + 4;    // row pitches (16-byte aligned rows)
  constexpr int HPC = COLS + 4;
  constexpr int NQ = RP * COLS / 4;        // float4 items of a block
  constexpr int NI = (NQ + 255) / 256;     // items per thread
  __shared__ __attribute__((aligned(16))) float Gs[RP * GP];   // G (rounded in BF16)
  __shared__ __attribute__((aligned(16))) float Hs[RP * HPC];  // H block (rounded in BF16)
  __shared__ __attribute__((aligned(16))) float Ds[RP * HPC];  // G H, then the new H
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const bool gram = gout != nullptr;
  // the caller's H takes float4 stores when its rows keep 16-byte alignment
  const bool hc4 = (n % 4 == 0) && (reinterpret_cast<uintptr_t>(Hc) % 16 == 0);

  // G once per workgroup (none for gram_only).  EG: loaded into registers
  // here and stored to LDS after the first block's own loads have been
  // issued, so that all of them share one memory round trip (the registers
  // this holds cost occupancy, so the host picks EG only when the grid is
  // one workgroup per CU); else staged first, each store waiting for its load.
  constexpr int NG = EG ? (RP * RP / 4 + 255) / 256 : 1;
  float4 gq[NG];
  if constexpr (EG) {
#pragma unroll
    for (int e = 0; e < NG; ++e) {
      const int idx = tid + 256 * e;
      gq[e] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!gram_only && idx < RP * RP / 4) gq[e] = *reinterpret_cast<const float4*>(&G[4 * idx]);
    }
  } else {
    for (int idx = tid; idx < (gram_only ? 0 : RP * RP / 4); idx += 256) {
      const int k = (4 * idx) / RP, l = (4 * idx) % RP;
      float4 v = *reinterpret_cast<const float4*>(&G[4 * idx]);
      if (bf16) {
        v.x = bf16_val(v.x); v.y = bf16_val(v.y); v.z = bf16_val(v.z); v.w = bf16_val(v.w);
      }
      *reinterpret_cast<float4*>(&Gs[k * GP + l]) = v;
    }
  }
  bool g_staged = !EG || gram_only != 0;

  v4f gacc[MT];
#pragma unroll
  for (int nt = 0; nt < MT; ++nt) gacc[nt] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int64_t blk = blockIdx.x; blk * COLS < n; blk += gridDim.x) {
    const int64_t j0 = blk * COLS;
    // item e of this thread: rank kk, columns j0 + j4 .. + 3 (float4); its
    // master values and split sums are loaded first
    float4 hr[NI], sv[NI];
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
    if (!gram_only) {
      split_sums<NI, (NI >= 4 ? 4 : 16 / NI)>(part, off, ok, sp, splits, sv);
    } else {
#pragma unroll
      for (int e = 0; e < NI; ++e) sv[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (EG && !g_staged) {  // first block only; read after the barriers below
#pragma unroll
      for (int e = 0; e < NG; ++e) {
        const int idx = tid + 256 * e;
        if (idx >= RP * RP / 4) continue;
        const int k = (4 * idx) / RP, l = (4 * idx) % RP;
        float4 v = gq[e];
        if (bf16) {
          v.x = bf16_val(v.x); v.y = bf16_val(v.y); v.z = bf16_val(v.z); v.w = bf16_val(v.w);
        }
        *reinterpret_cast<float4*>(&Gs[k * GP + l]) = v;
      }
      g_staged = true;
    }
    __syncthreads();  // the previous block's Hs / Ds reads are done
#pragma unroll
    for (int e = 0; e < NI; ++e) {
      const int idx = tid + 256 * e;
      if (NQ % 256 != 0 && idx >= NQ) continue;
      const int kk = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
      float4 v = hr[e];
      if (bf16) {
        v.x = bf16_val(v.x); v.y = bf16_val(v.y); v.z = bf16_val(v.z); v.w = bf16_val(v.w);
      }
      *reinterpret_cast<float4*>(&Hs[kk * HPC + j4]) = v;
    }
    __syncthreads();
    if (!gram_only) {
      // D = G H_block: wave w the 16-column strip w, every rank tile
      if (w < JT) {
        v4f acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int l0 = 0; l0 < RP; l0 += 16) {
          float b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) b[s] = Hs[(l0 + 4 * g + s) * HPC + 16 * w + c];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const float4 a =
                *reinterpret_cast<const float4*>(&Gs[(16 * mt + c) * GP + l0 + 4 * g]);
            acc[mt] = mfma_f32(a.x, b[0], acc[mt]);
            acc[mt] = mfma_f32(a.y, b[1], acc[mt]);
            acc[mt] = mfma_f32(a.z, b[2], acc[mt]);
            acc[mt] = mfma_f32(a.w, b[3], acc[mt]);
          }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v) Ds[(16 * mt + 4 * g + v) * HPC + 16 * w + c] = acc[mt][v];
      }
      __syncthreads();
    }
    // ratio update of this thread's items, then the new values (rounded in
    // BF16) into Ds for the Gram
#pragma unroll
    for (int e = 0; e < NI; ++e) {
      const int idx = tid + 256 * e;
      if (NQ % 256 != 0 && idx >= NQ) continue;
      const int kk = idx / (COLS / 4), j4 = 4 * (idx % (COLS / 4));
      float4 hn = make_float4(0.f, 0.f, 0.f, 0.f);
      if (ok[e]) {
        const float4 h = hr[e];
        if (gram_only) {
          hn = h;
        } else {
          const float4 d = *reinterpret_cast<const float4*>(&Ds[kk * HPC + j4]);
          const float4 sm = sv[e];
          hn.x = (d.x > 0.f) ? h.x * (sm.x / d.x) : h.x;
          hn.y = (d.y > 0.f) ? h.y * (sm.y / d.y) : h.y;
          hn.z = (d.z > 0.f) ? h.z * (sm.z / d.z) : h.z;
          hn.w = (d.w > 0.f) ? h.w * (sm.w / d.w) : h.w;
          const int64_t j = j0 + j4;
          *reinterpret_cast<float4*>(&Hp[(int64_t)kk * ldh + j]) = hn;
          // the bf16 copy has the padded pitch too (its padded columns get
          // the zeros the padded H holds); the caller's H has pitch n
          if (Hb)
            *reinterpret_cast<uint2*>(&Hb[(int64_t)kk * ldh + j]) =
                make_uint2((uint32_t)to_bf16(hn.x) | ((uint32_t)to_bf16(hn.y) << 16),
                           (uint32_t)to_bf16(hn.z) | ((uint32_t)to_bf16(hn.w) << 16));
          if (kk < r) {
            if (hc4 && j + 3 < n) {
              *reinterpret_cast<float4*>(&Hc[(int64_t)kk * n + j]) = hn;
            } else {
              const float hv[4] = {hn.x, hn.y, hn.z, hn.w};
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (j + u < n) Hc[(int64_t)kk * n + j + u] = hv[u];
            }
          }
        }
      }
      if (bf16) {
        hn.x = bf16_val(hn.x); hn.y = bf16_val(hn.y); hn.z = bf16_val(hn.z); hn.w = bf16_val(hn.w);
      }
      // (each thread rewrites only the entries of its own items, after
      // reading their denominators)
      if (gram) *reinterpret_cast<float4*>(&Ds[kk * HPC + j4]) = hn;
    }
    if (!gram) continue;
    __syncthreads();
    // partial Gram: rank tile w against every rank tile, K = the block's columns
    if (w < MT) {
#pragma unroll
      for (int j4 = 0; j4 < COLS; j4 += 16) {
        const float4 a = *reinterpret_cast<const float4*>(&Ds[(16 * w + c) * HPC + j4 + 4 * g]);
#pragma unroll
        for (int nt = 0; nt < MT; ++nt) {
          const float4 b = *reinterpret_cast<const float4*>(&Ds[(16 * nt + c) * HPC + j4 + 4 * g]);
          gacc[nt] = mfma_f32(a.x, b.x, gacc[nt]);
          gacc[nt] = mfma_f32(a.y, b.y, gacc[nt]);
          gacc[nt] = mfma_f32(a.z, b.z, gacc[nt]);
          gacc[nt] = mfma_f32(a.w, b.w, gacc[nt]);
        }
      }
    }
  }
  if (gram && w < MT) {
    float* out = gout + (int64_t)blockIdx.x * RP * RP;
#pragma unroll
    for (int nt = 0; nt < MT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(16 * w + 4 * g + v) * RP + 16 * nt + c] = gacc[nt][v];
  }
}

}  // namespace

hipError_t launch_update_h_mf(int rp, int64_t n, int r, const float* part, int64_t ldp,
                              int64_t sp, int splits, const float* G, float* Hp, int64_t ldh,
                              float* Hcaller, uint16_t* Hb, bool bf16, float* gout, int grid,
                              int cols, bool gram_only, bool early_g, hipStream_t st) {
#define UHF(R, C)                                                                          \
  do {                                                                                     \
    if (early_g)                                                                           \
      hipLaunchKernelGGL((k_update_h_mf<R, C, true>), dim3(grid), dim3(256), 0, st, n, r, part, \
                         ldp, sp, splits, G, Hp, ldh, Hcaller, Hb, (int)bf16, gout,         \
                         (int)gram_only);                                                  \
    else                                                                                   \
      hipLaunchKernelGGL((k_update_h_mf<R, C, false>), dim3(grid), dim3(256), 0, st, n, r,   \
                         part, ldp, sp, splits, G, Hp, ldh, Hcaller, Hb, (int)bf16, gout,   \
                         (int)gram_only);                                                  \
  } while (0)
#define UHC(R)                     \
  do {                             \
    if (cols == 64) UHF(R, 64);    \
    else if (cols == 32) UHF(R, 32); \
    else UHF(R, 16);               \
  } while (0)
  switch (rp) {
    case 16: UHC(16); break;
    case 32: UHC(32); break;
    case 64: UHC(64); break;
    default: return hipErrorInvalidValue;
  }
#undef UHC
#undef UHF
  return hipGetLastError();
}

}  // namespace nmfk
