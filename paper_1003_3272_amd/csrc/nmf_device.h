// Device helpers shared by the gfx950 kernel sources: MFMA wrappers,
// bfloat16 rounding, and the waits and barrier of the asynchronous
// global -> LDS copy ring.  Internal linkage: every source gets its own copy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// s_waitcnt vmcnt(VM) (gfx9 encoding, vmcnt split over bits 3:0 and
// 15:14), leaving expcnt and lgkmcnt unconstrained.
template <int VM>
__device__ __forceinline__ void wait_vm() {
  static_assert(VM >= 0 && VM < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((VM & 0xF) | (0x7 << 4) | (0xF << 8) | (((VM >> 4) & 0x3) << 14));
}

// Workgroup barrier for the copy ring.  __syncthreads() (and any LDS
// release fence) would drain every outstanding global->LDS copy, because
// their completion is counted by vmcnt; the ring instead waits for exactly
// its own stage (wait_stage) and then meets at a bare s_barrier.  The empty
// asm statements keep the compiler from moving LDS accesses across it, and
// lgkmcnt(0) retires this wave's own LDS reads first.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int L, int S>
__device__ __forceinline__ void wait_stage(int after) {
  // my loads of the stage being consumed are done once at most
  // L * after loads (those of the `after` later stages, after <= S - 2)
  // are outstanding
  static_assert((S - 2) * L < 64, "vmcnt holds at most 63 outstanding loads");
  if (S >= 6 && after >= 4) wait_vm<(S >= 6 ? 4 * L : 0)>();
  else if (S >= 5 && after >= 3) wait_vm<(S >= 5 ? 3 * L : 0)>();
  else if (S >= 4 && after >= 3) wait_vm<(S >= 4 ? 3 * L : 0)>();
  else if (after >= 2) wait_vm<2 * L>();
  else if (after == 1) wait_vm<L>();
  else wait_vm<0>();
}

}  // namespace
}  // namespace nmfk
