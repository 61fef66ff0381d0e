/*
 * nmf_ceiling.h -- measured rate ceilings of the device (a measurement aid
 * of libnmf.so, not a step of the method).
 *
 * The published peaks of a GPU assume a clock and an issue rate that the
 * chip need not sustain under load.  nmf_ceiling measures what it does
 * sustain for the operations the library's kernels are built on, so that a
 * kernel's achieved rate can be read against both: the published peak (the
 * roofline) and the measured ceiling.  The measurement is not part of any
 * solver call.
 */
#ifndef NMF_CEILING_H
#define NMF_CEILING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NMF_CEIL_HBM_READ = 0,   /* bytes/s streaming a buffer once, read only     */
  NMF_CEIL_MFMA_F32 = 1,   /* flop/s of v_mfma_f32_16x16x4f32                */
  NMF_CEIL_MFMA_BF16 = 2,  /* flop/s of v_mfma_f32_16x16x32_bf16             */
  NMF_CEIL_MFMA_F64 = 3,   /* flop/s of v_mfma_f64_16x16x4f64                */
  NMF_CEIL_FMA_F64 = 4,    /* flop/s of the float64 vector FMA               */
  NMF_CEIL_MFMA_F32_32 = 5,  /* flop/s of v_mfma_f32_32x32x2f32              */
  NMF_CEIL_MFMA_BF16_32 = 6  /* flop/s of v_mfma_f32_32x32x16_bf16           */
} nmf_ceiling_kind;

/* Measures one rate of the current device: one untimed launch, then reps
 * launches on `stream` timed by two HIP events; *rate_host gets the work of
 * the reps launches (bytes read, or 2 flops per multiply-add) divided by
 * the time between the events.  The compute kinds run 2048 workgroups of 4
 * waves, each wave with independent accumulator chains and no memory
 * traffic but one 8-byte store per lane.
 *   buf        device memory of `bytes` bytes, 256-byte aligned, owned by
 *              the caller; its contents are overwritten.  The read kind
 *              streams its first bytes - 4 MiB bytes and writes per-
 *              workgroup sums after them; the compute kinds write their
 *              stores into its first 4 MiB.
 *   bytes      >= 64 MiB and a multiple of 256 (a read stream should exceed
 *              the caches: give that kind several hundred MiB or more).
 *   reps       1 ... 1000.
 * Returns 0; -1 (an argument out of range, nothing launched) or -3 (a HIP
 * call failed).  Synchronizes `stream`. */
int32_t nmf_ceiling(int32_t kind, void* buf, int64_t bytes, int32_t reps, double* rate_host,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NMF_CEILING_H */
