/* fpe_probe.h — microbenchmarks of the MI355X (gfx950) rates that the
 * kernels of libfpe are measured against (libfpe_probe.so; measurement only,
 * nothing in libfpe calls it).
 *
 * Each probe is one kernel launch of `blocks` workgroups of 256 threads that
 * runs `iters` iterations of independent chains of one operation, so that the
 * issue rate, not a dependency, bounds it.  The caller times the launch (for
 * example with HIP events on `stream`) and divides the returned operation
 * count by the time:
 *   FPE_PROBE_FMA_F64    FP64 fused multiply-adds (v_fma_f64)
 *   FPE_PROBE_FMA_F32    FP32 fused multiply-adds, not packed (v_fma_f32)
 *   FPE_PROBE_DF32_STEP  compensated (double-float) multiply-add steps a X + b
 *                        of the compensated walk, the running bound included
 *   FPE_PROBE_M61_MAC    multiply-adds modulo 2^61 - 1 as the modular walk does them
 *   FPE_PROBE_MAD_U64    32 x 32 + 64 -> 64-bit integer multiply-adds (v_mad_u64_u32)
 *   FPE_PROBE_MFMA_I8    int8 matrix multiply-accumulate operations (2 per
 *                        multiply-add) of v_mfma_i32_32x32x32_i8
 *   FPE_PROBE_COPY       bytes moved (read + written) by a copy of `bytes`
 *                        bytes from src to dst (16-byte vector loads and stores)
 * sink: device buffer of at least blocks * 256 * 16 bytes (each thread stores
 * its chains there, so the compiler keeps the work).  src/dst/bytes: COPY only
 * (bytes a multiple of 16, buffers 16-byte aligned).
 * Returns the operation count of the launch, or a negative value on an
 * invalid argument or a failed launch. */
#ifndef FPE_PROBE_H
#define FPE_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FPE_PROBE_FMA_F64 = 0,
  FPE_PROBE_FMA_F32 = 1,
  FPE_PROBE_DF32_STEP = 2,
  FPE_PROBE_M61_MAC = 3,
  FPE_PROBE_MAD_U64 = 4,
  FPE_PROBE_MFMA_I8 = 5,
  FPE_PROBE_COPY = 6
} fpe_probe_kind;

double fpe_probe_launch(int32_t kind, int64_t blocks, int64_t iters, void* sink, const void* src, void* dst,
                        size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FPE_PROBE_H */
