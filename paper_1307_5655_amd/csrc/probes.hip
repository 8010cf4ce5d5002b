// Rate probes (libfpe_probe.so): one kernel per operation, independent
// chains per thread so that issue, not latency, bounds each.  The double-float
// step and the modular multiply-add are the walks' own (walk_core.h).
#include <hip/hip_runtime.h>

#include "../../include/fpe_probe.h"
#include "walk_core.h"

namespace fpe {
namespace {

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void p_fma_f64(int64_t iters, double* sink) {
  const int t = blockIdx.x * kT + threadIdx.x;
  double a[8];
  const double b = 1.0 + 1e-9 * (t & 7), c = 1e-12 * (1 + (t & 3));   // VGPR operands
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.0 + k;
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = __builtin_fma(a[k], b, c);
  }
  double s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  sink[t] = s;
}

__global__ __launch_bounds__(kT) void p_fma_f32(int64_t iters, float* sink) {
  const int t = blockIdx.x * kT + threadIdx.x;
  float a[16];
  const float b = 1.0f + 1e-6f * (t & 7), c = 1e-7f * (float)(1 + (t & 3));   // VGPR operands
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = 1.0f + k;
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = __builtin_fmaf(a[k], b, c);
  }
  float s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += a[k];
  sink[t] = s;
}

__global__ __launch_bounds__(kT) void p_df32(int64_t iters, float* sink) {
  const int t = blockIdx.x * kT + threadIdx.x;
  DF acc[4];
  const P2 X{0.999f + 1e-6f * (t & 7), 1e-9f};
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = DF{0.5f + k, 0.f, 0.f, 1.f};
  DF b{0.25f, 1e-9f, 1e-20f, 0.25f};
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = df_step<true, true>(acc[k].h, acc[k].l, acc[k].e, acc[k].t, X, b.h, b.l, b.e, b.t);
  }
  float s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k].h + acc[k].l + acc[k].e + acc[k].t;
  sink[t] = s;
}

__global__ __launch_bounds__(kT) void p_m61(int64_t iters, uint64_t* sink) {
  const int t = blockIdx.x * kT + threadIdx.x;
  uint64_t a[4];
  const uint64_t x = (0x123456789abcdefull + t) % kP61, b = 0x0fedcba987654321ull % kP61;
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = (uint64_t)(t + k + 1);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = m61_add(m61_mul(a[k], x), b);
  }
  sink[t] = a[0] ^ a[1] ^ a[2] ^ a[3];
}

__global__ __launch_bounds__(kT) void p_mad_u64(int64_t iters, uint64_t* sink) {
  const int t = blockIdx.x * kT + threadIdx.x;
  uint64_t a[8];
  const uint32_t x = 0x9e3779b9u + t, y = 0x7f4a7c15u;
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (uint64_t)(t + k);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (uint64_t)(x ^ (uint32_t)a[k]) * y + a[k];
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  sink[t] = s;
}

typedef int8_t i8x16 __attribute__((ext_vector_type(16)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(kT) void p_mfma_i8(int64_t iters, int32_t* sink) {
  const int t = blockIdx.x * kT + threadIdx.x;
  i8x16 a, b;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    a[k] = (int8_t)((t + k) & 0x7f);
    b[k] = (int8_t)((3 * t + k) & 0x7f);
  }
  i32x16 c[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) c[k] = i32x16{};
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c[k], 0, 0, 0);
  }
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int r = 0; r < 16; ++r) s += c[k][r];
  }
  sink[t] = s;
}

__global__ __launch_bounds__(kT) void p_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) dst[i] = src[i];
}

}  // namespace
}  // namespace fpe

extern "C" double fpe_probe_launch(int32_t kind, int64_t blocks, int64_t iters, void* sink, const void* src,
                                   void* dst, size_t bytes, void* stream) {
  using namespace fpe;
  hipStream_t st = (hipStream_t)stream;
  if (blocks < 1 || blocks > (1 << 20) || iters < 0) return -1;
  if (kind != FPE_PROBE_COPY && !sink) return -1;
  const double threads = (double)blocks * kT;
  double ops = 0;
  switch (kind) {
    case FPE_PROBE_FMA_F64:
      hipLaunchKernelGGL(p_fma_f64, dim3((unsigned)blocks), dim3(kT), 0, st, iters, (double*)sink);
      ops = threads * (double)iters * 8;
      break;
    case FPE_PROBE_FMA_F32:
      hipLaunchKernelGGL(p_fma_f32, dim3((unsigned)blocks), dim3(kT), 0, st, iters, (float*)sink);
      ops = threads * (double)iters * 16;
      break;
    case FPE_PROBE_DF32_STEP:
      hipLaunchKernelGGL(p_df32, dim3((unsigned)blocks), dim3(kT), 0, st, iters, (float*)sink);
      ops = threads * (double)iters * 4;
      break;
    case FPE_PROBE_M61_MAC:
      hipLaunchKernelGGL(p_m61, dim3((unsigned)blocks), dim3(kT), 0, st, iters, (uint64_t*)sink);
      ops = threads * (double)iters * 4;
      break;
    case FPE_PROBE_MAD_U64:
      hipLaunchKernelGGL(p_mad_u64, dim3((unsigned)blocks), dim3(kT), 0, st, iters, (uint64_t*)sink);
      ops = threads * (double)iters * 8;
      break;
    case FPE_PROBE_MFMA_I8:
      hipLaunchKernelGGL(p_mfma_i8, dim3((unsigned)blocks), dim3(kT), 0, st, iters, (int32_t*)sink);
      // per wavefront and instruction: 32 x 32 x 32 multiply-adds = 65536 operations
      ops = (double)blocks * (kT / 64) * (double)iters * 4 * 65536.0;
      break;
    case FPE_PROBE_COPY:
      if (!src || !dst || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) & 15) return -1;
      hipLaunchKernelGGL(p_copy, dim3((unsigned)blocks), dim3(kT), 0, st, (const uint4*)src, (uint4*)dst,
                         (int64_t)(bytes / 16));
      ops = 2.0 * (double)bytes;
      break;
    default:
      return -1;
  }
  return hipGetLastError() == hipSuccess ? ops : -1;
}
