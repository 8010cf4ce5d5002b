// Plain FP64 walk kernel: one fused multiply-add per node and point.
#include "walk_core.h"

namespace fpe {

// The depth-6 walk with the LDS tier needs one VGPR more than five waves
// per SIMD allow; asking for five keeps that occupancy.
template <int DMAX, int PPL>
constexpr int f64_waves_per_eu() { return DMAX == 6 && PPL == 4 ? 5 : 1; }

template <int DMAX, int PPL, bool OFFT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(f64_waves_per_eu<DMAX, PPL>())))
void k_eval_f64(DevTree tr, Pts<double> P, int64_t npts, double* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t base = (int64_t)blockIdx.x * kBlock * PPL + threadIdx.x;
  double x[PPL][8];
  load_points<double, PPL>(P, tr.nvars, base, npts, x);
  double y[PPL];
  walk_points<ArF64, DMAX, PPL, OFFT>(tr, x, lds, y);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int64_t i = base + (int64_t)j * kWave;
    if (i < npts) out[i] = y[j];
  }
}

template <int DMAX, int PPL, bool OFFT>
static void go(const KernelLaunch& L, double* out) {
  Pts<double> P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const double*)L.pts[j];
  hipLaunchKernelGGL((k_eval_f64<DMAX, PPL, OFFT>), dim3((unsigned)blocks_for(L.npts, PPL)), dim3(kBlock),
                     (walk_lds_bytes<ArF64, DMAX, PPL>()), L.stream, L.tr, P, L.npts, out);
}

void launch_f64(const KernelLaunch& L, double* out) {
  const bool d2 = L.tr.depth <= 2, d6 = L.tr.depth <= 6, d8 = L.tr.depth <= 8;
  // the chain-like kernels read the program with runs (every width, so the
  // bits do not depend on the points per lane)
  KernelLaunch R = L;
  R.tr.ops64 = L.tr.ops64r;
  if (L.offt) {
    if (d8) go<8, 1, true>(L, out); else go<kMaxDepth, 1, true>(L, out);
  } else if (d2) {
    if (L.ppl >= 8) go<2, 8, false>(R, out);
    else if (L.ppl >= 4) go<2, 4, false>(R, out);
    else if (L.ppl >= 2) go<2, 2, false>(R, out);
    else go<2, 1, false>(R, out);
  } else if (L.ppl >= 4 && d6) {
    go<6, 4, false>(L, out);
  } else if (L.ppl >= 4 && d8) {
    go<8, 4, false>(L, out);
  } else if (L.ppl >= 2) {
    if (d8) go<8, 2, false>(L, out); else go<kMaxDepth, 2, false>(L, out);
  } else {
    if (d8) go<8, 1, false>(L, out); else go<kMaxDepth, 1, false>(L, out);
  }
}

}  // namespace fpe
