// Exact walk kernel modulo the Mersenne prime 2^61 - 1.
#include "walk_core.h"

namespace fpe {

template <int DMAX, int PPL, bool OFFT>
__global__ __launch_bounds__(kBlock) void k_eval_m61(DevTree tr, Pts<uint64_t> P, int64_t npts,
                                                     uint64_t* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t base = (int64_t)blockIdx.x * kBlock * PPL + threadIdx.x;
  uint64_t x[PPL][8];
  load_points<uint64_t, PPL>(P, tr.nvars, base, npts, x);
  uint64_t y[PPL];
  walk_points<ArM61, DMAX, PPL, OFFT>(tr, x, lds, y);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int64_t i = base + (int64_t)j * kWave;
    if (i < npts) out[i] = y[j];
  }
}

template <int DMAX, int PPL, bool OFFT>
static void go(const KernelLaunch& L, uint64_t* out) {
  Pts<uint64_t> P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const uint64_t*)L.pts[j];
  hipLaunchKernelGGL((k_eval_m61<DMAX, PPL, OFFT>), dim3((unsigned)blocks_for(L.npts, PPL)), dim3(kBlock),
                     (walk_lds_bytes<ArM61, DMAX, PPL>()), L.stream, L.tr, P, L.npts, out);
}

void launch_m61(const KernelLaunch& L, uint64_t* out) {
  const bool d2 = L.tr.depth <= 2, d8 = L.tr.depth <= 8;
  if (L.offt) {
    if (d8) go<8, 1, true>(L, out); else go<kMaxDepth, 1, true>(L, out);
  } else if (L.ppl >= 2 && d2) {
    go<2, 2, false>(L, out);
  } else if (L.ppl >= 2 && d8) {
    go<8, 2, false>(L, out);
  } else {
    if (d8) go<8, 1, false>(L, out); else go<kMaxDepth, 1, false>(L, out);
  }
}

}  // namespace fpe
