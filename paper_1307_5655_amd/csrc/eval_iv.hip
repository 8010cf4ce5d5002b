// Interval walk kernel: one point (a box of intervals) per lane; the result
// is an outward-rounded enclosure [lo, hi] of the tree's interval evaluation.
#include "walk_core.h"

namespace fpe {

// Intervals are stored as (lo, hi) pairs: a lane reads 16 contiguous bytes.
struct IvPts {
  const double* p[8];
};

template <int DMAX, bool OFFT>
__global__ __launch_bounds__(kBlock) void k_eval_iv(DevTree tr, IvPts P, int64_t npts, double* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool in = i < npts;
  IV x[1][8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    if (v < tr.nvars && in) {
      const double2 q = *(const double2*)(P.p[v] + 2 * i);
      x[0][v] = IV{q.x, q.y};
    } else {
      x[0][v] = IV{0.0, 0.0};
    }
  }
  IV y[1];
  walk_points<ArIV, DMAX, 1, OFFT>(tr, x, lds, y);
  if (in) {
    // a non-finite bound (overflow, or an infinity met by a zero) gives no
    // information: the whole line
    IV r = y[0];
    if (!(isfinite(r.lo) && isfinite(r.hi))) r = IV{-INFINITY, INFINITY};
    *(double2*)(out + 2 * i) = double2{r.lo, r.hi};
  }
}

template <int DMAX, bool OFFT>
static void go(const KernelLaunch& L, double* out) {
  IvPts P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const double*)L.pts[j];
  hipLaunchKernelGGL((k_eval_iv<DMAX, OFFT>), dim3((unsigned)blocks_for(L.npts, 1)), dim3(kBlock),
                     (walk_lds_bytes<ArIV, DMAX, 1>()), L.stream, L.tr, P, L.npts, out);
}

void launch_iv(const KernelLaunch& L, double* out) {
  const bool d2 = L.tr.depth <= 2, d8 = L.tr.depth <= 8;
  if (L.offt) {
    if (d8) go<8, true>(L, out); else go<kMaxDepth, true>(L, out);
  } else if (d2) {
    go<2, false>(L, out);
  } else if (d8) {
    go<8, false>(L, out);
  } else {
    go<kMaxDepth, false>(L, out);
  }
}

}  // namespace fpe
