// Compensated FP32 (double-float) walk kernel and the FP64 (double-double)
// re-evaluation of the points it flags.
#include "walk_core.h"

namespace fpe {

// COND: the condition numbers are written (o.cond); without it the walk's
// condition sums are dead and the compiler drops them.  (The two-point walks
// with the LDS tier hold 7 KB of LDS per wave, which caps them at five waves
// per SIMD; no register budget is asked beyond that.)
template <int DMAX, int PPL, bool OFFT, bool COND>
__global__ __launch_bounds__(kBlock) void k_eval_df32(DevTree tr, Pts<double> P, int64_t npts, F32COut o) {
  extern __shared__ __align__(16) char lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t base = (int64_t)blockIdx.x * kBlock * PPL + threadIdx.x;
  double x[PPL][8];
  load_points<double, PPL>(P, tr.nvars, base, npts, x);
  DF r[PPL];
  walk_points<ArDF32, DMAX, PPL, OFFT>(tr, x, lds, r);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int64_t i = base + (int64_t)j * kWave;
    bool flag = false;
    if (i < npts) {
      // the coordinates are read again here rather than kept live across the walk
      const double eabs = df32_abs_bound(tr, [&](int v) { return P.p[v][i]; });
      double y, bnd;
      float cond;
      flag = df32_finish<COND>(r[j], eabs, o.tol, tr.bound_scale, o.force, y, cond, bnd);
      o.out[i] = y;
      if constexpr (COND) o.cond[i] = cond;
      if (o.bound) o.bound[i] = bnd;
    }
    if (o.flags) {
      const uint64_t ballot = __ballot(flag);
      const int64_t wbase = i - lane;
      if (lane == 0 && wbase < npts) {
        o.flags[wbase >> 5] = (uint32_t)ballot;
        if (wbase + 32 < npts) o.flags[(wbase >> 5) + 1] = (uint32_t)(ballot >> 32);
      }
    }
    append_flagged(flag, i, o.list, o.count);
  }
}

// FP64 fallback: double-double walk over the flagged points, PPL of them per
// lane.  The grid is fixed; wavefronts stride over the count read from
// device memory.
template <int DMAX, int PPL, bool OFFT>
__global__ __launch_bounds__(kBlock) void k_fallback_dd(DevTree tr, Pts<double> P,
                                                        const int32_t* __restrict__ list,
                                                        const int64_t* __restrict__ count,
                                                        double* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t n = *count;
  const int64_t stride = (int64_t)gridDim.x * kBlock * PPL;
  for (int64_t base = (int64_t)blockIdx.x * kBlock * PPL; base < n; base += stride) {
    double x[PPL][8];
    int64_t idx[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int64_t k = base + (int64_t)j * kWave + threadIdx.x;
      idx[j] = k < n ? list[k] : -1;
#pragma unroll
      for (int v = 0; v < 8; ++v) x[j][v] = (idx[j] >= 0 && v < tr.nvars) ? P.p[v][idx[j]] : 0.0;
    }
    DD r[PPL];
    walk_points<ArDD, DMAX, PPL, OFFT>(tr, x, lds, r);
#pragma unroll
    for (int j = 0; j < PPL; ++j)
      if (idx[j] >= 0) out[idx[j]] = r[j].h + r[j].l;
  }
}

template <int DMAX, int PPL, bool OFFT>
static void go(const KernelLaunch& L, const F32COut& o) {
  Pts<double> P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const double*)L.pts[j];
  if (o.cond)
    hipLaunchKernelGGL((k_eval_df32<DMAX, PPL, OFFT, true>), dim3((unsigned)blocks_for(L.npts, PPL)), dim3(kBlock),
                       (walk_lds_bytes<ArDF32, DMAX, PPL>()), L.stream, L.tr, P, L.npts, o);
  else
    hipLaunchKernelGGL((k_eval_df32<DMAX, PPL, OFFT, false>), dim3((unsigned)blocks_for(L.npts, PPL)), dim3(kBlock),
                       (walk_lds_bytes<ArDF32, DMAX, PPL>()), L.stream, L.tr, P, L.npts, o);
}

void launch_df32(const KernelLaunch& L, const F32COut& o) {
  const bool d2 = L.tr.depth <= 2, d6 = L.tr.depth <= 6, d8 = L.tr.depth <= 8;
  // the chain-like kernels read the program with runs (both widths, so the
  // bits do not depend on the points per lane)
  KernelLaunch R = L;
  R.tr.ops32 = L.tr.ops32r;
  if (L.offt) {
    if (d8) go<8, 1, true>(L, o); else go<kMaxDepth, 1, true>(L, o);
  } else if (d2) {
    if (L.ppl >= 2) go<2, 2, false>(R, o);
    else go<2, 1, false>(R, o);
  } else if (L.ppl >= 2 && d6) {
    go<6, 2, false>(L, o);
  } else if (L.ppl >= 2 && d8) {
    go<8, 2, false>(L, o);
  } else {
    if (d8) go<8, 1, false>(L, o); else go<kMaxDepth, 1, false>(L, o);
  }
}

template <int DMAX, int PPL, bool OFFT>
static void gofb(const KernelLaunch& L, const int32_t* list, const int64_t* count, double* out) {
  Pts<double> P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const double*)L.pts[j];
  hipLaunchKernelGGL((k_fallback_dd<DMAX, PPL, OFFT>), dim3((unsigned)L.nblocks), dim3(kBlock),
                     (walk_lds_bytes<ArDD, DMAX, PPL>()), L.stream, L.tr, P, list, count, out);
}

void launch_fallback(const KernelLaunch& L, const int32_t* list, const int64_t* count, double* out) {
  const bool d2 = L.tr.depth <= 2, d6 = L.tr.depth <= 6, d8 = L.tr.depth <= 8;
  // the chain-like kernels read the FP64 program with runs
  KernelLaunch R = L;
  R.tr.ops64 = L.tr.ops64r;
  if (L.offt) {
    if (d8) gofb<8, 1, true>(L, list, count, out); else gofb<kMaxDepth, 1, true>(L, list, count, out);
  } else if (d2) {
    if (L.ppl >= 2) gofb<2, 2, false>(R, list, count, out);
    else gofb<2, 1, false>(R, list, count, out);
  } else if (L.ppl >= 2 && d6) {
    gofb<6, 2, false>(L, list, count, out);
  } else if (L.ppl >= 2 && d8) {
    gofb<8, 2, false>(L, list, count, out);
  } else {
    if (d8) gofb<8, 1, false>(L, list, count, out); else gofb<kMaxDepth, 1, false>(L, list, count, out);
  }
}

}  // namespace fpe
