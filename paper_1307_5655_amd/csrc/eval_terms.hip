// Few points, big trees: the terms of p in parallel.
//
// The tree walk gives one lane one point and runs the tree's ops in order,
// so with few points most of the chip idles while each lane runs a long
// chain of dependent steps.  Here one workgroup takes one point and spreads
// the polynomial's terms over its lanes: each lane evaluates its terms
// c * prod_j x_j^{e_j} (powers by fast exponentiation, Section 2.2), and
// the partial sums meet in a wavefront reduction (DPP row shifts within the
// rows of 16 lanes, then the rows' last lanes) and across the workgroup's
// wavefronts in LDS.  This is the direct scheme's evaluation of the same
// polynomial (every term a child of the root, Section 1), whatever scheme
// the tree was compiled with: exact modulo 2^61 - 1, and in FP64 within
// (nvars (2 log2 deg + 1) + terms per lane + 8) u of p~(|x|) = sum |c| |x|^m.
#include <cmath>

#include "walk_core.h"

namespace fpe {

namespace {

constexpr int kTermThreads = 256;

// v of the lane kShr places lower in the same row of 16 (0 for the row's
// first kShr lanes), 64 bits as two DPP moves.
template <int kShr>
__device__ __forceinline__ uint64_t row_shr(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x110 + kShr, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x110 + kShr, 0xF, 0xF, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t read_lane(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

struct AddF64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const {
    return (uint64_t)__double_as_longlong(__longlong_as_double((long long)a) + __longlong_as_double((long long)b));
  }
};
struct AddM61 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return m61_add(a, b); }
};

// The wavefront's sum (every lane active): inclusive scans within the rows
// of 16 lanes leave each row's sum in its last lane; the four are added in a
// fixed order, so the result does not depend on timing.
template <class Add>
__device__ __forceinline__ uint64_t wave_sum(uint64_t v, Add add) {
  v = add(v, row_shr<1>(v));
  v = add(v, row_shr<2>(v));
  v = add(v, row_shr<4>(v));
  v = add(v, row_shr<8>(v));
  return add(add(read_lane(v, 15), read_lane(v, 31)), add(read_lane(v, 47), read_lane(v, 63)));
}

// kDom 0: FP64 (values as their bits), 1: residues mod 2^61 - 1.
template <int kDom>
__global__ __launch_bounds__(kTermThreads) void k_eval_terms(DevTree tr, Pts<uint64_t> P, uint64_t* __restrict__ out) {
  __shared__ uint64_t wsum[kTermThreads / kWave];
  const int64_t pt = blockIdx.x;
  const int nv = tr.nvars;
  uint64_t x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = j < nv ? P.p[j][pt] : 0u;
  double accd = 0.0;
  uint64_t accm = 0;
  for (int k = threadIdx.x; k < tr.n_nodes; k += kTermThreads) {
    const uint64_t c = tr.tc[k];
    if (c == 0) continue;   // junction nodes
    const int32_t* e = tr.te + (int64_t)k * nv;
    if constexpr (kDom == 0) {
      double v = __longlong_as_double((long long)c);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < nv && e[j] != 0) v *= pow_f64(__longlong_as_double((long long)x[j]), (uint32_t)e[j]);
      accd += v;
    } else {
      uint64_t v = c;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < nv && e[j] != 0) v = m61_mul(v, pow_m61(x[j], (uint32_t)e[j]));
      accm = m61_add(accm, v);
    }
  }
  uint64_t s;
  if constexpr (kDom == 0) s = wave_sum((uint64_t)__double_as_longlong(accd), AddF64{});
  else s = wave_sum(accm, AddM61{});
  const int wave = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    if constexpr (kDom == 0) {
      const AddF64 add;
      out[pt] = add(add(wsum[0], wsum[1]), add(wsum[2], wsum[3]));
    } else {
      const AddM61 add;
      out[pt] = add(add(wsum[0], wsum[1]), add(wsum[2], wsum[3]));
    }
  }
}
static_assert(kTermThreads == 4 * kWave, "four wavefront sums");

inline int bit_length(int32_t v) {
  int b = 0;
  while (v > 0) {
    ++b;
    v >>= 1;
  }
  return b;
}

}  // namespace

bool terms_eligible(const fpe_tree* t) { return !t->term_c.empty(); }

// A cost model of the two paths, calibrated on MI355X with the trivariate
// degree-40 tree (12,341 terms): with few points the walk is one chain of
// n_ops dependent steps per lane, ≈ 100 ns a step in FP64 and 200 ns mod p
// (all lanes in parallel up to ~2.6e5 points); the term path costs npts x
// nodes x (powers + 2) operations, each ≈ 4 FP64 lane-operations (20 mod p)
// at 3.9e13 per second, plus 5 us.  The terms are taken below half the
// walk's estimate.
bool terms_preferred(const fpe_tree* t, int64_t npts) {
  if (!terms_eligible(t) || npts <= 0) return false;
  double pw = 0;
  for (int j = 0; j < t->nvars; ++j) pw += 2.0 * bit_length(t->deg_max[j]);
  const bool f64 = t->domain == FPE_F64;
  const double t_terms = (double)npts * (double)t->nodes.size() * (pw + 2.0) * (f64 ? 4.0 : 20.0) / 3.9e13 + 5e-6;
  const double t_walk = (double)t->ops64.size() * (f64 ? 100e-9 : 200e-9) * std::max(1.0, (double)npts / 262144.0);
  return t_terms < 0.5 * t_walk;
}

void launch_terms(const KernelLaunch& L, int32_t domain, void* out) {
  Pts<uint64_t> P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const uint64_t*)L.pts[j];
  if (domain == FPE_F64)
    hipLaunchKernelGGL(k_eval_terms<0>, dim3((unsigned)L.npts), dim3(kTermThreads), 0, L.stream, L.tr, P,
                       (uint64_t*)out);
  else
    hipLaunchKernelGGL(k_eval_terms<1>, dim3((unsigned)L.npts), dim3(kTermThreads), 0, L.stream, L.tr, P,
                       (uint64_t*)out);
}

}  // namespace fpe
