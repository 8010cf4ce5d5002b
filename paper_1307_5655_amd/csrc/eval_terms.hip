// Few points, big trees: the terms of p in parallel.
//
// The tree walk gives one lane one point and runs the tree's ops in order,
// so with few points most of the chip idles while each lane runs a long
// chain of dependent steps.  Here one workgroup takes one point and spreads
// the polynomial's terms over its lanes: each lane evaluates its terms
// c * prod_j x_j^{e_j} and the partial sums meet in a wavefront reduction
// (DPP row shifts within the rows of 16 lanes, then the rows' last lanes)
// and across the workgroup's wavefronts in LDS.  This is the direct scheme's
// evaluation of the same polynomial (every term a child of the root,
// Section 1), whatever scheme the tree was compiled with: exact modulo
// 2^61 - 1, and in FP64 within (nvars (2 log2 deg + 1) + terms per lane + 8) u
// of p~(|x|) = sum |c| |x|^m.
//
// The workgroup first fills an LDS table of its point's powers x_j^k,
// k = 0..deg_max(j), each by fast exponentiation (Section 2.2), so a term
// costs one table read and one product per variable (x^0 = 1 makes the
// product exact where an exponent is 0); trees whose table would not fit in
// 64 KB take each power by fast exponentiation in the term itself, with the
// same values.  A lane loads the coefficients and exponents of four of its
// terms before it evaluates them, so their loads are in flight together.
#include <algorithm>
#include <climits>
#include <cmath>

#include "walk_core.h"

namespace fpe {

namespace {

// Variable j's powers x_j^0 .. x_j^deg_max(j) sit at entries off[j] ..
// off[j + 1] - 1 of a point's table.
struct TermTab {
  int32_t off[9];
};
constexpr int kTermTableMax = 8000;   // entries (8 B each) a workgroup's LDS tables may hold
// From this many points on, a workgroup takes kTermPts of them (the grid
// still fills the chip), so each term record it loads serves them all.
constexpr int kTermPts = 4;
constexpr int64_t kTermMultiMin = 2048;

constexpr int kTermThreads = 256;
constexpr int kTermUnroll = 4;

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

template <int kDom>
__device__ __forceinline__ uint64_t term_pow(uint64_t x, uint32_t e) {
  if constexpr (kDom == 0) return (uint64_t)__double_as_longlong(pow_f64(u2d(x), e));
  else return pow_m61(x, e);
}
template <int kDom>
__device__ __forceinline__ uint64_t term_mul(uint64_t a, uint64_t b) {
  if constexpr (kDom == 0) return (uint64_t)__double_as_longlong(u2d(a) * u2d(b));
  else return m61_mul(a, b);
}

// kDom 0: FP64 (values as their bits), 1: residues mod 2^61 - 1.  kTab: the
// powers come from the points' LDS tables (point p's variable j at
// p * tt.off[nvars] + tt.off[j] ..).  kPts points per workgroup share each
// loaded term record (kPts > 1 only with the tables).
template <int kDom, bool kTab, int kPts>
__global__ __launch_bounds__(kTermThreads) void k_eval_terms(DevTree tr, Pts<uint64_t> P, int64_t npts,
                                                             uint64_t* __restrict__ out, TermTab tt) {
  static_assert(kTab || kPts == 1, "powers per term: one point per workgroup");
  extern __shared__ uint64_t ptab[];
  __shared__ uint64_t wsum[kPts][kTermThreads / kWave];
  const int64_t pt0 = (int64_t)blockIdx.x * kPts;
  const int nv = tr.nvars;
  uint64_t x[8];
  if constexpr (kTab) {
    const int ne = tt.off[nv];
    for (int i = threadIdx.x; i < kPts * ne; i += kTermThreads) {
      const int p = i / ne, r = i - p * ne;
      int j = 0;
#pragma unroll
      for (int q = 1; q < 8; ++q) j += (q < nv && r >= tt.off[q]) ? 1 : 0;
      const int64_t pt = pt0 + p;
      const uint64_t xj = pt < npts ? P.p[j][pt] : 0u;
      ptab[i] = term_pow<kDom>(xj, (uint32_t)(r - tt.off[j]));
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = j < nv ? P.p[j][pt0] : 0u;
  }
  double accd[kPts];
  uint64_t accm[kPts];
#pragma unroll
  for (int p = 0; p < kPts; ++p) {
    accd[p] = 0.0;
    accm[p] = 0;
  }
  const int n = tr.n_nodes;
  for (int k0 = threadIdx.x; k0 < n; k0 += kTermUnroll * kTermThreads) {
    uint64_t c[kTermUnroll];
    int32_t e[kTermUnroll][8];
#pragma unroll
    for (int u = 0; u < kTermUnroll; ++u) {
      const int k = k0 + u * kTermThreads;
      c[u] = k < n ? tr.tc[k] : 0u;
#pragma unroll
      for (int j = 0; j < 8; ++j) e[u][j] = (k < n && j < nv) ? tr.te[(int64_t)k * nv + j] : 0;
    }
#pragma unroll
    for (int u = 0; u < kTermUnroll; ++u) {
      if (c[u] == 0) continue;   // junction nodes and the tail
#pragma unroll
      for (int p = 0; p < kPts; ++p) {
        uint64_t v = c[u];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (j >= nv) break;
          if constexpr (kTab) v = term_mul<kDom>(v, ptab[p * tt.off[nv] + tt.off[j] + e[u][j]]);
          else if (e[u][j] != 0) v = term_mul<kDom>(v, term_pow<kDom>(x[j], (uint32_t)e[u][j]));
        }
        if constexpr (kDom == 0) accd[p] += u2d(v);
        else accm[p] = m61_add(accm[p], v);
      }
    }
  }
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int p = 0; p < kPts; ++p) {
    uint64_t s;
    if constexpr (kDom == 0) s = wave_sum((uint64_t)__double_as_longlong(accd[p]), AddF64{});
    else s = wave_sum(accm[p], AddM61{});
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[p][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < kPts && pt0 + threadIdx.x < npts) {
    const int p = threadIdx.x;
    if constexpr (kDom == 0) {
      const AddF64 add;
      out[pt0 + p] = add(add(wsum[p][0], wsum[p][1]), add(wsum[p][2], wsum[p][3]));
    } else {
      const AddM61 add;
      out[pt0 + p] = add(add(wsum[p][0], wsum[p][1]), add(wsum[p][2], wsum[p][3]));
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
// (all lanes in parallel up to ~2.6e5 points).  The term path costs 5 us,
// plus one workgroup's pass over the terms (≈ 1 ns a term in FP64, 2 ns mod
// p), plus, over the whole chip, each point's operations (its terms'
// nvars + 1 and its table's exponentiations, about 2 log2(deg + 1) products
// an entry) at ≈ 0.12 ps each in FP64 and 0.6 ps mod p.  The terms are
// taken below half the walk's estimate.
bool terms_preferred(const fpe_tree* t, int64_t npts) {
  if (!terms_eligible(t) || npts <= 0) return false;
  double table = 0;
  for (int j = 0; j < t->nvars; ++j) table += (t->deg_max[j] + 1.0) * 2.0 * bit_length(t->deg_max[j]);
  const bool f64 = t->domain == FPE_F64;
  const double nodes = (double)t->nodes.size();
  const double per_point = nodes * (t->nvars + 1.0) + table;
  const double t_terms = 5e-6 + nodes * (f64 ? 1e-9 : 2e-9) + (double)npts * per_point * (f64 ? 0.12e-12 : 0.6e-12);
  const double t_walk = (double)t->ops64.size() * (f64 ? 100e-9 : 200e-9) * std::max(1.0, (double)npts / 262144.0);
  return t_terms < 0.5 * t_walk;
}

void launch_terms(const KernelLaunch& L, int32_t domain, void* out) {
  Pts<uint64_t> P{};
  for (int j = 0; j < L.tr.nvars; ++j) P.p[j] = (const uint64_t*)L.pts[j];
  TermTab tt{};
  int64_t entries = 0;
  for (int j = 0; j < L.tr.nvars; ++j) {
    entries += (int64_t)L.tr.deg_max[j] + 1;
    tt.off[j + 1] = (int32_t)std::min<int64_t>(entries, INT32_MAX);
  }
  const dim3 block(kTermThreads);
  uint64_t* o = (uint64_t*)out;
  const int64_t n = L.npts;
  const bool f64 = domain == FPE_F64;
  if (n >= kTermMultiMin && kTermPts * entries <= kTermTableMax) {
    // enough points to fill the chip with kTermPts per workgroup
    const dim3 grid((unsigned)((n + kTermPts - 1) / kTermPts));
    const size_t lds = (size_t)(kTermPts * entries) * sizeof(uint64_t);
    if (f64) hipLaunchKernelGGL((k_eval_terms<0, true, kTermPts>), grid, block, lds, L.stream, L.tr, P, n, o, tt);
    else hipLaunchKernelGGL((k_eval_terms<1, true, kTermPts>), grid, block, lds, L.stream, L.tr, P, n, o, tt);
  } else if (entries <= kTermTableMax) {
    const size_t lds = (size_t)entries * sizeof(uint64_t);
    if (f64) hipLaunchKernelGGL((k_eval_terms<0, true, 1>), dim3((unsigned)n), block, lds, L.stream, L.tr, P, n, o, tt);
    else hipLaunchKernelGGL((k_eval_terms<1, true, 1>), dim3((unsigned)n), block, lds, L.stream, L.tr, P, n, o, tt);
  } else {
    if (f64) hipLaunchKernelGGL((k_eval_terms<0, false, 1>), dim3((unsigned)n), block, 0, L.stream, L.tr, P, n, o, tt);
    else hipLaunchKernelGGL((k_eval_terms<1, false, 1>), dim3((unsigned)n), block, 0, L.stream, L.tr, P, n, o, tt);
  }
}

}  // namespace fpe
