// Fused served launches: one work table of requests (different trees, point
// counts and forms) in one launch over a fixed grid that strides over the
// 64-point blocks of all requests.  Served trees may hold powers outside the
// table (computed on the fly), so these kernels carry that path too.
#include "walk_core.h"

namespace fpe {

__device__ __forceinline__ int find_item(const int64_t* __restrict__ prefix, int n, int64_t b) {
  int lo = 0, hi = n;   // prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_serve_zero(WorkTable* wt) {
  const int n = wt->n_items;
  int64_t* cnt = table_counters(wt);
  for (int r = threadIdx.x; r < n; r += blockDim.x) cnt[r] = 0;
}

// The shallow kernel asks for eight waves per SIMD (64 VGPRs; a few values
// of the rare paths spill), measured 2 % faster than the seven its registers
// would otherwise give.
template <int DMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(DMAX <= 8 ? 8 : 1)))
void k_serve_walk(WorkTable* wt) {
  const int n = wt->n_items;
  const int64_t total = wt->total_blocks;
  const WorkItem* items = table_items(wt);
  const int64_t* prefix = table_prefix(wt);
  int64_t* counters = table_counters(wt);
  extern __shared__ __align__(16) char lds[];
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    const int r = find_item(prefix, n, b);
    const WorkItem& it = items[r];
    const int64_t i = (b - prefix[r]) * kBlock + (threadIdx.x & (kWave - 1));
    const bool in = i < it.npts;
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (in && j < it.tree.nvars) ? it.pts[j][i] : 0.0;
    bool flag = false;
    if (it.domain == FPE_F64) {
      // the same programs as fpe_evaluate: chain-like trees walk their
      // program with runs (the item's op pointer), the others their ops
      double y;
      if (it.tree.n_offtable != 0) y = walk_point<ArF64, DMAX, true>(it.tree, x, lds);
      else if (DMAX > 2 && it.tree.depth <= 2) y = walk_point<ArF64, 2, false>(it.tree, x, lds);
      else y = walk_point<ArF64, DMAX, false>(it.tree, x, lds);
      if (in) it.out[i] = y;
    } else {
      // the walk without on-the-fly powers (no coordinates kept) when the
      // tree has none, which is the usual case
      DF rr;
      if (it.tree.n_offtable != 0) rr = walk_point<ArDF32, DMAX, true>(it.tree, x, lds);
      else if (DMAX > 2 && it.tree.depth <= 2) rr = walk_point<ArDF32, 2, false>(it.tree, x, lds);
      else rr = walk_point<ArDF32, DMAX, false>(it.tree, x, lds);
      if (in) {
        const double eabs = df32_abs_bound(it.tree, [&](int v) { return it.pts[v][i]; });
        double y, bnd;
        float cond;
        flag = df32_finish<true>(rr, eabs, it.tol, it.tree.bound_scale, 0, y, cond, bnd);
        it.out[i] = y;
        if (it.cond) it.cond[i] = cond;
      }
    }
    append_flagged(flag, i, it.list, &counters[r]);
  }
}

// The flagged points of all requests of the batch, cut into 64-point blocks
// per request, form one index space: each workgroup builds the prefix of the
// per-request block counts in LDS, then the grid strides over the blocks
// (binary search for the request), so the work is spread evenly whatever the
// mix of request sizes, and every wavefront walks one request's tree.
template <int DMAX>
__global__ __launch_bounds__(kBlock) void k_serve_fallback(WorkTable* wt) {
  const int n = wt->n_items;
  const WorkItem* items = table_items(wt);
  const int64_t* counters = table_counters(wt);
  extern __shared__ __align__(16) char lds[];
  __shared__ int64_t pre[kMaxServe + 1];
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int r = 0; r < n; ++r) {
      pre[r] = acc;
      acc += items[r].domain == FPE_F32C ? (counters[r] + kBlock - 1) / kBlock : 0;
    }
    pre[n] = acc;
  }
  __syncthreads();
  const int64_t total = pre[n];
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    const int r = find_item(pre, n, b);
    const WorkItem& it = items[r];
    const int64_t k = (b - pre[r]) * kBlock + threadIdx.x;
    const int64_t i = k < counters[r] ? it.list[k] : -1;
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (i >= 0 && j < it.tree.nvars) ? it.pts[j][i] : 0.0;
    // as in the walk: no coordinates kept when every power is in the table,
    // and the chain-like walk for trees of depth <= 2
    DD rr;
    if (it.tree.n_offtable != 0) rr = walk_point<ArDD, DMAX, true>(it.tree, x, lds);
    else if (DMAX > 2 && it.tree.depth <= 2) rr = walk_point<ArDD, 2, false>(it.tree, x, lds);
    else rr = walk_point<ArDD, DMAX, false>(it.tree, x, lds);
    if (i >= 0) it.out[i] = rr.h + rr.l;
  }
}

ServeKernels serve_kernels() {
  ServeKernels k;
  k.zero = (const void*)k_serve_zero;
  k.walk8 = (const void*)k_serve_walk<8>;
  k.walk16 = (const void*)k_serve_walk<kMaxDepth>;
  k.fallback8 = (const void*)k_serve_fallback<8>;
  k.fallback16 = (const void*)k_serve_fallback<kMaxDepth>;
  k.walk_lds = std::max({walk_lds_bytes<ArF64, kMaxDepth, 1>(), walk_lds_bytes<ArDF32, kMaxDepth, 1>(),
                         walk_lds_bytes<ArF64, 8, 1>(), walk_lds_bytes<ArDF32, 8, 1>(),
                         walk_lds_bytes<ArF64, 2, 1>(), walk_lds_bytes<ArDF32, 2, 1>()});
  k.fallback_lds = std::max(walk_lds_bytes<ArDD, 8, 1>(), walk_lds_bytes<ArDD, kMaxDepth, 1>());
  return k;
}

size_t work_table_bytes() {
  return 256 + sizeof(WorkItem) * kMaxServe + sizeof(int64_t) * (2 * kMaxServe + 1);
}

}  // namespace fpe
