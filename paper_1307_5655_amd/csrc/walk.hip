// Host-side launch of the pointwise walks (fpe_evaluate): picks the kernel
// by domain, walk depth, points per lane and whether any power is computed
// on the fly; the kernels' launchers size the LDS tier of the power tables.
#include <mutex>

#include "walk_core.h"

namespace fpe {

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

size_t eval_workspace_bytes(const fpe_tree* t, int64_t npts) {
  if (!t || t->domain != FPE_F32C) return 0;
  // [count int64 | pad to 256 | list int32[npts]]
  return 256 + (size_t)std::max<int64_t>(npts, 0) * sizeof(int32_t);
}

namespace {


// Points per lane: one op drives PPL independent multiply-adds, which
// amortises the wave-uniform dispatch; tables beyond kTableCapMulti entries
// and trees with on-the-fly powers use the one-point kernels.
int pick_ppl(const fpe_tree* t, const fpe_eval_opts* opts) {
  if (t->n_offtable > 0 || t->n_table > kTableCapMulti || t->domain == FPE_IVAL) return 1;
  // Default: 4 points per lane for FP64 (8 for chain-like walks of depth
  // <= 2, whose per-op cost is the wave-uniform dispatch: 4.7 -> 3.8 ms for
  // Hörner at degree 5000 and 1e7 points, while the depth-6 walks gain nothing
  // at 8 for the registers they lose), 2 otherwise (measured best on MI355X
  // once the power table lives in private memory); walks deeper than 8 hold
  // twice the accumulators and take half as many points.
  const int dflt = t->domain != FPE_F64 ? 2 : t->depth <= 2 ? 8 : 4;
  int p = opts && opts->points_per_lane > 0 ? opts->points_per_lane : dflt;
  if (t->depth > 8) p = std::min(p, t->domain == FPE_F64 ? 2 : 1);
  if (t->domain != FPE_F64) p = std::min(p, 2);
  return p >= 8 ? 8 : p >= 4 ? 4 : p >= 2 ? 2 : 1;
}

}  // namespace

fpe_status launch_eval(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                       const fpe_eval_opts* opts, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (t->depth > kMaxDepth) return fail(FPE_EUNSUPPORTED, "walk deeper than the kernels hold");
  if (npts == 0) return FPE_OK;
  if (npts > 0x7fffffff) return fail(FPE_EINVAL, "too many points for one launch");
  KernelLaunch L{};
  L.tr = dev_view(t);
  for (int j = 0; j < t->nvars; ++j) L.pts[j] = pts[j];
  L.npts = npts;
  L.ppl = pick_ppl(t, opts);
  L.offt = t->n_offtable > 0;
  L.stream = st;
  hipEvent_t eb = opts ? (hipEvent_t)opts->ev_walk_begin : nullptr;
  hipEvent_t ee = opts ? (hipEvent_t)opts->ev_walk_end : nullptr;
  const int32_t path = opts ? opts->path : 0;
  if (path < 0 || path > 2) return fail(FPE_EINVAL, "opts->path must be 0, 1 or 2");
  if (path == 2 && !terms_eligible(t))
    return fail(FPE_EUNSUPPORTED, "the term-parallel path takes FPE_F64 and FPE_MODP (2^61-1) trees");
  if (path == 2 || (path == 1 && terms_preferred(t, npts))) {
    if (t->domain == FPE_MODP && t->modulus != kP61) return fail(FPE_EUNSUPPORTED, "evaluation modulus must be 2^61-1");
    if (eb) (void)hipEventRecord(eb, st);
    launch_terms(L, t->domain, out);
    if (ee) (void)hipEventRecord(ee, st);
  } else if (t->domain == FPE_F64) {
    if (eb) (void)hipEventRecord(eb, st);
    launch_f64(L, (double*)out);
    if (ee) (void)hipEventRecord(ee, st);
  } else if (t->domain == FPE_IVAL) {
    // intervals are read and written as 16-byte (lo, hi) pairs
    for (int j = 0; j < t->nvars; ++j)
      if (((uintptr_t)pts[j]) & 15) return fail(FPE_EINVAL, "interval point arrays must be 16-byte aligned");
    if (((uintptr_t)out) & 15) return fail(FPE_EINVAL, "interval output must be 16-byte aligned");
    if (eb) (void)hipEventRecord(eb, st);
    launch_iv(L, (double*)out);
    if (ee) (void)hipEventRecord(ee, st);
  } else if (t->domain == FPE_MODP) {
    if (t->modulus != kP61) return fail(FPE_EUNSUPPORTED, "evaluation modulus must be 2^61-1");
    if (eb) (void)hipEventRecord(eb, st);
    launch_m61(L, (uint64_t*)out);
    if (ee) (void)hipEventRecord(ee, st);
  } else {
    if (!opts || !opts->workspace) return fail(FPE_EINVAL, "FPE_F32C needs opts->workspace");
    if (opts->workspace_bytes < eval_workspace_bytes(t, npts))
      return fail(FPE_ENOMEM, "workspace smaller than fpe_workspace_bytes()");
    if (((uintptr_t)opts->workspace) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
    F32COut o;
    o.out = (double*)out;
    o.cond = opts->cond_out;
    o.flags = opts->flags_out;
    o.bound = opts->bound_out;
    o.count = (int64_t*)opts->workspace;
    o.list = (int32_t*)((char*)opts->workspace + 256);
    o.tol = opts->tol > 0 ? opts->tol : 1e-12;
    o.force = opts->force;
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, o.count);
    if (eb) (void)hipEventRecord(eb, st);
    launch_df32(L, o);
    if (ee) (void)hipEventRecord(ee, st);
    // the fallback grid is fixed (the count is on the device): enough
    // wavefronts to fill the chip at its occupancy, fewer for small inputs
    KernelLaunch F = L;
    F.nblocks = std::min<int64_t>(blocks_for(npts, F.ppl), 8192);
    launch_fallback(F, o.list, o.count, (double*)out);
    if (opts->nfallback_out) {
      hipError_t e = hipMemcpyAsync(opts->nfallback_out, o.count, sizeof(int64_t),
                                    hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("copy: ") + hipGetErrorString(e));
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return FPE_OK;
}

}  // namespace fpe

// ----------------------------------------------------------------------------
// Allocation-free evaluation (fpe_evaluate_noalloc).
//
// The compensated form needs a scratch buffer beyond the caller's inputs and
// outputs: the fallback counter and the list of flagged point indices.  This
// entry point takes it from a file-scope device array instead of a
// workspace argument, so it calls no allocator.  Each GPU the library runs
// on holds its own copy of the array (at its own address) until the process
// ends.  In host code the array's name is only a stand-in for the device
// symbol: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels.
// ----------------------------------------------------------------------------

namespace fpe {
namespace {

constexpr int64_t kNoAllocScratchBytes = 256 + (int64_t)sizeof(int32_t) * FPE_NOALLOC_MAX_POINTS;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of the scratch array (looked up
// on the first call on each device, with that device current).
fpe_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(FPE_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FPE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FPE_OK;
}

}  // namespace
}  // namespace fpe

extern "C" fpe_status fpe_evaluate_noalloc(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                                           const fpe_eval_opts* opts, void* stream) {
  using namespace fpe;
  if (!t) return fail(FPE_EINVAL, "tree is NULL");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (npts < 0) return fail(FPE_EINVAL, "npts < 0");
  if (t->batch != 1) return fail(FPE_EINVAL, "a batch tree is for fpe_compose");
  if (t->domain == FPE_BIGINT) return fail(FPE_EINVAL, "a big-integer tree is evaluated by fpe_eval_bigint");
  if (npts > FPE_NOALLOC_MAX_POINTS)
    return fail(FPE_EINVAL, "npts exceeds FPE_NOALLOC_MAX_POINTS, the allocation-free maximum");
  if (npts == 0) return FPE_OK;
  if (!pts || !out) return fail(FPE_EINVAL, "NULL points or output");
  for (int j = 0; j < t->nvars; ++j)
    if (!pts[j]) return fail(FPE_EINVAL, "NULL point array");
  fpe_eval_opts o{};
  if (opts) o = *opts;
  if (t->domain == FPE_F32C) {
    void* p = nullptr;
    fpe_status st = scratch_address(&p);
    if (st != FPE_OK) return st;
    o.workspace = p;
    o.workspace_bytes = (size_t)kNoAllocScratchBytes;
  }
  return launch_eval(t, pts, npts, out, &o, stream);
}
