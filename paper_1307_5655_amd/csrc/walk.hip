// Host-side launch of the pointwise walks (fpe_evaluate): picks the kernel
// by domain, walk depth, points per lane and whether any power is computed
// on the fly, and sizes each wavefront's LDS power table.
#include "walk_core.h"

namespace fpe {

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

// LDS of one wavefront's power table (one point per lane) for a kernel kind:
// FPE_F64, FPE_F32C (three-float powers), FPE_MODP, or kLdsFallback (the
// double-double re-evaluation; also the size every served kernel reserves).
size_t lds_bytes(const fpe_tree* t, int kind) {
  size_t per = kind == FPE_MODP ? TabM61::bytes_per_entry
             : kind == FPE_F32C ? TabP3::bytes_per_entry
             : kind == kLdsFallback ? std::max(TabDD::bytes_per_entry, TabP3::bytes_per_entry)
             : t->n_table > kTableCap ? TabF64::bytes_per_entry_big
                                    : TabF64::bytes_per_entry;
  return std::max<size_t>(16, per * (size_t)lds_entries(t->n_table));
}

size_t eval_workspace_bytes(const fpe_tree* t, int64_t npts) {
  if (!t || t->domain != FPE_F32C) return 0;
  // [count int64 | pad to 256 | list int32[npts]]
  return 256 + (size_t)std::max<int64_t>(npts, 0) * sizeof(int32_t);
}

namespace {

inline int64_t blocks_for(int64_t n, int ppl) { return (n + kBlock * ppl - 1) / (kBlock * ppl); }

// Points per lane: FP64 walks take 2 (an op drives two independent fused
// multiply-adds); the heavier double-float and modular steps take 1.
int pick_ppl(const fpe_tree* t, const fpe_eval_opts* opts) {
  if (t->n_offtable > 0) return 1;
  // Default: a chain-like walk (depth <= 2, e.g. Hörner) keeps few
  // accumulators and gains from more points per lane (4 FP64, 2 otherwise);
  // deeper walks spend those registers on the stack (2 FP64, 1 otherwise).
  const bool shallow = t->depth <= 2;
  int p = opts && opts->points_per_lane > 0 ? opts->points_per_lane
          : t->domain == FPE_F64               ? (shallow ? 4 : 2)
                                               : (shallow ? 2 : 1);
  if (t->depth > 8) p = std::min(p, t->domain == FPE_F64 ? 2 : 1);
  if (t->domain != FPE_F64) p = std::min(p, 2);
  return p >= 4 ? 4 : p >= 2 ? 2 : 1;
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
  L.nblocks = blocks_for(npts, L.ppl);
  L.stream = st;
  L.lds = lds_bytes(t, t->domain) * L.ppl;
  hipEvent_t eb = opts ? (hipEvent_t)opts->ev_walk_begin : nullptr;
  hipEvent_t ee = opts ? (hipEvent_t)opts->ev_walk_end : nullptr;
  if (t->domain == FPE_F64) {
    if (eb) (void)hipEventRecord(eb, st);
    launch_f64(L, (double*)out);
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
    o.count = (int64_t*)opts->workspace;
    o.list = (int32_t*)((char*)opts->workspace + 256);
    o.tol = opts->tol > 0 ? opts->tol : 1e-12;
    o.force = opts->force;
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, o.count);
    if (eb) (void)hipEventRecord(eb, st);
    launch_df32(L, o);
    if (ee) (void)hipEventRecord(ee, st);
    KernelLaunch F = L;
    F.ppl = 1;
    F.nblocks = std::min<int64_t>(blocks_for(npts, 1), 4096);
    F.lds = lds_bytes(t, kLdsFallback);
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
