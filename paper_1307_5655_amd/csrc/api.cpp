// C-ABI entry points of libfpe.so (declared in include/fpe.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "fpe_internal.h"

namespace fpe {
fpe_status compile_tree(int32_t nvars, int64_t nterms, const int32_t* exps, const void* coeffs,
                        int64_t batch, int32_t domain, uint64_t modulus, const fpe_scheme* fs,
                        fpe_tree** out);
const char* last_error();

namespace {
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// The chain walk's program for chain-like trees (depth <= 2, every power in
// the table), FP64 and double-float: maximal sequences of at least
// kRunMinOps depth-1 NODE_OPEN steps by powers of the first table entry
// become run records (kRunCode).  Other trees keep their ops.
void build_runs(fpe_tree* t) {
  t->ops64r.clear();
  t->ops32r.clear();
  t->runc.clear();
  t->runc64.clear();
  const bool f32 = t->domain == FPE_F32C;
  if ((t->domain != FPE_F64 && !f32) || t->depth > 2 || t->n_offtable > 0 || t->n_table < 1 ||
      t->table_deg[0] <= 0 || (f32 && t->ops32.size() != t->ops64.size()))
    return;
  const int32_t v0 = t->table_var[0], d0 = t->table_deg[0];
  auto unit_steps = [&](const OpF64& o, int max_gap) -> int {   // steps of x^d0 the op is; 0: not a chain step
    if (op_kind(o.info) != kNodeOpen || op_level(o.info) != 1 || op_pidx2(o.info) != kNoPair) return 0;
    const uint32_t p = op_pidx(o.info);
    if (p == kOffTable || (int32_t)p >= t->n_table || t->table_var[p] != v0 || t->table_deg[p] % d0) return 0;
    const int k = t->table_deg[p] / d0;
    return k <= max_gap ? k : 0;
  };
  auto word2 = [](float a, float b) {
    uint32_t ua, ub;
    std::memcpy(&ua, &a, 4);
    std::memcpy(&ub, &b, 4);
    return (uint64_t)ua | ((uint64_t)ub << 32);
  };
  auto bits32 = [](uint32_t v) {
    float f;
    std::memcpy(&f, &v, 4);
    return f;
  };
  const size_t n = t->ops64.size();
  // the FP64 program with runs (FP64 trees' walk; a compensated tree's
  // double-double fallback, which reads the FP64 records): gaps of up to
  // kRunMaxGap steps of x^d0
  {
    std::vector<OpF64> prog;
    std::vector<uint64_t> coefs;
    bool any = false;
    for (size_t i = 0; i < n;) {
      size_t j = i;
      while (j < n && unit_steps(t->ops64[j], kRunMaxGap) > 0) ++j;
      if (j - i >= (size_t)kRunMinOps) {
        OpF64 r = t->ops64[i];
        r.a = coefs.size();
        for (size_t k = i; k < j; ++k) {
          for (int z = 1; z < unit_steps(t->ops64[k], kRunMaxGap); ++z) coefs.push_back(0);   // +0.0
          coefs.push_back(t->ops64[k].b);
        }
        r.b = coefs.size() - r.a;
        r.deg = kRunCode << 20;
        prog.push_back(r);
        any = true;
        i = j;
      } else {
        prog.push_back(t->ops64[i]);
        ++i;
      }
    }
    if (any && coefs.size() <= 0x7fffffffu) {
      t->ops64r = std::move(prog);
      if (f32) t->runc64 = std::move(coefs);
      else t->runc = std::move(coefs);
    }
  }
  if (!f32) return;
  // the double-float program with runs: gap-free (a compensated step costs
  // more than the dispatch a gap step would save)
  std::vector<OpF32> prog32;
  std::vector<uint64_t> coefs;
  bool any = false;
  for (size_t i = 0; i < n;) {
    size_t j = i;
    while (j < n && unit_steps(t->ops64[j], kRunMaxGapF32) > 0) ++j;
    if (j - i >= (size_t)kRunMinOps) {
      OpF32 r = t->ops32[i];
      const size_t first = coefs.size() / kRunWordsF32;
      for (size_t k = i; k < j; ++k) {
        for (int z = 1; z < unit_steps(t->ops64[k], kRunMaxGapF32); ++z) {   // b = 0, no bound term
          coefs.push_back(0);
          coefs.push_back(0);
        }
        coefs.push_back(word2(t->ops32[k].bh, t->ops32[k].bl));
        coefs.push_back(word2(t->ops32[k].bk2, 0.f));
      }
      r.ah = bits32((uint32_t)first);
      r.al = bits32((uint32_t)(coefs.size() / kRunWordsF32 - first));
      r.deg = kRunCode << 20;
      prog32.push_back(r);
      any = true;
      i = j;
    } else {
      prog32.push_back(t->ops32[i]);
      ++i;
    }
  }
  if (!any || coefs.size() / 2 > 0x7fffffffu) return;
  t->ops32r = std::move(prog32);
  t->runc = std::move(coefs);
}

void layout(fpe_tree* t) {
  // bound data of the compensated walk, from the node array
  for (int j = 0; j < 8; ++j) t->deg_max[j] = 0;
  double c1 = 0;
  for (size_t i = 0; i < t->nodes.size(); ++i) {
    for (int j = 0; j < t->nvars; ++j) t->deg_max[j] = std::max(t->deg_max[j], t->exps[i * t->nvars + j]);
    if (t->domain == FPE_F32C) c1 += std::fabs(t->nodes[i].coef.f);
  }
  // the FP64 sum of n non-negative terms is within n 2^-53 of the exact one
  c1 *= 1.0 + (double)(t->nodes.size() + 1) * std::ldexp(1.0, -52);
  t->abs_scale = df32_abs_scale((int64_t)t->ops64.size(), c1);
  // the composition rows as the kernel reads them (32-bit residues), kept by
  // the tree so that the upload is an asynchronous copy from live memory
  t->coef_rows32.clear();
  if (t->domain == FPE_MODP && t->modulus == kP31) t->coef_rows32.assign(t->coef_rows.begin(), t->coef_rows.end());
  build_runs(t);
  // the few-point path's term coefficients (exponents: t->exps)
  t->term_c.clear();
  if (t->domain == FPE_F64 || (t->domain == FPE_MODP && t->modulus == kP61 && t->batch == 1))
    for (const fpe_node& nd : t->nodes) t->term_c.push_back(nd.coef.u);
  size_t off = 0;
  // each op array is followed by kOpTail zero records (the walk reads ahead)
  t->off_ops64 = off;
  off = align256(off + (t->ops64.size() + kOpTail) * sizeof(OpF64));
  t->off_ops32 = off;
  off = align256(off + (t->ops32.size() + kOpTail) * sizeof(OpF32));
  t->off_chain = off;
  off = align256(off + std::max<size_t>(t->chain.size(), 1) * sizeof(ChainStep));
  t->off_coef = off;
  if (t->domain == FPE_MODP && t->modulus == kP31) off = align256(off + t->coef_rows.size() * sizeof(uint32_t));
  t->off_ops64r = off;
  if (!t->ops64r.empty()) off = align256(off + (t->ops64r.size() + kOpTail) * sizeof(OpF64));
  t->off_ops32r = off;
  if (!t->ops32r.empty()) off = align256(off + (t->ops32r.size() + kOpTail) * sizeof(OpF32));
  t->off_runc = off;
  if (!t->runc.empty()) off = align256(off + t->runc.size() * sizeof(uint64_t));
  t->off_runc64 = off;
  if (!t->runc64.empty()) off = align256(off + t->runc64.size() * sizeof(uint64_t));
  t->off_term_c = off;
  if (!t->term_c.empty()) off = align256(off + t->term_c.size() * sizeof(uint64_t));
  t->off_term_e = off;
  if (!t->term_c.empty()) off = align256(off + t->exps.size() * sizeof(int32_t));
  t->dev_bytes = std::max<size_t>(off, 256);
}
}  // namespace

DevTree dev_view(const fpe_tree* t) {
  DevTree d{};
  const char* b = (const char*)t->dev;
  d.ops64 = (const OpF64*)(b + t->off_ops64);
  d.ops64r = t->ops64r.empty() ? d.ops64 : (const OpF64*)(b + t->off_ops64r);
  d.ops32r = t->ops32r.empty() ? (const OpF32*)(b + t->off_ops32) : (const OpF32*)(b + t->off_ops32r);
  d.runc = (const uint64_t*)(b + t->off_runc);
  d.runc64 = (const uint64_t*)(b + t->off_runc64);
  d.tc = (const uint64_t*)(b + t->off_term_c);
  d.te = (const int32_t*)(b + t->off_term_e);
  d.ops32 = (const OpF32*)(b + t->off_ops32);
  d.chain = (const ChainStep*)(b + t->off_chain);
  d.coef_rows = (const uint32_t*)(b + t->off_coef);
  d.n_ops = (int32_t)t->ops64.size();
  d.n_chain = (int32_t)t->chain.size();
  d.n_table = t->n_table;
  d.nvars = t->nvars;
  d.depth = t->depth;
  d.n_nodes = (int32_t)t->nodes.size();
  d.n_offtable = t->n_offtable;
  d.bound_scale = df32_bound_scale(d.n_ops);
  d.batch = t->batch;
  d.abs_scale = t->abs_scale;
  for (int j = 0; j < 8; ++j) d.deg_max[j] = t->deg_max[j];
  return d;
}

}  // namespace fpe

using namespace fpe;

extern "C" {

const char* fpe_last_error(void) { return fpe::last_error(); }

const char* fpe_version(void) { return "fpe 1.0 gfx950"; }

fpe_status fpe_compile(int32_t nvars, int64_t nterms, const int32_t* exps, const void* coeffs,
                       int64_t batch, int32_t domain, uint64_t modulus, const fpe_scheme* f,
                       fpe_tree** out) {
  try {
    fpe_status s = compile_tree(nvars, nterms, exps, coeffs, batch, domain, modulus, f, out);
    if (s == FPE_OK) layout(*out);
    return s;
  } catch (const std::bad_alloc&) {
    return fail(FPE_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(FPE_EINVAL, "unexpected error in compile");
  }
}

void fpe_tree_free(fpe_tree* t) {
  if (!t) return;
  bigpoint_forget(t);
  compose_levels_forget(t);
  delete t;
}

fpe_status fpe_tree_nodes(const fpe_tree* t, const fpe_node** nodes, int64_t* n, int32_t* max_slot) {
  if (!t) return fail(FPE_EINVAL, "tree is NULL");
  if (nodes) *nodes = t->nodes.data();
  if (n) *n = (int64_t)t->nodes.size();
  if (max_slot) *max_slot = t->max_slot;
  return FPE_OK;
}

fpe_status fpe_tree_get_info(const fpe_tree* t, fpe_tree_info* info) {
  if (!t || !info) return fail(FPE_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof *info);
  info->n_nodes = (int64_t)t->nodes.size();
  info->n_terms = t->n_terms;
  info->nvars = t->nvars;
  info->max_slot = t->max_slot;
  info->max_lazy_height = t->max_lh;
  info->walk_depth = t->depth;
  info->n_powers = t->n_powers;
  info->n_table = t->n_table;
  info->n_chain = (int32_t)t->chain.size();
  info->n_offtable = t->n_offtable;
  info->n_pair_ops = t->n_pairs;
  for (int k = 0; k < 5; ++k) info->n_ops_kind[k] = t->n_kind[k];
  info->domain = t->domain;
  info->modulus = t->modulus;
  info->batch = t->batch;
  return FPE_OK;
}

fpe_status fpe_tree_node_exps(const fpe_tree* t, int64_t i, int32_t* exps_out) {
  if (!t || !exps_out) return fail(FPE_EINVAL, "NULL argument");
  if (i < 0 || i >= (int64_t)t->nodes.size()) return fail(FPE_EINVAL, "node index out of range");
  std::memcpy(exps_out, &t->exps[i * t->nvars], sizeof(int32_t) * t->nvars);
  return FPE_OK;
}

size_t fpe_tree_device_bytes(const fpe_tree* t) { return t ? t->dev_bytes : 0; }

fpe_status fpe_tree_upload(fpe_tree* t, void* dev_buf, size_t bytes, void* stream) {
  if (!t || !dev_buf) return fail(FPE_EINVAL, "NULL argument");
  if (bytes < t->dev_bytes) return fail(FPE_ENOMEM, "device buffer smaller than fpe_tree_device_bytes()");
  if (((uintptr_t)dev_buf) & 255) return fail(FPE_EINVAL, "device buffer must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char* b = (char*)dev_buf;
  // the zero records after each op array (read ahead by the walk), copied
  // from a static zero block so the call records no memset
  static const OpF64 kZero64[kOpTail] = {};
  static const OpF32 kZero32[kOpTail] = {};
  hipError_t e = hipMemcpyAsync(b + t->off_ops64 + t->ops64.size() * sizeof(OpF64), kZero64, sizeof kZero64,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + t->off_ops32 + t->ops32.size() * sizeof(OpF32), kZero32, sizeof kZero32,
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !t->ops64.empty())
    e = hipMemcpyAsync(b + t->off_ops64, t->ops64.data(), t->ops64.size() * sizeof(OpF64),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !t->ops32.empty())
    e = hipMemcpyAsync(b + t->off_ops32, t->ops32.data(), t->ops32.size() * sizeof(OpF32),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !t->chain.empty())
    e = hipMemcpyAsync(b + t->off_chain, t->chain.data(), t->chain.size() * sizeof(ChainStep),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && t->domain == FPE_MODP && t->modulus == kP31)
    e = hipMemcpyAsync(b + t->off_coef, t->coef_rows32.data(), t->coef_rows32.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !t->ops64r.empty()) {
    e = hipMemcpyAsync(b + t->off_ops64r, t->ops64r.data(), t->ops64r.size() * sizeof(OpF64), hipMemcpyHostToDevice,
                       st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b + t->off_ops64r + t->ops64r.size() * sizeof(OpF64), kZero64, sizeof kZero64,
                         hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess && !t->ops32r.empty()) {
    e = hipMemcpyAsync(b + t->off_ops32r, t->ops32r.data(), t->ops32r.size() * sizeof(OpF32), hipMemcpyHostToDevice,
                       st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b + t->off_ops32r + t->ops32r.size() * sizeof(OpF32), kZero32, sizeof kZero32,
                         hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess && !t->runc.empty())
    e = hipMemcpyAsync(b + t->off_runc, t->runc.data(), t->runc.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !t->runc64.empty())
    e = hipMemcpyAsync(b + t->off_runc64, t->runc64.data(), t->runc64.size() * sizeof(uint64_t),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !t->term_c.empty()) {
    e = hipMemcpyAsync(b + t->off_term_c, t->term_c.data(), t->term_c.size() * sizeof(uint64_t),
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b + t->off_term_e, t->exps.data(), t->exps.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                         st);
  }
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
  t->dev = dev_buf;
  return FPE_OK;
}

size_t fpe_workspace_bytes(const fpe_tree* t, int64_t npts) { return eval_workspace_bytes(t, npts); }

int32_t fpe_eval_path(const fpe_tree* t, int64_t npts) {
  if (!t) return 0;
  return terms_preferred(t, npts) ? 2 : 1;
}

fpe_status fpe_evaluate(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                        const fpe_eval_opts* opts, void* stream) {
  if (!t) return fail(FPE_EINVAL, "tree is NULL");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (npts < 0) return fail(FPE_EINVAL, "npts < 0");
  if (t->batch != 1) return fail(FPE_EINVAL, "a batch tree is for fpe_compose");
  if (t->domain == FPE_BIGINT) return fail(FPE_EINVAL, "a big-integer tree is evaluated by fpe_eval_bigint");
  if (npts == 0) return FPE_OK;
  if (!pts || !out) return fail(FPE_EINVAL, "NULL points or output");
  for (int j = 0; j < t->nvars; ++j)
    if (!pts[j]) return fail(FPE_EINVAL, "NULL point array");
  return launch_eval(t, pts, npts, out, opts, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serialisation of the host tree: a flat little-endian byte image
// ---------------------------------------------------------------------------
namespace {
constexpr uint64_t kMagic = 0x3130455246505845ull;  // "EXPFREE01"-like tag
struct Writer {
  std::vector<char> b;
  template <class T> void pod(const T& v) {
    const char* p = (const char*)&v;
    b.insert(b.end(), p, p + sizeof(T));
  }
  template <class T> void vec(const std::vector<T>& v) {
    pod<uint64_t>(v.size());
    const char* p = (const char*)v.data();
    b.insert(b.end(), p, p + v.size() * sizeof(T));
  }
};
struct Reader {
  const char* p;
  size_t n, o = 0;
  bool ok = true;
  template <class T> void pod(T& v) {
    if (o + sizeof(T) > n) { ok = false; return; }
    std::memcpy(&v, p + o, sizeof(T));
    o += sizeof(T);
  }
  template <class T> void vec(std::vector<T>& v) {
    uint64_t k = 0;
    pod(k);
    if (!ok || k > (n - o) / std::max<size_t>(sizeof(T), 1)) { ok = false; return; }
    v.resize(k);
    std::memcpy(v.data(), p + o, k * sizeof(T));
    o += k * sizeof(T);
  }
};
void write_tree(const fpe_tree* t, Writer& w) {
  w.pod(kMagic);
  w.pod(t->nvars); w.pod(t->domain); w.pod(t->modulus); w.pod(t->batch); w.pod(t->n_terms);
  w.pod(t->n_table); w.pod(t->n_powers); w.pod(t->depth); w.pod(t->max_slot); w.pod(t->max_lh);
  w.pod(t->n_offtable); w.pod(t->n_pairs);
  w.vec(t->nodes); w.vec(t->exps); w.vec(t->coef_rows); w.vec(t->ops64); w.vec(t->ops32);
  w.vec(t->chain); w.vec(t->table_var); w.vec(t->table_deg);
}
}  // namespace

extern "C" {

fpe_status fpe_tree_serialize(const fpe_tree* t, void* buf, size_t* bytes) {
  if (!t || !bytes) return fail(FPE_EINVAL, "NULL argument");
  Writer w;
  write_tree(t, w);
  if (!buf) {
    *bytes = w.b.size();
    return FPE_OK;
  }
  if (*bytes < w.b.size()) {
    *bytes = w.b.size();
    return fail(FPE_ENOMEM, "buffer too small");
  }
  std::memcpy(buf, w.b.data(), w.b.size());
  *bytes = w.b.size();
  return FPE_OK;
}

fpe_status fpe_tree_deserialize(const void* buf, size_t bytes, fpe_tree** out) {
  if (!buf || !out) return fail(FPE_EINVAL, "NULL argument");
  Reader r{(const char*)buf, bytes};
  uint64_t magic = 0;
  r.pod(magic);
  if (!r.ok || magic != kMagic) return fail(FPE_EINVAL, "not a serialised tree");
  auto* t = new fpe_tree();
  r.pod(t->nvars); r.pod(t->domain); r.pod(t->modulus); r.pod(t->batch); r.pod(t->n_terms);
  r.pod(t->n_table); r.pod(t->n_powers); r.pod(t->depth); r.pod(t->max_slot); r.pod(t->max_lh);
  r.pod(t->n_offtable); r.pod(t->n_pairs);
  r.vec(t->nodes); r.vec(t->exps); r.vec(t->coef_rows); r.vec(t->ops64); r.vec(t->ops32);
  r.vec(t->chain); r.vec(t->table_var); r.vec(t->table_deg);
  if (!r.ok || r.o != bytes || t->nvars < 1 || t->nvars > 8 ||
      t->exps.size() != t->nodes.size() * (size_t)t->nvars || t->ops64.size() != t->nodes.size() ||
      t->n_table < 0 || t->n_table > kMaxTable) {
    delete t;
    return fail(FPE_EINVAL, "corrupt serialised tree");
  }
  for (const auto& c : t->chain)
    if (c.dst >= t->n_table ||
        (chain_is_mul(c.kind) && (c.s1 >= t->n_table || c.s2 >= t->n_table || chain_var(c.kind) >= (uint32_t)t->nvars)) ||
        (!chain_is_mul(c.kind) && (c.kind != kChainLoad || c.s1 >= t->nvars))) {
      delete t;
      return fail(FPE_EINVAL, "corrupt serialised tree (power chain)");
    }
  // the program is a balanced stack walk that ends with exactly one END
  int32_t depth = 0, maxd = 0;
  for (size_t k = 0; k < t->ops64.size(); ++k) {
    uint32_t kind = op_kind(t->ops64[k].info);
    if ((kind == kEnd) != (k + 1 == t->ops64.size())) depth = -1000;
    if (kind == kLeafOpen) maxd = std::max(maxd, ++depth);
    if (kind == kNodeAdd) --depth;
    if ((kind == kLeafAdd || kind == kNodeOpen) && depth < 1) depth = -1000;
    if (depth < 0) break;
  }
  if (depth < 0 || maxd > kMaxDepth || std::max(maxd, 1) != t->depth) {
    delete t;
    return fail(FPE_EINVAL, "corrupt serialised tree (walk)");
  }
  for (const auto& o : t->ops64) {
    uint32_t p = op_pidx(o.info);
    const uint32_t p2 = op_pidx2(o.info);
    if (op_kind(o.info) > kEnd || (p != kOffTable && p >= (uint32_t)t->n_table) ||
        (p2 != kNoPair && (p2 >= (uint32_t)t->n_table || p == kOffTable)) ||
        (p2 != kNoPair && (op_deg(o.deg) & kThirdBit) && (op_deg(o.deg) & 0xFFu) >= (uint32_t)t->n_table) ||
        op_var(o.info) >= (uint32_t)t->nvars || (int)op_level(o.info) > kMaxDepth ||
        op_code(o.deg) != dispatch_code(o.info)) {
      delete t;
      return fail(FPE_EINVAL, "corrupt serialised tree (program)");
    }
  }
  // domain, modulus, batch and the coefficient rows agree: the composition
  // kernel indexes coef_rows by instance and node, the modular walks take
  // residues below the modulus
  const bool intcoef = t->domain == FPE_MODP || t->domain == FPE_BIGINT;
  bool meta = t->domain >= FPE_F64 && t->domain <= FPE_BIGINT && t->batch >= 1 && t->n_terms >= 1 &&
              t->n_terms <= (int64_t)t->nodes.size() && t->table_var.size() == (size_t)t->n_table &&
              t->table_deg.size() == (size_t)t->n_table;
  if (meta && t->domain == FPE_MODP) meta = t->modulus == kP61 || t->modulus == kP31;
  if (meta && t->domain != FPE_MODP) meta = t->modulus == 0;
  if (meta && t->batch != 1) meta = t->domain == FPE_MODP && t->modulus == kP31;
  if (meta && t->batch > ((int64_t)1 << 40) / (int64_t)std::max<size_t>(t->nodes.size(), 1)) meta = false;
  if (meta) meta = t->coef_rows.size() == (intcoef ? (size_t)t->batch * t->nodes.size() : 0);
  if (meta && t->domain == FPE_MODP)
    for (uint64_t c : t->coef_rows)
      if (c >= t->modulus) { meta = false; break; }
  for (size_t k = 0; meta && k < t->exps.size(); ++k) meta = t->exps[k] >= 0 && t->exps[k] < (1 << 20);
  if (!meta) {
    delete t;
    return fail(FPE_EINVAL, "corrupt serialised tree (domain, batch or coefficients)");
  }
  // the counts the launchers select kernels by are recounted from the
  // program: on-the-fly powers (kernels without that path would read a table
  // entry that does not exist), products of entries, steps by kind; a
  // composition program's constants are node indices into the rows
  int32_t offt = 0, pairs = 0, kinds[5] = {0, 0, 0, 0, 0};
  const bool index_ops = t->domain == FPE_MODP && t->modulus == kP31;
  for (const auto& o : t->ops64) {
    const uint32_t kind = op_kind(o.info);
    const bool haspow = kind != kEnd || (o.info & kEndHasPow);
    if (haspow && op_pidx(o.info) == kOffTable) ++offt;
    if (op_pidx2(o.info) != kNoPair) ++pairs;
    ++kinds[kind];
    if (index_ops && (o.a >= t->nodes.size() || o.b >= t->nodes.size())) offt = -1;
  }
  if (offt != t->n_offtable || pairs != t->n_pairs) {
    delete t;
    return fail(FPE_EINVAL, "corrupt serialised tree (power counts or node indices)");
  }
  for (int k = 0; k < 5; ++k) t->n_kind[k] = kinds[k];
  // the FP32 records repeat the program of the FP64 ones, with the dispatch
  // codes of the double-float walk's deeper LDS tier
  bool same = t->ops32.empty() || t->ops32.size() == t->ops64.size();
  for (size_t k = 0; same && k < t->ops32.size(); ++k)
    same = t->ops32[k].info == t->ops64[k].info &&
           t->ops32[k].deg == ((t->ops64[k].deg & 0xFFFFFu) | (dispatch_code(t->ops64[k].info, kLdsPowersF32) << 20));
  if (!same || (t->domain == FPE_F32C) != !t->ops32.empty()) {
    delete t;
    return fail(FPE_EINVAL, "corrupt serialised tree (program)");
  }
  layout(t);
  *out = t;
  return FPE_OK;
}

size_t fpe_compose_workspace_bytes(const fpe_tree* t, int32_t dq) { return compose_workspace_bytes(t, dq); }

// Limbs that p(x) needs at most for points of lx limbs: deg * lx for x^deg,
// four for the coefficient, and enough for the sum of the terms.
static int64_t bigint_limbs_needed(const fpe_tree* t, int32_t lx) {
  int64_t dp = 0;
  for (size_t i = 0; i < t->nodes.size(); ++i) dp = std::max<int64_t>(dp, t->exps[i]);
  int64_t extra = 1;
  for (int64_t n = t->n_terms; n > 1; n >>= 16) ++extra;
  return dp * lx + 4 + extra;
}

int32_t fpe_bigint_out_limbs(const fpe_tree* t, int32_t lx) {
  if (!t || t->domain != FPE_BIGINT || lx < 1) return 0;
  const int64_t n = bigint_limbs_needed(t, lx);
  return n > kBigMaxLimbs ? 0 : (int32_t)n;
}

size_t fpe_bigint_workspace_bytes(const fpe_tree* t, int32_t lout, int64_t batch) {
  if (!t || t->domain != FPE_BIGINT) return 0;
  return bigint_workspace_bytes(t, lout, batch);
}

fpe_status fpe_eval_bigint(const fpe_tree* t, const uint32_t* x, int32_t lx, int64_t batch, uint32_t* out,
                           int32_t lout, void* workspace, size_t workspace_bytes, void* stream) {
  if (!t || !x || !out) return fail(FPE_EINVAL, "NULL argument");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (t->domain != FPE_BIGINT) return fail(FPE_EINVAL, "the tree is not compiled for FPE_BIGINT");
  if (lx < 1) return fail(FPE_EINVAL, "points need at least one limb");
  if (lout > kBigMaxLimbs) return fail(FPE_EUNSUPPORTED, "more output limbs than the kernel's columns hold");
  if (lout < bigint_limbs_needed(t, lx)) return fail(FPE_EINVAL, "lout smaller than fpe_bigint_out_limbs()");
  return launch_bigint(t, x, lx, batch, out, lout, workspace, workspace_bytes, stream);
}

int64_t fpe_bigpoint_out_limbs(const fpe_tree* t, int32_t lx) {
  if (!t || t->domain != FPE_BIGINT || lx < 1) return 0;
  return bigpoint_out_limbs(t, lx);
}

size_t fpe_bigpoint_workspace_bytes(const fpe_tree* t, int32_t lx) {
  if (!t || t->domain != FPE_BIGINT || lx < 1) return 0;
  return bigpoint_workspace_bytes(t, lx);
}

fpe_status fpe_eval_bigpoint(const fpe_tree* t, const uint32_t* x, int32_t lx, uint32_t* out, int64_t lout,
                             void* workspace, size_t workspace_bytes, void* stream) {
  if (!t || !x || !out) return fail(FPE_EINVAL, "NULL argument");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (t->domain != FPE_BIGINT) return fail(FPE_EINVAL, "the tree is not compiled for FPE_BIGINT");
  if (lx < 1) return fail(FPE_EINVAL, "the point needs at least one limb");
  return launch_bigpoint(t, x, lx, out, lout, workspace, workspace_bytes, stream);
}

int32_t fpe_compose_bigint_coef_limbs(const fpe_tree* t, const uint64_t* q, int32_t dq) {
  return compose_bigint_plan(t, q, dq).lc;
}

int64_t fpe_compose_bigint_out_limbs(const fpe_tree* t, const uint64_t* q, int32_t dq) {
  return compose_bigint_plan(t, q, dq).nout;
}

size_t fpe_compose_bigint_workspace_bytes(const fpe_tree* t, const uint64_t* q, int32_t dq) {
  return compose_bigint_plan(t, q, dq).bytes;
}

fpe_status fpe_compose_bigint(const fpe_tree* t, const uint64_t* q, int32_t dq, uint32_t* out, int64_t lout,
                              void* workspace, size_t workspace_bytes, void* stream) {
  if (!t || !q || !out) return fail(FPE_EINVAL, "NULL argument");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (t->domain != FPE_BIGINT) return fail(FPE_EINVAL, "the tree is not compiled for FPE_BIGINT");
  if (dq < 0) return fail(FPE_EINVAL, "dq < 0");
  return launch_compose_bigint(t, q, dq, out, lout, workspace, workspace_bytes, stream);
}

fpe_status fpe_bigint_status(const void* workspace, void* stream) {
  if (!workspace) return fail(FPE_EINVAL, "NULL workspace");
  int32_t flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, workspace, sizeof flag, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("bigint status: ") + hipGetErrorString(e));
  if (flag) return fail(FPE_ENOMEM, "a big-integer value needed more than lout limbs (result truncated)");
  return FPE_OK;
}

size_t fpe_compose_ex_workspace_bytes(const fpe_tree* t, int32_t dq, int32_t product) {
  return compose_workspace_bytes_ex(t, dq, product);
}

fpe_status fpe_compose_ex(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, int32_t product,
                          void* workspace, size_t workspace_bytes, void* stream) {
  if (!t || !q || !out) return fail(FPE_EINVAL, "NULL argument");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (t->domain != FPE_MODP || t->modulus != kP31 || t->nvars != 1)
    return fail(FPE_EINVAL, "composition needs a univariate tree compiled mod 2^31-1");
  if (dq < 1) return fail(FPE_EINVAL, "deg q must be >= 1");
  if (product < FPE_PRODUCT_AUTO || product > FPE_PRODUCT_MFMA) return fail(FPE_EINVAL, "unknown product method");
  return launch_compose_ex(t, q, dq, out, workspace, workspace_bytes, product, stream);
}

fpe_status fpe_compose(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (!t || !q || !out) return fail(FPE_EINVAL, "NULL argument");
  if (!t->dev) return fail(FPE_EINVAL, "tree is not uploaded");
  if (t->domain != FPE_MODP || t->modulus != kP31 || t->nvars != 1)
    return fail(FPE_EINVAL, "composition needs a univariate tree compiled mod 2^31-1");
  if (dq < 1) return fail(FPE_EINVAL, "deg q must be >= 1");
  return launch_compose(t, q, dq, out, workspace, workspace_bytes, stream);
}

}  // extern "C"
