// Composition p(q(x)) over Z/(2^31 - 1) through the evaluation tree of p
// (evaluation at a polynomial: the title problem of the paper; Section 1.2
// notes that divide-and-conquer schemes suit elements, such as polynomials,
// whose size grows linearly with each multiplication).
//
// The walk is the same stack program as the pointwise kernels, with
// polynomial-valued accumulators: a step a * X + b becomes a polynomial
// product with a power q^d of q plus a constant.  One wavefront walks one
// instance, so all instances of a batch are resident at once and the latency
// of one instance's chain of dependent steps is hidden by the others; the
// polynomials live in a per-instance workspace in HBM (L2-resident while the
// instance runs) and every product is a register-blocked convolution over the
// wavefront.  The powers q^d are computed by the tree's power chain
// (q^{d1 + d2} = q^{d1} q^{d2}).
#include <hip/hip_runtime.h>

#include "fpe_internal.h"

namespace fpe {

namespace {

constexpr int kCB = 64;   // threads per instance: one wavefront

__device__ __forceinline__ uint32_t m31_fold(uint64_t v) {
  v = (v & kP31) + (v >> 31);
  v = (v & kP31) + (v >> 31);
  return (uint32_t)(v >= kP31 ? v - kP31 : v);
}

struct ComposeArgs {
  DevTree tr;
  const uint32_t* q;      // batch x (dq + 1)
  uint32_t* out;          // batch x (dp * dq + 1)
  uint32_t* ws;           // batch x per_instance words
  int32_t dq;
  int32_t dp;
  int64_t lmax;           // dp * dq + 1
  int64_t per_instance;   // words of workspace per instance
  int32_t nbuf;           // stack buffers per instance (depth + 2)
};

// out[0 .. la + lb - 1) (+)= a * b, plus c0 at degree 0.  When accumulate is
// set, out holds a polynomial of length lout that is extended with zeros.
//
// Register-blocked convolution by one wavefront: lane l owns kR consecutive
// output coefficients of a tile of 64 kR, and the loop runs over the shorter
// operand a in chunks of kChunk coefficients.  For each chunk the slice of the
// longer operand b that the tile needs (64 kR + kChunk - 1 words) and the
// chunk of a are staged in LDS with coalesced loads; then, block by block of
// kR coefficients of a, each lane reads a window of 2 kR - 1 words of b
// (stride kR across lanes) and does kR * kR multiply-adds.  Products of
// 31-bit residues are < 2^62, so a 64-bit accumulator takes three of them
// between folds (2^31 = 1 mod p).
constexpr int kR = 6;
constexpr int kChunk = 11 * kR;   // a multiple of kR: windows stay inside the staged slice
constexpr int kSpan = 64 * kR + kChunk;   // staged words of b per chunk

__device__ __forceinline__ uint64_t m31_fold64(uint64_t v) { return (v & kP31) + (v >> 31); }

__device__ void poly_mac(const uint32_t* a, int la, const uint32_t* b, int lb, uint32_t* out, int lout,
                         bool accumulate, uint32_t c0, uint32_t* sb, uint32_t* sa) {
  if (la > lb) {   // loop over the shorter operand
    const uint32_t* t = a;
    a = b;
    b = t;
    const int tl = la;
    la = lb;
    lb = tl;
  }
  const int lp = la + lb - 1;
  const int lane = threadIdx.x & 63;
  for (int tile = 0; tile < lp; tile += 64 * kR) {
    const int k0 = tile + lane * kR;
    int i_lo = tile - (lb - 1);   // a's coefficients that reach this tile
    if (i_lo < 0) i_lo = 0;
    int i_hi = tile + 64 * kR - 1;
    if (i_hi > la - 1) i_hi = la - 1;
    uint64_t acc[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) acc[r] = 0;
    for (int ic = i_lo; ic <= i_hi; ic += kChunk) {
      // stage b[j0 .. j0 + kSpan) with j0 = tile - ic - (kChunk - 1), and
      // a[ic .. ic + kChunk) (zero outside the operands)
      const int j0 = tile - ic - (kChunk - 1);
      __syncthreads();
      for (int u = lane; u < kSpan; u += 64) {
        const int j = j0 + u;
        sb[u] = (j >= 0 && j < lb) ? b[j] : 0u;
      }
      for (int u = lane; u < kChunk; u += 64) {
        const int i = ic + u;
        sa[u] = (i <= i_hi) ? a[i] : 0u;
      }
      __syncthreads();
      // window indices: base + m in [0, kSpan) because ib <= kChunk - kR
      for (int ib = 0; ib < kChunk && ic + ib <= i_hi; ib += kR) {
        // window bw[m] = b[k0 - (ic + ib) - (kR - 1) + m] = sb[base + m]
        const int base = lane * kR + (kChunk - 1) - ib - (kR - 1);
        uint32_t bw[2 * kR - 1];
#pragma unroll
        for (int m = 0; m < 2 * kR - 1; ++m) bw[m] = sb[base + m];
#pragma unroll
        for (int s2 = 0; s2 < kR; ++s2) {
          const uint32_t av = sa[ib + s2];
#pragma unroll
          for (int r = 0; r < kR; ++r) acc[r] += (uint64_t)av * bw[r - s2 + kR - 1];
          if (s2 % 3 == 2) {
#pragma unroll
            for (int r = 0; r < kR; ++r) acc[r] = m31_fold64(acc[r]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int k = k0 + r;
      if (k < lp) {
        uint64_t v = m31_fold64(acc[r]);
        if (accumulate && k < lout) v += out[k];
        if (k == 0) v += c0;
        out[k] = m31_fold(v);
      }
    }
  }
}

__device__ void poly_scale(uint32_t c, const uint32_t* b, int lb, uint32_t* out, int lout,
                           bool accumulate, uint32_t c0) {
  for (int k = threadIdx.x; k < lb; k += kCB) {
    uint64_t acc = (uint64_t)c * b[k];
    if (accumulate && k < lout) acc += out[k];
    if (k == 0) acc += c0;
    out[k] = m31_fold(acc);
  }
}

__global__ __launch_bounds__(kCB) void k_compose_walk(ComposeArgs A) {
  const int64_t inst = blockIdx.x;
  const DevTree& tr = A.tr;
  uint32_t* W = A.ws + inst * A.per_instance;
  uint32_t* table = W + (int64_t)A.nbuf * A.lmax;          // n_table polynomials
  const uint32_t* coef = tr.coef_rows + inst * (int64_t)tr.n_nodes;
  const uint32_t* qi = A.q + inst * (int64_t)(A.dq + 1);
  __shared__ uint32_t sb[kSpan], sa[kChunk];   // product staging (see poly_mac)
  __shared__ int32_t tab_len[kMaxTable];
  __shared__ int32_t buf[kMaxDepth + 2];   // stack level -> buffer
  __shared__ int32_t len[kMaxDepth + 2];   // length of the polynomial at each level

  // powers q^d by the chain
  for (int c = 0; c < tr.n_chain; ++c) {
    const ChainStep st = tr.chain[c];
    uint32_t* dst = table + (int64_t)st.dst * A.lmax;
    if (st.kind == kChainLoad) {
      for (int k = threadIdx.x; k <= A.dq; k += kCB) dst[k] = qi[k];
      if (threadIdx.x == 0) tab_len[st.dst] = A.dq + 1;
    } else {
      const int la = tab_len[st.s1], lb = tab_len[st.s2];
      poly_mac(table + (int64_t)st.s1 * A.lmax, la, table + (int64_t)st.s2 * A.lmax, lb, dst, 0, false, 0, sb, sa);
      if (threadIdx.x == 0) tab_len[st.dst] = la + lb - 1;
    }
    __syncthreads();
  }
  if (threadIdx.x < kMaxDepth + 2) {
    buf[threadIdx.x] = threadIdx.x;
    len[threadIdx.x] = 0;
  }
  __syncthreads();

  int top = 0;   // number of open accumulators (uniform)
  for (int pc = 0; pc < tr.n_ops; ++pc) {
    const OpF64 o = tr.ops64[pc];
    const uint32_t kind = op_kind(o.info);
    const uint32_t pidx = op_pidx(o.info);
    const bool haspow = pidx != kOffTable;
    const uint32_t* X = haspow ? table + (int64_t)pidx * A.lmax : nullptr;
    const int lx = haspow ? tab_len[pidx] : 1;
    const uint32_t cN = coef[o.a];
    const uint32_t cP = coef[o.b];
    if (kind == kLeafAdd) {
      uint32_t* d = W + (int64_t)buf[top - 1] * A.lmax;
      poly_scale(cN, X, lx, d, len[top - 1], true, 0);
      __syncthreads();
      if (threadIdx.x == 0) len[top - 1] = max(len[top - 1], lx);
    } else if (kind == kNodeOpen) {
      uint32_t* s = W + (int64_t)buf[top - 1] * A.lmax;
      uint32_t* d = W + (int64_t)buf[top] * A.lmax;   // free buffer above the top
      poly_mac(s, len[top - 1], X, lx, d, 0, false, cP, sb, sa);
      __syncthreads();
      if (threadIdx.x == 0) {
        const int b = buf[top - 1];
        buf[top - 1] = buf[top];
        buf[top] = b;
        len[top - 1] = len[top - 1] + lx - 1;
      }
    } else if (kind == kLeafOpen) {
      uint32_t* d = W + (int64_t)buf[top] * A.lmax;
      poly_scale(cN, X, lx, d, 0, false, cP);
      __syncthreads();
      if (threadIdx.x == 0) len[top] = lx;
      ++top;
    } else if (kind == kNodeAdd) {
      uint32_t* s = W + (int64_t)buf[top - 1] * A.lmax;
      uint32_t* d = W + (int64_t)buf[top - 2] * A.lmax;
      poly_mac(s, len[top - 1], X, lx, d, len[top - 2], true, 0, sb, sa);
      __syncthreads();
      if (threadIdx.x == 0) len[top - 2] = max(len[top - 2], len[top - 1] + lx - 1);
      --top;
    } else {   // END
      uint32_t* res = A.out + inst * A.lmax;
      const bool leaf_root = (o.info & kEndLeafRoot) != 0;
      const bool pw = (o.info & kEndHasPow) != 0;
      int lr;
      if (leaf_root) {
        if (pw) poly_scale(cN, X, lx, res, 0, false, 0);
        else if (threadIdx.x == 0) res[0] = cN;
        lr = pw ? lx : 1;
      } else {
        const uint32_t* s = W + (int64_t)buf[top - 1] * A.lmax;
        if (pw) {
          poly_mac(s, len[top - 1], X, lx, res, 0, false, 0, sb, sa);
          lr = len[top - 1] + lx - 1;
        } else {
          for (int k = threadIdx.x; k < len[top - 1]; k += kCB) res[k] = s[k];
          lr = len[top - 1];
        }
      }
      for (int64_t k = lr + threadIdx.x; k < A.lmax; k += kCB) res[k] = 0;
      break;
    }
    __syncthreads();
  }
}

}  // namespace

size_t compose_fused_workspace_bytes(const fpe_tree* t, int32_t dq) {
  if (!t || t->nodes.empty() || dq < 1) return 0;
  int32_t dp = 0;
  for (size_t i = 0; i < t->nodes.size(); ++i) dp = std::max(dp, t->exps[i * t->nvars]);
  const int64_t lmax = (int64_t)dp * dq + 1;
  const int64_t per = (int64_t)(t->depth + 2 + t->n_table) * lmax;
  return (size_t)(per * t->batch) * sizeof(uint32_t);
}

fpe_status launch_compose_fused(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                                size_t ws_bytes, void* stream) {
  if (t->n_offtable > 0) return fail(FPE_EUNSUPPORTED, "composition needs every power in the table");
  if (t->depth + 2 > kMaxDepth + 2) return fail(FPE_EUNSUPPORTED, "walk deeper than the kernels hold");
  const size_t need = compose_fused_workspace_bytes(t, dq);
  if (!ws || ws_bytes < need) return fail(FPE_ENOMEM, "workspace smaller than fpe_compose_workspace_bytes()");
  if (t->batch > 0x7fffffff) return fail(FPE_EINVAL, "batch too large");
  ComposeArgs A{};
  A.tr = dev_view(t);
  A.q = q;
  A.out = out;
  A.ws = (uint32_t*)ws;
  A.dq = dq;
  int32_t dp = 0;
  for (size_t i = 0; i < t->nodes.size(); ++i) dp = std::max(dp, t->exps[i * t->nvars]);
  A.dp = dp;
  A.lmax = (int64_t)dp * dq + 1;
  A.nbuf = t->depth + 2;
  A.per_instance = (int64_t)(t->depth + 2 + t->n_table) * A.lmax;
  hipLaunchKernelGGL(k_compose_walk, dim3((unsigned)t->batch), dim3(kCB), 0, (hipStream_t)stream, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("compose launch: ") + hipGetErrorString(e));
  return FPE_OK;
}

// The product method of a composition: for outputs that fit one node's four
// matrix tiles, the level walk with matrix-core products when the tree has
// few levels (divide-and-conquer schemes), else the fused walk (one
// wavefront per instance, all products schoolbook); beyond, the op-by-op
// walk with transform products.
constexpr int64_t kFusedMaxOut = 4096;
constexpr int32_t kNttMinOperand = 64;
constexpr int64_t kLevelsMaxLaunches = 64;
int32_t compose_method(const fpe_tree* t, int32_t dq, int32_t product) {
  if (product != FPE_PRODUCT_AUTO) return product;
  int32_t dp = 0;
  for (size_t i = 0; i < t->nodes.size(); ++i) dp = std::max(dp, t->exps[i * t->nvars]);
  if ((int64_t)dp * dq + 1 > kFusedMaxOut) return FPE_PRODUCT_NTT;
  int64_t launches = 0;
  if (t->n_offtable == 0 && compose_levels_ok(t, dq, &launches) && launches <= kLevelsMaxLaunches)
    return FPE_PRODUCT_MFMA;
  return FPE_PRODUCT_FUSED;
}

size_t compose_workspace_bytes_ex(const fpe_tree* t, int32_t dq, int32_t product) {
  if (!t || dq < 1) return 0;
  switch (compose_method(t, dq, product)) {
    case FPE_PRODUCT_FUSED: return compose_fused_workspace_bytes(t, dq);
    case FPE_PRODUCT_SCHOOLBOOK: return compose_ops_workspace_bytes(t, dq, 1 << 30);
    case FPE_PRODUCT_NTT: return compose_ops_workspace_bytes(t, dq, kNttMinOperand);
    case FPE_PRODUCT_MFMA: return compose_levels_workspace_bytes(t, dq);
  }
  return 0;
}
size_t compose_workspace_bytes(const fpe_tree* t, int32_t dq) {
  return compose_workspace_bytes_ex(t, dq, FPE_PRODUCT_AUTO);
}

fpe_status launch_compose_ex(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                             size_t ws_bytes, int32_t product, void* stream) {
  switch (compose_method(t, dq, product)) {
    case FPE_PRODUCT_FUSED: return launch_compose_fused(t, q, dq, out, ws, ws_bytes, stream);
    case FPE_PRODUCT_SCHOOLBOOK: return launch_compose_ops(t, q, dq, out, ws, ws_bytes, 1 << 30, stream);
    case FPE_PRODUCT_NTT: return launch_compose_ops(t, q, dq, out, ws, ws_bytes, kNttMinOperand, stream);
    case FPE_PRODUCT_MFMA: return launch_compose_levels(t, q, dq, out, ws, ws_bytes, stream);
  }
  return fail(FPE_EINVAL, "unknown product method");
}
fpe_status launch_compose(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                          size_t ws_bytes, void* stream) {
  return launch_compose_ex(t, q, dq, out, ws, ws_bytes, FPE_PRODUCT_AUTO, stream);
}

}  // namespace fpe
