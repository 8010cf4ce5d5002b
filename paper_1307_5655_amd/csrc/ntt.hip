// Long convolutions by number-theoretic transforms, and the composition walk
// that uses them for its large polynomial products (subquadratic
// multiplication: Section 1.2 notes that the divide-and-conquer schemes suit
// elements whose size grows linearly with each multiplication, such as
// polynomials; with fast products their top levels dominate the cost).
//
// A product of two rows of residues (< 2^31, lengths up to kNttMax / 2) is
// computed exactly over the integers as three cyclic convolutions modulo the
// NTT primes below (each 2^25 | p - 1 at least; their product exceeds
// 2^92, while a product coefficient is below 2^14 * 2^62 = 2^76), then
// recombined by Garner's method and reduced modulo 2^31 - 1.  Each
// transform of one row modulo one prime runs in one workgroup, with the row
// held in LDS (kNttMax = 2^14 words = 64 KB): a radix-2 decimation-in-frequency
// forward transform (natural order in, bit-reversed order out), the
// pointwise product in that order, and a decimation-in-time inverse
// (bit-reversed in, natural out), so no bit reversal pass is needed.
// Residue arithmetic is Montgomery's (R = 2^32), with the twiddle factors
// kept in Montgomery form so the data stays in ordinary form.
//
// The composition walk here is the stack program of the tree (as in
// compose.hip) executed op by op from the host, each op one batched launch
// over all instances: scalings for leaves, and for inner nodes products
// that go to the transforms when both operands have at least `ntt_min`
// coefficients, otherwise to a batched schoolbook kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fpe_internal.h"
#include "ntt_core.h"

namespace fpe {

namespace {

// Forward transform of row blockIdx.x (src + row * src_stride, `len`
// residues < 2^31, zero-padded to n) modulo prime blockIdx.y, into
// dst + (prime * rows + row) * n.
__global__ __launch_bounds__(kNttThreads) void k_ntt_fwd(const uint32_t* __restrict__ src, int64_t src_stride, int len,
                                                         int n, int logn, const uint32_t* __restrict__ tw_all,
                                                         uint32_t* __restrict__ dst, int rows) {
  extern __shared__ uint32_t x[];
  const int prime = blockIdx.y;
  const NttPrime P = kPrimes[prime];
  const uint32_t* tw = tw_all + (size_t)prime * kNttMax;
  const uint32_t* s = src + (int64_t)blockIdx.x * src_stride;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint32_t v = i < len ? s[i] : 0u;
    while (v >= P.p) v -= P.p;   // residues < 2^31 < 2p
    x[i] = v;
  }
  __syncthreads();
  for (int lh = logn - 1; lh >= 0; --lh) {
    const int h = 1 << lh;
    const int tstep = kNttLogMax - 1 - lh;   // twiddle index j * kNttMax / (2h)
    for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
      const int j = b & (h - 1);
      const int i0 = ((b >> lh) << (lh + 1)) + j, i1 = i0 + h;
      const uint32_t u = x[i0], v = x[i1];
      x[i0] = madd(u, v, P.p);
      x[i1] = mmul(msub(u, v, P.p), tw[j << tstep], P.p, P.pinv);
    }
    __syncthreads();
  }
  uint32_t* d = dst + ((size_t)prime * rows + blockIdx.x) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = x[i];
}

// Pointwise product of the transforms a (row blockIdx.x) and b (row
// blockIdx.x, or row 0 when b_rows == 1), then the inverse transform, scaled
// so that the result is the cyclic convolution itself; into c.
__global__ __launch_bounds__(kNttThreads) void k_ntt_mul_inv(const uint32_t* __restrict__ a,
                                                             const uint32_t* __restrict__ b, int b_rows, int n,
                                                             int logn, Scales sc, const uint32_t* __restrict__ tw_all,
                                                             uint32_t* __restrict__ c, int rows) {
  extern __shared__ uint32_t x[];
  const int prime = blockIdx.y;
  const NttPrime P = kPrimes[prime];
  const uint32_t scale = sc.s[prime];
  const uint32_t* twi = tw_all + (size_t)prime * kNttMax + kNttMax / 2;
  const uint32_t* ar = a + ((size_t)prime * rows + blockIdx.x) * n;
  const uint32_t* br = b + ((size_t)prime * b_rows + (b_rows == 1 ? 0 : blockIdx.x)) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = mmul(ar[i], br[i], P.p, P.pinv);
  __syncthreads();
  for (int lh = 0; lh < logn; ++lh) {
    const int h = 1 << lh;
    const int tstep = kNttLogMax - 1 - lh;
    for (int bb = threadIdx.x; bb < n / 2; bb += blockDim.x) {
      const int j = bb & (h - 1);
      const int i0 = ((bb >> lh) << (lh + 1)) + j, i1 = i0 + h;
      const uint32_t u = x[i0], v = mmul(x[i1], twi[j << tstep], P.p, P.pinv);
      x[i0] = madd(u, v, P.p);
      x[i1] = msub(u, v, P.p);
    }
    __syncthreads();
  }
  // scale = n^-1 R^2 mod p: the pointwise products carried a factor R^-1
  uint32_t* d = c + ((size_t)prime * rows + blockIdx.x) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = mmul(x[i], scale, P.p, P.pinv);
}

// Garner's recombination of the three residues of each coefficient into the
// exact integer x = a1 + p1 t1 + p1 p2 t2 (< p1 p2 p3), reduced modulo
// 2^31 - 1; dst[k] = (accumulate ? dst[k] : 0) + x_k (+ c0 at k = 0) for
// k < len, and, when accumulating into a shorter row, the row is extended:
// positions in [old_len, len) start from 0.
struct CrtConst {
  uint32_t inv12, inv13, inv23;   // p1^-1 mod p2, p1^-1 mod p3, p2^-1 mod p3 (Montgomery form)
  uint64_t p1p2_m31;              // p1 p2 mod 2^31 - 1
};

__device__ __forceinline__ uint32_t m31_fold(uint64_t v) {
  v = (v & kP31) + (v >> 31);
  v = (v & kP31) + (v >> 31);
  return (uint32_t)(v >= kP31 ? v - kP31 : v);
}

__global__ void k_crt_m31(const uint32_t* __restrict__ res, int n, int rows, int len, uint32_t* __restrict__ dst,
                          int64_t dst_stride, int old_len, const uint32_t* __restrict__ c0_rows, int64_t c0_stride,
                          int c0_index, CrtConst K) {
  const int row = blockIdx.y;
  const NttPrime P1 = kPrimes[0], P2 = kPrimes[1], P3 = kPrimes[2];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < len; k += gridDim.x * blockDim.x) {
    const uint32_t a1 = res[((size_t)0 * rows + row) * n + k];
    const uint32_t a2 = res[((size_t)1 * rows + row) * n + k];
    const uint32_t a3 = res[((size_t)2 * rows + row) * n + k];
    // t1 = (a2 - a1) / p1 mod p2; t2 = ((a3 - a1) / p1 - t1) / p2 mod p3
    // (a1 < p1 may exceed p2 or p3: reduce first)
    const uint32_t a1m2 = a1 >= P2.p ? a1 - P2.p : a1;
    const uint32_t a1m3 = a1 >= P3.p ? a1 - P3.p : a1;
    const uint32_t t1 = mmul(msub(a2, a1m2, P2.p), K.inv12, P2.p, P2.pinv);
    const uint32_t u = mmul(msub(a3, a1m3, P3.p), K.inv13, P3.p, P3.pinv);
    const uint32_t t1m3 = t1 >= P3.p ? t1 - P3.p : t1;
    const uint32_t t2 = mmul(msub(u, t1m3, P3.p), K.inv23, P3.p, P3.pinv);
    uint64_t v = (uint64_t)a1 + (uint64_t)P1.p * t1;
    v = (uint64_t)m31_fold(v) + K.p1p2_m31 * t2;
    uint32_t* d = dst + (int64_t)row * dst_stride;
    if (k < old_len) v += d[k];
    if (k == 0 && c0_index >= 0) v += c0_rows[(int64_t)row * c0_stride + c0_index];
    d[k] = m31_fold(v);
  }
}

// dst[row][k] = (k < old_len ? dst : 0) + c * X[row][k] (+ c0 at k = 0), k < lx,
// with c = coef[row][ci] (or 1 when ci < 0), c0 = coef[row][c0i] if c0i >= 0;
// positions [lx, new_len) of a row that was longer keep their values.
__global__ void k_scale_rows(const uint32_t* __restrict__ X, int64_t x_stride, int lx, uint32_t* __restrict__ dst,
                             int64_t dst_stride, int old_len, const uint32_t* __restrict__ coef, int64_t coef_stride,
                             int ci, int c0i) {
  const int row = blockIdx.y;
  const uint32_t c = ci >= 0 ? coef[(int64_t)row * coef_stride + ci] : 1u;
  const uint32_t* xr = X + (int64_t)row * x_stride;
  uint32_t* d = dst + (int64_t)row * dst_stride;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < lx; k += gridDim.x * blockDim.x) {
    uint64_t v = (uint64_t)c * xr[k];
    if (k < old_len) v += d[k];
    if (k == 0 && c0i >= 0) v += coef[(int64_t)row * coef_stride + c0i];
    d[k] = m31_fold(v);
  }
}

// Batched schoolbook product: dst[row][k] = (k < old_len ? dst : 0) +
// sum_i a[i] b[k - i] (+ c0 at k = 0), one workgroup per row, each thread a
// set of output coefficients; 64-bit sums folded every third product.
__global__ __launch_bounds__(256) void k_mul_rows(const uint32_t* __restrict__ a, int64_t a_stride, int la,
                                                  const uint32_t* __restrict__ b, int64_t b_stride, int lb,
                                                  uint32_t* __restrict__ dst, int64_t dst_stride, int old_len,
                                                  const uint32_t* __restrict__ coef, int64_t coef_stride, int c0i) {
  const int row = blockIdx.y;
  const uint32_t* ar = a + (int64_t)row * a_stride;
  const uint32_t* br = b + (int64_t)row * b_stride;
  uint32_t* d = dst + (int64_t)row * dst_stride;
  const int lp = la + lb - 1;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < lp; k += gridDim.x * blockDim.x) {
    const int i0 = k - (lb - 1) > 0 ? k - (lb - 1) : 0, i1 = k < la - 1 ? k : la - 1;
    uint64_t acc = 0;
    int cnt = 0;
    for (int i = i0; i <= i1; ++i) {
      acc += (uint64_t)ar[i] * br[k - i];
      if (++cnt == 3) {
        acc = (acc & kP31) + (acc >> 31);
        cnt = 0;
      }
    }
    uint64_t v = (uint64_t)m31_fold(acc);
    if (k < old_len) v += d[k];
    if (k == 0 && c0i >= 0) v += coef[(int64_t)row * coef_stride + c0i];
    d[k] = m31_fold(v);
  }
}

// dst[row][0] = coef[row][ci] (the value of a root that is a leaf).
__global__ void k_set_const(uint32_t* __restrict__ dst, int64_t dst_stride, const uint32_t* __restrict__ coef,
                            int64_t coef_stride, int ci, int rows) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row < rows) dst[(int64_t)row * dst_stride] = coef[(int64_t)row * coef_stride + ci];
}

// dst[row][k] = src[row][k] for k < len, 0 for len <= k < total.
__global__ void k_copy_rows(const uint32_t* __restrict__ src, int64_t src_stride, int len, uint32_t* __restrict__ dst,
                            int64_t dst_stride, int total) {
  const int row = blockIdx.y;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x)
    dst[(int64_t)row * dst_stride + k] = k < len ? src[(int64_t)row * src_stride + k] : 0u;
}

struct Plan {
  int64_t batch = 0, lmax = 0, nmax = 0;   // nmax: the largest transform length used (0: none)
  size_t off_stack = 0, off_table = 0, off_a = 0, off_b = 0, off_c = 0, off_tw = 0, bytes = 0;
};

inline size_t al256(size_t v) { return (v + 255) & ~size_t(255); }
inline int ceil_log2(int64_t v) {
  int l = 0;
  while (((int64_t)1 << l) < v) ++l;
  return l;
}

int32_t deg_p(const fpe_tree* t) {
  int32_t dp = 0;
  for (size_t i = 0; i < t->nodes.size(); ++i) dp = std::max(dp, t->exps[i * t->nvars]);
  return dp;
}

// The lengths of every product of the walk, to size the transforms: the
// walk is simulated on lengths only (the same stack program).
struct LenSim {
  std::vector<int> tab_len;
  int64_t max_n = 0;
  void product(int la, int lb, int ntt_min) {
    if (std::min(la, lb) >= ntt_min) max_n = std::max<int64_t>(max_n, (int64_t)1 << ceil_log2(la + lb - 1));
  }
};

Plan make_plan(const fpe_tree* t, int32_t dq, int ntt_min) {
  Plan P;
  P.batch = t->batch;
  P.lmax = (int64_t)deg_p(t) * dq + 1;
  LenSim S;
  S.tab_len.assign(t->n_table, 0);
  for (const auto& st : t->chain) {
    if (st.kind == kChainLoad) {
      S.tab_len[st.dst] = dq + 1;
    } else {
      S.product(S.tab_len[st.s1], S.tab_len[st.s2], ntt_min);
      S.tab_len[st.dst] = S.tab_len[st.s1] + S.tab_len[st.s2] - 1;
    }
  }
  std::vector<int> len(kMaxDepth + 2, 0);
  int top = 0;
  for (const auto& o : t->ops64) {
    const uint32_t kind = op_kind(o.info), p = op_pidx(o.info);
    const int lx = p != kOffTable ? S.tab_len[p] : 1;
    if (kind == kLeafAdd) len[top - 1] = std::max(len[top - 1], lx);
    else if (kind == kNodeOpen) {
      S.product(len[top - 1], lx, ntt_min);
      len[top - 1] = len[top - 1] + lx - 1;
    } else if (kind == kLeafOpen) len[top++] = lx;
    else if (kind == kNodeAdd) {
      S.product(len[top - 1], lx, ntt_min);
      len[top - 2] = std::max(len[top - 2], len[top - 1] + lx - 1);
      --top;
    } else if ((o.info & kEndHasPow) && !(o.info & kEndLeafRoot)) {
      S.product(len[top - 1], lx, ntt_min);
    }
  }
  P.nmax = S.max_n;
  size_t off = 0;
  const size_t row = (size_t)P.batch * P.lmax * sizeof(uint32_t);
  P.off_stack = off;
  off = al256(off + (size_t)(t->depth + 2) * row);
  P.off_table = off;
  off = al256(off + (size_t)std::max(t->n_table, 1) * row);
  const size_t ntt_bytes = (size_t)3 * P.batch * P.nmax * sizeof(uint32_t);
  P.off_a = off;
  off = al256(off + ntt_bytes);
  P.off_b = off;
  off = al256(off + ntt_bytes);
  P.off_c = off;
  off = al256(off + ntt_bytes);
  P.off_tw = off;
  off = al256(off + (P.nmax ? (size_t)3 * kNttMax * sizeof(uint32_t) : 0));
  P.bytes = std::max<size_t>(off, 256);
  return P;
}

CrtConst crt_consts() {
  const uint64_t p1 = kPrimes[0].p, p2 = kPrimes[1].p, p3 = kPrimes[2].p;
  auto mont = [](uint64_t v, const NttPrime& P) {   // v R mod p
    return (uint32_t)(((unsigned __int128)v << 32) % P.p);
  };
  CrtConst K;
  K.inv12 = mont(host_pow(p1 % p2, p2 - 2, p2), kPrimes[1]);
  K.inv13 = mont(host_pow(p1 % p3, p3 - 2, p3), kPrimes[2]);
  K.inv23 = mont(host_pow(p2 % p3, p3 - 2, p3), kPrimes[2]);
  K.p1p2_m31 = (uint64_t)((unsigned __int128)p1 * p2 % kP31);
  return K;
}

// Executes the composition walk op by op, each op one batched launch.
struct Runner {
  const fpe_tree* t;
  hipStream_t st;
  int ntt_min;
  Plan P;
  char* ws;
  const uint32_t* coef;   // device: batch x n_nodes
  int64_t nn;             // coefficients per row (n_nodes)
  CrtConst K{};

  uint32_t* stack(int b) const { return (uint32_t*)(ws + P.off_stack) + (size_t)b * P.batch * P.lmax; }
  uint32_t* table(int i) const { return (uint32_t*)(ws + P.off_table) + (size_t)i * P.batch * P.lmax; }
  dim3 grid_rows(int64_t len) const {
    const int64_t g = std::min<int64_t>((len + 255) / 256, 64);
    return dim3((unsigned)std::max<int64_t>(g, 1), (unsigned)P.batch);
  }

  // dst = (dst of length old_len, extended with zeros) + a * b (+ c0),
  // for every row of the batch; the product has la + lb - 1 coefficients
  void product(const uint32_t* a, int la, const uint32_t* b, int lb, uint32_t* dst, int old_len, int c0i) {
    const int lp = la + lb - 1;
    if (std::min(la, lb) >= ntt_min) {
      const int logn = ceil_log2(lp);
      const int n = 1 << logn;
      uint32_t* A = (uint32_t*)(ws + P.off_a);
      uint32_t* B = (uint32_t*)(ws + P.off_b);
      uint32_t* C = (uint32_t*)(ws + P.off_c);
      const uint32_t* tw = (const uint32_t*)(ws + P.off_tw);
      const int thr = std::min(kNttThreads, std::max(64, n / 2));
      const size_t lds = (size_t)n * sizeof(uint32_t);
      const dim3 g((unsigned)P.batch, 3);
      hipLaunchKernelGGL(k_ntt_fwd, g, dim3(thr), lds, st, a, (int64_t)P.lmax, la, n, logn, tw, A, (int)P.batch);
      hipLaunchKernelGGL(k_ntt_fwd, g, dim3(thr), lds, st, b, (int64_t)P.lmax, lb, n, logn, tw, B, (int)P.batch);
      hipLaunchKernelGGL(k_ntt_mul_inv, g, dim3(thr), lds, st, A, B, (int)P.batch, n, logn, scales_for(n), tw, C,
                         (int)P.batch);
      hipLaunchKernelGGL(k_crt_m31, grid_rows(lp), dim3(256), 0, st, C, n, (int)P.batch, lp, dst, (int64_t)P.lmax,
                         old_len, coef, nn, c0i, K);
    } else {
      hipLaunchKernelGGL(k_mul_rows, grid_rows(lp), dim3(256), 0, st, a, (int64_t)P.lmax, la, b, (int64_t)P.lmax,
                         lb, dst, (int64_t)P.lmax, old_len, coef, nn, c0i);
    }
  }
  // dst = (dst, old_len) + c X (+ c0)
  void scale(const uint32_t* X, int lx, uint32_t* dst, int old_len, int ci, int c0i) {
    hipLaunchKernelGGL(k_scale_rows, grid_rows(lx), dim3(256), 0, st, X, (int64_t)P.lmax, lx, dst, (int64_t)P.lmax,
                       old_len, coef, nn, ci, c0i);
  }

  void run(const uint32_t* q, int32_t dq, uint32_t* out) {
    K = crt_consts();
    if (P.nmax) launch_twiddles((uint32_t*)(ws + P.off_tw), 3, st);
    // powers q^d by the chain
    std::vector<int> tab_len(t->n_table, 0);
    for (const auto& c : t->chain) {
      if (c.kind == kChainLoad) {
        hipLaunchKernelGGL(k_copy_rows, grid_rows(P.lmax), dim3(256), 0, st, q, (int64_t)(dq + 1), dq + 1,
                           table(c.dst), (int64_t)P.lmax, dq + 1);
        tab_len[c.dst] = dq + 1;
      } else {
        product(table(c.s1), tab_len[c.s1], table(c.s2), tab_len[c.s2], table(c.dst), 0, -1);
        tab_len[c.dst] = tab_len[c.s1] + tab_len[c.s2] - 1;
      }
    }
    // the walk: stack levels map to buffers (a NODE_OPEN writes into the free
    // buffer above the top and swaps)
    int buf[kMaxDepth + 2], len[kMaxDepth + 2];
    for (int k = 0; k < kMaxDepth + 2; ++k) {
      buf[k] = k;
      len[k] = 0;
    }
    int top = 0;
    for (const auto& o : t->ops64) {
      const uint32_t kind = op_kind(o.info), p = op_pidx(o.info);
      const uint32_t* X = p != kOffTable ? table(p) : nullptr;
      const int lx = p != kOffTable ? tab_len[p] : 1;
      const int cN = (int)o.a, cP = (int)o.b;   // node indices into the coefficient rows
      if (kind == kLeafAdd) {
        scale(X, lx, stack(buf[top - 1]), len[top - 1], cN, -1);
        len[top - 1] = std::max(len[top - 1], lx);
      } else if (kind == kNodeOpen) {
        product(stack(buf[top - 1]), len[top - 1], X, lx, stack(buf[top]), 0, cP);
        std::swap(buf[top - 1], buf[top]);
        len[top - 1] = len[top - 1] + lx - 1;
      } else if (kind == kLeafOpen) {
        scale(X, lx, stack(buf[top]), 0, cN, cP);
        len[top++] = lx;
      } else if (kind == kNodeAdd) {
        product(stack(buf[top - 1]), len[top - 1], X, lx, stack(buf[top - 2]), len[top - 2], -1);
        len[top - 2] = std::max(len[top - 2], len[top - 1] + lx - 1);
        --top;
      } else {   // END: the root's value times its own power, zero-padded
        const bool leaf = (o.info & kEndLeafRoot) != 0, pw = (o.info & kEndHasPow) != 0;
        if (leaf && pw) {
          scale(X, lx, out, 0, cN, -1);
          hipLaunchKernelGGL(k_copy_rows, grid_rows(P.lmax), dim3(256), 0, st, out, (int64_t)P.lmax, lx, out,
                             (int64_t)P.lmax, (int)P.lmax);
        } else if (leaf) {
          hipLaunchKernelGGL(k_copy_rows, grid_rows(P.lmax), dim3(256), 0, st, (const uint32_t*)nullptr, 0, 0, out,
                             (int64_t)P.lmax, (int)P.lmax);
          hipLaunchKernelGGL(k_set_const, dim3((unsigned)((P.batch + 255) / 256)), dim3(256), 0, st, out,
                             (int64_t)P.lmax, coef, nn, cN, (int)P.batch);
        } else if (pw) {
          product(stack(buf[top - 1]), len[top - 1], X, lx, out, 0, -1);
          const int lr = len[top - 1] + lx - 1;
          hipLaunchKernelGGL(k_copy_rows, grid_rows(P.lmax), dim3(256), 0, st, out, (int64_t)P.lmax, lr, out,
                             (int64_t)P.lmax, (int)P.lmax);
        } else {
          hipLaunchKernelGGL(k_copy_rows, grid_rows(P.lmax), dim3(256), 0, st, stack(buf[top - 1]),
                             (int64_t)P.lmax, len[top - 1], out, (int64_t)P.lmax, (int)P.lmax);
        }
        break;
      }
    }
  }
};

}  // namespace

size_t compose_ops_workspace_bytes(const fpe_tree* t, int32_t dq, int32_t ntt_min) {
  if (!t || t->nodes.empty() || dq < 1) return 0;
  return make_plan(t, dq, ntt_min).bytes;
}

fpe_status launch_compose_ops(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                              size_t ws_bytes, int32_t ntt_min, void* stream) {
  if (t->n_offtable > 0) return fail(FPE_EUNSUPPORTED, "composition needs every power in the table");
  if (t->batch > 65535) return fail(FPE_EUNSUPPORTED, "the transform path takes at most 65535 instances");
  const Plan P = make_plan(t, dq, ntt_min);
  if (P.nmax > kNttMax) return fail(FPE_EUNSUPPORTED, "a product is longer than the largest transform (2^14)");
  if (!ws || ws_bytes < P.bytes) return fail(FPE_ENOMEM, "workspace smaller than the composition needs");
  if (((uintptr_t)ws) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
  Runner R{t, (hipStream_t)stream, ntt_min, P, (char*)ws, dev_view(t).coef_rows, (int64_t)t->nodes.size()};
  R.run(q, dq, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition launch: ") + hipGetErrorString(e));
  return FPE_OK;
}

}  // namespace fpe
