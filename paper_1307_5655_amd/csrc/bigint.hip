// Exact evaluation over the natural numbers at big-integer points: the
// workload of the paper's Benchmarks section (Figure 1: the balanced scheme
// against Estrin's over multiprecision integers).
//
// The walk is the stack program of the pointwise kernels with big-integer
// accumulators, one workgroup of 8 or 16 wavefronts per point.  A big integer
// is an array of 16-bit limbs (least significant first) held in 32-bit
// words, so a product of two limbs fits in 32 bits and a column of up to
// 2^16 products fits in 64.  A multiply-add out (+)= a b + c0 is a
// convolution over the workgroup (each thread sums blocks of four adjacent
// columns) into 64-bit columns, then a carry-lookahead turns the columns into
// limbs (one wavefront for one chunk of 64 columns, every chunk at once over
// the wavefronts for up to 64 chunks, ranges of chunks beyond).
// Coefficients are uint64 (four limbs); with
// coefficients and points >= 0 every partial value is at most p(x), so every
// value fits the output's limb count.
#include <hip/hip_runtime.h>

#include "fpe_internal.h"

namespace fpe {

namespace {

constexpr int kLanes = 64;     // a wavefront
constexpr int kBigWaves = 8;        // wavefronts per point
constexpr int kBigWavesFew = 16;    // wavefronts per point when the points fit the compute units once

__global__ void k_zero_flag(int32_t* p) { *p = 0; }

inline int64_t align64(int64_t words) { return (words + 63) & ~int64_t(63); }

// Per-point workspace (32-bit words): the stack buffers and the power table
// (lout limbs each), then the 64-bit columns (2 lout words), 256-byte aligned.
inline int64_t col_offset(const fpe_tree* t, int32_t lout) {
  return align64((int64_t)(t->depth + 2 + t->n_table) * lout);
}
inline int64_t per_point_words(const fpe_tree* t, int32_t lout) {
  return align64(col_offset(t, lout) + 2 * (int64_t)lout);
}

struct BigArgs {
  DevTree tr;
  const uint32_t* x;      // batch x lx limbs
  uint32_t* out;          // batch x lout limbs
  uint32_t* ws;           // batch x per_instance words
  int32_t lx;
  int32_t lout;           // limbs of every value (output capacity)
  int64_t per_instance;   // words of workspace per point
  int32_t nbuf;           // stack buffers (depth + 2)
  int64_t col_off;        // words from the point's workspace to its 64-bit columns
  int32_t* overflow;      // set if a value needs more than lout limbs (cannot happen
                          // when lout is at least the host's bound)
};

// Each operand of up to kBigStage limbs is staged in LDS for the product,
// and results of up to kBigCols limbs keep their columns in LDS for the carry
// pass (its reads would otherwise wait on L2).
constexpr int kBigStage = 3072;
constexpr int kBigCols = 4096;

// Carry, 64 columns at a time (lane l: column base + l), as a carry-lookahead
// over the wavefront.  Column k's 64-bit sum is four 16-bit digits, digit i
// weighing 2^16 in column k + i, so the digit sum D of a column (digit i of
// column k - i) is below 2^18; its bits above 16 (at most 3) move up one
// column, leaving E = (D mod 2^16) + (D of column k - 1) / 2^16 < 2^16 + 3,
// whose carry out is at most 1: generated where E > 0xFFFF, propagated where
// E = 0xFFFF.  With G and P those lanes' ballots, (G | P) + G + c_in is a
// binary sum whose carry into bit l is exactly column l's carry in.  Columns
// nhi .. nhi + 2 take the top digits of the last three: anything left there
// is an overflow (the value needs more than lout limbs).  Col reads a column
// from LDS or global memory by its own kind of load (a generic pointer would
// take flat loads, whose aperture is chosen from the base address, which may
// lie below the column array when the compiler folds an offset into the load).
template <class Col>
__device__ __forceinline__ uint32_t digit_sum(int k, int nhi, Col col_at) {
  uint32_t D = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int kk = k - i;
    if (kk >= 0 && kk < nhi) D += (uint32_t)((col_at(kk) >> (16 * i)) & 0xFFFFu);
  }
  return D;
}

// One wavefront carries the columns [b0, b1) (b0 a multiple of 64), entering
// with carry cin into column b0 and hprev = D(b0 - 1) / 2^16; on return cin
// and hprev are those of the column after the last chunk.  kWrite: write the
// limbs below nhi, raise ovf for a nonzero limb above and keep lenv (highest
// nonzero limb + 1); otherwise only clear allp if some column of the range
// does not propagate (the range's carry out is then independent of cin).
template <bool kWrite, class Col>
__device__ __forceinline__ void carry_range(int nhi, int b0, int b1, uint32_t& cin, uint32_t& hprev, uint32_t* out,
                                            int& lenv, bool& ovf, bool& allp, Col col_at) {
  const int lane = threadIdx.x & (kLanes - 1);
  for (int base = b0; base < b1; base += kLanes) {
    const int k = base + lane;
    const uint32_t D = digit_sum(k, nhi, col_at);
    const uint32_t hi = D >> 16;
    uint32_t hb = (uint32_t)__shfl_up((int)hi, 1);
    if (lane == 0) hb = hprev;
    const uint32_t E = (D & 0xFFFFu) + hb;
    const uint64_t G = __ballot(E > 0xFFFFu), Pm = __ballot(E == 0xFFFFu);
    const uint64_t Am = G | Pm;
    const uint64_t cm = (Am + G + cin) ^ Am ^ G;   // bit l: carry into column base + l
    if (kWrite) {
      const uint32_t limb = (E + (uint32_t)((cm >> lane) & 1u)) & 0xFFFFu;
      if (k < nhi) out[k] = limb;
      else if (limb) ovf = true;
      const uint64_t nz = __ballot(k < nhi && limb != 0);
      if (nz) lenv = base + 64 - __clzll((long long)nz);
    } else if (Pm != ~0ull) {
      allp = false;
    }
    cin = (uint32_t)(((G >> 63) | ((Pm >> 63) & (cm >> 63))) & 1u);
    hprev = (uint32_t)__shfl((int)hi, kLanes - 1);
  }
}

// The carry of at most 64 chunks of 64 columns, all chunks at once: the
// wavefronts take chunks w, w + kW, ... and keep each chunk's E values in
// registers; a chunk's ballots G and P give its carry out with no carry in,
// g = bit 63 of G | (P & ((G | P) + G ^ (G | P) ^ G)), and whether it
// propagates a carry in, p = (P == all ones).  Over the chunks (one lane
// each) the same lookahead, (g | p) + g, gives every chunk's carry in, and a
// second look at each chunk writes its limbs.  Returns the result's length
// in every thread; every thread of the workgroup calls it.
template <int kW, class Col>
__device__ __forceinline__ int carry_chunks(int nhi, uint32_t* out, int32_t* overflow, Col col_at) {
  constexpr int kOwn = kLanes / kW;   // chunks per wavefront at most
  __shared__ uint64_t cg[kLanes], cp[kLanes];
  __shared__ int clen[kW];
  const int lane = threadIdx.x & (kLanes - 1), w = threadIdx.x / kLanes;
  const int ncol = nhi + 3, nch = (ncol + kLanes - 1) / kLanes;
  uint32_t E[kOwn];
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const int c = w + kW * j;
    E[j] = 0u;
    if (c < nch) {
      const uint32_t D = digit_sum(kLanes * c + lane, nhi, col_at);
      uint32_t hb = (uint32_t)__shfl_up((int)(D >> 16), 1);
      if (lane == 0) hb = c > 0 ? digit_sum(kLanes * c - 1, nhi, col_at) >> 16 : 0u;
      E[j] = (D & 0xFFFFu) + hb;
      const uint64_t G = __ballot(E[j] > 0xFFFFu), P = __ballot(E[j] == 0xFFFFu);
      if (lane == 0) {
        cg[c] = G;
        cp[c] = P;
      }
    }
  }
  __syncthreads();
  bool g = false, pr = false;
  if (lane < nch) {
    const uint64_t G = cg[lane], P = cp[lane], A = G | P;
    const uint64_t cm0 = (A + G) ^ A ^ G;
    g = (((G >> 63) | ((P >> 63) & (cm0 >> 63))) & 1u) != 0;
    pr = P == ~0ull;
  }
  const uint64_t Gc = __ballot(g), Pc = __ballot(pr), Ac = Gc | Pc;
  const uint64_t cin_mask = (Ac + Gc) ^ Ac ^ Gc;   // bit c: carry into chunk c
  int lenv = 1;
  bool ovf = false;
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const int c = w + kW * j;
    if (c < nch) {
      const uint64_t G = __ballot(E[j] > 0xFFFFu), P = __ballot(E[j] == 0xFFFFu), A = G | P;
      const uint64_t cm = (A + G + ((cin_mask >> c) & 1u)) ^ A ^ G;
      const uint32_t limb = (E[j] + (uint32_t)((cm >> lane) & 1u)) & 0xFFFFu;
      const int k = kLanes * c + lane;
      if (k < nhi) out[k] = limb;
      else if (limb) ovf = true;
      const uint64_t nz = __ballot(k < nhi && limb != 0);
      if (nz) lenv = max(lenv, kLanes * c + 64 - __clzll((long long)nz));
      if (c == nch - 1 && (((G >> 63) | ((P >> 63) & (cm >> 63))) & 1u)) ovf = true;
    }
  }
  if (ovf) *overflow = 1;
  if (lane == 0) clen[w] = lenv;
  __syncthreads();
  int n = clen[0];
#pragma unroll
  for (int i = 1; i < kW; ++i) n = max(n, clen[i]);
  return n;
}

// Carries columns 0 .. nhi + 2 into the nhi limbs of out and returns the
// result's length (at least 1) in every thread; every thread of the workgroup
// calls it.  One chunk of 64 columns is one wavefront's; 2 to 64 chunks go
// to carry_chunks.  Longer results (columns in global memory) are split into
// kW contiguous ranges, one per wavefront: a first pass gives each range's
// carry out with no carry in and whether every column of it propagates; a
// range's carry in is then the carry out of the ranges below, composed in
// order (g_w | (p_w & c)), and a second pass writes the limbs.
template <int kW, class Col>
__device__ __forceinline__ int carry_columns(int nhi, uint32_t* out, int32_t* overflow, Col col_at) {
  __shared__ uint32_t rg[kW], rp[kW];
  __shared__ int rlen[kW];
  const int lane = threadIdx.x & (kLanes - 1), w = threadIdx.x / kLanes;
  const int ncol = nhi + 3, nch = (ncol + kLanes - 1) / kLanes;
  int lenv = 1;
  bool ovf = false, allp = true;
  if (nch >= 2 && nch <= kLanes) return carry_chunks<kW>(nhi, out, overflow, col_at);
  if (kW == 1 || nch < 2 * kW) {
    if (w == 0) {
      uint32_t cin = 0, hprev = 0;
      carry_range<true>(nhi, 0, ncol, cin, hprev, out, lenv, ovf, allp, col_at);
      if (cin || hprev) ovf = true;
      if (ovf) *overflow = 1;
      if (lane == 0) rlen[0] = lenv;
    }
    __syncthreads();
    return rlen[0];
  }
  const int q = (nch + kW - 1) / kW * kLanes;   // columns per wavefront
  const int b0 = w * q, b1 = min(b0 + q, ncol);
  const uint32_t h0 = b0 > 0 && b0 < ncol ? digit_sum(b0 - 1, nhi, col_at) >> 16 : 0u;
  uint32_t cin = 0, hprev = h0;
  carry_range<false>(nhi, b0, b1, cin, hprev, out, lenv, ovf, allp, col_at);
  if (lane == 0) {
    rg[w] = cin;
    rp[w] = allp ? 1u : 0u;
  }
  __syncthreads();
  cin = 0;
  for (int i = 0; i < w; ++i) cin = rg[i] | (rp[i] & cin);
  hprev = h0;
  carry_range<true>(nhi, b0, b1, cin, hprev, out, lenv, ovf, allp, col_at);
  if (b0 < ncol && b1 == ncol && (cin || hprev)) ovf = true;   // the top range
  if (ovf) *overflow = 1;
  if (lane == 0) rlen[w] = lenv;
  __syncthreads();
  int n = rlen[0];
#pragma unroll
  for (int i = 1; i < kW; ++i) n = max(n, rlen[i]);
  return n;
}

// Staged operands sit between zero limbs (a[i] at sa[kPadA + i], b[i] at
// sb[kPadB + i], kPadHi zeros after each), so the blocked product loop below
// reads across an operand's ends without bounds checks, by aligned 16-byte
// LDS loads.
constexpr int kPadA = 15;
constexpr int kPadB = 16;
constexpr int kPadHi = 8;
constexpr int kColBlock = 4;   // adjacent columns per thread

struct alignas(16) Limbs4 {
  uint32_t v[4];
};

// out (+)= a[0 .. la) * b[0 .. lb) + c0, where out holds lacc limbs when
// accumulating; returns the length of the result (index of the highest
// nonzero limb + 1, at least 1).  Only the limbs below the result's length
// bound max(la + lb, lacc, 4) + 2 are written: a value is read below its
// length only.  col is 64-bit scratch of lout words.  a == nullptr: the
// first operand is the coefficient ca as four limbs (la = 4).  All lanes
// call it.
//
// A thread sums four adjacent columns k0 .. k0 + 3 over blocks of four limbs
// of a: with w[m] = b[k0 - i - 3 + m] (m = 0 .. 6), column k0 + j gets
// a[i + t] w[j - t + 3] for t = 0 .. 3, and the next block's window is this
// one moved by four (three limbs kept, four loaded).  Blocks start at i = 1
// (mod 4), which aligns every load; limbs outside an operand read as zero,
// so the products a block adds outside a column's range are zero.
template <int kW>
__device__ int big_mac(const uint32_t* a, int la, const uint32_t* b, int lb, uint32_t* out, int lout,
                       bool accumulate, int lacc, uint64_t c0, uint64_t* col, int32_t* overflow, uint64_t ca = 0) {
  constexpr int kThreads = kW * kLanes;
  __shared__ alignas(16) uint32_t sa[kPadA + kBigStage + kPadHi + 1];
  __shared__ alignas(16) uint32_t sb[kPadB + kBigStage + kPadHi];
  __shared__ uint64_t scol[kBigCols];
  const int lane = threadIdx.x;
  // limbs the result can reach: the product, the accumulated value and the
  // four limbs of c0, plus carries
  const int nhi = min(max(max(la + lb, accumulate ? lacc : 0), 4) + 2, lout);
  const bool stage_a = la <= kBigStage, stage_b = lb <= kBigStage;
  const bool lds_cols = nhi <= kBigCols;
  if (stage_a)
    for (int k = lane; k < kPadA + la + kPadHi; k += kThreads) {
      const int i = k - kPadA;
      sa[k] = (unsigned)i < (unsigned)la ? (a ? a[i] : (uint32_t)((ca >> (16 * (i & 3))) & 0xFFFFu)) : 0u;
    }
  if (stage_b)
    for (int k = lane; k < kPadB + lb + kPadHi; k += kThreads)
      sb[k] = k >= kPadB && k < kPadB + lb ? b[k - kPadB] : 0u;
  __syncthreads();
  // the column sums; ld_a(i) gives a[i .. i + 3] and ld_b(i) b[i .. i + 3],
  // zero outside the operands
  auto columns = [&](auto ld_a, auto ld_b) {
    for (int k0 = lane * kColBlock; k0 < nhi; k0 += kThreads * kColBlock) {
      uint64_t s[kColBlock] = {0u, 0u, 0u, 0u};
      const int i_lo = max(0, k0 - (lb - 1)), i_hi = min(la - 1, k0 + kColBlock - 1);
      if (i_lo <= i_hi) {
        int i = i_lo - ((i_lo - 1) & 3);
        const Limbs4 lo = ld_b(k0 - i - 3), hi = ld_b(k0 - i + 1);
        uint32_t w[7] = {lo.v[0], lo.v[1], lo.v[2], lo.v[3], hi.v[0], hi.v[1], hi.v[2]};
        for (; i <= i_hi; i += 4) {
          const Limbs4 av = ld_a(i);
          const Limbs4 nb = ld_b(k0 - i - 7);
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < kColBlock; ++j) s[j] += (uint64_t)av.v[t] * w[j - t + 3];
          w[6] = w[2];
          w[5] = w[1];
          w[4] = w[0];
#pragma unroll
          for (int m = 0; m < 4; ++m) w[m] = nb.v[m];
        }
      }
#pragma unroll
      for (int j = 0; j < kColBlock; ++j) {
        const int k = k0 + j;
        if (k >= nhi) break;
        uint64_t v = s[j];
        if (accumulate && k < lacc) v += out[k];
        if (k < 4) v += (c0 >> (16 * k)) & 0xFFFFu;
        if (lds_cols) scol[k] = v;
        else col[k] = v;
      }
    }
  };
  // staged operands: one aligned LDS load per four limbs; others (longer
  // than the staging arrays) from global memory, limb by limb with bounds
  auto lds_a = [&](int i) { return *(const Limbs4*)&sa[kPadA + i]; };
  auto lds_b = [&](int i) { return *(const Limbs4*)&sb[kPadB + i]; };
  auto mem_a = [&](int i) {
    Limbs4 r;
#pragma unroll
    for (int t = 0; t < 4; ++t) r.v[t] = (unsigned)(i + t) < (unsigned)la ? a[i + t] : 0u;
    return r;
  };
  auto mem_b = [&](int i) {
    Limbs4 r;
#pragma unroll
    for (int t = 0; t < 4; ++t) r.v[t] = (unsigned)(i + t) < (unsigned)lb ? b[i + t] : 0u;
    return r;
  };
  if (stage_a) {
    if (stage_b) columns(lds_a, lds_b);
    else columns(lds_a, mem_b);
  } else {
    if (stage_b) columns(mem_a, lds_b);
    else columns(mem_a, mem_b);
  }
  __syncthreads();
  if (lds_cols) return carry_columns<kW>(nhi, out, overflow, [&](int kk) { return scol[kk]; });
  return carry_columns<kW>(nhi, out, overflow, [&](int kk) { return col[kk]; });
}

// kW wavefronts per point: their lanes share a product's columns and, for
// long results, its carry.
template <int kW>
__global__ __launch_bounds__(kW * kLanes) void k_bigint_walk(BigArgs A) {
  constexpr int kThreads = kW * kLanes;
  const int64_t inst = blockIdx.x;
  const DevTree& tr = A.tr;
  const int L = A.lout;
  uint32_t* W = A.ws + inst * A.per_instance;
  uint32_t* table = W + (int64_t)A.nbuf * L;                       // n_table values
  uint64_t* col = (uint64_t*)(W + A.col_off);                      // 64-bit columns, L of them
  const uint32_t* xi = A.x + inst * (int64_t)A.lx;
  __shared__ int32_t tab_len[kMaxTable];
  __shared__ int32_t buf[kMaxDepth + 2];
  __shared__ int32_t len[kMaxDepth + 2];

  // powers x^d by the chain
  for (int c = 0; c < tr.n_chain; ++c) {
    const ChainStep st = tr.chain[c];
    uint32_t* dst = table + (int64_t)st.dst * L;
    if (!chain_is_mul(st.kind)) {
      int lx = 1;
      for (int k = 0; k < A.lx; ++k)
        if (xi[k]) lx = k + 1;
      for (int k = threadIdx.x; k < L; k += kThreads) dst[k] = k < A.lx ? xi[k] : 0u;
      if (threadIdx.x == 0) tab_len[st.dst] = lx;
    } else {
      const int la = tab_len[st.s1], lb = tab_len[st.s2];
      const int n = big_mac<kW>(table + (int64_t)st.s1 * L, la, table + (int64_t)st.s2 * L, lb, dst, L, false, 0, 0,
                            col, A.overflow);
      if (threadIdx.x == 0) tab_len[st.dst] = n;
    }
    __syncthreads();
  }
  if (threadIdx.x < kMaxDepth + 2) {
    buf[threadIdx.x] = threadIdx.x;
    len[threadIdx.x] = 1;
  }
  __syncthreads();

  int top = 0;   // open accumulators (uniform)
  // each op's record is loaded one op ahead (the op array ends on zero
  // records, so the load past END stays inside it)
  OpF64 nx = tr.ops64[0];
  for (int pc = 0; pc < tr.n_ops; ++pc) {
    const OpF64 o = nx;
    nx = tr.ops64[pc + 1];
    const uint32_t kind = op_kind(o.info);
    const uint32_t pidx = op_pidx(o.info);
    const bool haspow = pidx != kOffTable;
    const uint32_t* X = haspow ? table + (int64_t)pidx * L : nullptr;
    const int lx = haspow ? tab_len[pidx] : 1;
    if (kind == kLeafAdd) {                       // top += c(N) X
      uint32_t* d = W + (int64_t)buf[top - 1] * L;
      const int n = big_mac<kW>(nullptr, 4, X, lx, d, L, true, len[top - 1], 0, col, A.overflow, o.a);
      if (threadIdx.x == 0) len[top - 1] = n;
    } else if (kind == kNodeOpen) {               // top = top X + c(P)
      uint32_t* s = W + (int64_t)buf[top - 1] * L;
      uint32_t* d = W + (int64_t)buf[top] * L;   // free buffer above the top
      const int n = big_mac<kW>(s, len[top - 1], X, lx, d, L, false, 0, o.b, col, A.overflow);
      if (threadIdx.x == 0) {
        const int b = buf[top - 1];
        buf[top - 1] = buf[top];
        buf[top] = b;
        len[top - 1] = n;
      }
    } else if (kind == kLeafOpen) {               // push c(N) X + c(P)
      uint32_t* d = W + (int64_t)buf[top] * L;
      const int n = big_mac<kW>(nullptr, 4, X, lx, d, L, false, 0, o.b, col, A.overflow, o.a);
      if (threadIdx.x == 0) len[top] = n;
      ++top;
    } else if (kind == kNodeAdd) {                // below += top X; pop
      uint32_t* s = W + (int64_t)buf[top - 1] * L;
      uint32_t* d = W + (int64_t)buf[top - 2] * L;
      const int n = big_mac<kW>(s, len[top - 1], X, lx, d, L, true, len[top - 2], 0, col, A.overflow);
      if (threadIdx.x == 0) len[top - 2] = n;
      --top;
    } else {                                      // END: y = (children ? top : c(R)) X_R
      uint32_t* res = A.out + inst * (int64_t)L;
      const bool leaf_root = (o.info & kEndLeafRoot) != 0;
      const bool pw = (o.info & kEndHasPow) != 0;
      int n = 4;                                  // limbs written below (the rest are zeroed)
      if (leaf_root) {
        if (pw) {
          n = min(4 + lx + 2, L);
          big_mac<kW>(nullptr, 4, X, lx, res, L, false, 0, 0, col, A.overflow, o.a);
        } else {
          for (int k = threadIdx.x; k < 4; k += kThreads) res[k] = (uint32_t)((o.a >> (16 * k)) & 0xFFFFu);
        }
      } else {
        const uint32_t* s = W + (int64_t)buf[top - 1] * L;
        if (pw) {
          n = min(len[top - 1] + lx + 2, L);
          big_mac<kW>(s, len[top - 1], X, lx, res, L, false, 0, 0, col, A.overflow);
        } else {
          n = len[top - 1];
          for (int k = threadIdx.x; k < n; k += kThreads) res[k] = s[k];
        }
      }
      for (int k = n + threadIdx.x; k < L; k += kThreads) res[k] = 0;
      break;
    }
    __syncthreads();
  }
}

}  // namespace

size_t bigint_workspace_bytes(const fpe_tree* t, int32_t lout, int64_t batch) {
  if (!t || lout < 1 || batch < 1) return 0;
  // 256 bytes for the overflow flag, then every point's workspace
  return 256 + (size_t)per_point_words(t, lout) * sizeof(uint32_t) * (size_t)batch;
}

fpe_status launch_bigint(const fpe_tree* t, const uint32_t* x, int32_t lx, int64_t batch, uint32_t* out,
                         int32_t lout, void* ws, size_t ws_bytes, void* stream) {
  if (t->n_offtable > 0) return fail(FPE_EUNSUPPORTED, "big-integer evaluation needs every power in the table");
  if (t->depth + 2 > kMaxDepth + 2) return fail(FPE_EUNSUPPORTED, "walk deeper than the kernels hold");
  if (batch < 1 || batch > 0x7fffffff) return fail(FPE_EINVAL, "batch out of range");
  if (!ws || ws_bytes < bigint_workspace_bytes(t, lout, batch))
    return fail(FPE_ENOMEM, "workspace smaller than fpe_bigint_workspace_bytes()");
  if (((uintptr_t)ws) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
  BigArgs A{};
  A.tr = dev_view(t);
  A.x = x;
  A.out = out;
  A.overflow = (int32_t*)ws;                       // first 256 bytes: the overflow flag
  A.ws = (uint32_t*)((char*)ws + 256);
  A.lx = lx;
  A.lout = lout;
  A.per_instance = per_point_words(t, lout);
  A.col_off = col_offset(t, lout);
  A.nbuf = t->depth + 2;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, A.overflow);
  // A workgroup's 59 KB of LDS allow two per compute unit, and a point's walk
  // is a chain of dependent products, so the wavefronts of one point are what
  // hides its latencies: eight per point, and sixteen when there are no more
  // points than compute units (one workgroup each).  Measured at 256-bit
  // points (balanced / Horner, 256 terms): 256 points 1.34 / 2.80 ms with
  // four, 1.15 / 1.75 with eight, 1.12 / 1.40 with sixteen; 4,096 points
  // 11.5 / 23.8, 10.2 / 16.2 and 17.6 / 22.5 ms.
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(FPE_EDEVICE, "big-integer launch: cannot query the device");
  if (batch <= ncu)
    hipLaunchKernelGGL(k_bigint_walk<kBigWavesFew>, dim3((unsigned)batch), dim3(kBigWavesFew * kLanes), 0, st, A);
  else
    hipLaunchKernelGGL(k_bigint_walk<kBigWaves>, dim3((unsigned)batch), dim3(kBigWaves * kLanes), 0, st, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("big-integer launch: ") + hipGetErrorString(e));
  return FPE_OK;
}

}  // namespace fpe
