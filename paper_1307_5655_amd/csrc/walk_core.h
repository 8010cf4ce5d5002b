// Evaluation-tree walk core for gfx950 (CDNA4), shared by the kernels.
//
// One point per lane; the node program (the walk of Section 2.1 in stack
// form, see fpe_internal.h) is wave-uniform and read with scalar loads, so
// the whole wavefront shares each op.  The accumulators of the walk live in
// VGPRs: the kernel is a nest of loops, one per stack depth, so every
// accumulator index is a compile-time constant.  The per-point powers x_j^d
// (Section 2.2, fast exponentiation) are computed once per point by the
// tree's power chain into a register table before the walk.
//
// Arithmetic policies:
//   F64   plain FP64, one fused multiply-add per node;
//   DF32  compensated FP32: double-float accumulators (error-free TwoProd
//         by fma, TwoSum, FastTwoSum renormalisation), powers as three
//         floats, a running error bound and the condition sum
//         ptilde(|x|) = sum |c_m| |x|^m in FP32; the result hi + lo in FP64;
//   DD64  double-double (TwoProd by FP64 fma): the fallback re-evaluation;
//   M61   exact arithmetic modulo the Mersenne prime 2^61 - 1.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "fpe_internal.h"

namespace fpe {

// ----------------------------------------------------------------------------
// small device helpers
// ----------------------------------------------------------------------------

__device__ __forceinline__ double u2d(uint64_t u) { return __longlong_as_double((long long)u); }

struct DD {
  double h, l;
};

// (a.h + a.l) * (b.h + b.l) in double-double (Dekker product by fma).
__device__ __forceinline__ DD dd_mul(DD a, DD b) {
  double p = a.h * b.h;
  double e = __builtin_fma(a.h, b.h, -p);
  e = __builtin_fma(a.h, b.l, e);
  e = __builtin_fma(a.l, b.h, e);
  double s = p + e;
  return {s, e - (s - p)};
}

__device__ __forceinline__ DD dd_fma(DD a, DD x, DD b) {
  // a * x + b
  double p = a.h * x.h;
  double pe = __builtin_fma(a.h, x.h, -p);
  pe = __builtin_fma(a.h, x.l, pe);
  pe = __builtin_fma(a.l, x.h, pe);
  double s = p + b.h;
  double bb = s - p;
  double se = (p - (s - bb)) + (b.h - bb);
  se = se + (pe + b.l);
  double h = s + se;
  return {h, se - (h - s)};
}

__device__ __forceinline__ uint64_t m61_reduce128(uint64_t lo, uint64_t hi) {
  // value = hi * 2^64 + lo < 2^122; 2^61 = 1 (mod p)
  uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
  r = (r & kP61) + (r >> 61);
  return r >= kP61 ? r - kP61 : r;
}
__device__ __forceinline__ uint64_t m61_mul(uint64_t a, uint64_t b) {
  return m61_reduce128(a * b, __umul64hi(a, b));
}
__device__ __forceinline__ uint64_t m61_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  return s >= kP61 ? s - kP61 : s;
}

// Off-table power x^d by binary exponentiation (FP64), used only for the
// rare ops whose power did not fit the table.
__device__ __forceinline__ double pow_f64(double x, uint32_t d) {
  double r = 1.0, b = x;
  while (d) {
    if (d & 1u) r *= b;
    b *= b;
    d >>= 1;
  }
  return r;
}
__device__ __forceinline__ uint64_t pow_m61(uint64_t x, uint32_t d) {
  uint64_t r = 1, b = x;
  while (d) {
    if (d & 1u) r = m61_mul(r, b);
    b = m61_mul(b, b);
    d >>= 1;
  }
  return r;
}

// ----------------------------------------------------------------------------
// arithmetic policies
// ----------------------------------------------------------------------------

struct ArF64 {
  using Op = OpF64;
  using Acc = double;
  using Pow = double;
  using In = double;
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops64; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, Pow X, Acc top) {   // a*X + top
    return __builtin_fma(u2d(o.a), X, top);
  }
  static __device__ __forceinline__ Acc fma_tb(Acc top, Pow X, const Op& o) {   // top*X + b
    return __builtin_fma(top, X, u2d(o.b));
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, Pow X) {           // a*X + b
    return __builtin_fma(u2d(o.a), X, u2d(o.b));
  }
  static __device__ __forceinline__ Acc fma_tt(Acc top, Pow X, Acc below) {
    return __builtin_fma(top, X, below);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return u2d(o.a); }
  static __device__ __forceinline__ Acc mul(Acc a, Pow X) { return a * X; }
  static __device__ __forceinline__ Pow off_table(const In* x, const Op& o) {
    return pow_f64(x[op_var(o.info)], o.deg);
  }
};

struct ArDD {   // double-double walk (fallback), double-double powers
  using Op = OpF64;
  using Acc = DD;
  using Pow = DD;
  using In = double;
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops64; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, const Pow& X, const Acc& top) {
    return dd_fma(DD{u2d(o.a), 0.0}, X, top);
  }
  static __device__ __forceinline__ Acc fma_tb(const Acc& top, const Pow& X, const Op& o) {
    return dd_fma(top, X, DD{u2d(o.b), 0.0});
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, const Pow& X) {
    return dd_fma(DD{u2d(o.a), 0.0}, X, DD{u2d(o.b), 0.0});
  }
  static __device__ __forceinline__ Acc fma_tt(const Acc& top, const Pow& X, const Acc& below) {
    return dd_fma(top, X, below);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return DD{u2d(o.a), 0.0}; }
  static __device__ __forceinline__ Acc mul(const Acc& a, const Pow& X) { return dd_mul(a, X); }
  static __device__ __forceinline__ Pow off_table(const In* x, const Op& o) {
    // binary exponentiation in double-double
    DD r{1.0, 0.0}, b{x[op_var(o.info)], 0.0};
    for (uint32_t d = o.deg; d; d >>= 1) {
      if (d & 1u) r = dd_mul(r, b);
      b = dd_mul(b, b);
    }
    return r;
  }
};

struct ArM61 {
  using Op = OpF64;
  using Acc = uint64_t;
  using Pow = uint64_t;
  using In = uint64_t;
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops64; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, Pow X, Acc top) {
    return m61_add(m61_mul(o.a, X), top);
  }
  static __device__ __forceinline__ Acc fma_tb(Acc top, Pow X, const Op& o) {
    return m61_add(m61_mul(top, X), o.b);
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, Pow X) {
    return m61_add(m61_mul(o.a, X), o.b);
  }
  static __device__ __forceinline__ Acc fma_tt(Acc top, Pow X, Acc below) {
    return m61_add(m61_mul(top, X), below);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return o.a; }
  static __device__ __forceinline__ Acc mul(Acc a, Pow X) { return m61_mul(a, X); }
  static __device__ __forceinline__ Pow off_table(const In* x, const Op& o) {
    return pow_m61(x[op_var(o.info)], o.deg);
  }
};

// Compensated FP32.  A value is hi + lo (double-float); alongside it the
// walk carries e, a bound on |value - exact value of the subtree|, and t,
// the subtree's sum of |c| |x|^m (for the condition number).
//
// One step a * X + b with X = X.h + X.m + X.l (a power split into three
// floats, accurate to about 2^-70):
//   p  = fl(a.h X.h), pe = a.h X.h - p exactly (fma),
//   pe += a.h X.m + a.l X.h + a.h X.l        (three fmas, a.l X.m dropped)
//   (s, se) = TwoSum(p, b.h),  se += pe + b.l,  (hi, lo) = FastTwoSum(s, se).
// With u = 2^-24: |pe| <= 3u|p| along the way, so the three fma roundings
// add at most 8u^2|p|; the dropped term u^2|p|; pe + b.l and the final sum
// round by at most u^2 (7|p| + 3|b|); the 48-bit constants a and b add
// u^2 (|p| + |b|).  The new error is therefore at most u^2 (17|p| + 4|b|);
// the bound uses 20 and 6 for margin, and inherited errors propagate as
// e_a |X| + e_b.  The FP32 evaluation of the bound itself loses at most a
// factor (1 - u)^n, covered by the final factor 1.01.
struct DF {
  float h, l, e, t;
};
struct P3 {
  float h, m, l;
};

constexpr float kU2 = 3.5527136788005009e-15f;   // 2^-48
constexpr float kK1 = 20.0f * kU2;
constexpr float kK2 = 6.0f * kU2;

__device__ __forceinline__ DF df_step(float ah, float al, float ea, float ta, const P3& X,
                                      float bh, float bl, float eb, float tb) {
  float p = ah * X.h;
  float pe = __builtin_fmaf(ah, X.h, -p);
  pe = __builtin_fmaf(ah, X.m, pe);
  pe = __builtin_fmaf(al, X.h, pe);
  pe = __builtin_fmaf(ah, X.l, pe);
  float s = p + bh;
  float bb = s - p;
  float se = (p - (s - bb)) + (bh - bb);
  se = se + (pe + bl);
  float hi = s + se;
  float lo = se - (hi - s);
  float ax = __builtin_fabsf(X.h) * 1.0000001f;
  float e = __builtin_fmaf(ea, ax, eb);
  e = __builtin_fmaf(kK1, __builtin_fabsf(p), e);
  e = __builtin_fmaf(kK2, __builtin_fabsf(bh), e);
  float t = __builtin_fmaf(ta, ax, tb);
  return DF{hi, lo, e, t};
}

struct ArDF32 {
  using Op = OpF32;
  using Acc = DF;
  using Pow = P3;
  using In = double;
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops32; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, const Pow& X, const Acc& top) {
    return df_step(o.ah, o.al, 0.f, o.aabs, X, top.h, top.l, top.e, top.t);
  }
  static __device__ __forceinline__ Acc fma_tb(const Acc& top, const Pow& X, const Op& o) {
    return df_step(top.h, top.l, top.e, top.t, X, o.bh, o.bl, 0.f, o.babs);
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, const Pow& X) {
    return df_step(o.ah, o.al, 0.f, o.aabs, X, o.bh, o.bl, 0.f, o.babs);
  }
  static __device__ __forceinline__ Acc fma_tt(const Acc& top, const Pow& X, const Acc& below) {
    return df_step(top.h, top.l, top.e, top.t, X, below.h, below.l, below.e, below.t);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return DF{o.ah, o.al, 0.f, o.aabs}; }
  static __device__ __forceinline__ Acc mul(const Acc& a, const Pow& X) {
    return df_step(a.h, a.l, a.e, a.t, X, 0.f, 0.f, 0.f, 0.f);
  }
  static __device__ __forceinline__ Pow off_table(const In* x, const Op& o) {
    double v = pow_f64(x[op_var(o.info)], o.deg);
    return split3(v);
  }
  static __device__ __forceinline__ P3 split3(double v) {
    float h = (float)v;
    double r = v - (double)h;
    float m = (float)r;
    float l = (float)(r - (double)m);
    return P3{h, m, l};
  }
};

// ----------------------------------------------------------------------------
// power tables
// ----------------------------------------------------------------------------
//
// Each point owns one column of a per-wavefront table in LDS: entry e of
// column c (= point-in-lane j * 64 + lane) at [e][c], so a wavefront reads 64
// consecutive words (no bank conflict).  The two most used entries are also
// kept in registers.  The chain runs in double-double with the low word
// stored as a float relative to the high word (lo / hi, so it cannot overflow
// where hi is large): about 77 bits, so every power is accurate to a few units
// in 2^-70 before it is rounded.

constexpr int kWave = 64;

struct TabF64 {
  double* hi;          // [n_table][stride]
  float* lo;           // [n_table][stride], low word / high word
  int col, stride;
  double r0, r1;
  static constexpr size_t bytes_per_entry = kWave * (sizeof(double) + sizeof(float));
  __device__ __forceinline__ void bind(char* lds, int n_table, int j, int ppl) {
    stride = ppl * kWave;
    col = j * kWave + (threadIdx.x & (kWave - 1));
    hi = (double*)lds;
    lo = (float*)(lds + (size_t)n_table * stride * sizeof(double));
  }
  __device__ __forceinline__ DD dd_at(uint32_t i) const {
    const double h = hi[i * stride + col];
    return DD{h, h * (double)lo[i * stride + col]};
  }
  __device__ __forceinline__ void build(const DevTree& tr, const double* x) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      double h;
      float l;
      if (st.kind == kChainLoad) {
        h = x[st.s1];
        l = 0.f;
      } else {
        DD r = dd_mul(dd_at(st.s1), dd_at(st.s2));
        h = r.h;
        l = (r.h != 0.0 && isfinite(r.h)) ? (float)(r.l / r.h) : 0.f;
      }
      hi[st.dst * stride + col] = h;
      lo[st.dst * stride + col] = l;
    }
    r0 = tr.n_table > 0 ? hi[col] : 0.0;
    r1 = tr.n_table > 1 ? hi[stride + col] : 0.0;
  }
  __device__ __forceinline__ double get0() const { return r0; }
  __device__ __forceinline__ double get1() const { return r1; }
  __device__ __forceinline__ double get(uint32_t i) const { return hi[i * stride + col]; }
};

// The fallback reads the powers as double-double (hi + lo).
struct TabDD : TabF64 {
  DD d0, d1;
  __device__ __forceinline__ void build(const DevTree& tr, const double* x) {
    TabF64::build(tr, x);
    d0 = tr.n_table > 0 ? dd_at(0) : DD{0.0, 0.0};
    d1 = tr.n_table > 1 ? dd_at(1) : DD{0.0, 0.0};
  }
  __device__ __forceinline__ DD get0() const { return d0; }
  __device__ __forceinline__ DD get1() const { return d1; }
  __device__ __forceinline__ DD get(uint32_t i) const { return dd_at(i); }
};

struct TabM61 {
  uint64_t* v;         // [n_table][stride]
  int col, stride;
  uint64_t r0, r1;
  static constexpr size_t bytes_per_entry = kWave * sizeof(uint64_t);
  __device__ __forceinline__ void bind(char* lds, int, int j, int ppl) {
    stride = ppl * kWave;
    col = j * kWave + (threadIdx.x & (kWave - 1));
    v = (uint64_t*)lds;
  }
  __device__ __forceinline__ void build(const DevTree& tr, const uint64_t* x) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      v[st.dst * stride + col] =
          st.kind == kChainLoad ? x[st.s1] : m61_mul(v[st.s1 * stride + col], v[st.s2 * stride + col]);
    }
    r0 = tr.n_table > 0 ? v[col] : 0;
    r1 = tr.n_table > 1 ? v[stride + col] : 0;
  }
  __device__ __forceinline__ uint64_t get0() const { return r0; }
  __device__ __forceinline__ uint64_t get1() const { return r1; }
  __device__ __forceinline__ uint64_t get(uint32_t i) const { return v[i * stride + col]; }
};

// Three-float powers for the double-float walk: the double-double value of
// the chain split into h + m + l (72 bits).
__device__ __forceinline__ P3 split3_dd(DD r) {
  float h = (float)r.h;
  double d = (r.h - (double)h) + r.l;
  float m = (float)d;
  float l = (float)(d - (double)m);
  return P3{h, m, l};
}

struct TabP3 {
  float* f;            // [n_table][3][stride]
  int col, stride;
  P3 r0, r1;
  static constexpr size_t bytes_per_entry = kWave * 3 * sizeof(float);
  __device__ __forceinline__ void bind(char* lds, int, int j, int ppl) {
    stride = ppl * kWave;
    col = j * kWave + (threadIdx.x & (kWave - 1));
    f = (float*)lds;
  }
  __device__ __forceinline__ P3 load(uint32_t i) const {
    const float* p = f + i * (3 * stride) + col;
    return P3{p[0], p[stride], p[2 * stride]};
  }
  __device__ __forceinline__ void store(uint32_t i, P3 v) {
    float* p = f + i * (3 * stride) + col;
    p[0] = v.h;
    p[stride] = v.m;
    p[2 * stride] = v.l;
  }
  __device__ __forceinline__ void build(const DevTree& tr, const double* x) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      if (st.kind == kChainLoad) {
        store(st.dst, split3_dd(DD{x[st.s1], 0.0}));
      } else {
        const P3 a = load(st.s1), b = load(st.s2);
        DD r = dd_mul(DD{(double)a.h + (double)a.m, (double)a.l},
                      DD{(double)b.h + (double)b.m, (double)b.l});
        store(st.dst, split3_dd(r));
      }
    }
    r0 = tr.n_table > 0 ? load(0) : P3{0.f, 0.f, 0.f};
    r1 = tr.n_table > 1 ? load(1) : P3{0.f, 0.f, 0.f};
  }
  __device__ __forceinline__ P3 get0() const { return r0; }
  __device__ __forceinline__ P3 get1() const { return r1; }
  __device__ __forceinline__ P3 get(uint32_t i) const { return load(i); }
};

template <class Ar> struct TabFor;
template <> struct TabFor<ArF64> { using T = TabF64; };
template <> struct TabFor<ArDD> { using T = TabDD; };
template <> struct TabFor<ArM61> { using T = TabM61; };
template <> struct TabFor<ArDF32> { using T = TabP3; };

// ----------------------------------------------------------------------------
// the walk
// ----------------------------------------------------------------------------
//
// PPL points per lane share every op: the op (one scalar load) drives PPL
// independent multiply-adds, which amortises the wave-uniform dispatch and
// gives the VALU independent work to interleave.

// OFFT: the tree has ops whose power is not in the table (computed on the
// fly from the coordinates); without it the coordinates are dead after the
// power chain.
template <class Ar, int DMAX, int PPL, bool OFFT>
struct Walker {
  using Op = typename Ar::Op;
  using Acc = typename Ar::Acc;
  using Pow = typename Ar::Pow;
  using In = typename Ar::In;
  using Tab = typename TabFor<Ar>::T;

  const Op* __restrict__ ops;
  const In (*x)[8];   // x[j][var]: the coordinates of point j (kernel locals)
  Tab* tab;           // tab[j]: the power table of point j (kernel locals)
  Acc m[DMAX][PPL];
  Acc y[PPL];

  __device__ __forceinline__ Walker(const In (*x_)[8], Tab* t_) : ops(nullptr), x(x_), tab(t_) {}

#define FPE_FOR_J _Pragma("unroll") for (int j = 0; j < PPL; ++j)
  // Apply body(j, X_j) for every point j with the op's power.  The two most
  // used powers come from registers, the rest from the LDS column; each case
  // is its own code path.
#define FPE_WITH_POW(o, BODY)                                              \
  do {                                                                     \
    const uint32_t pidx_ = op_pidx((o).info);                              \
    if (pidx_ == 0) {                                                      \
      FPE_FOR_J { const Pow X = tab[j].get0(); BODY; }                      \
    } else if (pidx_ == 1) {                                               \
      FPE_FOR_J { const Pow X = tab[j].get1(); BODY; }                      \
    } else if (!OFFT || pidx_ != kOffTable) {                              \
      FPE_FOR_J { const Pow X = tab[j].get(pidx_); BODY; }                  \
    } else {                                                               \
      if constexpr (OFFT) {                                                \
        FPE_FOR_J { const Pow X = Ar::off_table(x[j], (o)); BODY; }         \
      }                                                                    \
    }                                                                      \
  } while (0)

  // One op at stack depth L (L accumulators open, the top is m[L - 1]).
  template <int L>
  __device__ __forceinline__ void step(const Op& o) {
    const uint32_t info = o.info;
    if (info & kBitLeaf) {
      if (info & kBitFirst) {              // LEAF_OPEN: push a * X + b
        if constexpr (L < DMAX) FPE_WITH_POW(o, m[L][j] = Ar::fma_ab(o, X));
      } else {                             // LEAF_ADD: top += a * X
        if constexpr (L >= 1) FPE_WITH_POW(o, m[L - 1][j] = Ar::fma_ca(o, X, m[L - 1][j]));
      }
    } else if (info & kBitFirst) {         // NODE_OPEN: top = top * X + b
      if constexpr (L >= 1) FPE_WITH_POW(o, m[L - 1][j] = Ar::fma_tb(m[L - 1][j], X, o));
    } else {                               // NODE_ADD: below += top * X; pop
      if constexpr (L >= 2) FPE_WITH_POW(o, m[L - 2][j] = Ar::fma_tt(m[L - 1][j], X, m[L - 2][j]));
    }
  }

  // The root: y = (children ? m[0] : a) * X_root.
  __device__ __forceinline__ void finish(const Op& o) {
    const uint32_t info = o.info;
    FPE_FOR_J { y[j] = m[0][j]; }
    if (info & kEndLeafRoot) {
      FPE_FOR_J { y[j] = Ar::leaf_root(o); }
    }
    if (info & kEndHasPow) FPE_WITH_POW(o, y[j] = Ar::mul(y[j], X));
  }

  // The walk: one flat loop over the ops; the op's depth (set by the host)
  // selects the code with the right compile-time accumulator indices.
  __device__ __forceinline__ void walk() {
    int pc = 0;
#pragma unroll 1
    for (;;) {
      const Op o = ops[pc];
      ++pc;
      const uint32_t info = o.info;
      if (info & kBitEnd) {
        finish(o);
        return;
      }
      const uint32_t L = op_level(info);
      {
        switch (L) {
          case 0: step<0>(o); break;
          case 1: step<1>(o); break;
          case 2: step<2>(o); break;
          case 3: step<3>(o); break;
          case 4: step<4>(o); break;
          case 5: step<5>(o); break;
          case 6: step<6>(o); break;
          case 7: step<7>(o); break;
          default:
            if constexpr (DMAX > 8) {
              switch (L) {
          case 8: step<8>(o); break;
          case 9: step<9>(o); break;
          case 10: step<10>(o); break;
          case 11: step<11>(o); break;
          case 12: step<12>(o); break;
          case 13: step<13>(o); break;
          case 14: step<14>(o); break;
          default: step<15>(o); break;
              }
            }
        }
      }
    }
  }
#undef FPE_WITH_POW
#undef FPE_FOR_J

  __device__ __forceinline__ void run(const DevTree& tr) {
    ops = Ar::ops(tr);
#pragma unroll
    for (int j = 0; j < PPL; ++j) tab[j].build(tr, x[j]);
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
#pragma unroll
      for (int j = 0; j < PPL; ++j) m[k][j] = Acc{};
    }
    walk();
  }
};

// Evaluate PPL points of this lane (their columns of the LDS power table).
template <class Ar, int DMAX, int PPL, bool OFFT>
__device__ __forceinline__ void walk_points(const DevTree& tr, const typename Ar::In (*x)[8], char* lds,
                                            typename Ar::Acc* y) {
  typename TabFor<Ar>::T tab[PPL];
#pragma unroll
  for (int j = 0; j < PPL; ++j) tab[j].bind(lds, tr.n_table, j, PPL);
  Walker<Ar, DMAX, PPL, OFFT> w(x, tab);
  w.run(tr);
#pragma unroll
  for (int j = 0; j < PPL; ++j) y[j] = w.y[j];
}

template <class Ar, int DMAX, bool OFFT>
__device__ __forceinline__ typename Ar::Acc walk_point(const DevTree& tr, const typename Ar::In* x,
                                                       char* lds) {
  typename Ar::In xx[1][8];
#pragma unroll
  for (int v = 0; v < 8; ++v) xx[0][v] = x[v];
  typename Ar::Acc y[1];
  walk_points<Ar, DMAX, 1, OFFT>(tr, xx, lds, y);
  return y[0];
}

// ----------------------------------------------------------------------------
// shared kernel helpers
// ----------------------------------------------------------------------------

constexpr int kBlock = kWave;   // one wavefront per workgroup

template <class T>
struct Pts {
  const T* p[8];
};

template <class T, int PPL>
__device__ __forceinline__ void load_points(const Pts<T>& P, int nvars, int64_t base, int64_t npts,
                                            T (*x)[8]) {
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int64_t i = base + (int64_t)j * kWave;
#pragma unroll
    for (int v = 0; v < 8; ++v) x[j][v] = (v < nvars && i < npts) ? P.p[v][i] : T(0);
  }
}

// Compensated FP32 outputs: y = hi + lo (FP64), the condition number and,
// for every point whose bound exceeds tol |y| (or that left the FP32 range),
// a bit in the fallback mask and its index in the fallback list.
struct F32COut {
  double* out;
  float* cond;
  uint32_t* flags;       // optional bitmask, 32 points per word
  int32_t* list;         // fallback indices
  int64_t* count;        // fallback count (device)
  double tol;
  int32_t force;
};

__device__ __forceinline__ bool df32_finish(const DF& r, double tol, int force, double& y, float& cond) {
  y = (double)r.h + (double)r.l;
  const double ay = fabs(y);
  const double bound = (double)r.e * 1.01;
  const bool finite = isfinite(r.h) && isfinite(r.l) && isfinite(r.e) && isfinite(r.t);
  cond = (float)((double)r.t / ay);
  bool flag = !finite || !(bound <= tol * ay) || ay < 1e-30;
  if (force == 1) flag = true;
  if (force == 2) flag = false;
  return flag;
}

// Append the flagged lanes of this wavefront to the fallback list (one
// atomic per wavefront: ballot + popcount).
__device__ __forceinline__ void append_flagged(bool flag, int64_t i, int32_t* list, int64_t* count) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t ballot = __ballot(flag);
  if (ballot) {
    unsigned long long cbase = 0;
    if (lane == 0) cbase = atomicAdd((unsigned long long*)count, (unsigned long long)__popcll(ballot));
    cbase = __shfl(cbase, 0);
    if (flag) list[(int64_t)cbase + __popcll(ballot & ((uint64_t(1) << lane) - 1))] = (int32_t)i;
  }
}

}  // namespace fpe
