// Evaluation-tree walk kernels for gfx950 (CDNA4).
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
// Each lane owns one column of a per-wavefront table in LDS (entry e of lane
// l at [e][l], so a wavefront reads 64 consecutive words: no bank conflict).
// The two most used entries are also kept in registers.  The chain runs in
// double-double with the low word stored as a float relative to the high
// word (lo / hi, so it cannot overflow where hi is large): about 77 bits, so
// every power is accurate to a few units in 2^-70 before it is rounded.

constexpr int kWave = 64;

struct TabF64 {
  double* hi;          // [n_table][64]
  float* lo;           // [n_table][64], low word / high word
  int lane;
  double r0, r1;
  static constexpr size_t bytes_per_entry = kWave * (sizeof(double) + sizeof(float));
  __device__ __forceinline__ void bind(char* lds, int n_table) {
    lane = threadIdx.x & (kWave - 1);
    hi = (double*)lds;
    lo = (float*)(lds + (size_t)n_table * kWave * sizeof(double));
  }
  __device__ __forceinline__ DD dd_at(uint32_t i) const {
    const double h = hi[i * kWave + lane];
    return DD{h, h * (double)lo[i * kWave + lane]};
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
      hi[st.dst * kWave + lane] = h;
      lo[st.dst * kWave + lane] = l;
    }
    r0 = tr.n_table > 0 ? hi[lane] : 0.0;
    r1 = tr.n_table > 1 ? hi[kWave + lane] : 0.0;
  }
  __device__ __forceinline__ double get0() const { return r0; }
  __device__ __forceinline__ double get1() const { return r1; }
  __device__ __forceinline__ double get(uint32_t i) const { return hi[i * kWave + lane]; }
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
  uint64_t* v;         // [n_table][64]
  int lane;
  uint64_t r0, r1;
  static constexpr size_t bytes_per_entry = kWave * sizeof(uint64_t);
  __device__ __forceinline__ void bind(char* lds, int) {
    lane = threadIdx.x & (kWave - 1);
    v = (uint64_t*)lds;
  }
  __device__ __forceinline__ void build(const DevTree& tr, const uint64_t* x) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      v[st.dst * kWave + lane] =
          st.kind == kChainLoad ? x[st.s1] : m61_mul(v[st.s1 * kWave + lane], v[st.s2 * kWave + lane]);
    }
    r0 = tr.n_table > 0 ? v[lane] : 0;
    r1 = tr.n_table > 1 ? v[kWave + lane] : 0;
  }
  __device__ __forceinline__ uint64_t get0() const { return r0; }
  __device__ __forceinline__ uint64_t get1() const { return r1; }
  __device__ __forceinline__ uint64_t get(uint32_t i) const { return v[i * kWave + lane]; }
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
  float* f;            // [n_table][3][64]
  int lane;
  P3 r0, r1;
  static constexpr size_t bytes_per_entry = kWave * 3 * sizeof(float);
  __device__ __forceinline__ void bind(char* lds, int) {
    lane = threadIdx.x & (kWave - 1);
    f = (float*)lds;
  }
  __device__ __forceinline__ P3 load(uint32_t i) const {
    const float* p = f + i * (3 * kWave) + lane;
    return P3{p[0], p[kWave], p[2 * kWave]};
  }
  __device__ __forceinline__ void store(uint32_t i, P3 v) {
    float* p = f + i * (3 * kWave) + lane;
    p[0] = v.h;
    p[kWave] = v.m;
    p[2 * kWave] = v.l;
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

template <class Ar, int DMAX>
struct Walker {
  using Op = typename Ar::Op;
  using Acc = typename Ar::Acc;
  using Pow = typename Ar::Pow;
  using In = typename Ar::In;
  using Tab = typename TabFor<Ar>::T;

  const Op* __restrict__ ops;
  const In* x;        // this point's coordinates (a local array of the kernel)
  Tab& tab;           // the power table (a local of the kernel)
  Acc m[DMAX];
  Acc y;

  __device__ __forceinline__ Walker(const In* x_, Tab& t_) : ops(nullptr), x(x_), tab(t_) {}

  // The power of op o: the two most used table entries are read from fixed
  // registers, the rest by a wave-uniform index.
  template <class F>
  __device__ __forceinline__ void with_pow(const Op& o, F&& f) {
    const uint32_t pidx = op_pidx(o.info);
    if (pidx == 0) {
      f(tab.get0());
    } else if (pidx == 1) {
      f(tab.get1());
    } else if (pidx != kOffTable) {
      f(tab.get(pidx));
    } else {
      f(Ar::off_table(x, o));
    }
  }

  // Walk ops at stack depth L until the op that pops below L (returns
  // false) or the root (returns true).
  template <int L>
  __device__ __forceinline__ bool level(int& pc) {
    for (;;) {
      const Op o = ops[pc];
      ++pc;
      const uint32_t kind = op_kind(o.info);
      if (kind == kLeafAdd) {
        if constexpr (L >= 1) with_pow(o, [&](const Pow& X) { m[L - 1] = Ar::fma_ca(o, X, m[L - 1]); });
      } else if (kind == kNodeOpen) {
        if constexpr (L >= 1) with_pow(o, [&](const Pow& X) { m[L - 1] = Ar::fma_tb(m[L - 1], X, o); });
      } else if (kind == kLeafOpen) {
        if constexpr (L < DMAX) {
          with_pow(o, [&](const Pow& X) { m[L] = Ar::fma_ab(o, X); });
          if (level<L + 1>(pc)) return true;
        }
      } else if (kind == kNodeAdd) {
        if constexpr (L >= 2) {
          with_pow(o, [&](const Pow& X) { m[L - 2] = Ar::fma_tt(m[L - 1], X, m[L - 2]); });
        }
        return false;
      } else {   // END: the root
        Acc r;
        if constexpr (L >= 1) r = m[0];
        if (o.info & kEndLeafRoot) r = Ar::leaf_root(o);
        if (o.info & kEndHasPow) with_pow(o, [&](const Pow& X) { r = Ar::mul(r, X); });
        y = r;
        return true;
      }
    }
  }

  __device__ __forceinline__ void run(const DevTree& tr) {
    ops = Ar::ops(tr);
    tab.build(tr, x);
    int pc = 0;
    level<0>(pc);
  }
};

// Evaluate one point (this lane's column of the LDS power table).
template <class Ar, int DMAX>
__device__ __forceinline__ typename Ar::Acc walk_point(const DevTree& tr, const typename Ar::In* x,
                                                       char* lds) {
  typename TabFor<Ar>::T tab;
  tab.bind(lds, tr.n_table);
  Walker<Ar, DMAX> w(x, tab);
  w.run(tr);
  return w.y;
}

// ----------------------------------------------------------------------------
// kernels
// ----------------------------------------------------------------------------
//
// One wavefront per workgroup: each wavefront owns its slice of LDS for the
// power table, sized at launch from the tree (n_table entries).

constexpr int kBlock = kWave;

template <class T>
struct Pts {
  const T* p[8];
};

template <class T>
__device__ __forceinline__ void load_point(const Pts<T>& P, int nvars, int64_t i, T* x) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < nvars) x[j] = P.p[j][i];
}

template <int DMAX>
__global__ __launch_bounds__(kBlock) void k_eval_f64(DevTree tr, Pts<double> P, int64_t npts,
                                                     double* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= npts) return;
  double x[8];
  load_point(P, tr.nvars, i, x);
  out[i] = walk_point<ArF64, DMAX>(tr, x, lds);
}

template <int DMAX>
__global__ __launch_bounds__(kBlock) void k_eval_m61(DevTree tr, Pts<uint64_t> P, int64_t npts,
                                                     uint64_t* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= npts) return;
  uint64_t x[8];
  load_point(P, tr.nvars, i, x);
  out[i] = walk_point<ArM61, DMAX>(tr, x, lds);
}

// Compensated FP32 walk.  Writes y = hi + lo (FP64), the condition number
// and, for every point whose bound exceeds tol |y| (or that left the FP32
// range), a bit in the fallback mask and its index in the fallback list
// (one atomic per wavefront: ballot + popcount).
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

template <int DMAX>
__global__ __launch_bounds__(kBlock) void k_eval_df32(DevTree tr, Pts<double> P, int64_t npts,
                                                      F32COut o) {
  extern __shared__ __align__(16) char lds[];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool flag = false;
  if (i < npts) {
    double x[8];
    load_point(P, tr.nvars, i, x);
    const DF r = walk_point<ArDF32, DMAX>(tr, x, lds);
    double y;
    float cond;
    flag = df32_finish(r, o.tol, o.force, y, cond);
    o.out[i] = y;
    if (o.cond) o.cond[i] = cond;
  }
  const uint64_t ballot = __ballot(flag);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wbase = i - lane;
  if (o.flags && lane == 0) {
    o.flags[wbase >> 5] = (uint32_t)ballot;
    if (wbase + 32 < npts) o.flags[(wbase >> 5) + 1] = (uint32_t)(ballot >> 32);
  }
  if (ballot) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long*)o.count, (unsigned long long)__popcll(ballot));
    base = __shfl(base, 0);
    if (flag) {
      const int64_t rank = __popcll(ballot & ((uint64_t(1) << lane) - 1));
      o.list[(int64_t)base + rank] = (int32_t)i;
    }
  }
}

// FP64 fallback: double-double walk over the flagged points.  The grid is
// fixed; wavefronts stride over the count read from device memory.
template <int DMAX>
__global__ __launch_bounds__(kBlock) void k_fallback_dd(DevTree tr, Pts<double> P,
                                                        const int32_t* __restrict__ list,
                                                        const int64_t* __restrict__ count,
                                                        double* __restrict__ out) {
  extern __shared__ __align__(16) char lds[];
  const int64_t n = *count;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
    const int64_t k = base + threadIdx.x;
    if (k < n) {
      const int64_t i = list[k];
      double x[8];
      load_point(P, tr.nvars, i, x);
      const DD r = walk_point<ArDD, DMAX>(tr, x, lds);
      out[i] = r.h + r.l;
    }
  }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

namespace {

template <class F>
bool dispatch_depth(int depth, F&& f) {
  if (depth <= 8) f(std::integral_constant<int, 8>{});
  else if (depth <= kMaxDepth) f(std::integral_constant<int, kMaxDepth>{});
  else return false;
  return true;
}

inline int64_t blocks_for(int64_t n) { return (n + kBlock - 1) / kBlock; }

template <class T>
Pts<T> make_pts(const void* const* pts, int nvars) {
  Pts<T> P{};
  for (int j = 0; j < nvars; ++j) P.p[j] = (const T*)pts[j];
  return P;
}

}  // namespace

size_t lds_bytes(const fpe_tree* t, int domain) {
  size_t per = domain == FPE_MODP ? TabM61::bytes_per_entry
             : domain == FPE_F32C ? std::max(TabP3::bytes_per_entry, TabF64::bytes_per_entry)
                                  : TabF64::bytes_per_entry;
  return std::max<size_t>(16, per * (size_t)t->n_table);
}

size_t eval_workspace_bytes(const fpe_tree* t, int64_t npts) {
  if (!t || t->domain != FPE_F32C) return 0;
  // [count int64 | pad to 256 | list int32[npts]]
  return 256 + (size_t)std::max<int64_t>(npts, 0) * sizeof(int32_t);
}

fpe_status launch_eval(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                       const fpe_eval_opts* opts, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (t->depth > kMaxDepth) return fail(FPE_EUNSUPPORTED, "walk deeper than the kernels hold");
  if (npts == 0) return FPE_OK;
  DevTree tr = dev_view(t);
  const int64_t nb = blocks_for(npts);
  if (nb > 0x7fffffff || npts > 0x7fffffff) return fail(FPE_EINVAL, "too many points for one launch");
  if (t->domain == FPE_F64) {
    const size_t sh = lds_bytes(t, FPE_F64);
    auto P = make_pts<double>(pts, t->nvars);
    if (opts && opts->ev_walk_begin) (void)hipEventRecord((hipEvent_t)opts->ev_walk_begin, st);
    dispatch_depth(t->depth, [&](auto D) {
      hipLaunchKernelGGL((k_eval_f64<decltype(D)::value>), dim3((unsigned)nb), dim3(kBlock), sh, st,
                         tr, P, npts, (double*)out);
    });
    if (opts && opts->ev_walk_end) (void)hipEventRecord((hipEvent_t)opts->ev_walk_end, st);
  } else if (t->domain == FPE_MODP) {
    if (t->modulus != kP61) return fail(FPE_EUNSUPPORTED, "evaluation modulus must be 2^61-1");
    const size_t sh = lds_bytes(t, FPE_MODP);
    auto P = make_pts<uint64_t>(pts, t->nvars);
    if (opts && opts->ev_walk_begin) (void)hipEventRecord((hipEvent_t)opts->ev_walk_begin, st);
    dispatch_depth(t->depth, [&](auto D) {
      hipLaunchKernelGGL((k_eval_m61<decltype(D)::value>), dim3((unsigned)nb), dim3(kBlock), sh, st,
                         tr, P, npts, (uint64_t*)out);
    });
    if (opts && opts->ev_walk_end) (void)hipEventRecord((hipEvent_t)opts->ev_walk_end, st);
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
    auto P = make_pts<double>(pts, t->nvars);
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, o.count);
    dispatch_depth(t->depth, [&](auto D) {
      constexpr int DM = decltype(D)::value;
      if (opts->ev_walk_begin) (void)hipEventRecord((hipEvent_t)opts->ev_walk_begin, st);
      hipLaunchKernelGGL((k_eval_df32<DM>), dim3((unsigned)nb), dim3(kBlock), lds_bytes(t, FPE_F32C),
                         st, tr, P, npts, o);
      if (opts->ev_walk_end) (void)hipEventRecord((hipEvent_t)opts->ev_walk_end, st);
      const int64_t fb = std::min<int64_t>(nb, 4096);
      hipLaunchKernelGGL((k_fallback_dd<DM>), dim3((unsigned)fb), dim3(kBlock), lds_bytes(t, FPE_F64),
                         st, tr, P, (const int32_t*)o.list, (const int64_t*)o.count, (double*)out);
    });
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
