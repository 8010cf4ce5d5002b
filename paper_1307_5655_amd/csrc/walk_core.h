// Evaluation-tree walk core for gfx950 (CDNA4), shared by the kernels.
//
// PPL points per lane; the node program (the walk of Section 2.1 in stack
// form, see fpe_internal.h) is wave-uniform and read with scalar loads, so
// the whole wavefront shares each op.  The accumulators of the walk live in
// VGPRs: one switch on each op's dispatch code, whose cases carry the stack
// depth as a compile-time constant, so every accumulator index is static.
// The per-point powers x_j^d (Section 2.2, fast exponentiation) are computed
// once per point by the tree's power chain into a per-point table before the
// walk (registers, an LDS tier and private memory; see "power tables").
//
// Arithmetic policies:
//   F64   plain FP64, one fused multiply-add per node;
//   DF32  compensated FP32: double-float accumulators (error-free TwoProd
//         by fma, TwoSum, FastTwoSum renormalisation), powers as three
//         floats, a running error bound and the condition sum
//         ptilde(|x|) = sum |c_m| |x|^m in FP32; the result hi + lo in FP64;
//   DD64  double-double (TwoProd by FP64 fma): the fallback re-evaluation;
//   M61   exact arithmetic modulo the Mersenne prime 2^61 - 1;
//   IV    FP64 intervals rounded outward (point coefficients, interval points).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

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

// a * x + b in double-double; AL / BL: whether a / b have a low word (a
// coefficient is a plain double, so its terms are left out).
template <bool AL = true, bool BL = true>
__device__ __forceinline__ DD dd_fma(DD a, DD x, DD b) {
  double p = a.h * x.h;
  double pe = __builtin_fma(a.h, x.h, -p);
  pe = __builtin_fma(a.h, x.l, pe);
  if constexpr (AL) pe = __builtin_fma(a.l, x.h, pe);
  double s = p + b.h;
  double bb = s - p;
  double se = (p - (s - bb)) + (b.h - bb);
  if constexpr (BL) se = se + (pe + b.l);
  else se = se + pe;
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

// Coordinate v of a point (v is wave-uniform; a switch keeps x in registers).
template <class T>
__device__ __forceinline__ T coord(const T* x, uint32_t v) {
  switch (v) {
    case 0: return x[0];
    case 1: return x[1];
    case 2: return x[2];
    case 3: return x[3];
    case 4: return x[4];
    case 5: return x[5];
    case 6: return x[6];
    default: return x[7];
  }
}

// ----------------------------------------------------------------------------
// arithmetic policies
// ----------------------------------------------------------------------------

struct ArF64 {
  using Op = OpF64;
  using Acc = double;
  using Pow = double;
  using In = double;
  using Full = Pow;
  static __device__ __forceinline__ Pow to_pow(const Pow& f) { return f; }
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
  static __device__ __forceinline__ Pow off_table(In xv, const Op& o) { return pow_f64(xv, op_deg(o.deg)); }
  static __device__ __forceinline__ Pow pair(Pow a, Pow b) { return a * b; }
};

struct ArDD {   // double-double walk (fallback), double-double powers
  using Op = OpF64;
  using Acc = DD;
  using Pow = DD;
  using In = double;
  using Full = Pow;
  static __device__ __forceinline__ Pow to_pow(const Pow& f) { return f; }
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops64; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, const Pow& X, const Acc& top) {
    return dd_fma<false, true>(DD{u2d(o.a), 0.0}, X, top);
  }
  static __device__ __forceinline__ Acc fma_tb(const Acc& top, const Pow& X, const Op& o) {
    return dd_fma<true, false>(top, X, DD{u2d(o.b), 0.0});
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, const Pow& X) {
    return dd_fma<false, false>(DD{u2d(o.a), 0.0}, X, DD{u2d(o.b), 0.0});
  }
  static __device__ __forceinline__ Acc fma_tt(const Acc& top, const Pow& X, const Acc& below) {
    return dd_fma(top, X, below);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return DD{u2d(o.a), 0.0}; }
  static __device__ __forceinline__ Acc mul(const Acc& a, const Pow& X) { return dd_mul(a, X); }
  static __device__ __forceinline__ Pow off_table(In xv, const Op& o) {
    // binary exponentiation in double-double
    DD r{1.0, 0.0}, b{xv, 0.0};
    for (uint32_t d = op_deg(o.deg); d; d >>= 1) {
      if (d & 1u) r = dd_mul(r, b);
      b = dd_mul(b, b);
    }
    return r;
  }
  static __device__ __forceinline__ Pow pair(const Pow& a, const Pow& b) { return dd_mul(a, b); }
};

struct ArM61 {
  using Op = OpF64;
  using Acc = uint64_t;
  using Pow = uint64_t;
  using In = uint64_t;
  using Full = Pow;
  static __device__ __forceinline__ Pow to_pow(const Pow& f) { return f; }
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
  static __device__ __forceinline__ Pow off_table(In xv, const Op& o) { return pow_m61(xv, op_deg(o.deg)); }
  static __device__ __forceinline__ Pow pair(Pow a, Pow b) { return m61_mul(a, b); }
};

// Compensated FP32.  A value is hi + lo (double-float); alongside it the
// walk carries e, a bound on |value - exact value of the subtree|, and t,
// the subtree's sum of |c| |x|^m (for the condition number).
//
// One step a * X + b with X = X.h + X.m (a power rounded to two floats,
// within u^2 |X| of the exact power, u = 2^-24: the table keeps each power
// to about 2^-70 and the walk reads its two leading floats):
//   p  = fl(a.h X.h), pe = a.h X.h - p exactly (fma),
//   pe += a.h X.m + a.l X.h                  (two fmas, a.l X.m dropped)
//   (s, se) = TwoSum(p, b.h),  se += pe + b.l,  (hi, lo) = FastTwoSum(s, se).
// |pe| <= 3u|p| along the way, so the fma roundings add at most 8u^2|p|; the
// dropped term u^2|p|; the power's rounding to two floats u^2|p|; pe + b.l
// and the final sum round by at most u^2 (7|p| + 3|b|); the 48-bit
// constants a and b add u^2 (|p| + |b|).  The new error is therefore at most
// u^2 (18|p| + 4|b|); the bound uses 20 and 6 for margin, and inherited
// errors propagate as
// e_a |X| + e_b.  When b is a coefficient (exact), the host stores 6 u^2 |b.h|
// rounded up in the op, so that term costs nothing on the device.
// The bound is evaluated in FP32 with |X.h| in place of |X|
// (|X| <= |X.h| (1 + u + u^2)) and at most three roundings per step, each
// shrinking a sum of non-negative terms by at most (1 - u): after n steps the
// computed bound falls short of the exact one by at most
// g^n, g = (1 + u + u^2) / (1 - u)^3 < 1 + 4.001 u.  The host gives every
// tree the factor g^(n_ops) (with a little margin) as DevTree::bound_scale, and
// the final test scales the bound by it.
struct DF {
  float h, l, e, t;
};
struct P3 {   // a table power to about 2^-70: h + m + l
  float h, m, l;
};
struct P2 {   // the power as the walk reads it: h + m
  float h, m;
};

constexpr float kU2 = 3.5527136788005009e-15f;   // 2^-48
constexpr float kK1 = 20.0f * kU2;
constexpr float kK2 = 6.0f * kU2;

// EA / EB: whether a / b carry an inherited error bound (accumulators do;
// the coefficients of a node are exact and have no inherited term).
template <bool EA, bool EB>
__device__ __forceinline__ DF df_step(float ah, float al, float ea, float ta, const P2& X,
                                      float bh, float bl, float eb, float tb) {
  float p = ah * X.h;
  float pe = __builtin_fmaf(ah, X.h, -p);
  pe = __builtin_fmaf(ah, X.m, pe);
  pe = __builtin_fmaf(al, X.h, pe);
  float s = p + bh;
  float bb = s - p;
  float se = (p - (s - bb)) + (bh - bb);
  se = se + (pe + bl);
  float hi = s + se;
  float lo = se - (hi - s);
  const float ax = __builtin_fabsf(X.h);
  // eb: the inherited bound of b (EB), else b's own bound term 6 u^2 |b.h|
  float e = EA ? __builtin_fmaf(ea, ax, eb) : eb;
  e = __builtin_fmaf(kK1, __builtin_fabsf(p), e);
  if constexpr (EB) e = __builtin_fmaf(kK2, __builtin_fabsf(bh), e);
  float t = __builtin_fmaf(ta, ax, tb);
  return DF{hi, lo, e, t};
}

struct ArDF32 {
  using Op = OpF32;
  using Acc = DF;
  using Pow = P2;
  using Full = P3;   // table entries at full precision, for products of entries
  using In = double;
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops32; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, const Pow& X, const Acc& top) {
    return df_step<false, true>(o.ah, o.al, 0.f, __builtin_fabsf(o.ah), X, top.h, top.l, top.e, top.t);
  }
  static __device__ __forceinline__ Acc fma_tb(const Acc& top, const Pow& X, const Op& o) {
    return df_step<true, false>(top.h, top.l, top.e, top.t, X, o.bh, o.bl, o.bk2, __builtin_fabsf(o.bh));
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, const Pow& X) {
    return df_step<false, false>(o.ah, o.al, 0.f, __builtin_fabsf(o.ah), X, o.bh, o.bl, o.bk2,
                                  __builtin_fabsf(o.bh));
  }
  static __device__ __forceinline__ Acc fma_tt(const Acc& top, const Pow& X, const Acc& below) {
    return df_step<true, true>(top.h, top.l, top.e, top.t, X, below.h, below.l, below.e, below.t);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return DF{o.ah, o.al, 0.f, __builtin_fabsf(o.ah)}; }
  static __device__ __forceinline__ Acc mul(const Acc& a, const Pow& X) {
    return df_step<true, false>(a.h, a.l, a.e, a.t, X, 0.f, 0.f, 0.f, 0.f);
  }
  static __device__ __forceinline__ Pow off_table(In xv, const Op& o) {
    // binary exponentiation in double-double, rounded to two floats
    DD r{1.0, 0.0}, b{xv, 0.0};
    for (uint32_t d = op_deg(o.deg); d; d >>= 1) {
      if (d & 1u) r = dd_mul(r, b);
      b = dd_mul(b, b);
    }
    const float h = (float)r.h;
    return P2{h, (float)((r.h - (double)h) + r.l)};
  }
  // the product of two full-precision table powers, in double-double, split
  // into three floats again
  static __device__ __forceinline__ Full pair(const Full& a, const Full& b) {
    const DD r = dd_mul(DD{(double)a.h + (double)a.m, (double)a.l}, DD{(double)b.h + (double)b.m, (double)b.l});
    const float h = (float)r.h;
    const double d = (r.h - (double)h) + r.l;
    const float m = (float)d;
    return P3{h, m, (float)(d - (double)m)};
  }
  static __device__ __forceinline__ Pow to_pow(const Full& f) { return P2{f.h, f.m}; }
};

// Interval walk.  A value is an interval [lo, hi] of FP64 numbers; the
// coefficients are exact points.  Every bound comes from one
// round-to-nearest operation r (a product, an fma or a sum) and is then moved
// outward: dn(r) = RN(RN(r - |r| 2^-52) - 2^-1074) <= exact <= up(r).  For a
// normal r, |r| 2^-52 is at least one unit in the last place of r, twice the
// worst round-to-nearest error, and subtracting it rounds to a float at or
// below r - ulp; the 2^-1074 term covers results at or below the subnormal
// range.  A bound that overflows turns the point's result into
// [-inf, +inf] (see iv_finish).
struct IV {
  double lo, hi;
};
__device__ __forceinline__ double iv_dn(double r) {
  return __builtin_fma(-__builtin_fabs(r), 0x1p-52, r) - 0x1p-1074;
}
__device__ __forceinline__ double iv_up(double r) {
  return __builtin_fma(__builtin_fabs(r), 0x1p-52, r) + 0x1p-1074;
}
// a * X + [bl, bh] for a point a: the ends of a X are a times the ends of X,
// swapped when a < 0 (a is wave-uniform, so the choice is a select).
__device__ __forceinline__ IV iv_axb(double a, const IV& X, double bl, double bh) {
  const bool neg = a < 0.0;
  const double xl = neg ? X.hi : X.lo, xh = neg ? X.lo : X.hi;
  return IV{iv_dn(__builtin_fma(a, xl, bl)), iv_up(__builtin_fma(a, xh, bh))};
}
// U * X + [bl, bh]: the product's ends are the least and greatest of the four
// end products; each is fused with the matching end of b, and rounding outward
// after the min / max keeps the bound (dn and up are monotone).
__device__ __forceinline__ IV iv_mad(const IV& U, const IV& X, double bl, double bh) {
  const double l1 = __builtin_fma(U.lo, X.lo, bl), l2 = __builtin_fma(U.lo, X.hi, bl);
  const double l3 = __builtin_fma(U.hi, X.lo, bl), l4 = __builtin_fma(U.hi, X.hi, bl);
  const double h1 = __builtin_fma(U.lo, X.lo, bh), h2 = __builtin_fma(U.lo, X.hi, bh);
  const double h3 = __builtin_fma(U.hi, X.lo, bh), h4 = __builtin_fma(U.hi, X.hi, bh);
  return IV{iv_dn(fmin(fmin(l1, l2), fmin(l3, l4))), iv_up(fmax(fmax(h1, h2), fmax(h3, h4)))};
}
// Bounds [lo, hi] on m^d for m >= 0 from bounds on m^a and m^b, a + b = d.
__device__ __forceinline__ IV mag_mul(const IV& a, const IV& b) {
  return IV{fmax(iv_dn(a.lo * b.lo), 0.0), iv_up(a.hi * b.hi)};
}
// The range of x^d over X = [l, h] from bounds ml on |l|^d and mh on |h|^d:
// odd d is increasing; even d is decreasing below 0 and increasing above, with
// its least value 0 when 0 lies in X.
__device__ __forceinline__ IV power_range(const IV& X, const IV& ml, const IV& mh, bool odd) {
  if (odd) return IV{X.lo >= 0.0 ? ml.lo : -ml.hi, X.hi >= 0.0 ? mh.hi : -mh.lo};
  if (X.lo >= 0.0) return IV{ml.lo, mh.hi};
  if (X.hi <= 0.0) return IV{mh.lo, ml.hi};
  return IV{0.0, fmax(ml.hi, mh.hi)};
}
// Bounds on m^d by binary exponentiation (powers outside the table).
__device__ __forceinline__ IV mag_pow(double m, uint32_t d) {
  IV r{1.0, 1.0}, b{m, m};
  for (; d; d >>= 1) {
    if (d & 1u) r = mag_mul(r, b);
    b = mag_mul(b, b);
  }
  return r;
}

struct ArIV {
  using Op = OpF64;
  using Acc = IV;
  using Pow = IV;
  using In = IV;
  using Full = Pow;
  static __device__ __forceinline__ Pow to_pow(const Pow& f) { return f; }
  static __device__ __forceinline__ const Op* ops(const DevTree& t) { return t.ops64; }
  static __device__ __forceinline__ Acc fma_ca(const Op& o, const Pow& X, const Acc& top) {
    return iv_axb(u2d(o.a), X, top.lo, top.hi);
  }
  static __device__ __forceinline__ Acc fma_tb(const Acc& top, const Pow& X, const Op& o) {
    const double b = u2d(o.b);
    return iv_mad(top, X, b, b);
  }
  static __device__ __forceinline__ Acc fma_ab(const Op& o, const Pow& X) {
    const double b = u2d(o.b);
    return iv_axb(u2d(o.a), X, b, b);
  }
  static __device__ __forceinline__ Acc fma_tt(const Acc& top, const Pow& X, const Acc& below) {
    return iv_mad(top, X, below.lo, below.hi);
  }
  static __device__ __forceinline__ Acc leaf_root(const Op& o) { return IV{u2d(o.a), u2d(o.a)}; }
  static __device__ __forceinline__ Acc mul(const Acc& a, const Pow& X) { return iv_mad(a, X, 0.0, 0.0); }
  static __device__ __forceinline__ Pow off_table(const In& xv, const Op& o) {
    const uint32_t d = op_deg(o.deg);
    return power_range(xv, mag_pow(__builtin_fabs(xv.lo), d), mag_pow(__builtin_fabs(xv.hi), d), (d & 1u) != 0);
  }
  // interval trees are compiled without power products; this product of two
  // enclosures is still an enclosure
  static __device__ __forceinline__ Pow pair(const Pow& a, const Pow& b) { return iv_mad(a, b, 0.0, 0.0); }
};

// ----------------------------------------------------------------------------
// power tables
// ----------------------------------------------------------------------------
//
// The chain runs in double-double (the FP64 table keeps the low word as a
// float relative to the high word, lo / hi, so it cannot overflow where hi is
// large: about 77 bits), so every power is accurate to a few units in 2^-70
// before it is rounded.

constexpr int kWave = 64;

__device__ __forceinline__ float rel_lo(const DD& r) {
  return (r.h != 0.0 && isfinite(r.h)) ? (float)(r.l / r.h) : 0.f;
}

// Where the entries of a table live: the whole table lives in a per-lane
// private array (scratch memory, cached in L1/L2 and sized by the runtime
// for the resident waves), where the power chain runs once per point and
// from which the rarely used entries are read; entries 0..kRegPowers-1 (the
// most used powers, ordered so by the compiler) are copied into registers
// for the walk.  The table takes no LDS and no registers beyond those
// copies, so occupancy is set by the walk's accumulators.

// Register copies of entries 0..kRegPowers-1 (static indices) and the
// dynamic reader.
template <class E>
struct RegPow {
  E r[kRegPowers];
  template <class Get>
  __device__ __forceinline__ E any(uint32_t i, Get&& mem) const {
    switch (i) {
      case 0: return r[0];
      case 1: return r[1];
      case 2: return r[2];
      case 3: return r[3];
      default: return mem(i);
    }
  }
};

template <int CAP>
struct TabF64 {
  double pm[CAP];         // entry i at pm[i] (private)
  float pl[CAP];          // low word / high word, for the chain
  __device__ __forceinline__ void build(const DevTree& tr, const double* x, RegPow<double>& rp) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      DD r;
      if (st.kind == kChainLoad) {
        r = DD{coord(x, st.s1), 0.0};
      } else {
        const double h1 = pm[st.s1], h2 = pm[st.s2];
        r = dd_mul(DD{h1, h1 * (double)pl[st.s1]}, DD{h2, h2 * (double)pl[st.s2]});
      }
      pm[st.dst] = r.h;
      pl[st.dst] = rel_lo(r);
    }
#pragma unroll
    for (int k = 0; k < kRegPowers; ++k) rp.r[k] = k < tr.n_table ? pm[k] : 0.0;
  }
  __device__ __forceinline__ double get(uint32_t i) const { return pm[i]; }
};

// The fallback reads the powers as double-double (hi + lo).
template <int CAP>
struct TabDD {
  DD pm[CAP];             // entry i at pm[i] (private)
  __device__ __forceinline__ void build(const DevTree& tr, const double* x, RegPow<DD>& rp) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      pm[st.dst] = st.kind == kChainLoad ? DD{coord(x, st.s1), 0.0} : dd_mul(pm[st.s1], pm[st.s2]);
    }
#pragma unroll
    for (int k = 0; k < kRegPowers; ++k) rp.r[k] = k < tr.n_table ? pm[k] : DD{0.0, 0.0};
  }
  __device__ __forceinline__ DD get(uint32_t i) const { return pm[i]; }
};

template <int CAP>
struct TabM61 {
  uint64_t pm[CAP];         // entry i at pm[i] (private)
  __device__ __forceinline__ void build(const DevTree& tr, const uint64_t* x, RegPow<uint64_t>& rp) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      pm[st.dst] = st.kind == kChainLoad ? coord(x, st.s1) : m61_mul(pm[st.s1], pm[st.s2]);
    }
#pragma unroll
    for (int k = 0; k < kRegPowers; ++k) rp.r[k] = k < tr.n_table ? pm[k] : 0;
  }
  __device__ __forceinline__ uint64_t get(uint32_t i) const { return pm[i]; }
};

// Three-float powers for the double-float walk's table: the double-double
// value of the chain split into h + m + l (72 bits); the walk reads h + m.
__device__ __forceinline__ P3 split3_dd(DD r) {
  float h = (float)r.h;
  double d = (r.h - (double)h) + r.l;
  float m = (float)d;
  float l = (float)(d - (double)m);
  return P3{h, m, l};
}

template <int CAP>
struct TabP3 {
  P3 pm[CAP];             // entry i at pm[i] (private)
  __device__ __forceinline__ void build(const DevTree& tr, const double* x, RegPow<P2>& rp) {
    // the chain runs on the three-float values (h + m is exact in FP64, so
    // each product is a double-double one)
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      if (st.kind == kChainLoad) {
        pm[st.dst] = split3_dd(DD{coord(x, st.s1), 0.0});
      } else {
        const P3 a = pm[st.s1], b = pm[st.s2];
        pm[st.dst] = split3_dd(dd_mul(DD{(double)a.h + (double)a.m, (double)a.l},
                                      DD{(double)b.h + (double)b.m, (double)b.l}));
      }
    }
#pragma unroll
    for (int k = 0; k < kRegPowers; ++k) rp.r[k] = k < tr.n_table ? get(k) : P2{0.f, 0.f};
  }
  __device__ __forceinline__ P2 get(uint32_t i) const { return P2{pm[i].h, pm[i].m}; }
  __device__ __forceinline__ P3 full(uint32_t i) const { return pm[i]; }
};

// Interval tables: the chain runs on bounds of |l|^d and |h|^d (l, h the ends
// of the entry's variable), and each entry's enclosure of the range of x^d is
// formed from them as the step that makes it runs (a MUL step's kind carries
// the entry's variable and the parity of its degree).
template <int CAP>
struct TabIV {
  IV pm[CAP];             // entry i: enclosure of the range of x_var^d (private)
  IV ml[CAP], mh[CAP];    // bounds on |l|^d and |h|^d
  __device__ __forceinline__ void build(const DevTree& tr, const IV* x, RegPow<IV>& rp) {
    for (int c = 0; c < tr.n_chain; ++c) {
      const ChainStep st = tr.chain[c];
      if (!chain_is_mul(st.kind)) {
        const IV X = coord(x, st.s1);
        const double l = __builtin_fabs(X.lo), h = __builtin_fabs(X.hi);
        ml[st.dst] = IV{l, l};
        mh[st.dst] = IV{h, h};
        pm[st.dst] = X;
      } else {
        const IV a = mag_mul(ml[st.s1], ml[st.s2]), b = mag_mul(mh[st.s1], mh[st.s2]);
        ml[st.dst] = a;
        mh[st.dst] = b;
        pm[st.dst] = power_range(coord(x, chain_var(st.kind)), a, b, (st.kind & kChainOdd) != 0);
      }
    }
#pragma unroll
    for (int k = 0; k < kRegPowers; ++k) rp.r[k] = k < tr.n_table ? pm[k] : IV{0.0, 0.0};
  }
  __device__ __forceinline__ IV get(uint32_t i) const { return pm[i]; }
};

// LDS tier of the tables: entries kRegPowers .. kRegPowers+T-1 (the next
// most used after the register copies; T = tier_entries<Ar>()) of every
// point of a wavefront, stored as 32-bit planes [entry][word][point j][lane]
// so a wavefront reads 64 consecutive words (no bank conflicts).  One
// wavefront per workgroup, so a workgroup's dynamic LDS is
// walk_lds_bytes<Ar, DMAX, PPL>(): 7 KB for the double-float walk (seven
// two-float powers) at two points per lane, so that its five waves per SIMD
// (20 per compute unit) fit in 160 KB (measured on MI355X: eight entries,
// 8 KB, lost occupancy and ran slower than four).  Entries beyond the tier stay in
// private memory; the tier keeps the table's hot part out of it, whose
// working set is far beyond the caches at full occupancy.
template <class E, int PPL>
struct LdsTier {
  static constexpr int kWords = (int)(sizeof(E) / 4);
  static constexpr int kStride = PPL * kWave;
  uint32_t* base;   // the workgroup's dynamic LDS
  int col;          // j * 64 + lane is added per access
  __device__ __forceinline__ uint32_t* at(uint32_t i, int w, int j) const {
    return base + ((i - kRegPowers) * kWords + w) * kStride + j * kWave + col;
  }
  __device__ __forceinline__ void put(uint32_t i, int j, const E& v) const {
    uint32_t u[kWords];
    __builtin_memcpy(u, &v, sizeof v);
#pragma unroll
    for (int w = 0; w < kWords; ++w) *at(i, w, j) = u[w];
  }
  __device__ __forceinline__ E get(uint32_t i, int j) const {
    uint32_t u[kWords];
#pragma unroll
    for (int w = 0; w < kWords; ++w) u[w] = *at(i, w, j);
    E v;
    __builtin_memcpy(&v, u, sizeof v);
    return v;
  }
};
// Whether a kernel uses the tier: not for chain-like walks (depth <= 2, whose
// few powers all sit in registers).  (The FP64 depth-6 kernel asks for five
// waves per SIMD, which the tier's addressing would otherwise lower by one.)
template <class Ar, int DMAX>
constexpr bool lds_tier() {
  return DMAX > 2;
}
// Entries in the tier: the double-float walk's two-float powers take half the
// bytes of the double-double and interval ones, so it holds more (its op
// records are coded for that).
template <class Ar>
constexpr int tier_entries() {
  return std::is_same_v<Ar, ArDF32> ? kLdsPowersF32 : kLdsPowers;
}
template <class Ar, int DMAX, int PPL>
constexpr size_t walk_lds_bytes() {
  return lds_tier<Ar, DMAX>() ? (size_t)tier_entries<Ar>() * sizeof(typename Ar::Pow) * PPL * kWave : 0;
}

// CAP: entries a table can hold; kernels with several points per lane only
// take tables of at most kTableCapMulti entries (the launcher sends larger
// ones to the one-point kernels), which keeps their private arrays small.
template <class Ar, int CAP> struct TabFor;
template <int CAP> struct TabFor<ArF64, CAP> { using T = TabF64<CAP>; };
template <int CAP> struct TabFor<ArDD, CAP> { using T = TabDD<CAP>; };
template <int CAP> struct TabFor<ArM61, CAP> { using T = TabM61<CAP>; };
template <int CAP> struct TabFor<ArDF32, CAP> { using T = TabP3<CAP>; };
template <int CAP> struct TabFor<ArIV, CAP> { using T = TabIV<CAP>; };
template <int PPL> constexpr int table_cap() { return PPL > 1 ? kTableCapMulti : kMaxTable; }

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
  using Full = typename Ar::Full;
  using In = typename Ar::In;
  using Tab = typename TabFor<Ar, table_cap<PPL>()>::T;

  const Op* __restrict__ ops;
  const uint64_t* runc;   // run coefficients (plain FP64 chain walk)
  const In (*x)[8];   // x[j][var]: the coordinates of point j (kernel locals)
  Tab* tab;           // tab[j]: the power table of point j (private memory)
  RegPow<Pow> rp[PPL];   // rp[j]: entries 0..kRegPowers-1 of point j (registers)
  LdsTier<Pow, PPL> lt;  // entries kRegPowers.. of the LDS tier
  Acc m[DMAX][PPL];
  Acc y[PPL];
  In xv[OFFT ? PPL : 1][8];   // coordinates by value, for powers computed on the fly

  // coordinate v of point j (j is unrolled; v is wave-uniform)
  __device__ __forceinline__ In xvar(int j, uint32_t v) const {
    switch (v) {
      case 0: return xv[j][0];
      case 1: return xv[j][1];
      case 2: return xv[j][2];
      case 3: return xv[j][3];
      case 4: return xv[j][4];
      case 5: return xv[j][5];
      case 6: return xv[j][6];
      default: return xv[j][7];
    }
  }

  __device__ __forceinline__ Walker(const In (*x_)[8], Tab* t_, char* lds)
      : ops(nullptr), runc(nullptr), x(x_), tab(t_) {
    lt.base = (uint32_t*)lds;
    lt.col = (int)(threadIdx.x & (kWave - 1));
    if constexpr (OFFT) {
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
#pragma unroll
        for (int v = 0; v < 8; ++v) xv[j][v] = x_[j][v];
      }
    }
  }

#define FPE_FOR_J _Pragma("unroll") for (int j = 0; j < PPL; ++j)
  // X for point j in power class PC (see PowClass): a register entry, an
  // entry of the LDS tier (kPowMem; private without the tier) or of the
  // private table (kPowPriv), or (kPowOther) the product of two or three
  // entries / a power computed on the fly.
  // Tier and private entries read by their own loads (an LDS or a private
  // load); the plain FP64 walk keeps one read for both (a flat load from the
  // selected address), which measured 5-7 % faster for it, while the split
  // reads made the double-float walks 3-4 % faster.
  static constexpr bool kSplitMem = !std::is_same_v<Ar, ArF64>;
  template <uint32_t PC>
  __device__ __forceinline__ Pow power(const Op& o, int j) const {
    if constexpr (PC < (uint32_t)kRegPowers) {
      return rp[j].r[PC];
    } else if constexpr ((PC == kPowMem || PC == kPowPriv) && !kSplitMem) {
      return mem(j, op_pidx(o.info));
    } else if constexpr (PC == kPowMem) {
      if constexpr (lds_tier<Ar, DMAX>()) return lt.get(op_pidx(o.info), j);
      else return tab[j].get(op_pidx(o.info));
    } else if constexpr (PC == kPowPriv) {
      return tab[j].get(op_pidx(o.info));
    } else {
      const uint32_t p1 = op_pidx(o.info), p2 = op_pidx2(o.info);
      if (p2 != kNoPair) {
        const Full a = Ar::pair(full(j, p1), full(j, p2));
        if (op_deg(o.deg) & kThirdBit) return Ar::to_pow(Ar::pair(a, full(j, op_deg(o.deg) & 0xFFu)));
        return Ar::to_pow(a);
      }
      if constexpr (OFFT) return Ar::off_table(xvar(j, op_var(o.info)), o);
      return getany(j, p1);
    }
  }

  // entry i >= kRegPowers of point j's table: the LDS tier or private memory
  __device__ __forceinline__ Pow mem(int j, uint32_t i) const {
    if constexpr (lds_tier<Ar, DMAX>())
      if (i < (uint32_t)(kRegPowers + tier_entries<Ar>())) return lt.get(i, j);
    return tab[j].get(i);
  }
  // entry i of point j's table at full precision (for products of entries)
  __device__ __forceinline__ Full full(int j, uint32_t i) const {
    if constexpr (std::is_same_v<Full, Pow>) return getany(j, i);
    else return tab[j].full(i);
  }
  // entry i of point j's table, wherever it lives
  __device__ __forceinline__ Pow getany(int j, uint32_t i) const {
    return rp[j].any(i, [&](uint32_t k) { return mem(j, k); });
  }

  // One op with dispatch code C: depth L (L accumulators open, the top is
  // m[L - 1]), kind K, power class PC.
  template <uint32_t C>
  __device__ __forceinline__ void step(const Op& o) {
    constexpr int L = (int)(C & 15u);
    constexpr uint32_t K = (C >> 4) & 3u;
    constexpr uint32_t PC = C >> 6;
    if constexpr (K == kLeafOpen) {              // push a * X + b
      if constexpr (L < DMAX) {
        FPE_FOR_J { m[L][j] = Ar::fma_ab(o, power<PC>(o, j)); }
      }
    } else if constexpr (K == kLeafAdd) {         // top += a * X
      if constexpr (L >= 1 && L <= DMAX) {
        FPE_FOR_J { m[L - 1][j] = Ar::fma_ca(o, power<PC>(o, j), m[L - 1][j]); }
      }
    } else if constexpr (K == kNodeOpen) {        // top = top * X + b
      if constexpr (L >= 1 && L <= DMAX) {
        FPE_FOR_J { m[L - 1][j] = Ar::fma_tb(m[L - 1][j], power<PC>(o, j), o); }
      }
    } else {                                      // NODE_ADD: below += top * X; pop
      if constexpr (L >= 2 && L <= DMAX) {
        FPE_FOR_J { m[L - 2][j] = Ar::fma_tt(m[L - 1][j], power<PC>(o, j), m[L - 2][j]); }
      }
    }
  }

  // The root: y = (children ? m[0] : a) * X_root.
  template <uint32_t PC>
  __device__ __forceinline__ void finish(const Op& o) {
    const uint32_t info = o.info;
    FPE_FOR_J { y[j] = m[0][j]; }
    if (info & kEndLeafRoot) {
      FPE_FOR_J { y[j] = Ar::leaf_root(o); }
    }
    if (info & kEndHasPow) {
      FPE_FOR_J { y[j] = Ar::mul(y[j], power<PC>(o, j)); }
    }
  }

  // The walk: one flat loop over the ops and one switch on the op's dispatch
  // code (set by the host), whose cases carry compile-time accumulator
  // indices.
  // Waits for the outstanding scalar load of the next ops (s_waitcnt
  // lgkmcnt(0); vmcnt and expcnt left at their maxima).  Without this wait
  // after the ops that the load overlaps, the compiler would wait at the loop
  // head, right after issuing the load.
  static __device__ __forceinline__ void settle() { __builtin_amdgcn_s_waitcnt(0xC07F); }

  // A run record (kRunCode): steps top = top * X0 + c, the coefficients read
  // with scalar loads (FP64: eight at a time; double-float: four steps of
  // two words), the next group in flight while the current one is applied.
  static constexpr bool kRuns =
      (std::is_same_v<Ar, ArF64> || std::is_same_v<Ar, ArDF32> || std::is_same_v<Ar, ArDD>) && DMAX <= 2;
  __device__ __forceinline__ void run_chain(const Op& o) {
    if constexpr (std::is_same_v<Ar, ArF64>) run_chain_f64(o);
    else if constexpr (std::is_same_v<Ar, ArDD>) run_chain_dd(o);
    else run_chain_df32(o);
  }
  // double-float: o.ah, o.al carry the stream offset and the step count
  // (as bits); each step is the NODE_OPEN step with b = (b.h, b.l) and its
  // bound term from the stream (b = 0 and no bound term in a gap)
  __device__ __forceinline__ void run_chain_df32(const Op& o) {
    using CW = const __attribute__((address_space(4))) uint64_t;
    CW* __restrict__ c = (CW*)runc + (int64_t)kRunWordsF32 * __float_as_uint(o.ah);
    const int64_t K = (int64_t)__float_as_uint(o.al);
    Pow X[PPL];
    FPE_FOR_J { X[j] = rp[j].r[0]; }
    auto step = [&](uint64_t w0, uint64_t w1) {
      const float bh = __uint_as_float((uint32_t)w0), bl = __uint_as_float((uint32_t)(w0 >> 32));
      const float k2 = __uint_as_float((uint32_t)w1);
      FPE_FOR_J {
        const Acc t = m[0][j];
        m[0][j] = df_step<true, false>(t.h, t.l, t.e, t.t, X[j], bh, bl, k2, __builtin_fabsf(bh));
      }
    };
    int64_t i = 0;
    if (K >= 4) {
      uint64_t cur[8], nxt[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) cur[k] = c[k];
      settle();
#pragma unroll 1
      for (; i + 8 <= K; i += 4) {
#pragma unroll
        for (int k = 0; k < 8; ++k) nxt[k] = c[2 * (i + 4) + k];
#pragma unroll
        for (int q = 0; q < 4; ++q) step(cur[2 * q], cur[2 * q + 1]);
        settle();
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) step(cur[2 * q], cur[2 * q + 1]);
      i += 4;
    }
#pragma unroll 1
    for (; i < K; ++i) step(c[2 * i], c[2 * i + 1]);
  }
  __device__ __forceinline__ void run_chain_f64(const Op& o) {
    using CW = const __attribute__((address_space(4))) uint64_t;
    CW* __restrict__ c = (CW*)runc + o.a;
    const int64_t K = (int64_t)o.b;
    Pow X[PPL];
    FPE_FOR_J { X[j] = rp[j].r[0]; }
    auto apply = [&](const uint64_t (&cc)[8]) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double ck = u2d(cc[k]);
        FPE_FOR_J { m[0][j] = __builtin_fma(m[0][j], X[j], ck); }
      }
    };
    int64_t i = 0;
    if (K >= 8) {
      uint64_t cur[8], nxt[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) cur[k] = c[k];
      settle();
#pragma unroll 1
      for (; i + 16 <= K; i += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) nxt[k] = c[i + 8 + k];
        apply(cur);
        settle();
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
      }
      apply(cur);
      i += 8;
    }
#pragma unroll 1
    for (; i < K; ++i) {
      const double ck = u2d(c[i]);
      FPE_FOR_J { m[0][j] = __builtin_fma(m[0][j], X[j], ck); }
    }
  }

  // double-double (the compensated walk's fallback): the FP64 runs, each
  // step exactly the walk's NODE_OPEN step top = top X0 + c
  __device__ __forceinline__ void run_chain_dd(const Op& o) {
    using CW = const __attribute__((address_space(4))) uint64_t;
    CW* __restrict__ c = (CW*)runc + o.a;
    const int64_t K = (int64_t)o.b;
    Pow X[PPL];
    FPE_FOR_J { X[j] = rp[j].r[0]; }
    auto apply = [&](const uint64_t (&cc)[8]) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const DD ck{u2d(cc[k]), 0.0};
        FPE_FOR_J { m[0][j] = dd_fma<true, false>(m[0][j], X[j], ck); }
      }
    };
    int64_t i = 0;
    if (K >= 8) {
      uint64_t cur[8], nxt[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) cur[k] = c[k];
      settle();
#pragma unroll 1
      for (; i + 16 <= K; i += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) nxt[k] = c[i + 8 + k];
        apply(cur);
        settle();
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
      }
      apply(cur);
      i += 8;
    }
#pragma unroll 1
    for (; i < K; ++i) {
      const DD ck{u2d(c[i]), 0.0};
      FPE_FOR_J { m[0][j] = dd_fma<true, false>(m[0][j], X[j], ck); }
    }
  }

  // One op; true at END.
  __device__ __forceinline__ bool run_op(const Op& o) {
    if constexpr (kRuns) {
      if (op_code(o.deg) == kRunCode) {
        run_chain(o);
        return false;
      }
    }
    if constexpr (DMAX <= 2) {
      // chain-like walks (Hörner): almost every op is NODE_OPEN at depth 1
      // with the first register power; test it before the switch
      constexpr uint32_t kHot = make_code(1, kNodeOpen, 0);
      if (op_code(o.deg) == kHot) {
        step<kHot>(o);
        return false;
      }
    }
    switch (op_code(o.deg)) {
#define FPE_END(c) \
  case c: finish<((c) >> 6)>(o); return true;
#define FPE_OP(c)                                                          \
  case c:                                                                  \
    if constexpr (((c) & 15) <= DMAX) step<(c)>(o);                        \
    break;
#define FPE_L(k, p)                                                        \
  FPE_OP(1 + 16 * (k) + 64 * (p)) FPE_OP(2 + 16 * (k) + 64 * (p))          \
  FPE_OP(3 + 16 * (k) + 64 * (p)) FPE_OP(4 + 16 * (k) + 64 * (p))          \
  FPE_OP(5 + 16 * (k) + 64 * (p)) FPE_OP(6 + 16 * (k) + 64 * (p))          \
  FPE_OP(7 + 16 * (k) + 64 * (p)) FPE_OP(8 + 16 * (k) + 64 * (p))          \
  FPE_OP(9 + 16 * (k) + 64 * (p)) FPE_OP(10 + 16 * (k) + 64 * (p))         \
  FPE_OP(11 + 16 * (k) + 64 * (p)) FPE_OP(12 + 16 * (k) + 64 * (p))        \
  FPE_OP(13 + 16 * (k) + 64 * (p)) FPE_OP(14 + 16 * (k) + 64 * (p))        \
  FPE_OP(15 + 16 * (k) + 64 * (p))
#define FPE_P(p)                                                           \
  FPE_END(64 * (p)) FPE_L(0, p)                                            \
  FPE_OP(16 + 64 * (p)) FPE_L(1, p)                                        \
  FPE_OP(32 + 64 * (p)) FPE_L(2, p)                                        \
  FPE_OP(48 + 64 * (p)) FPE_L(3, p)
      FPE_P(0) FPE_P(1) FPE_P(2) FPE_P(3) FPE_P(4) FPE_P(5) FPE_P(6)
#undef FPE_P
#undef FPE_L
#undef FPE_OP
#undef FPE_END
      default:
        break;
    }
    return false;
  }

  // The next op record is loaded before the current op runs and settled
  // after it, so the load's latency overlaps the op's dispatch and
  // arithmetic.  Scalar loads may return out of order, so only a full wait is
  // safe and one load is outstanding at a time.  The FP64 walk, whose ops
  // carry one fused multiply-add per point, runs the ops in pairs: the two
  // records of the next pair come in one 64-byte load, which then has two
  // ops of arithmetic to arrive (measured 7-23 % faster).  The walks with
  // more arithmetic per op (compensated, double-double, mod p) were measured
  // slower in pairs (a second copy of the switch, more registers) and run
  // single ops.  The op arrays end with kOpTail zero records after END, so
  // the loads past END stay in bounds.
  static constexpr bool kPairs = std::is_same_v<Ar, ArF64>;
  __device__ __forceinline__ void walk() {
    // the op array is read-only while a kernel runs: reading it through the
    // constant address space keeps its loads scalar whatever the kernel
    // stores or waits on
    using CW = const __attribute__((address_space(4))) uint64_t;
    CW* __restrict__ op = (CW*)ops;
    static_assert(sizeof(Op) == 4 * sizeof(uint64_t), "op records are 32 bytes");
    auto fetch = [](CW* p) {
      uint64_t w[4] = {p[0], p[1], p[2], p[3]};
      Op r;
      __builtin_memcpy(&r, w, sizeof r);
      return r;
    };
    if constexpr (kPairs) {
      Op a = fetch(op), b = fetch(op + 4);
      settle();
#pragma unroll 1
      for (;;) {
        const Op o0 = a, o1 = b;
        op += 8;
        a = fetch(op);
        b = fetch(op + 4);
        if (run_op(o0)) return;
        if (run_op(o1)) return;
        settle();
      }
    } else {
      Op next = fetch(op);
      settle();
#pragma unroll 1
      for (;;) {
        const Op o = next;
        op += 4;
        next = fetch(op);
        if (run_op(o)) return;
        settle();
      }
    }
  }
#undef FPE_FOR_J

  __device__ __forceinline__ void run(const DevTree& tr) {
    ops = Ar::ops(tr);
    runc = std::is_same_v<Ar, ArDD> ? tr.runc64 : tr.runc;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      tab[j].build(tr, x[j], rp[j]);
      if constexpr (lds_tier<Ar, DMAX>())
        for (int i = kRegPowers; i < kRegPowers + tier_entries<Ar>() && i < tr.n_table; ++i)
          lt.put(i, j, tab[j].get(i));
    }
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
#pragma unroll
      for (int j = 0; j < PPL; ++j) m[k][j] = Acc{};
    }
    walk();
  }
};

// Evaluate PPL points of this lane (one power table each).
template <class Ar, int DMAX, int PPL, bool OFFT>
__device__ __forceinline__ void walk_points(const DevTree& tr, const typename Ar::In (*x)[8], char* lds,
                                            typename Ar::Acc* y) {
  typename TabFor<Ar, table_cap<PPL>()>::T tab[PPL];
  Walker<Ar, DMAX, PPL, OFFT> w(x, tab, lds);
  w.run(tr);
#pragma unroll
  for (int j = 0; j < PPL; ++j) y[j] = w.y[j];
}

template <class Ar, int DMAX, bool OFFT>
__device__ __forceinline__ typename Ar::Acc walk_point(const DevTree& tr, const typename Ar::In* x, char* lds) {
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
  double* bound;         // optional: the error bound the test used, per point
  double tol;
  int32_t force;
};

// The absolute part of the double-float walk's error bound at point x (the
// relative per-step terms assume normal FP32 numbers; this covers roundings
// in the subnormal range, constants split below the normal range and
// powers that underflow, carried up the tree): abs_scale times
// prod_j max(1, |x_j|)^deg_max[j], with pow's rounding covered by a
// 2^-40 margin.  A NaN coordinate gives NaN, and the point is flagged.
template <class X>
__device__ __forceinline__ double df32_abs_bound(const DevTree& tr, X&& xv) {
  double m = tr.abs_scale;
  for (int v = 0; v < tr.nvars; ++v) {
    const double a = fabs(xv(v));
    if (!(a <= 1.0) && tr.deg_max[v] > 0) m *= pow(a, (double)tr.deg_max[v]) * (1.0 + 0x1p-40);
  }
  return m;
}

// The result hi + lo in FP64 and whether it must be re-evaluated: the bound
// (running relative terms times the tree's scale, plus the absolute part
// eabs) does not certify tol relative accuracy, or a component is not
// finite.  The decision does not use the condition sum, so it is the same
// whether or not COND (the condition number p~(|x|) / |y| as output) is
// computed.
template <bool COND>
__device__ __forceinline__ bool df32_finish(const DF& r, double eabs, double tol, float scale, int force,
                                            double& y, float& cond, double& bound) {
  y = (double)r.h + (double)r.l;
  const double ay = fabs(y);
  bound = (double)r.e * (double)scale + eabs;
  const bool finite = isfinite(r.h) && isfinite(r.l) && isfinite(r.e);
  if constexpr (COND) cond = (float)((double)r.t / ay);
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
