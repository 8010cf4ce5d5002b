/* Plain C oracle (test infrastructure only).
 *
 * The plain definitions from the paper, written out for full-size samples and
 * for the timed CPU baseline.  Compiled with -O2 -fno-fast-math
 * -ffp-contract=off so that no FMA is formed unless fma() is called.
 *
 *  orc_horner_f64    textbook Hörner over the dense coefficient vector, with
 *                    or without a fused multiply-add (Hörner scheme H(k) = 1,
 *                    Section 1.1).
 *  orc_dd_horner     double-double Hörner (TwoProd by fma, TwoSum by Knuth):
 *                    the definition sum c_m x^m to about 2n 2^-104 ptilde.
 *  orc_ptilde        sum |c_m| |x|^m.
 *  orc_modp_eval     sum_m c_m prod_j x_j^{m_j} mod p for p < 2^63, with
 *                    unsigned __int128 products (the definition, term by term).
 *  orc_compose_modp  p(q(x)) mod p by schoolbook Hörner expansion.
 *
 * Parallel over points / instances with OpenMP when built with -fopenmp.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void orc_horner_f64(const double* c, int64_t deg, const double* x, int64_t npts,
                    double* y, int use_fma) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npts; ++i) {
    double xi = x[i];
    double acc = c[deg];
    if (use_fma) {
      for (int64_t k = deg - 1; k >= 0; --k) acc = fma(acc, xi, c[k]);
    } else {
      for (int64_t k = deg - 1; k >= 0; --k) acc = acc * xi + c[k];
    }
    y[i] = acc;
  }
}

static inline void two_sum(double a, double b, double* s, double* e) {
  double ss = a + b;
  double bb = ss - a;
  *e = (a - (ss - bb)) + (b - bb);
  *s = ss;
}

static inline void fast_two_sum(double a, double b, double* s, double* e) {
  double ss = a + b;
  *e = b - (ss - a);
  *s = ss;
}

void orc_dd_horner(const double* c, int64_t deg, const double* x, int64_t npts,
                   double* yhi, double* ylo) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npts; ++i) {
    double xi = x[i];
    double hi = c[deg], lo = 0.0;
    for (int64_t k = deg - 1; k >= 0; --k) {
      /* (hi, lo) * xi */
      double p = hi * xi;
      double pe = fma(hi, xi, -p);
      pe = pe + lo * xi;
      double s, e;
      fast_two_sum(p, pe, &s, &e);
      /* + c[k] */
      double t, te;
      two_sum(s, c[k], &t, &te);
      te = te + e;
      fast_two_sum(t, te, &hi, &lo);
    }
    yhi[i] = hi;
    ylo[i] = lo;
  }
}

void orc_ptilde(const double* c, int64_t deg, const double* x, int64_t npts, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npts; ++i) {
    double ax = fabs(x[i]);
    double acc = fabs(c[deg]);
    for (int64_t k = deg - 1; k >= 0; --k) acc = acc * ax + fabs(c[k]);
    y[i] = acc;
  }
}

static inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) {
  return (uint64_t)(((unsigned __int128)a * b) % p);
}

static uint64_t powmod(uint64_t b, int64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  b %= p;
  while (e > 0) {
    if (e & 1) r = mulmod(r, b, p);
    b = mulmod(b, b, p);
    e >>= 1;
  }
  return r;
}

/* exps: nterms x nvars row-major; pts: nvars x npts (SoA) */
void orc_modp_eval(int32_t nvars, int64_t nterms, const int32_t* exps, const uint64_t* coeffs,
                   uint64_t p, const uint64_t* pts, int64_t npts, uint64_t* out) {
  int32_t maxe = 0;
  for (int64_t t = 0; t < nterms * nvars; ++t)
    if (exps[t] > maxe) maxe = exps[t];
#pragma omp parallel
  {
    uint64_t* tab = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nvars * (size_t)(maxe + 1));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
      for (int32_t j = 0; j < nvars; ++j) {
        uint64_t xj = pts[(int64_t)j * npts + i] % p;
        for (int32_t e = 0; e <= maxe; ++e) tab[j * (maxe + 1) + e] = powmod(xj, e, p);
      }
      uint64_t acc = 0;
      for (int64_t t = 0; t < nterms; ++t) {
        uint64_t v = coeffs[t] % p;
        for (int32_t j = 0; j < nvars; ++j) v = mulmod(v, tab[j * (maxe + 1) + exps[t * nvars + j]], p);
        acc = (uint64_t)(((unsigned __int128)acc + v) % p);
      }
      out[i] = acc;
    }
    free(tab);
  }
}

/* p: batch x (dp+1), q: batch x (dq+1), out: batch x (dp*dq+1); values mod p < 2^32 */
void orc_compose_modp(const uint32_t* pc, int32_t dp, const uint32_t* qc, int32_t dq,
                      int64_t batch, uint64_t p, uint32_t* out) {
  int64_t dout = (int64_t)dp * dq + 1;
#pragma omp parallel
  {
    uint64_t* r = (uint64_t*)calloc((size_t)dout, sizeof(uint64_t));
    uint64_t* t = (uint64_t*)calloc((size_t)dout, sizeof(uint64_t));
#pragma omp for schedule(static)
    for (int64_t b = 0; b < batch; ++b) {
      const uint32_t* P = pc + b * (dp + 1);
      const uint32_t* Q = qc + b * (dq + 1);
      int64_t len = 1;
      r[0] = P[dp] % p;
      for (int32_t k = dp - 1; k >= 0; --k) {
        /* r <- r * q + P[k] */
        int64_t nlen = len + dq;
        memset(t, 0, sizeof(uint64_t) * (size_t)nlen);
        for (int64_t i = 0; i < len; ++i)
          for (int32_t j = 0; j <= dq; ++j) t[i + j] = (t[i + j] + r[i] * (uint64_t)(Q[j] % p)) % p;
        t[0] = (t[0] + P[k]) % p;
        memcpy(r, t, sizeof(uint64_t) * (size_t)nlen);
        len = nlen;
      }
      for (int64_t i = 0; i < dout; ++i) out[b * dout + i] = (uint32_t)(i < len ? r[i] : 0);
    }
    free(r);
    free(t);
  }
}
