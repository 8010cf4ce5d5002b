// Host compiler: polynomial + function scheme -> evaluation tree -> walk
// program.  Everything here runs once per polynomial ("preprocessing" before
// "subsequent fast evaluation", abstract and Section 1), on the CPU.
//
//  * terms are sorted in decreasing lexicographic order (the order <_t of
//    Section 1: index 0 is the biggest monomial, the root is last);
//  * the tree T_p^f is built by the split p = a x^{f(n)} + b of Section 1.1,
//    with T_a grafted as a child of the root of T_b, applied to each variable
//    in turn (Remark in Section 1.1), x1 outermost;
//  * partial degrees are d(N) = exp(N) - exp(parent(N));
//  * lazy heights follow Section 1.3; the walk itself uses the stack depth;
//  * the distinct powers x_j^d are planned as a chain of multiplications
//    (fast exponentiation, Section 2.2, Table 1).
//
// Readings where the paper is silent: f takes the degree n of the current
// sub-polynomial measured from its exponent origin; if b = 0 the split adds
// no node (the origin of a moves by f(n)); the balanced scheme is
// B(n) = ceil(n/2) on the degree; a nested block whose coefficient polynomial
// has no constant term gets a junction node with coefficient 0.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <unordered_map>

#include "fpe_internal.h"

namespace fpe {

namespace {

thread_local std::string g_err;

struct Scheme {
  int32_t kind;
  int32_t threshold;
  std::vector<int32_t> table;
  // f(n) for n >= 1; returns <= 0 or > n for an illegal scheme
  int64_t operator()(int64_t n) const {
    switch (kind) {
      case FPE_DIRECT: return n;
      case FPE_HORNER: return 1;
      case FPE_ESTRIN: {
        int64_t e = 1;
        while (e * 2 <= n) e *= 2;
        return e;
      }
      case FPE_BALANCED: return (n + 1) / 2;
      case FPE_BALANCED_FLOOR: return std::max<int64_t>(1, n / 2);
      case FPE_THRESHOLD: {
        if (n <= threshold) return 1;
        int64_t e = 1;
        while (e * 2 <= n) e *= 2;
        return e;
      }
      case FPE_TABLE: return n < (int64_t)table.size() ? table[n] : -1;
    }
    return -1;
  }
};

// Split a double into two floats whose sum rounds it to 48 bits.
inline void split_f32(double v, float& h, float& l) {
  h = (float)v;
  l = (float)(v - (double)h);
}

// K2 |bh| rounded up, bh = b rounded to float: the running-bound term of an
// exact constant b in one double-float step (see the double-float walk: the
// step's new error is at most u^2 (17 |p| + 4 |b|) with u = 2^-24, taken with
// constants 20 and 6).
inline float bound_term_up(double b) {
  const double v = 6.0 * std::ldexp(1.0, -48) * std::fabs((double)(float)b);   // exact in FP64
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
fpe_status fail(fpe_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
const char* last_error() { return g_err.c_str(); }

namespace {

struct Builder {
  int32_t nv;
  const std::vector<int32_t>& E;  // sorted terms x nv
  const Scheme& f;
  int64_t T;
  std::vector<int64_t> parent;    // per node id (terms 0..T-1, then junctions)
  std::vector<std::vector<int32_t>> jexps;
  std::unordered_map<int64_t, int64_t> jmemo;  // (k * T + lo) -> node id
  std::string err;

  int32_t e(int64_t t, int k) const { return E[t * nv + k]; }

  // first t in [lo, hi) with e(t, k) < v  (e(., k) is non-increasing on the range)
  int64_t first_below(int64_t lo, int64_t hi, int k, int64_t v) const {
    while (lo < hi) {
      int64_t m = lo + (hi - lo) / 2;
      if (e(m, k) < v) hi = m; else lo = m + 1;
    }
    return lo;
  }
  int64_t lowest_block(int64_t lo, int64_t hi, int k) const {
    int32_t last = e(hi - 1, k);
    // first t with e(t,k) <= last, i.e. first with e < last + 1
    return first_below(lo, hi, k, (int64_t)last + 1);
  }
  int64_t junction(int k, int64_t lo) {
    int64_t key = (int64_t)k * T + lo;
    auto it = jmemo.find(key);
    if (it != jmemo.end()) return it->second;
    std::vector<int32_t> ex(nv, 0);
    for (int j = 0; j <= k; ++j) ex[j] = e(lo, j);
    int64_t id = T + (int64_t)jexps.size();
    jexps.push_back(ex);
    parent.push_back(-1);
    jmemo[key] = id;
    return id;
  }
  // node standing for the block [lo, hi) (one value of x_k) at level k
  int64_t block_node(int k, int64_t lo, int64_t hi) {
    for (;;) {
      if (k == nv - 1) return lo;
      if (e(hi - 1, k + 1) > 0) return junction(k, lo);
      lo = lowest_block(lo, hi, k + 1);
      ++k;
    }
  }

  bool build() {
    parent.assign(T, -1);
    struct Task { int k; int64_t lo, hi, origin; };
    std::vector<Task> st;
    st.push_back({0, 0, T, 0});
    while (!st.empty()) {
      Task tk = st.back();
      st.pop_back();
      int k = tk.k;
      if (e(tk.lo, k) == e(tk.hi - 1, k)) {   // one term in x_k: one node
        if (k < nv - 1) {
          if (e(tk.hi - 1, k + 1) > 0) {
            int64_t J = junction(k, tk.lo);
            int64_t inner = block_node(k + 1, lowest_block(tk.lo, tk.hi, k + 1), tk.hi);
            parent[inner] = J;
          }
          st.push_back({k + 1, tk.lo, tk.hi, 0});
        }
        continue;
      }
      int64_t n = (int64_t)e(tk.lo, k) - tk.origin;
      int64_t s = f(n);
      if (s <= 0 || s > n) {
        err = "scheme returned f(" + std::to_string(n) + ") = " + std::to_string(s) +
              ", outside [1, n]";
        return false;
      }
      int64_t mid = first_below(tk.lo, tk.hi, k, tk.origin + s);
      if (mid == tk.hi) {                      // b = 0: p = a x^{f(n)}
        st.push_back({k, tk.lo, tk.hi, tk.origin + s});
        continue;
      }
      int64_t ra = block_node(k, lowest_block(tk.lo, mid, k), mid);
      int64_t rb = block_node(k, lowest_block(mid, tk.hi, k), tk.hi);
      parent[ra] = rb;                          // T_a under the root of T_b
      st.push_back({k, tk.lo, mid, tk.origin + s});
      st.push_back({k, mid, tk.hi, tk.origin});
    }
    return true;
  }
};

// Plan the power table and chain (fast exponentiation): every used
// (var, degree) gets a table entry; missing intermediate degrees are added by
// halving, so x^d = x^{floor(d/2)} * x^{ceil(d/2)}.
struct PowerPlan {
  std::vector<std::pair<int32_t, int32_t>> entries;  // (var, deg)
  std::vector<ChainStep> chain;
  std::map<std::pair<int32_t, int32_t>, int32_t> index;
  bool ok = true;

  int32_t ensure(int32_t var, int32_t d, int32_t cap) {
    auto key = std::make_pair(var, d);
    auto it = index.find(key);
    if (it != index.end()) return it->second;
    int32_t a = -1, b = -1;
    if (d > 1) {
      int32_t h = d / 2;
      a = ensure(var, h, cap);
      b = ensure(var, d - h, cap);
      if (a < 0 || b < 0) return -1;
    }
    if ((int32_t)entries.size() >= cap) {
      ok = false;
      return -1;
    }
    int32_t id = (int32_t)entries.size();
    entries.push_back(key);
    index[key] = id;
    if (d == 1) chain.push_back({(uint8_t)kChainLoad, (uint8_t)id, (uint8_t)var, 0});
    else chain.push_back({(uint8_t)kChainMul, (uint8_t)id, (uint8_t)a, (uint8_t)b});
    return id;
  }
};

// Pointwise walks: choose at most `cap` table powers greedily so that as many
// walk steps as possible read their power either from the table or as the
// product of two table entries.  An entry is added only when the chain can
// compute it (x itself, or the product of two entries already chosen); each
// round adds the computable power that newly covers the most steps, or, when
// none covers anything new, the next missing intermediate (halving chain) of
// the most used uncovered power.
struct CoverPlan {
  std::vector<std::pair<int32_t, int32_t>> entries;   // in chain order
  std::vector<ChainStep> chain;
  std::map<std::pair<int32_t, int32_t>, int32_t> index;

  bool has(int32_t v, int32_t d) const { return index.count({v, d}) != 0; }
  // a pair (a, b) of entries with a + b = d, or (-1, -1)
  std::pair<int32_t, int32_t> split(int32_t v, int32_t d) const {
    for (auto& e : entries) {
      if (e.first != v || e.second >= d) continue;
      auto it = index.find({v, d - e.second});
      if (it != index.end()) return {index.at(e), it->second};
    }
    return {-1, -1};
  }
  bool computable(int32_t v, int32_t d) const { return d == 1 || split(v, d).first >= 0; }
  // a triple (a, b, c) of entries with a + b + c = d, or a = -1
  std::array<int32_t, 3> split3(int32_t v, int32_t d) const {
    for (auto& e : entries) {
      if (e.first != v || e.second >= d) continue;
      auto ab = split(v, d - e.second);
      if (ab.first >= 0) return {index.at(e), ab.first, ab.second};
    }
    return {-1, -1, -1};
  }
  bool covered(int32_t v, int32_t d) const {
    return has(v, d) || split(v, d).first >= 0 || split3(v, d)[0] >= 0;
  }
  void add(int32_t v, int32_t d) {
    int32_t id = (int32_t)entries.size();
    if (d == 1) {
      chain.push_back({(uint8_t)kChainLoad, (uint8_t)id, (uint8_t)v, 0});
    } else {
      auto ab = split(v, d);
      chain.push_back({(uint8_t)kChainMul, (uint8_t)id, (uint8_t)ab.first, (uint8_t)ab.second});
    }
    entries.push_back({v, d});
    index[{v, d}] = id;
  }

  void build(const std::map<std::pair<int32_t, int32_t>, int64_t>& freq, int32_t cap) {
    // candidates: used powers and their halving intermediates
    std::set<std::pair<int32_t, int32_t>> cand;
    for (auto& kv : freq) {
      std::vector<int32_t> st{kv.first.second};
      while (!st.empty()) {
        int32_t d = st.back();
        st.pop_back();
        if (!cand.insert({kv.first.first, d}).second || d == 1) continue;
        st.push_back(d / 2);
        st.push_back(d - d / 2);
      }
    }
    while ((int32_t)entries.size() < cap) {
      // uncovered steps
      std::vector<std::pair<std::pair<int32_t, int32_t>, int64_t>> un;
      for (auto& kv : freq)
        if (!covered(kv.first.first, kv.first.second)) un.push_back(kv);
      if (un.empty()) break;
      std::pair<int32_t, int32_t> best{-1, -1};
      int64_t bestgain = 0;
      for (auto& c : cand) {
        if (has(c.first, c.second) || !computable(c.first, c.second)) continue;
        int64_t gain = 0;
        for (auto& u : un) {
          if (u.first.first != c.first) continue;
          const int32_t d = u.first.second;
          if (d == c.second || (d > c.second && (has(c.first, d - c.second) || d - c.second == c.second)))
            gain += u.second;
        }
        if (gain > bestgain || (gain == bestgain && gain > 0 && c.second < best.second)) {
          bestgain = gain;
          best = c;
        }
      }
      if (bestgain == 0) {
        // build towards the most used uncovered power along its halving chain
        auto top = *std::max_element(un.begin(), un.end(),
                                     [](auto& a, auto& b) { return a.second < b.second; });
        const int32_t v = top.first.first;
        int32_t d = top.first.second;
        // descend to the first computable missing intermediate
        for (;;) {
          if (!has(v, d) && computable(v, d)) break;
          int32_t h = d - d / 2;   // the larger half
          if (!has(v, h)) d = h;
          else if (!has(v, d / 2)) d = d / 2;
          else break;
        }
        if (has(v, d) || !computable(v, d)) break;
        best = {v, d};
      }
      add(best.first, best.second);
    }
    // room left: turn the most used products into direct entries
    while ((int32_t)entries.size() < cap) {
      std::pair<int32_t, int32_t> best{-1, -1};
      int64_t bf = 0;
      for (auto& kv : freq)
        if (!has(kv.first.first, kv.first.second) && computable(kv.first.first, kv.first.second) &&
            kv.second > bf) {
          bf = kv.second;
          best = kv.first;
        }
      if (bf == 0) break;
      add(best.first, best.second);
    }
  }
};

}  // namespace

fpe_status compile_tree(int32_t nvars, int64_t nterms, const int32_t* exps, const void* coeffs,
                        int64_t batch, int32_t domain, uint64_t modulus, const fpe_scheme* fs,
                        fpe_tree** out) {
  if (!out) return fail(FPE_EINVAL, "out is NULL");
  *out = nullptr;
  if (nvars < 1 || nvars > 8) return fail(FPE_EINVAL, "nvars must be in 1..8");
  if (nterms < 1) return fail(FPE_EINVAL, "nterms must be >= 1");
  if (!exps || !coeffs || !fs) return fail(FPE_EINVAL, "NULL exps, coeffs or scheme");
  if (domain != FPE_F64 && domain != FPE_F32C && domain != FPE_MODP && domain != FPE_IVAL &&
      domain != FPE_BIGINT)
    return fail(FPE_EINVAL, "unknown domain");
  if (domain == FPE_BIGINT && nvars != 1) return fail(FPE_EUNSUPPORTED, "big-integer evaluation is univariate");
  // integer coefficients (uint64): residues mod p, or the big-integer walk's
  const bool intcoef = domain == FPE_MODP || domain == FPE_BIGINT;
  if (batch < 1) return fail(FPE_EINVAL, "batch must be >= 1");
  if (domain != FPE_MODP && batch != 1) return fail(FPE_EINVAL, "batch > 1 needs FPE_MODP");
  if (domain == FPE_MODP && modulus != kP61 && modulus != kP31)
    return fail(FPE_EUNSUPPORTED, "modulus must be 2^61-1 or 2^31-1");
  if (domain == FPE_MODP && batch > 1 && modulus != kP31)
    return fail(FPE_EINVAL, "a batch of polynomials is compiled for composition mod 2^31-1");
  Scheme f{fs->kind, fs->threshold, {}};
  if (fs->kind < FPE_DIRECT || fs->kind > FPE_TABLE) return fail(FPE_EINVAL, "unknown scheme");
  if (fs->kind == FPE_TABLE) {
    if (!fs->table || fs->table_len < 2) return fail(FPE_EINVAL, "scheme table is empty");
    f.table.assign(fs->table, fs->table + fs->table_len);
    for (int32_t n = 1; n < fs->table_len; ++n)
      if (f.table[n] < 1 || f.table[n] > n)
        return fail(FPE_EINVAL, "scheme table entry f(" + std::to_string(n) + ") outside [1, n]");
  }

  // ---- validate and keep the nonzero terms
  const double* cf = (const double*)coeffs;
  const uint64_t* cu = (const uint64_t*)coeffs;
  std::vector<int64_t> keep;
  keep.reserve(nterms);
  for (int64_t t = 0; t < nterms; ++t) {
    for (int j = 0; j < nvars; ++j) {
      int32_t v = exps[t * nvars + j];
      if (v < 0 || v >= (1 << 20)) return fail(FPE_EINVAL, "exponent outside [0, 2^20)");
    }
    bool nz = false;
    if (domain == FPE_MODP) {
      for (int64_t r = 0; r < batch; ++r) {
        uint64_t c = cu[r * nterms + t];
        if (c >= modulus) return fail(FPE_EINVAL, "residue >= modulus");
        nz |= c != 0;
      }
    } else if (domain == FPE_BIGINT) {
      nz = cu[t] != 0;
    } else {
      if (!std::isfinite(cf[t])) return fail(FPE_EINVAL, "non-finite coefficient");
      nz = cf[t] != 0.0;
    }
    if (nz) keep.push_back(t);
  }
  if (keep.empty()) return fail(FPE_EINVAL, "the polynomial is zero");

  // ---- order <_t: decreasing lexicographic order of the monomials
  std::sort(keep.begin(), keep.end(), [&](int64_t x, int64_t y) {
    for (int j = 0; j < nvars; ++j) {
      int32_t a = exps[x * nvars + j], b = exps[y * nvars + j];
      if (a != b) return a > b;
    }
    return x < y;
  });
  int64_t T = (int64_t)keep.size();
  std::vector<int32_t> E(T * nvars);
  for (int64_t t = 0; t < T; ++t)
    for (int j = 0; j < nvars; ++j) E[t * nvars + j] = exps[keep[t] * nvars + j];
  for (int64_t t = 1; t < T; ++t)
    if (std::memcmp(&E[(t - 1) * nvars], &E[t * nvars], sizeof(int32_t) * nvars) == 0)
      return fail(FPE_EINVAL, "duplicate monomial");

  // ---- tree
  Builder B{nvars, E, f, T, {}, {}, {}, {}};
  if (!B.build()) return fail(FPE_EINVAL, B.err);
  int64_t N = T + (int64_t)B.jexps.size();
  auto ex_of = [&](int64_t id) -> const int32_t* {
    return id < T ? &E[id * nvars] : B.jexps[id - T].data();
  };
  std::vector<int64_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    const int32_t* a = ex_of(x);
    const int32_t* b = ex_of(y);
    for (int j = 0; j < nvars; ++j)
      if (a[j] != b[j]) return a[j] > b[j];
    return false;
  });
  std::vector<int64_t> pos(N);
  for (int64_t i = 0; i < N; ++i) pos[order[i]] = i;

  auto* t = new fpe_tree();
  t->nvars = nvars;
  t->domain = domain;
  t->modulus = domain == FPE_MODP ? modulus : 0;
  t->batch = batch;
  t->n_terms = T;
  t->nodes.resize(N);
  t->exps.resize(N * nvars);
  std::vector<int64_t> par(N, -1);
  int64_t roots = 0;
  for (int64_t i = 0; i < N; ++i) {
    int64_t id = order[i];
    std::memcpy(&t->exps[i * nvars], ex_of(id), sizeof(int32_t) * nvars);
    par[i] = B.parent[id] < 0 ? -1 : pos[B.parent[id]];
    roots += par[i] < 0;
  }
  if (roots != 1 || par[N - 1] != -1) {
    delete t;
    return fail(FPE_EINVAL, "internal: the tree does not have the root last");
  }
  std::vector<std::vector<int32_t>> ch(N);
  for (int64_t i = 0; i < N - 1; ++i) {
    if (par[i] <= i) {
      delete t;
      return fail(FPE_EINVAL, "internal: <_t is not topological");
    }
    ch[par[i]].push_back((int32_t)i);   // ascending index = C_1 first
  }

  // coefficients in node order (junctions 0)
  std::vector<double> cnode(N, 0.0);
  if (intcoef) t->coef_rows.assign(batch * N, 0);
  for (int64_t id = 0; id < T; ++id) {
    int64_t i = pos[id];
    if (intcoef) {
      for (int64_t r = 0; r < batch; ++r) t->coef_rows[r * N + i] = cu[r * nterms + keep[id]];
    } else {
      cnode[i] = cf[keep[id]];
    }
  }

  // ---- node array: partial degrees, flags, slots, lazy heights, subtrees
  std::vector<int32_t> H(N, 0), lh(N, 0), slot(N, 0);
  std::vector<int64_t> sub(N);
  for (int64_t i = 0; i < N; ++i) {
    fpe_node& nd = t->nodes[i];
    std::memset(&nd, 0, sizeof nd);
    if (intcoef) nd.coef.u = t->coef_rows[i];
    else nd.coef.f = cnode[i];
    nd.parent = (int32_t)par[i];
    const int32_t* me = &t->exps[i * nvars];
    int nz = 0;
    for (int j = 0; j < nvars; ++j) {
      int32_t d = me[j] - (par[i] >= 0 ? t->exps[par[i] * nvars + j] : 0);
      if (d < 0) {
        delete t;
        return fail(FPE_EINVAL, "internal: negative partial degree");
      }
      if (d) {
        ++nz;
        nd.var = (uint8_t)j;
        nd.pdeg = d;
      }
    }
    if (nz > 1 || (par[i] >= 0 && nz == 0)) {
      delete t;
      return fail(FPE_EINVAL, "internal: partial degree with more than one variable");
    }
    if (ch[i].empty()) nd.flags |= FPE_NODE_LEAF;
    if (order[i] >= T) nd.flags |= FPE_NODE_JUNCTION;
    if (par[i] < 0) nd.flags |= FPE_NODE_ROOT;
    else if (ch[par[i]].front() == i) nd.flags |= FPE_NODE_FIRST_CHILD;
    sub[i] = i;
    for (int32_t c : ch[i]) sub[i] = std::min(sub[i], sub[c]);
    if (ch[i].size() >= 2) {
      int32_t mh = 0, ml = 0;
      for (size_t k = 1; k < ch[i].size(); ++k) {
        mh = std::max(mh, H[ch[i][k]]);
        ml = std::max(ml, lh[ch[i][k]]);
      }
      slot[i] = 1 + mh;
      lh[i] = 1 + ml;
    }
    H[i] = slot[i];
    for (int32_t c : ch[i]) H[i] = std::max(H[i], H[c]);
    nd.slot = (uint8_t)std::min(slot[i], 255);
    nd.lazy_height = (uint8_t)std::min(lh[i], 255);
    nd.sub_begin = (int32_t)sub[i];
    t->max_slot = std::max(t->max_slot, slot[i]);
    t->max_lh = std::max(t->max_lh, lh[i]);
  }
  // subtrees are contiguous ranges [sub_begin, i]
  for (int64_t i = 0; i < N; ++i) {
    int64_t cnt = 1;
    for (int32_t c : ch[i]) cnt += (c - sub[c] + 1);
    if (cnt != i - sub[i] + 1) {
      delete t;
      return fail(FPE_EINVAL, "internal: subtree is not contiguous");
    }
  }

  // ---- power usage
  std::map<std::pair<int32_t, int32_t>, int64_t> freq;
  for (int64_t i = 0; i < N; ++i) {
    const fpe_node& nd = t->nodes[i];
    if (nd.pdeg > 0) freq[{nd.var, nd.pdeg}] += 1;
  }
  t->n_powers = (int32_t)freq.size();
  std::vector<std::pair<int64_t, std::pair<int32_t, int32_t>>> byf;
  for (auto& kv : freq) byf.push_back({kv.second, kv.first});
  std::stable_sort(byf.begin(), byf.end(), [](auto& a, auto& b) { return a.first > b.first; });
  // The table holds the most used powers and the chain temporaries they
  // need, within a cap; a power left out is read as the product of two (or
  // three) entries when its degree is such a sum, else computed on the fly.
  // The per-point table lives in private memory and only its first entries
  // in registers, so a larger table costs little: the smallest of 16, 24,
  // 32, 48 entries is taken that covers every power with at most 1 in 64
  // walk steps reading a product.  A batch tree (composition) keeps its coefficients per
  // instance, so its ops carry node indices instead of coefficient values,
  // and its table may hold up to 48 entries without products.  So does an
  // interval tree: the product of two power enclosures is wider than the
  // range of the power when the interval contains 0, so its powers come only
  // from the table or, beyond it, are computed on the fly from the bounds.
  const bool index_ops = domain == FPE_MODP && modulus == kP31;
  const bool no_products = index_ops || domain == FPE_IVAL || domain == FPE_BIGINT;
  const int32_t cap = no_products ? kMaxTable : kTableCap;
  PowerPlan plan;
  if (no_products) {
    for (size_t k = 0; k < byf.size(); ++k) {
      PowerPlan tmp = plan;
      tmp.ensure(byf[k].second.first, byf[k].second.second, cap);
      if (tmp.ok) plan = std::move(tmp);
    }
  } else {
    std::map<std::pair<int32_t, int32_t>, int64_t> fr(freq.begin(), freq.end());
    int64_t nsteps = 0;
    for (auto& kv : fr) nsteps += kv.second;
    for (int32_t c : {16, 24, 32, kMaxTable}) {
      CoverPlan cp;
      cp.build(fr, c);
      int64_t missing = 0, products = 0;
      for (auto& kv : fr) {
        if (!cp.covered(kv.first.first, kv.first.second)) missing += kv.second;
        else if (!cp.index.count(kv.first)) products += kv.second;
      }
      plan.entries = cp.entries;
      plan.chain = cp.chain;
      plan.index = cp.index;
      if (missing == 0 && products * 64 <= nsteps) break;
    }
  }
  std::vector<std::pair<int32_t, int32_t>> pending;
  for (auto& kv : freq)
    if (!plan.index.count(kv.first)) pending.push_back(kv.first);
  // renumber: used entries by frequency first, chain temporaries after
  std::vector<int32_t> rank(plan.entries.size(), -1);
  int32_t nr = 0;
  for (size_t k = 0; k < byf.size(); ++k) {
    auto it = plan.index.find(byf[k].second);
    if (it != plan.index.end() && rank[it->second] < 0) rank[it->second] = nr++;
  }
  for (size_t id = 0; id < plan.entries.size(); ++id)
    if (rank[id] < 0) rank[id] = nr++;
  t->n_table = (int32_t)plan.entries.size();
  t->table_var.assign(t->n_table, 0);
  t->table_deg.assign(t->n_table, 0);
  for (size_t id = 0; id < plan.entries.size(); ++id) {
    t->table_var[rank[id]] = plan.entries[id].first;
    t->table_deg[rank[id]] = plan.entries[id].second;
  }
  for (auto s : plan.chain) {
    ChainStep c = s;
    c.dst = (uint8_t)rank[s.dst];
    if (s.kind == kChainMul) {
      c.s1 = (uint8_t)rank[s.s1];
      c.s2 = (uint8_t)rank[s.s2];
      const auto& en = plan.entries[s.dst];
      c.kind = (uint8_t)(kChainMul | ((en.second & 1) ? kChainOdd : 0u) | ((uint32_t)en.first << 4));
    }
    t->chain.push_back(c);
  }
  // pending powers: the product of two (or three) table entries of the same
  // variable
  std::map<std::pair<int32_t, int32_t>, std::array<uint32_t, 3>> pairs;
  if (!no_products) {
    auto find = [&](int32_t v, int32_t d) -> int32_t {
      auto it = plan.index.find({v, d});
      return it == plan.index.end() ? -1 : rank[it->second];
    };
    for (auto& pw : pending) {
      bool done = false;
      for (int32_t e = 0; e < t->n_table && !done; ++e) {
        if (t->table_var[e] != pw.first || t->table_deg[e] >= pw.second) continue;
        const int32_t f = find(pw.first, pw.second - t->table_deg[e]);
        if (f >= 0) {
          pairs[pw] = {(uint32_t)e, (uint32_t)f, kNoPair};
          done = true;
        }
      }
      for (int32_t e = 0; e < t->n_table && !done; ++e) {
        if (t->table_var[e] != pw.first || t->table_deg[e] >= pw.second) continue;
        for (int32_t g = 0; g < t->n_table && !done; ++g) {
          if (t->table_var[g] != pw.first || t->table_deg[e] + t->table_deg[g] >= pw.second) continue;
          const int32_t f = find(pw.first, pw.second - t->table_deg[e] - t->table_deg[g]);
          if (f >= 0) {
            pairs[pw] = {(uint32_t)e, (uint32_t)g, (uint32_t)f};
            done = true;
          }
        }
      }
    }
  }
  auto pidx_of = [&](const fpe_node& nd, uint32_t& p2, uint32_t& p3) -> uint32_t {
    p2 = kNoPair;
    p3 = kNoPair;
    auto it = plan.index.find({nd.var, nd.pdeg});
    if (it != plan.index.end()) return (uint32_t)rank[it->second];
    auto jt = pairs.find({nd.var, nd.pdeg});
    if (jt != pairs.end()) {
      p2 = jt->second[1];
      p3 = jt->second[2];
      return jt->second[0];
    }
    return kOffTable;
  };

  // ---- walk program (stack form of the walk of Section 2.1)
  auto bits = [&](int64_t i) -> uint64_t {
    if (index_ops) return (uint64_t)i;
    if (intcoef) return t->coef_rows[i];
    uint64_t u;
    std::memcpy(&u, &cnode[i], 8);
    return u;
  };
  int32_t depth = 0, maxd = 0;
  t->ops64.reserve(N);
  for (int64_t i = 0; i < N; ++i) {
    const fpe_node& nd = t->nodes[i];
    OpF64 op{};
    uint32_t pidx2 = kNoPair, pidx3 = kNoPair;
    uint32_t pidx = nd.pdeg > 0 ? pidx_of(nd, pidx2, pidx3) : kOffTable;
    if (nd.pdeg > 0 && pidx == kOffTable) t->n_offtable++;
    if (pidx2 != kNoPair) t->n_pairs++;
    uint32_t info = (pidx << 8) | ((uint32_t)nd.var << 16) | ((uint32_t)std::min(depth, 31) << 20) |
                    (pidx2 << 25);
    // deg: the partial degree (used on the fly), or a third table index
    op.deg = pidx3 != kNoPair ? (kThirdBit | pidx3) : (uint32_t)nd.pdeg;
    if (par[i] < 0) {
      info |= kEnd | kBitEnd;
      if (ch[i].empty()) {
        info |= kEndLeafRoot;
        op.a = bits(i);
      }
      if (nd.pdeg > 0) info |= kEndHasPow;
      if (depth != (ch[i].empty() ? 0 : 1)) {
        delete t;
        return fail(FPE_EINVAL, "internal: walk stack unbalanced at the root");
      }
    } else {
      bool leaf = ch[i].empty();
      bool first = (nd.flags & FPE_NODE_FIRST_CHILD) != 0;
      if (leaf && first) {
        info |= kLeafOpen | kBitLeaf | kBitFirst;
        op.a = bits(i);
        op.b = bits(par[i]);
        ++depth;
      } else if (leaf) {
        info |= kLeafAdd | kBitLeaf;
        op.a = bits(i);
      } else if (first) {
        info |= kNodeOpen | kBitFirst;
        op.b = bits(par[i]);
      } else {
        info |= kNodeAdd;
        --depth;
      }
      maxd = std::max(maxd, depth);
    }
    op.info = info;
    t->n_kind[op_kind(info)]++;
    // dispatch code: depth before the op, kind, power class (END: depth 0, kind 0)
    op.deg = (op.deg & 0xFFFFFu) | (dispatch_code(info) << 20);
    t->ops64.push_back(op);
  }
  t->depth = std::max(maxd, 1);
  if (domain == FPE_F32C) {
    t->ops32.resize(N);
    for (int64_t i = 0; i < N; ++i) {
      const OpF64& o = t->ops64[i];
      OpF32 q{};
      double a, b;
      std::memcpy(&a, &o.a, 8);
      std::memcpy(&b, &o.b, 8);
      split_f32(a, q.ah, q.al);
      split_f32(b, q.bh, q.bl);
      q.bk2 = bound_term_up(b);
      q.info = o.info;
      q.deg = (o.deg & 0xFFFFFu) | (dispatch_code(o.info, kLdsPowersF32) << 20);
      t->ops32[i] = q;
    }
  }
  *out = t;
  return FPE_OK;
}

}  // namespace fpe
