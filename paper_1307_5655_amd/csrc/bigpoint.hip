// Exact evaluation at one big natural number x (the setting of the
// Benchmarks section, Figure 1: one polynomial, one large point, the time
// dominated by the products at the top of the tree).
//
// The tree is walked level by level from its definition (Section 1):
// u(N) = c(N) + sum over the children C of u(C) x^{d(C)}, and p(x) =
// u(R) x^{d(R)} at the root R.  The nodes of one height are independent
// (the parallelism of the divide-and-conquer schemes that Section 2.3
// exploits with threads), so each level is one set of batched launches over
// all of its products: the powers x^d come first, by the tree's
// multiplication chain (Section 2.2), level by level too.  Values are arrays
// of 16-bit limbs (least significant first).  A product of two values is
// their exact convolution: by number-theoretic transforms modulo two primes
// below 2^31 (one workgroup per operand and prime, the row in LDS) and
// Garner's recombination (a convolution value is below 2^14 * 2^32 = 2^46
// < p1 p2), or, when one operand has fewer than 64 limbs, by a schoolbook
// kernel.  A node's value is then the sum of its children's convolutions and
// its coefficient, normalised to limbs by one workgroup: each 64-bit sum is
// split into 16-bit pieces that are added back at their positions (values
// below 2^16 + 3), and the remaining single carries are resolved by a
// carry-lookahead prefix over the workgroup (generate: a limb of at least
// 2^16; propagate: a limb of exactly 2^16 - 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fpe_internal.h"
#include "ntt_core.h"

namespace fpe {
namespace {

constexpr int kBigPrimes = 2;
constexpr int kSchoolMax = 64;   // a product whose shorter operand is shorter goes to the schoolbook kernel
constexpr int kCarryThreads = 1024;
constexpr int kCarryTable = 15360;   // digit sums t_k a carry workgroup keeps in LDS (60 KB)

// Where a limb array lives: the workspace, the caller's point, or the
// caller's output (the job lists hold offsets, so they depend only on the
// tree and the point's length).
enum Space : int32_t { kWs = 0, kX = 1, kOut = 2 };
struct Ref {
  int32_t space;
  int32_t pad;
  int64_t off;   // in 32-bit words
};
struct Bases {
  uint32_t* p[3];
};
__device__ __forceinline__ uint32_t* at(const Bases& B, const Ref& r) { return B.p[r.space] + r.off; }

struct Job {          // one product a * b, its exact convolution into conv (la + lb - 1 values)
  Ref a, b;
  int64_t conv;       // offset of the uint64 convolution in the workspace (in 64-bit words)
  int64_t scratch;    // offset of the transforms (words): kBigPrimes * 2 * 2^logn
  int32_t la, lb;
  int32_t logn;       // 0: schoolbook
  int32_t pad;
};
struct Parent {       // out = sum of the convolutions of jobs [job_begin, job_end) + coef
  Ref out;
  uint64_t coef;
  int32_t job_begin, job_end;
  int32_t len;        // limbs written (an upper bound of the value's length; zeros above)
  int32_t pad;
};
struct Scales2 {
  uint32_t s[kBigPrimes][kNttLogMax + 1];   // n^-1 R^2 mod p for n = 2^logn
};

__global__ __launch_bounds__(kNttThreads) void k_job_fwd(const Job* __restrict__ jobs, Bases B,
                                                         const uint32_t* __restrict__ tw_all,
                                                         uint32_t* __restrict__ ws) {
  extern __shared__ uint32_t x[];
  const Job J = jobs[blockIdx.x];
  if (J.logn == 0) return;
  const int prime = blockIdx.y, operand = blockIdx.z;
  const NttPrime P = kPrimes[prime];
  const uint32_t* tw = tw_all + (size_t)prime * kNttMax;
  const int logn = J.logn, n = 1 << logn;
  const uint32_t* s = operand ? at(B, J.b) : at(B, J.a);
  const int len = operand ? J.lb : J.la;
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = i < len ? s[i] : 0u;   // limbs < 2^16 < p
  __syncthreads();
  for (int lh = logn - 1; lh >= 0; --lh) {
    const int h = 1 << lh;
    const int tstep = kNttLogMax - 1 - lh;
    for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
      const int j = b & (h - 1);
      const int i0 = ((b >> lh) << (lh + 1)) + j, i1 = i0 + h;
      const uint32_t u = x[i0], v = x[i1];
      x[i0] = madd(u, v, P.p);
      x[i1] = mmul(msub(u, v, P.p), tw[j << tstep], P.p, P.pinv);
    }
    __syncthreads();
  }
  uint32_t* d = ws + J.scratch + (size_t)(operand * kBigPrimes + prime) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = x[i];
}

__global__ __launch_bounds__(kNttThreads) void k_job_mul_inv(const Job* __restrict__ jobs, Scales2 sc,
                                                             const uint32_t* __restrict__ tw_all,
                                                             uint32_t* __restrict__ ws) {
  extern __shared__ uint32_t x[];
  const Job J = jobs[blockIdx.x];
  if (J.logn == 0) return;
  const int prime = blockIdx.y;
  const NttPrime P = kPrimes[prime];
  const uint32_t* twi = tw_all + (size_t)prime * kNttMax + kNttMax / 2;
  const int logn = J.logn, n = 1 << logn;
  uint32_t* A = ws + J.scratch + (size_t)prime * n;
  const uint32_t* Bt = ws + J.scratch + (size_t)(kBigPrimes + prime) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = mmul(A[i], Bt[i], P.p, P.pinv);
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
  const uint32_t scale = sc.s[prime][logn];
  for (int i = threadIdx.x; i < n; i += blockDim.x) A[i] = mmul(x[i], scale, P.p, P.pinv);
}

// The exact convolution of every job: Garner's recombination of the two
// residues (transform jobs), or the schoolbook sums.
__global__ void k_job_finish(const Job* __restrict__ jobs, Bases B, uint32_t* __restrict__ ws, uint32_t inv12) {
  const Job J = jobs[blockIdx.y];
  const int lp = J.la + J.lb - 1;
  uint64_t* conv = (uint64_t*)ws + J.conv;
  if (J.logn) {
    const NttPrime P1 = kPrimes[0], P2 = kPrimes[1];
    const int n = 1 << J.logn;
    const uint32_t* r1 = ws + J.scratch;
    const uint32_t* r2 = ws + J.scratch + n;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < lp; k += gridDim.x * blockDim.x) {
      const uint32_t a1 = r1[k], a2 = r2[k];
      const uint32_t a1m = a1 >= P2.p ? a1 - P2.p : a1;
      const uint32_t t1 = mmul(msub(a2, a1m, P2.p), inv12, P2.p, P2.pinv);
      conv[k] = (uint64_t)a1 + (uint64_t)P1.p * t1;
    }
  } else {
    const uint32_t* a = at(B, J.a);
    const uint32_t* b = at(B, J.b);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < lp; k += gridDim.x * blockDim.x) {
      const int i0 = k - (J.lb - 1) > 0 ? k - (J.lb - 1) : 0, i1 = k < J.la - 1 ? k : J.la - 1;
      uint64_t acc = 0;
      for (int i = i0; i <= i1; ++i) acc += (uint64_t)a[i] * b[k - i];
      conv[k] = acc;
    }
  }
}

// The 64-bit sum at limb position k of a parent: its children's
// convolutions and its coefficient.
__device__ __forceinline__ uint64_t psum(const Parent& Pa, const Job* jobs, const uint32_t* ws, int64_t k) {
  if (k < 0) return 0;
  uint64_t s = k < 4 ? (Pa.coef >> (16 * k)) & 0xFFFFu : 0;
  for (int j = Pa.job_begin; j < Pa.job_end; ++j) {
    const Job& J = jobs[j];
    if (k < J.la + J.lb - 1) s += ((const uint64_t*)ws)[J.conv + k];
  }
  return s;
}
// t_k: the 16-bit pieces of the sums added at their positions (< 2^18)
__device__ __forceinline__ uint32_t tsum(const Parent& Pa, const Job* jobs, const uint32_t* ws, int64_t k) {
  uint64_t t = 0;
  for (int j = 0; j < 4; ++j) t += (psum(Pa, jobs, ws, k - j) >> (16 * j)) & 0xFFFFu;
  return (uint32_t)t;
}
// u_k = low 16 bits of t_k plus the high part of t_{k-1}: at most 2^16 + 2
__device__ __forceinline__ uint32_t usum(const Parent& Pa, const Job* jobs, const uint32_t* ws, int64_t k) {
  return (tsum(Pa, jobs, ws, k) & 0xFFFFu) + (k > 0 ? tsum(Pa, jobs, ws, k - 1) >> 16 : 0u);
}

__global__ __launch_bounds__(kCarryThreads) void k_sum_carry(const Parent* __restrict__ parents,
                                                             const Job* __restrict__ jobs, Bases B,
                                                             uint32_t* __restrict__ ws, int32_t* overflow) {
  const Parent Pa = parents[blockIdx.x];
  const int L = Pa.len;
  // t_k for k = 0..L, computed once with consecutive threads on consecutive
  // positions (coalesced reads of the children's columns) and kept in LDS;
  // values too long for it recompute t_k from the columns where needed
  __shared__ uint32_t ts[kCarryTable];
  const bool tab = L + 1 <= kCarryTable;
  if (tab) {
    for (int k = threadIdx.x; k <= L; k += kCarryThreads) ts[k] = tsum(Pa, jobs, ws, k);
    __syncthreads();
  }
  auto u_at = [&](int k) -> uint32_t {
    if (tab) return (ts[k] & 0xFFFFu) + (k > 0 ? ts[k - 1] >> 16 : 0u);
    return usum(Pa, jobs, ws, k);
  };
  const int per = (L + kCarryThreads - 1) / kCarryThreads;
  const int k0 = threadIdx.x * per, k1 = min(L, k0 + per);
  // this chunk's carry function: generate G (carry out with no carry in) and
  // propagate P (carry out = carry in)
  bool G = false, Pp = true;
  for (int k = k0; k < k1; ++k) {
    const uint32_t u = u_at(k);
    G = (u > 0xFFFFu) || (u == 0xFFFFu && G);
    Pp = Pp && u == 0xFFFFu;
  }
  __shared__ uint8_t g_s[kCarryThreads], p_s[kCarryThreads];
  g_s[threadIdx.x] = G;
  p_s[threadIdx.x] = k0 < k1 ? Pp : 1;
  __syncthreads();
  // inclusive prefix of the carry functions (Hillis-Steele): (G, P) of chunks
  // [i - 2^s + 1, i] composed with those before
  for (int off = 1; off < kCarryThreads; off <<= 1) {
    uint8_t g = g_s[threadIdx.x], p = p_s[threadIdx.x];
    if (threadIdx.x >= off) {
      const uint8_t g0 = g_s[threadIdx.x - off], p0 = p_s[threadIdx.x - off];
      g = g | (p & g0);
      p = p & p0;
    }
    __syncthreads();
    g_s[threadIdx.x] = g;
    p_s[threadIdx.x] = p;
    __syncthreads();
  }
  uint32_t c = threadIdx.x > 0 ? g_s[threadIdx.x - 1] : 0u;   // carry into this chunk
  uint32_t* out = at(B, Pa.out);
  for (int k = k0; k < k1; ++k) {
    const uint32_t u = u_at(k) + c;
    out[k] = u & 0xFFFFu;
    c = u >> 16;
  }
  // nothing may be left above the value's length (the host's bound)
  if (threadIdx.x == kCarryThreads - 1 &&
      (g_s[kCarryThreads - 1] || (tab ? ts[L] : tsum(Pa, jobs, ws, L)) != 0 || u_at(L) != 0))
    *overflow = 1;
}

__global__ void k_zero_flag32(int32_t* f) { *f = 0; }
__global__ void k_zero_tail(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// host: the schedule (levels of products and sums), cached per tree and
// point length
// ---------------------------------------------------------------------------

inline size_t al256b(size_t v) { return (v + 255) & ~size_t(255); }
inline int clog2(int64_t v) {
  int l = 0;
  while (((int64_t)1 << l) < v) ++l;
  return l;
}

struct Level {
  int32_t job_begin, job_end, par_begin, par_end;
  int32_t max_logn;
};
struct Schedule {
  int32_t lx = 0;
  std::vector<Job> jobs;
  std::vector<Parent> parents;
  std::vector<Level> levels;
  int64_t out_len = 0;
  size_t off_lists = 0, off_par = 0, bytes = 0;
  int64_t ntt_words = 0;   // scratch per level (max)
  size_t off_ntt = 0, off_tw = 0;
  std::string err;
};

struct ScheduleCache {
  std::mutex mu;
  std::vector<std::pair<const fpe_tree*, Schedule>> entries;   // per tree, last lx
};
ScheduleCache& cache() {
  static ScheduleCache c;
  return c;
}

// Builds the schedule of a tree at a point of lx limbs.
Schedule build_schedule(const fpe_tree* t, int32_t lx) {
  Schedule S;
  S.lx = lx;
  const int64_t N = (int64_t)t->nodes.size();
  std::vector<Job> jobs;
  std::vector<Parent> parents;
  // value arena in words; conv arena in 64-bit words (laid out after)
  int64_t words = 64;   // 256 bytes: the overflow flag
  int64_t conv_words = 0;
  auto alloc_val = [&](int64_t len) {
    const int64_t o = words;
    words += (len + 63) & ~int64_t(63);
    return o;
  };
  // powers: table entry -> (ref, len); a chain LOAD is the caller's point itself
  std::vector<Ref> tref(t->n_table);
  std::vector<int64_t> tlen(t->n_table, 0), tdepth(t->n_table, 0);
  std::vector<std::vector<int>> chain_levels;
  for (size_t c = 0; c < t->chain.size(); ++c) {
    const ChainStep& st = t->chain[c];
    if (st.kind == kChainLoad) {
      tref[st.dst] = Ref{kX, 0, 0};
      tlen[st.dst] = lx;
      tdepth[st.dst] = 0;
    } else {
      tdepth[st.dst] = 1 + std::max(tdepth[st.s1], tdepth[st.s2]);
      tlen[st.dst] = tlen[st.s1] + tlen[st.s2];
      if ((int64_t)chain_levels.size() < tdepth[st.dst]) chain_levels.resize(tdepth[st.dst]);
      chain_levels[tdepth[st.dst] - 1].push_back((int)c);
    }
  }
  for (int64_t e = 0; e < t->n_table; ++e)
    if (tref[e].space == kWs && tlen[e] > 0) tref[e].off = alloc_val(tlen[e]);
  auto add_job = [&](Ref a, int64_t la, Ref b, int64_t lb) -> bool {
    Job J{};
    J.a = a;
    J.b = b;
    J.la = (int32_t)la;
    J.lb = (int32_t)lb;
    const int64_t lp = la + lb - 1;
    if (std::min(la, lb) >= kSchoolMax) {
      J.logn = clog2(lp);
      if (J.logn > kNttLogMax) {
        S.err = "a product is longer than the largest transform (2^14 limbs)";
        return false;
      }
    }
    J.conv = conv_words;
    conv_words += (lp + 31) & ~int64_t(31);
    jobs.push_back(J);
    return true;
  };
  auto level_done = [&](int32_t jb, int32_t pb) {
    Level L{jb, (int32_t)jobs.size(), pb, (int32_t)parents.size(), 0};
    for (int32_t j = jb; j < L.job_end; ++j) L.max_logn = std::max(L.max_logn, jobs[j].logn);
    S.levels.push_back(L);
  };
  for (const auto& lvl : chain_levels) {
    const int32_t jb = (int32_t)jobs.size(), pb = (int32_t)parents.size();
    for (int c : lvl) {
      const ChainStep& st = t->chain[c];
      const int32_t j0 = (int32_t)jobs.size();
      if (!add_job(tref[st.s1], tlen[st.s1], tref[st.s2], tlen[st.s2])) return S;
      parents.push_back(Parent{tref[st.dst], 0, j0, j0 + 1, (int32_t)tlen[st.dst], 0});
    }
    level_done(jb, pb);
  }
  // nodes by height; children lists
  std::vector<std::vector<int64_t>> ch(N);
  for (int64_t i = 0; i < N; ++i)
    if (t->nodes[i].parent >= 0) ch[t->nodes[i].parent].push_back(i);
  std::vector<int64_t> height(N, 0), vlen(N, 0);
  std::vector<Ref> vref(N);
  int64_t hmax = 0;
  for (int64_t i = 0; i < N; ++i) {
    for (int64_t c : ch[i]) height[i] = std::max(height[i], height[c] + 1);
    hmax = std::max(hmax, height[i]);
  }
  auto pow_of = [&](int64_t i, Ref& r, int64_t& l) -> bool {
    const fpe_node& nd = t->nodes[i];
    for (int64_t e = 0; e < t->n_table; ++e)
      if (t->table_deg[e] == nd.pdeg && t->table_var[e] == nd.var) {
        r = tref[e];
        l = tlen[e];
        return true;
      }
    return false;
  };
  const int64_t R = N - 1;
  const bool root_pow = t->nodes[R].pdeg > 0;
  std::vector<std::vector<int64_t>> by_h(hmax + 1);
  for (int64_t i = 0; i < N; ++i) by_h[height[i]].push_back(i);
  for (int64_t h = 0; h <= hmax; ++h) {
    const int32_t jb = (int32_t)jobs.size(), pb = (int32_t)parents.size();
    for (int64_t i : by_h[h]) {
      const int32_t j0 = (int32_t)jobs.size();
      int64_t len = 4;
      for (int64_t c : ch[i]) {
        Ref X;
        int64_t lxp = 0;
        if (!pow_of(c, X, lxp)) {
          S.err = "a power outside the table";
          return S;
        }
        if (!add_job(vref[c], vlen[c], X, lxp)) return S;
        len = std::max(len, vlen[c] + lxp);
      }
      // the sum of the children and the coefficient may carry past the
      // longest term: one limb per factor 2^16 of their number, and one more
      int64_t extra = 1;
      for (int64_t k = (int64_t)ch[i].size() + 1; k > 1; k >>= 16) ++extra;
      len += extra;
      vlen[i] = len;
      // the root's value is the result when the root has no power of its own
      vref[i] = (i == R && !root_pow) ? Ref{kOut, 0, 0} : Ref{kWs, 0, alloc_val(len)};
      parents.push_back(Parent{vref[i], t->nodes[i].coef.u, j0, (int32_t)jobs.size(), (int32_t)len, 0});
    }
    level_done(jb, pb);
  }
  // the root's own power
  if (root_pow) {
    Ref X;
    int64_t lxp = 0;
    if (!pow_of(R, X, lxp)) {
      S.err = "a power outside the table";
      return S;
    }
    const int32_t jb = (int32_t)jobs.size(), pb = (int32_t)parents.size();
    if (!add_job(vref[R], vlen[R], X, lxp)) return S;
    S.out_len = vlen[R] + lxp;
    parents.push_back(Parent{Ref{kOut, 0, 0}, 0, jb, jb + 1, (int32_t)S.out_len, 0});
    level_done(jb, pb);
  } else {
    S.out_len = vlen[R];
  }
  // transform scratch per level, placed after the values and convolutions
  int64_t ntt_words = 0;
  for (const Level& L : S.levels) {
    int64_t w = 0;
    for (int32_t j = L.job_begin; j < L.job_end; ++j) {
      if (!jobs[j].logn) continue;
      jobs[j].scratch = w;   // relative; shifted below
      w += (int64_t)2 * kBigPrimes << jobs[j].logn;
    }
    ntt_words = std::max(ntt_words, w);
  }
  const int64_t conv_base = (words + 1) / 2 * 2;   // in 32-bit words, even
  const int64_t ntt_base = conv_base + 2 * conv_words;
  for (Job& J : jobs) {
    J.conv += conv_base / 2;
    if (J.logn) J.scratch += ntt_base;
  }
  S.jobs = std::move(jobs);
  S.parents = std::move(parents);
  S.ntt_words = ntt_words;
  S.off_tw = al256b((size_t)(ntt_base + ntt_words) * sizeof(uint32_t));
  S.off_lists = al256b(S.off_tw + (size_t)kBigPrimes * kNttMax * sizeof(uint32_t));
  S.off_par = al256b(S.off_lists + S.jobs.size() * sizeof(Job));
  S.bytes = al256b(S.off_par + S.parents.size() * sizeof(Parent));
  return S;
}

// The cached schedule of (t, lx) (rebuilt when lx changes).
const Schedule* schedule_for(const fpe_tree* t, int32_t lx) {
  ScheduleCache& C = cache();
  std::lock_guard<std::mutex> lk(C.mu);
  for (auto& e : C.entries)
    if (e.first == t && e.second.lx == lx) return &e.second;
  for (auto it = C.entries.begin(); it != C.entries.end(); ++it)
    if (it->first == t) {
      C.entries.erase(it);
      break;
    }
  C.entries.emplace_back(t, build_schedule(t, lx));
  return &C.entries.back().second;
}

}  // namespace

void bigpoint_forget(const fpe_tree* t) {
  ScheduleCache& C = cache();
  std::lock_guard<std::mutex> lk(C.mu);
  for (auto it = C.entries.begin(); it != C.entries.end(); ++it)
    if (it->first == t) {
      C.entries.erase(it);
      return;
    }
}

int64_t bigpoint_out_limbs(const fpe_tree* t, int32_t lx) {
  const Schedule* S = schedule_for(t, lx);
  if (!S->err.empty()) set_error(S->err);
  return S->err.empty() ? S->out_len : 0;
}

size_t bigpoint_workspace_bytes(const fpe_tree* t, int32_t lx) {
  const Schedule* S = schedule_for(t, lx);
  return S->err.empty() ? S->bytes : 0;
}

fpe_status launch_bigpoint(const fpe_tree* t, const uint32_t* x, int32_t lx, uint32_t* out, int64_t lout, void* ws,
                           size_t ws_bytes, void* stream) {
  if (t->n_offtable > 0) return fail(FPE_EUNSUPPORTED, "evaluation at a big point needs every power in the table");
  const Schedule* S = schedule_for(t, lx);
  if (!S->err.empty()) return fail(FPE_EUNSUPPORTED, S->err);
  if (lout < S->out_len) return fail(FPE_EINVAL, "lout smaller than fpe_bigpoint_out_limbs()");
  if (!ws || ws_bytes < S->bytes) return fail(FPE_ENOMEM, "workspace smaller than fpe_bigpoint_workspace_bytes()");
  if (((uintptr_t)ws) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  Bases B{{(uint32_t*)ws, const_cast<uint32_t*>(x), out}};
  uint32_t* tw = (uint32_t*)(base + S->off_tw);
  Job* jobs = (Job*)(base + S->off_lists);
  Parent* parents = (Parent*)(base + S->off_par);
  // the schedule lives as long as the tree's cache entry, so the copies read
  // live memory whenever they run
  hipError_t e = hipMemcpyAsync(jobs, S->jobs.data(), S->jobs.size() * sizeof(Job), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(parents, S->parents.data(), S->parents.size() * sizeof(Parent), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("big point: ") + hipGetErrorString(e));
  hipLaunchKernelGGL(k_zero_flag32, dim3(1), dim3(1), 0, st, (int32_t*)ws);
  launch_twiddles(tw, kBigPrimes, st);
  Scales2 sc{};
  for (int l = 0; l <= kNttLogMax; ++l) {
    const Scales s = scales_for(1 << l);
    for (int k = 0; k < kBigPrimes; ++k) sc.s[k][l] = s.s[k];
  }
  const uint64_t p1 = kPrimes[0].p, p2 = kPrimes[1].p;
  const uint32_t inv12 = (uint32_t)(((unsigned __int128)host_pow(p1 % p2, p2 - 2, p2) << 32) % p2);
  for (const Level& L : S->levels) {
    const int nj = L.job_end - L.job_begin, np = L.par_end - L.par_begin;
    if (nj > 0) {
      if (L.max_logn > 0) {
        const int n = 1 << L.max_logn;
        const int thr = std::min(kNttThreads, std::max(64, n / 2));
        const size_t lds = (size_t)n * sizeof(uint32_t);
        hipLaunchKernelGGL(k_job_fwd, dim3(nj, kBigPrimes, 2), dim3(thr), lds, st, jobs + L.job_begin, B, tw,
                           (uint32_t*)ws);
        hipLaunchKernelGGL(k_job_mul_inv, dim3(nj, kBigPrimes), dim3(thr), lds, st, jobs + L.job_begin, sc, tw,
                           (uint32_t*)ws);
      }
      hipLaunchKernelGGL(k_job_finish, dim3(8, nj), dim3(256), 0, st, jobs + L.job_begin, B, (uint32_t*)ws, inv12);
    }
    if (np > 0)
      hipLaunchKernelGGL(k_sum_carry, dim3(np), dim3(kCarryThreads), 0, st, parents + L.par_begin, jobs, B,
                         (uint32_t*)ws, (int32_t*)ws);
  }
  // limbs of the output beyond the value
  if (lout > S->out_len) {
    const int64_t extra = lout - S->out_len;
    hipLaunchKernelGGL(k_zero_tail, dim3((unsigned)std::min<int64_t>((extra + 255) / 256, 1024)), dim3(256), 0, st,
                       out + S->out_len, extra);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("big point launch: ") + hipGetErrorString(e));
  return FPE_OK;
}

}  // namespace fpe
