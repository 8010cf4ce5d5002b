// Composition p(q(x)) over Z/(2^31 - 1) by levels of the tree, with the
// large polynomial products on the matrix cores.
//
// The tree is walked from its definition (Section 1): u(N) = c(N) + sum over
// the children C of u(C) q^{d(C)}, and p(q) = u(R) q^{d(R)} at the root R.
// The nodes of one height are independent, so each height is one launch over
// all of its nodes and all instances; the powers q^d come first, by the
// tree's multiplication chain (Section 2.2), also level by level.  With
// divide-and-conquer trees the heights are few and their products grow
// geometrically towards the root (Section 1.2: such schemes suit elements
// whose size grows with each multiplication), so the top levels hold nearly
// all of the work, as dense products of polynomials with hundreds to
// thousands of coefficients.
//
// A large product is an integer matrix product.  Residues are centred
// (|v| < 2^30) and written as four balanced base-256 digits in [-128, 127];
// for digit planes s of h and t of the other operand, the convolution of the
// planes is a Toeplitz product: with output coefficient n = 32 m + u,
//   C[u][m] = sum_r sum_k t[32 r + u - k] h[32 (m - r) + k]   (k, u in [0, 32)),
// one 32 x 32 x 32 int8 MFMA per block r and tile of 32 blocks m, with the
// Toeplitz operand read from LDS at a per-lane offset and the h operand as
// aligned blocks.  The 16 digit pairs accumulate exactly in 32-bit integers
// by s + t (7 groups: 4 pairs x 2^14 x the summed operand lengths < 2^31,
// checked when the schedule is built), and the groups are recombined with
// 2^(8 g) = 2^(8 g mod 31) mod p.  Small levels run on a VALU schoolbook
// kernel (a thread per output coefficient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fpe_internal.h"

namespace fpe {

namespace {

typedef int8_t i8x16 __attribute__((ext_vector_type(16)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 1024;          // output coefficients of one MFMA tile (32 blocks of 32)
constexpr int kMaxTiles = 4;         // tiles of one node: one wavefront each
constexpr int kMfmaMinOut = 256;     // shorter outputs go to the VALU kernel
constexpr int kGroups = 7;           // digit pairs (s, t) grouped by s + t
constexpr int kMaxParentsPerLaunch = 65535;
constexpr int64_t kExactLimit = int64_t(1) << 15;   // summed min(lt, lh) of a node's products

// Where a polynomial lives: the instance's arena, the caller's q or output,
// or (length 1) the coefficient of a node.
enum CSpace : int32_t { cArena = 0, cQ = 1, cOut = 2, cCoef = 3 };
struct CRef {
  int32_t space;
  int32_t node;   // cCoef
  int64_t off;    // words within the instance's region
};
struct CChild {   // the product h * t (t the shorter operand)
  CRef h, t;
  int32_t lh, lt;
};
struct CParent {  // out = c(node) + sum of the products of children [child_begin, child_end)
  CRef out;
  int32_t coef_node;   // -1: no constant
  int32_t child_begin, child_end;
  int32_t lout;
};
struct CBases {
  uint32_t* arena;
  const uint32_t* q;
  uint32_t* out;
  const uint32_t* coef;
  int64_t arena_stride, q_stride, out_stride, n_nodes;
};

__device__ __forceinline__ const uint32_t* cptr(const CBases& B, const CRef& r, int64_t inst) {
  switch (r.space) {
    case cArena: return B.arena + inst * B.arena_stride + r.off;
    case cQ: return B.q + inst * B.q_stride + r.off;
    case cOut: return B.out + inst * B.out_stride + r.off;
    default: return B.coef + inst * B.n_nodes + r.node;
  }
}
__device__ __forceinline__ uint32_t* optr(const CBases& B, const CRef& r, int64_t inst) {
  return r.space == cOut ? B.out + inst * B.out_stride + r.off : B.arena + inst * B.arena_stride + r.off;
}

__device__ __forceinline__ uint64_t fold64(uint64_t v) { return (v & kP31) + (v >> 31); }
__device__ __forceinline__ uint32_t reduce31(uint64_t v) {
  v = (v & kP31) + (v >> 31);
  v = (v & kP31) + (v >> 31);
  return (uint32_t)(v >= kP31 ? v - kP31 : v);
}

// ---------------------------------------------------------------------------
// small levels: one thread per output coefficient of one node and instance
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cm_valu(const CParent* __restrict__ pars, const CChild* __restrict__ ch,
                                                 CBases B, int64_t batch) {
  const CParent P = pars[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= batch * P.lout) return;
  const int64_t inst = idx / P.lout;
  const int n = (int)(idx - inst * P.lout);
  uint64_t acc = (n == 0 && P.coef_node >= 0) ? B.coef[inst * B.n_nodes + P.coef_node] : 0u;
  for (int c = P.child_begin; c < P.child_end; ++c) {
    const CChild C = ch[c];
    const uint32_t* a = cptr(B, C.h, inst);
    const uint32_t* b = cptr(B, C.t, inst);
    const int i0 = max(0, n - (C.lt - 1)), i1 = min(n, C.lh - 1);
    int i = i0;
    // residues are below 2^31: three products and a folded sum stay below 2^64
    for (; i + 2 <= i1; i += 3)
      acc = fold64(acc + (uint64_t)a[i] * b[n - i] + (uint64_t)a[i + 1] * b[n - i - 1] +
                   (uint64_t)a[i + 2] * b[n - i - 2]);
    for (; i <= i1; ++i) acc = fold64(acc + (uint64_t)a[i] * b[n - i]);
  }
  optr(B, P.out, inst)[n] = reduce31(acc);
}

// ---------------------------------------------------------------------------
// large levels: one workgroup per node and instance, one wavefront per tile
// ---------------------------------------------------------------------------

// Four balanced base-256 digits of the centred residue of v (v < 2^31),
// byte-packed: digit s of value b (b = 0..3) lands in byte b of pk[s].
__device__ __forceinline__ void put_digits(uint32_t v, int b, uint32_t pk[4]) {
  int32_t x = v > (uint32_t)(kP31 >> 1) ? (int32_t)(v - (uint32_t)kP31) : (int32_t)v;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int32_t lo = ((x & 0xFF) ^ 0x80) - 0x80;
    pk[s] |= (uint32_t)(lo & 0xFF) << (8 * b);
    x = (x - lo) >> 8;
  }
}

// LDS: 16 planes of the Toeplitz operand (digit s, byte shift e at
// (4 s + e) * ntp), then 4 digit planes of h (hp bytes each).  Plane (s, e)
// holds byte y = digit s of trev[y + e], where trev[x] = t[X0 - x] (zero
// outside t), so that a lane whose read starts at a byte offset = e mod 4
// reads four aligned words.  Plane s of h holds digit s of h[i] at byte i,
// zero from lh up to 32 (J + 1) (the block J is the zero block that lanes
// outside the band read).
__global__ __launch_bounds__(256) void k_cm_mfma(const CParent* __restrict__ pars, const CChild* __restrict__ ch,
                                                 CBases B, int32_t ntp, int32_t hp) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint8_t* tpl = lds;
  uint8_t* hpl = lds + 16 * ntp;
  const CParent P = pars[blockIdx.y];
  const int64_t inst = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nthr = blockDim.x;
  const int ntiles = (P.lout + kTile - 1) / kTile;
  const int m0 = 32 * wave;        // first output block of this wavefront's tile
  const int u = lane & 31, hh = lane >> 5;
  i32x16 acc[kGroups];
#pragma unroll
  for (int g = 0; g < kGroups; ++g) acc[g] = i32x16{};

  for (int c = P.child_begin; c < P.child_end; ++c) {
    const CChild C = ch[c];
    const uint32_t* hv = cptr(B, C.h, inst);
    const uint32_t* tv = cptr(B, C.t, inst);
    const int J = (C.lh + 31) >> 5;
    const int rmax = (C.lt + 30) >> 5;   // blocks r with a nonzero t[32 r + u - k]
    const int X0 = 32 * rmax + 31;
    __syncthreads();   // the previous child's operands are no longer read
    for (int w = tid; w < 8 * (J + 1); w += nthr) {
      uint32_t pk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = 4 * w + b;
        put_digits(i < C.lh ? hv[i] : 0u, b, pk);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) ((uint32_t*)(hpl + s * hp))[w] = pk[s];
    }
    const int ntw = ntp >> 2;
    for (int it = tid; it < 4 * ntw; it += nthr) {
      const int e = it / ntw, w = it - e * ntw;
      uint32_t pk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = X0 - (4 * w + b) - e;
        put_digits((i >= 0 && i < C.lt) ? tv[i] : 0u, b, pk);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) ((uint32_t*)(tpl + (4 * s + e) * ntp))[w] = pk[s];
    }
    __syncthreads();
    if (wave < ntiles) {
      // this lane's row u of the Toeplitz operand holds k = 16 hh + j (byte
      // j): t[32 r + u - k] = trev[s0 - 32 r + j]
      const int s0 = X0 - u + 16 * hh;
      const int e = s0 & 3;
      const uint8_t* ta = tpl + e * ntp + (s0 - e);
      const int col = m0 + u;   // this lane's output block in the h operand's layout
      const int r_lo = max(0, m0 - J + 1), r_hi = min(rmax, m0 + 31);
      for (int r = r_lo; r <= r_hi; ++r) {
        i8x16 A[4], H[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const uint32_t* p = (const uint32_t*)(ta + 4 * s * ntp - 32 * r);
          const u32x4 v = {p[0], p[1], p[2], p[3]};
          A[s] = __builtin_bit_cast(i8x16, v);
        }
        const int jb = col - r;
        const int hoff = ((unsigned)jb < (unsigned)J ? 32 * jb : 32 * J) + 16 * hh;
#pragma unroll
        for (int s = 0; s < 4; ++s) H[s] = __builtin_bit_cast(i8x16, *(const u32x4*)(hpl + s * hp + hoff));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[a + s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], H[s], acc[a + s], 0, 0, 0);
      }
    }
  }
  if (wave < ntiles) {
    uint32_t* o = optr(B, P.out, inst);
    const uint64_t c0 = P.coef_node >= 0 ? B.coef[inst * B.n_nodes + P.coef_node] : 0u;
    const int col = m0 + u;
    constexpr int kShift[kGroups] = {0, 8, 16, 24, 1, 9, 17};   // 8 g mod 31
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int row = 8 * (rr >> 2) + 4 * hh + (rr & 3);
      const int n = 32 * col + row;
      int64_t v = 0;
#pragma unroll
      for (int g = 0; g < kGroups; ++g) v += (int64_t)acc[g][rr] * (int64_t(1) << kShift[g]);
      // |v| < 2^31 (2^24 + 2^17 + 2^16 + 2^9 + 2^8 + 3) < 2^56: add 2^27 p
      uint64_t w = (uint64_t)(v + ((int64_t)kP31 << 27)) + (n == 0 ? c0 : 0u);
      if (n < P.lout) o[n] = reduce31(w);
    }
  }
}

__global__ void k_cm_zero(uint32_t* out, int64_t stride, int64_t from, int64_t len, int64_t batch) {
  const int64_t n = len - from;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < batch * n; i += (int64_t)gridDim.x * blockDim.x)
    out[(i / n) * stride + from + i % n] = 0u;
}

// ---------------------------------------------------------------------------
// host: the schedule (levels of nodes), cached per tree and dq
// ---------------------------------------------------------------------------

struct CLevel {
  int32_t par_begin, par_end;
  int32_t mfma;
  int32_t waves;
  int32_t ntp, hp;
  int32_t max_lout;
};
struct CSched {
  int32_t dq = 0;
  std::vector<CParent> pars;
  std::vector<CChild> ch;
  std::vector<CLevel> levels;
  int64_t arena_words = 0;
  int64_t out_len = 0;
  int64_t lmax = 0;
  size_t off_ch = 0, off_arena = 0;
  std::string err;
};

struct CCache {
  std::mutex mu;
  std::vector<std::pair<const fpe_tree*, CSched>> entries;
};
CCache& ccache() {
  static CCache c;
  return c;
}

inline size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

CSched build_csched(const fpe_tree* t, int32_t dq) {
  CSched S;
  S.dq = dq;
  const int64_t N = (int64_t)t->nodes.size();
  int32_t dp = 0;
  for (int64_t i = 0; i < N; ++i) dp = std::max(dp, t->exps[i * t->nvars]);
  S.lmax = (int64_t)dp * dq + 1;
  int64_t words = 0;
  auto alloc = [&](int64_t len) {
    const int64_t o = words;
    words += (len + 3) & ~int64_t(3);
    return o;
  };
  std::vector<CParent> pars;
  std::vector<CChild> chl;
  // one dependency level: its nodes split into MFMA and VALU launches
  auto close_level = [&](std::vector<CParent>& lvl) {
    std::vector<CParent> big, small;
    for (CParent& p : lvl) {
      int64_t sum_min = 0;
      for (int32_t c = p.child_begin; c < p.child_end; ++c) sum_min += std::min(chl[c].lt, chl[c].lh);
      const bool mf = p.lout >= kMfmaMinOut && p.lout <= kMaxTiles * kTile && sum_min < kExactLimit;
      (mf ? big : small).push_back(p);
    }
    for (int kind = 0; kind < 2; ++kind) {
      std::vector<CParent>& v = kind ? small : big;
      for (size_t b = 0; b < v.size(); b += kMaxParentsPerLaunch) {
        CLevel L{(int32_t)pars.size(), 0, kind == 0, 1, 0, 0, 0};
        for (size_t k = b; k < std::min(v.size(), b + kMaxParentsPerLaunch); ++k) {
          const CParent& p = v[k];
          L.max_lout = std::max(L.max_lout, p.lout);
          for (int32_t c = p.child_begin; c < p.child_end; ++c) {
            const int32_t rmax = (chl[c].lt + 30) >> 5;
            const int32_t J = (chl[c].lh + 31) >> 5;
            L.ntp = std::max(L.ntp, (32 * rmax + 31 + 32 + 15) & ~15);
            L.hp = std::max(L.hp, 32 * (J + 1));
          }
          pars.push_back(p);
        }
        L.par_end = (int32_t)pars.size();
        L.waves = std::min(kMaxTiles, (L.max_lout + kTile - 1) / kTile);
        if (L.par_end > L.par_begin) S.levels.push_back(L);
      }
    }
    lvl.clear();
  };
  auto child = [&](CRef a, int64_t la, CRef b, int64_t lb) {
    CChild C{};
    if (la >= lb) {
      C.h = a, C.lh = (int32_t)la, C.t = b, C.lt = (int32_t)lb;
    } else {
      C.h = b, C.lh = (int32_t)lb, C.t = a, C.lt = (int32_t)la;
    }
    chl.push_back(C);
  };
  // powers: a LOAD is the caller's q itself
  std::vector<CRef> tref(t->n_table);
  std::vector<int64_t> tlen(t->n_table, 0), tdepth(t->n_table, 0);
  std::vector<std::vector<int>> chain_levels;
  for (size_t c = 0; c < t->chain.size(); ++c) {
    const ChainStep& st = t->chain[c];
    if (st.kind == kChainLoad) {
      tref[st.dst] = CRef{cQ, 0, 0};
      tlen[st.dst] = dq + 1;
    } else {
      tdepth[st.dst] = 1 + std::max(tdepth[st.s1], tdepth[st.s2]);
      tlen[st.dst] = tlen[st.s1] + tlen[st.s2] - 1;
      tref[st.dst] = CRef{cArena, 0, alloc(tlen[st.dst])};
      if ((int64_t)chain_levels.size() < tdepth[st.dst]) chain_levels.resize(tdepth[st.dst]);
      chain_levels[tdepth[st.dst] - 1].push_back((int)c);
    }
  }
  std::vector<CParent> lvl;
  for (const auto& cl : chain_levels) {
    for (int c : cl) {
      const ChainStep& st = t->chain[c];
      const int32_t j0 = (int32_t)chl.size();
      child(tref[st.s1], tlen[st.s1], tref[st.s2], tlen[st.s2]);
      lvl.push_back(CParent{tref[st.dst], -1, j0, j0 + 1, (int32_t)tlen[st.dst]});
    }
    close_level(lvl);
  }
  // nodes by height
  std::vector<std::vector<int64_t>> kids(N);
  for (int64_t i = 0; i < N; ++i)
    if (t->nodes[i].parent >= 0) kids[t->nodes[i].parent].push_back(i);
  std::vector<int64_t> height(N, 0), vlen(N, 1);
  std::vector<CRef> vref(N);
  int64_t hmax = 0;
  for (int64_t i = 0; i < N; ++i) {   // children have lower indices
    for (int64_t c : kids[i]) height[i] = std::max(height[i], height[c] + 1);
    hmax = std::max(hmax, height[i]);
    vref[i] = CRef{cCoef, (int32_t)i, 0};   // a leaf's value is its coefficient
  }
  auto pow_of = [&](int64_t i, CRef& r, int64_t& l) -> bool {
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
  for (int64_t h = 1; h <= hmax; ++h) {
    for (int64_t i : by_h[h]) {
      const int32_t j0 = (int32_t)chl.size();
      int64_t len = 1;
      for (int64_t c : kids[i]) {
        CRef X;
        int64_t lx = 0;
        if (!pow_of(c, X, lx)) {
          S.err = "composition needs every power in the table";
          return S;
        }
        child(vref[c], vlen[c], X, lx);
        len = std::max(len, vlen[c] + lx - 1);
      }
      vlen[i] = len;
      vref[i] = (i == R && !root_pow) ? CRef{cOut, 0, 0} : CRef{cArena, 0, alloc(len)};
      lvl.push_back(CParent{vref[i], (int32_t)i, j0, (int32_t)chl.size(), (int32_t)len});
    }
    close_level(lvl);
  }
  if (root_pow) {
    CRef X;
    int64_t lx = 0;
    if (!pow_of(R, X, lx)) {
      S.err = "composition needs every power in the table";
      return S;
    }
    const int32_t j0 = (int32_t)chl.size();
    child(vref[R], vlen[R], X, lx);
    S.out_len = vlen[R] + lx - 1;
    lvl.push_back(CParent{CRef{cOut, 0, 0}, -1, j0, j0 + 1, (int32_t)S.out_len});
    close_level(lvl);
  } else if (hmax == 0) {   // p is a constant: out = c(R)
    S.out_len = 1;
    lvl.push_back(CParent{CRef{cOut, 0, 0}, (int32_t)R, 0, 0, 1});
    close_level(lvl);
  } else {
    S.out_len = vlen[R];
  }
  if (S.out_len > S.lmax) {
    S.err = "internal: composition output longer than deg_p * dq + 1";
    return S;
  }
  S.pars = std::move(pars);
  S.ch = std::move(chl);
  S.arena_words = (words + 63) & ~int64_t(63);
  S.off_ch = al256(S.pars.size() * sizeof(CParent));
  S.off_arena = al256(S.off_ch + S.ch.size() * sizeof(CChild));
  return S;
}

const CSched* csched_for(const fpe_tree* t, int32_t dq) {
  CCache& C = ccache();
  std::lock_guard<std::mutex> lk(C.mu);
  for (auto& e : C.entries)
    if (e.first == t && e.second.dq == dq) return &e.second;
  for (auto it = C.entries.begin(); it != C.entries.end(); ++it)
    if (it->first == t) {
      C.entries.erase(it);
      break;
    }
  C.entries.emplace_back(t, build_csched(t, dq));
  return &C.entries.back().second;
}

}  // namespace

void compose_levels_forget(const fpe_tree* t) {
  CCache& C = ccache();
  std::lock_guard<std::mutex> lk(C.mu);
  for (auto it = C.entries.begin(); it != C.entries.end(); ++it)
    if (it->first == t) {
      C.entries.erase(it);
      return;
    }
}

size_t compose_levels_workspace_bytes(const fpe_tree* t, int32_t dq) {
  if (!t || t->nodes.empty() || dq < 1) return 0;
  const CSched* S = csched_for(t, dq);
  if (!S->err.empty()) return 0;
  return S->off_arena + (size_t)S->arena_words * (size_t)t->batch * sizeof(uint32_t);
}

// Whether the level walk applies (every product within its exactness and LDS
// limits, or else on the VALU kernel) and how many launches it takes.
bool compose_levels_ok(const fpe_tree* t, int32_t dq, int64_t* launches) {
  const CSched* S = csched_for(t, dq);
  if (launches) *launches = (int64_t)S->levels.size();
  return S->err.empty();
}

fpe_status launch_compose_levels(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (t->n_offtable > 0) return fail(FPE_EUNSUPPORTED, "composition needs every power in the table");
  if (t->batch > 0x7fffffff) return fail(FPE_EUNSUPPORTED, "batch too large");
  const CSched* S = csched_for(t, dq);
  if (!S->err.empty()) return fail(FPE_EUNSUPPORTED, S->err);
  const size_t need = S->off_arena + (size_t)S->arena_words * (size_t)t->batch * sizeof(uint32_t);
  if (!ws || ws_bytes < need) return fail(FPE_ENOMEM, "workspace smaller than the composition needs");
  if (((uintptr_t)ws) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  CParent* pars = (CParent*)base;
  CChild* chd = (CChild*)(base + S->off_ch);
  // the schedule lives as long as the tree's cache entry, so the copies read
  // live memory whenever they run
  hipError_t e = hipMemcpyAsync(pars, S->pars.data(), S->pars.size() * sizeof(CParent), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !S->ch.empty())
    e = hipMemcpyAsync(chd, S->ch.data(), S->ch.size() * sizeof(CChild), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition: ") + hipGetErrorString(e));
  CBases B{(uint32_t*)(base + S->off_arena), q, out, dev_view(t).coef_rows, S->arena_words, (int64_t)dq + 1,
           S->lmax, (int64_t)t->nodes.size()};
  for (const CLevel& L : S->levels) {
    const int np = L.par_end - L.par_begin;
    if (L.mfma) {
      const size_t lds = (size_t)16 * L.ntp + (size_t)4 * L.hp;
      hipLaunchKernelGGL(k_cm_mfma, dim3((unsigned)t->batch, np), dim3(64 * L.waves), lds, st, pars + L.par_begin,
                         chd, B, L.ntp, L.hp);
    } else {
      const int64_t gx = (t->batch * L.max_lout + 255) / 256;
      hipLaunchKernelGGL(k_cm_valu, dim3((unsigned)gx, np), dim3(256), 0, st, pars + L.par_begin, chd, B, t->batch);
    }
  }
  if (S->out_len < S->lmax) {
    const int64_t n = (S->lmax - S->out_len) * t->batch;
    hipLaunchKernelGGL(k_cm_zero, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st, out,
                       S->lmax, S->out_len, S->lmax, t->batch);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition launch: ") + hipGetErrorString(e));
  return FPE_OK;
}

}  // namespace fpe
