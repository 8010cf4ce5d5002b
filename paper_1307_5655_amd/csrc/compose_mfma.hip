// Composition p(q(x)) over Z/(2^31 - 1) by levels of the tree, with the
// polynomial products on the matrix cores.
//
// The tree is walked from its definition (Section 1): u(N) = c(N) + sum over
// the children C of u(C) q^{d(C)}, and p(q) = u(R) q^{d(R)} at the root R;
// the powers q^d come from the tree's multiplication chain (Section 2.2).
// Every value (a node's u, a power) is computed once its operands are, so
// the values of one dependency depth are independent and form one launch
// over all instances.  Divide-and-conquer trees have few depths and their
// products grow geometrically towards the root (Section 1.2: such schemes
// suit elements whose size grows with each multiplication), so nearly all of
// the work is dense products of polynomials with hundreds to thousands of
// coefficients.
//
// A product is an exact integer matrix product.  Residues are centred
// (|v| < 2^30) and written as four balanced base-256 digits in [-128, 127]
// (the bytes of v + 0x80808080, each offset by 128).  For digit planes s of
// h and a of t, with output coefficient n = 32 m + u,
//   C[u][m] = sum_r sum_k t[32 r + u - k] h[32 (m - r) + k]   (k, u in [0, 32)),
// one 32 x 32 x 32 int8 MFMA per block r and tile of 32 output blocks m: a
// Toeplitz operand read from LDS at a per-lane byte offset, and the h operand
// as aligned 32-byte blocks.  The 16 digit pairs accumulate exactly in 32-bit
// integers grouped by s + a (7 groups; 4 pairs x 2^14 x the summed lengths
// of a value's products < 2^31, checked when the schedule is built), and the
// groups are recombined with 2^(8 g) = 2^(8 g mod 31) mod p.
//
// A workgroup computes a group of values of one instance laid side by side
// in the columns (output blocks) of up to four tiles, one wavefront per tile.
// Their products are taken in rounds, one per power q^d: the power is the
// Toeplitz operand shared by every value of the group that multiplies it,
// and each value's factor sits in its own blocks of the h operand, so the
// small products of the lower levels fill the tiles as well as the large ones
// at the top.  Values beyond four tiles (4096 coefficients) or the exactness
// bound go to a VALU schoolbook kernel (a thread per output coefficient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "fpe_internal.h"

namespace fpe {

namespace {

typedef int8_t i8x16 __attribute__((ext_vector_type(16)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxTiles = 4;             // tiles of one workgroup: one wavefront each
constexpr int kCols = 32 * kMaxTiles;    // output blocks of 32 coefficients per workgroup
constexpr int kGroups = 7;               // digit pairs (s, a) grouped by s + a
constexpr int kMaxLaunchY = 65535;
constexpr size_t kMaxLds = 64 * 1024;
constexpr int64_t kExactLimit = int64_t(1) << 15;   // summed min(lt, lh) over a value's products

// Where a polynomial lives: the instance's arena, the caller's q or output,
// or (length 1) the coefficient of a node.
enum CSpace : int32_t { cArena = 0, cQ = 1, cOut = 2, cCoef = 3 };
struct CRef {
  int32_t space;
  int32_t node;   // cCoef
  int64_t off;    // words within the instance's region
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
// VALU schoolbook kernel: one thread per output coefficient
// ---------------------------------------------------------------------------
struct CChild {   // the product h * t
  CRef h, t;
  int32_t lh, lt;
};
struct CParent {  // out = c(node) + sum of the products of children [child_begin, child_end)
  CRef out;
  int32_t coef_node;   // -1: no constant
  int32_t child_begin, child_end;
  int32_t lout;
};

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
// matrix-core kernel: one workgroup per group of values and instance
// ---------------------------------------------------------------------------
struct GParent {   // a value of a group
  CRef out;
  int32_t coef_node;   // -1: no constant
  int32_t lout;
};
struct GRound {    // the products of a group by one power t
  CRef t;
  int32_t lt;
  int32_t e_begin, e_end;   // entries (the factors h)
  int32_t hblocks;          // 32-byte blocks of each h digit plane (block 0: zeros)
  int32_t b_begin;          // hblocks records: the entry of each block (-1: zeros)
  int32_t col_begin;        // kCols column records
  int32_t r_lo[kMaxTiles], r_hi[kMaxTiles];   // blocks r of t that reach each tile
};
struct GEntry {    // one factor: its blocks start at block hblk (>= 1) of the h planes
  CRef h;
  int32_t lh;
  int32_t hblk;
};
struct GCol {      // column m in a round: h block hblk + (m - base - r), if m - base - r < J
  int32_t hblk, base, J;
};
struct GOwn {      // column m of a group: its value (-1: none) and the value's first column
  int32_t parent, base;
};
struct GGroup {
  int32_t p_begin, p_end, rd_begin, rd_end;
  int32_t own_begin;
  int32_t ntiles;
};
struct GLists {
  const GGroup* groups;
  const GParent* pars;
  const GRound* rounds;
  const GEntry* ents;
  const GCol* cols;
  const GOwn* own;
  const int32_t* bent;
};

// The four balanced digits of the centred residue of v (v < p), byte s
// holding digit s as an int8.
__device__ __forceinline__ uint32_t digit_word(uint32_t v) {
  return (v + (v > (uint32_t)(kP31 >> 1) ? 0x00808081u : 0x80808080u)) ^ 0x80808080u;
}
// 4 x 4 byte transpose: d[s] byte b = byte s of w[b].
__device__ __forceinline__ void transpose4(const uint32_t w[4], uint32_t d[4]) {
  const uint32_t lo01 = (w[0] & 0x00FF00FFu) | ((w[1] & 0x00FF00FFu) << 8);
  const uint32_t hi01 = ((w[0] >> 8) & 0x00FF00FFu) | (w[1] & 0xFF00FF00u);
  const uint32_t lo23 = (w[2] & 0x00FF00FFu) | ((w[3] & 0x00FF00FFu) << 8);
  const uint32_t hi23 = ((w[2] >> 8) & 0x00FF00FFu) | (w[3] & 0xFF00FF00u);
  d[0] = (lo01 & 0xFFFFu) | (lo23 << 16);
  d[1] = (hi01 & 0xFFFFu) | (hi23 << 16);
  d[2] = (lo01 >> 16) | (lo23 & 0xFFFF0000u);
  d[3] = (hi01 >> 16) | (hi23 & 0xFFFF0000u);
}

// LDS: 16 planes of the Toeplitz operand (digit s, byte shift e, at
// (4 s + e) * ntp), then 4 digit planes of h (hp bytes each).  Plane (s, e)
// holds byte y = digit s of trev[y + e], where trev[x] = t[X0 - x] (zero
// outside t), so that a lane whose read starts at a byte = e mod 4 reads four
// aligned words; ntp = 64 mod 256, so the four copies fall in disjoint LDS
// banks.  An h plane holds 32-byte blocks (block 0 zeros, read by the lanes
// whose block falls outside their factor) as two halves: bytes 0..15 of every
// block, then bytes 16..31, so that the 16-byte reads of consecutive lanes
// are consecutive.  Three wavefronts per SIMD (the register budget of the
// accumulators plus one operand set).
__global__ __launch_bounds__(256, 3) void k_cm_mfma(GLists Ls, CBases B, int32_t ntp, int32_t hp) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint8_t* tpl = lds;
  uint8_t* hpl = lds + 16 * ntp;
  const GGroup G = Ls.groups[blockIdx.y];
  const int64_t inst = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int u = lane & 31, hh = lane >> 5;
  const int m = 32 * wave + u;   // this lane's output block (column) in the group
  i32x16 acc[kGroups];
#pragma unroll
  for (int g = 0; g < kGroups; ++g) acc[g] = i32x16{};

  for (int rd = G.rd_begin; rd < G.rd_end; ++rd) {
    const GRound R = Ls.rounds[rd];
    const uint32_t* tv = cptr(B, R.t, inst);
    const int rmax = (R.lt + 30) >> 5;   // blocks r with a nonzero t[32 r + u - k]
    const int X0 = 32 * rmax + 31;
    const int ntw = ((X0 + 31) >> 2) + 1;
    __syncthreads();   // the previous round's operands are no longer read
    for (int w = tid; w < ntw; w += nthr) {
      uint32_t pk[8], lo[4], hi[4];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int i = X0 - 4 * w - b;
        pk[b] = digit_word((i >= 0 && i < R.lt) ? tv[i] : 0u);
      }
      transpose4(pk, lo);
      transpose4(pk + 4, hi);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ((uint32_t*)(tpl + (4 * s + 0) * ntp))[w] = lo[s];
        ((uint32_t*)(tpl + (4 * s + 1) * ntp))[w] = __builtin_amdgcn_alignbyte(hi[s], lo[s], 1);
        ((uint32_t*)(tpl + (4 * s + 2) * ntp))[w] = __builtin_amdgcn_alignbyte(hi[s], lo[s], 2);
        ((uint32_t*)(tpl + (4 * s + 3) * ntp))[w] = __builtin_amdgcn_alignbyte(hi[s], lo[s], 3);
      }
    }
    const int hwords = 8 * R.hblocks;
    for (int W = tid; W < hwords; W += nthr) {
      uint32_t pk[4] = {0u, 0u, 0u, 0u}, d[4];
      const int blk = W >> 3, wi = W & 7;
      const int ei = Ls.bent[R.b_begin + blk];
      if (ei >= 0) {
        const GEntry E = Ls.ents[ei];
        const uint32_t* hv = cptr(B, E.h, inst);
        const int i0 = 32 * (blk - E.hblk) + 4 * wi;
#pragma unroll
        for (int b = 0; b < 4; ++b) pk[b] = digit_word(i0 + b < E.lh ? hv[i0 + b] : 0u);
      }
      transpose4(pk, d);
      const int dst = (wi >> 2) * 4 * R.hblocks + 4 * blk + (wi & 3);
#pragma unroll
      for (int s = 0; s < 4; ++s) ((uint32_t*)(hpl + s * hp))[dst] = d[s];
    }
    __syncthreads();
    if (wave < G.ntiles) {
      const int r_lo = R.r_lo[wave], r_hi = R.r_hi[wave];
      if (r_lo <= r_hi) {
        const GCol c = Ls.cols[R.col_begin + m];
        // this lane's row u of the Toeplitz operand holds k = 16 hh + j (byte
        // j): t[32 r + u - k] = trev[s0 - 32 r + j]
        const int s0 = X0 - u + 16 * hh;
        const int e = s0 & 3;
        const uint8_t* ta = tpl + e * ntp + (s0 - e);
        const int jb0 = m - c.base;
        for (int r = r_lo; r <= r_hi; ++r) {
          i8x16 A[4], H[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const uint32_t* p = (const uint32_t*)(ta + 4 * s * ntp - 32 * r);
            const u32x4 v = {p[0], p[1], p[2], p[3]};
            A[s] = __builtin_bit_cast(i8x16, v);
          }
          const int jb = jb0 - r;
          const int hoff = 16 * (((unsigned)jb < (unsigned)c.J ? c.hblk + jb : 0) + hh * R.hblocks);
#pragma unroll
          for (int s = 0; s < 4; ++s) H[s] = __builtin_bit_cast(i8x16, *(const u32x4*)(hpl + s * hp + hoff));
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s)
              acc[a + s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], H[s], acc[a + s], 0, 0, 0);
        }
      }
    }
  }
  if (wave < G.ntiles) {
    const GOwn o = Ls.own[G.own_begin + m];
    if (o.parent >= 0) {
      const GParent P = Ls.pars[G.p_begin + o.parent];
      uint32_t* out = optr(B, P.out, inst);
      const uint64_t c0 = P.coef_node >= 0 ? B.coef[inst * B.n_nodes + P.coef_node] : 0u;
      constexpr int kShift[kGroups] = {0, 8, 16, 24, 1, 9, 17};   // 8 g mod 31
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int row = 8 * (rr >> 2) + 4 * hh + (rr & 3);
        const int n = 32 * (m - o.base) + row;
        int64_t v = 0;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) v += (int64_t)acc[g][rr] * (int64_t(1) << kShift[g]);
        // |v| < 2^31 (2^24 + 2^17 + 2^16 + 2^9 + 2^8 + 3) < 2^56: add 2^27 p
        const uint64_t w = (uint64_t)(v + ((int64_t)kP31 << 27)) + (n == 0 ? c0 : 0u);
        if (n < P.lout) out[n] = reduce31(w);
      }
    }
  }
}

__global__ void k_cm_zero(uint32_t* out, int64_t stride, int64_t from, int64_t len, int64_t batch) {
  const int64_t n = len - from;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < batch * n; i += (int64_t)gridDim.x * blockDim.x)
    out[(i / n) * stride + from + i % n] = 0u;
}

// ---------------------------------------------------------------------------
// host: the schedule (depths, groups, rounds), cached per tree and dq
// ---------------------------------------------------------------------------

struct Prod {      // h * t, t the power table entry `key`
  int32_t key;
  CRef t;
  int32_t lt;
  CRef h;
  int32_t lh;
};
struct Value {     // out = c(coef_node) + sum of prods
  CRef out;
  int32_t coef_node;
  int32_t lout;
  std::vector<Prod> prods;
};

struct Launch {
  int32_t mfma;
  int32_t begin, end;   // groups (mfma) or VALU parents
  int32_t waves;
  int32_t ntp, hp;
  int32_t max_lout;
};
struct CSched {
  int32_t dq = 0;
  std::vector<GGroup> groups;
  std::vector<GParent> gpars;
  std::vector<GRound> rounds;
  std::vector<GEntry> ents;
  std::vector<GCol> cols;
  std::vector<GOwn> own;
  std::vector<int32_t> bent;
  std::vector<CParent> vpars;
  std::vector<CChild> vch;
  std::vector<Launch> launches;
  int64_t arena_words = 0, out_len = 0, lmax = 0;
  size_t off[9] = {}, bytes[9] = {};   // device copies of the nine lists, then the arena
  size_t off_arena = 0;
  std::string err;
};

inline size_t al256(size_t v) { return (v + 255) & ~size_t(255); }
inline int32_t rmax_of(int32_t lt) { return (lt + 30) >> 5; }
// bytes of one Toeplitz plane: the words the reads reach, rounded up to 64 mod 256
inline int32_t ntp_of(int32_t lt) {
  const int32_t need = (((32 * rmax_of(lt) + 31) + 31) / 4 + 1) * 4;
  return need + ((64 - need) % 256 + 256) % 256;
}

// The rounds of a set of values: (power, occurrence) -> products.
struct RoundKey {
  int32_t key, occ;
  bool operator<(const RoundKey& o) const { return key != o.key ? key < o.key : occ < o.occ; }
};
std::map<RoundKey, std::vector<std::pair<int32_t, const Prod*>>> rounds_of(const std::vector<const Value*>& vals) {
  std::map<RoundKey, std::vector<std::pair<int32_t, const Prod*>>> R;
  for (int32_t j = 0; j < (int32_t)vals.size(); ++j) {
    std::map<int32_t, int32_t> seen;
    for (const Prod& p : vals[j]->prods) R[RoundKey{p.key, seen[p.key]++}].push_back({j, &p});
  }
  return R;
}
size_t group_lds(const std::vector<const Value*>& vals, int32_t* ntp_out, int32_t* hp_out) {
  int32_t ntp = ntp_of(1), hp = 32;
  for (auto& kv : rounds_of(vals)) {
    int32_t blocks = 1;
    for (auto& e : kv.second) blocks += (e.second->lh + 31) >> 5;
    ntp = std::max(ntp, ntp_of(kv.second.front().second->lt));
    hp = std::max(hp, 32 * blocks);
  }
  if (ntp_out) *ntp_out = ntp;
  if (hp_out) *hp_out = hp;
  return (size_t)16 * ntp + (size_t)4 * hp;
}

void add_group(CSched& S, const std::vector<const Value*>& vals, Launch& L) {
  GGroup G{};
  G.p_begin = (int32_t)S.gpars.size();
  G.rd_begin = (int32_t)S.rounds.size();
  G.own_begin = (int32_t)S.own.size();
  std::vector<int32_t> base(vals.size());
  int32_t nb = 0;
  for (size_t j = 0; j < vals.size(); ++j) {
    base[j] = nb;
    nb += (vals[j]->lout + 31) >> 5;
    S.gpars.push_back(GParent{vals[j]->out, vals[j]->coef_node, vals[j]->lout});
  }
  G.p_end = (int32_t)S.gpars.size();
  G.ntiles = (nb + 31) >> 5;
  for (int32_t m = 0; m < kCols; ++m) {
    GOwn o{-1, 0};
    for (size_t j = 0; j < vals.size(); ++j)
      if (m >= base[j] && m < base[j] + ((vals[j]->lout + 31) >> 5)) o = GOwn{(int32_t)j, base[j]};
    S.own.push_back(o);
  }
  for (auto& kv : rounds_of(vals)) {
    GRound R{};
    const Prod* p0 = kv.second.front().second;
    R.t = p0->t;
    R.lt = p0->lt;
    R.e_begin = (int32_t)S.ents.size();
    R.col_begin = (int32_t)S.cols.size();
    R.b_begin = (int32_t)S.bent.size();
    const int32_t rmax = rmax_of(R.lt);
    std::vector<GCol> col(kCols, GCol{0, 0, 0});
    int32_t blocks = 1;
    S.bent.push_back(-1);
    for (auto& e : kv.second) {
      const int32_t j = e.first;
      const int32_t J = (e.second->lh + 31) >> 5;
      for (int32_t k = 0; k < J; ++k) S.bent.push_back((int32_t)S.ents.size());
      S.ents.push_back(GEntry{e.second->h, e.second->lh, blocks});
      const int32_t nbj = (vals[j]->lout + 31) >> 5;
      for (int32_t m = base[j]; m < base[j] + nbj; ++m) col[m] = GCol{blocks, base[j], J};
      blocks += J;
    }
    R.e_end = (int32_t)S.ents.size();
    R.hblocks = blocks;
    for (int32_t w = 0; w < kMaxTiles; ++w) {
      int32_t lo = 1 << 30, hi = -1;
      for (int32_t m = 32 * w; m < 32 * w + 32; ++m) {
        if (col[m].J == 0) continue;
        lo = std::min(lo, std::max(0, m - col[m].base - col[m].J + 1));
        hi = std::max(hi, std::min(rmax, m - col[m].base));
      }
      R.r_lo[w] = lo <= hi ? lo : 1;
      R.r_hi[w] = lo <= hi ? hi : 0;
    }
    S.cols.insert(S.cols.end(), col.begin(), col.end());
    S.rounds.push_back(R);
  }
  G.rd_end = (int32_t)S.rounds.size();
  S.groups.push_back(G);
  int32_t ntp = 0, hp = 0;
  group_lds(vals, &ntp, &hp);
  L.ntp = std::max(L.ntp, ntp);
  L.hp = std::max(L.hp, hp);
  L.waves = std::max(L.waves, G.ntiles);
}

// One dependency depth: its values packed into groups (matrix cores) or
// left to the VALU kernel.
void add_depth(CSched& S, const std::vector<Value>& vals) {
  std::vector<const Value*> mf, va;
  for (const Value& v : vals) {
    int64_t sum_min = 0;
    for (const Prod& p : v.prods) sum_min += std::min(p.lt, p.lh);
    bool ok = v.lout <= kCols * 32 && sum_min < kExactLimit;
    if (ok) ok = group_lds({&v}, nullptr, nullptr) <= kMaxLds;
    (ok ? mf : va).push_back(&v);
  }
  Launch L{1, (int32_t)S.groups.size(), 0, 1, 16, 32, 0};
  std::vector<const Value*> cur;
  int32_t blocks = 0;
  auto flush = [&]() {
    if (cur.empty()) return;
    if ((int32_t)S.groups.size() - L.begin == kMaxLaunchY) {
      L.end = (int32_t)S.groups.size();
      S.launches.push_back(L);
      L = Launch{1, (int32_t)S.groups.size(), 0, 1, 16, 32, 0};
    }
    add_group(S, cur, L);
    cur.clear();
    blocks = 0;
  };
  for (const Value* v : mf) {
    const int32_t nb = (v->lout + 31) >> 5;
    if (!cur.empty()) {
      std::vector<const Value*> trial = cur;
      trial.push_back(v);
      if (blocks + nb > kCols || group_lds(trial, nullptr, nullptr) > kMaxLds) flush();
    }
    cur.push_back(v);
    blocks += nb;
  }
  flush();
  L.end = (int32_t)S.groups.size();
  if (L.end > L.begin) S.launches.push_back(L);
  for (size_t b = 0; b < va.size(); b += kMaxLaunchY) {
    Launch V{0, (int32_t)S.vpars.size(), 0, 0, 0, 0, 0};
    for (size_t k = b; k < std::min(va.size(), b + kMaxLaunchY); ++k) {
      const Value* v = va[k];
      CParent P{v->out, v->coef_node, (int32_t)S.vch.size(), 0, v->lout};
      for (const Prod& p : v->prods) S.vch.push_back(CChild{p.h, p.t, p.lh, p.lt});
      P.child_end = (int32_t)S.vch.size();
      S.vpars.push_back(P);
      V.max_lout = std::max(V.max_lout, v->lout);
    }
    V.end = (int32_t)S.vpars.size();
    S.launches.push_back(V);
  }
}

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
  std::vector<std::vector<Value>> by_depth(1);
  auto put = [&](int64_t d, Value v) {
    if ((int64_t)by_depth.size() <= d) by_depth.resize(d + 1);
    by_depth[d].push_back(std::move(v));
  };
  // powers: a LOAD is the caller's q itself
  std::vector<CRef> tref(t->n_table);
  std::vector<int64_t> tlen(t->n_table, 0), tdepth(t->n_table, 0);
  for (size_t c = 0; c < t->chain.size(); ++c) {
    const ChainStep& st = t->chain[c];
    if (st.kind == kChainLoad) {
      tref[st.dst] = CRef{cQ, 0, 0};
      tlen[st.dst] = dq + 1;
      continue;
    }
    tdepth[st.dst] = 1 + std::max(tdepth[st.s1], tdepth[st.s2]);
    tlen[st.dst] = tlen[st.s1] + tlen[st.s2] - 1;
    tref[st.dst] = CRef{cArena, 0, alloc(tlen[st.dst])};
    Value v{tref[st.dst], -1, (int32_t)tlen[st.dst], {}};
    v.prods.push_back(Prod{st.s2, tref[st.s2], (int32_t)tlen[st.s2], tref[st.s1], (int32_t)tlen[st.s1]});
    put(tdepth[st.dst], std::move(v));
  }
  auto pow_of = [&](int64_t i) -> int32_t {
    const fpe_node& nd = t->nodes[i];
    for (int32_t e = 0; e < t->n_table; ++e)
      if (t->table_deg[e] == nd.pdeg && t->table_var[e] == nd.var) return e;
    return -1;
  };
  std::vector<std::vector<int64_t>> kids(N);
  for (int64_t i = 0; i < N; ++i)
    if (t->nodes[i].parent >= 0) kids[t->nodes[i].parent].push_back(i);
  std::vector<int64_t> vlen(N, 1), vdepth(N, 0);
  std::vector<CRef> vref(N);
  const int64_t R = N - 1;
  const bool root_pow = t->nodes[R].pdeg > 0;
  for (int64_t i = 0; i < N; ++i) {   // children have lower indices
    vref[i] = CRef{cCoef, (int32_t)i, 0};   // a leaf's value is its coefficient
    if (kids[i].empty()) continue;
    Value v{CRef{}, (int32_t)i, 1, {}};
    int64_t d = 0, len = 1;
    for (int64_t c : kids[i]) {
      const int32_t e = pow_of(c);
      if (e < 0) {
        S.err = "composition needs every power in the table";
        return S;
      }
      v.prods.push_back(Prod{e, tref[e], (int32_t)tlen[e], vref[c], (int32_t)vlen[c]});
      d = std::max({d, vdepth[c], tdepth[e]});
      len = std::max(len, vlen[c] + tlen[e] - 1);
    }
    vlen[i] = len;
    vdepth[i] = d + 1;
    vref[i] = (i == R && !root_pow) ? CRef{cOut, 0, 0} : CRef{cArena, 0, alloc(len)};
    v.out = vref[i];
    v.lout = (int32_t)len;
    put(vdepth[i], std::move(v));
  }
  if (root_pow) {
    const int32_t e = pow_of(R);
    if (e < 0) {
      S.err = "composition needs every power in the table";
      return S;
    }
    S.out_len = vlen[R] + tlen[e] - 1;
    Value v{CRef{cOut, 0, 0}, -1, (int32_t)S.out_len, {}};
    v.prods.push_back(Prod{e, tref[e], (int32_t)tlen[e], vref[R], (int32_t)vlen[R]});
    put(1 + std::max(vdepth[R], tdepth[e]), std::move(v));
  } else if (kids[R].empty()) {   // p is a constant: out = c(R)
    S.out_len = 1;
    put(1, Value{CRef{cOut, 0, 0}, (int32_t)R, 1, {}});
  } else {
    S.out_len = vlen[R];
  }
  if (S.out_len > S.lmax) {
    S.err = "internal: composition output longer than deg_p * dq + 1";
    return S;
  }
  for (size_t d = 1; d < by_depth.size(); ++d)
    if (!by_depth[d].empty()) add_depth(S, by_depth[d]);
  S.arena_words = (words + 63) & ~int64_t(63);
  const size_t sizes[9] = {S.groups.size() * sizeof(GGroup), S.gpars.size() * sizeof(GParent),
                           S.rounds.size() * sizeof(GRound), S.ents.size() * sizeof(GEntry),
                           S.cols.size() * sizeof(GCol),     S.own.size() * sizeof(GOwn),
                           S.vpars.size() * sizeof(CParent), S.vch.size() * sizeof(CChild),
                           S.bent.size() * sizeof(int32_t)};
  size_t o = 0;
  for (int k = 0; k < 9; ++k) {
    S.off[k] = o;
    S.bytes[k] = sizes[k];
    o = al256(o + sizes[k]);
  }
  S.off_arena = o;
  return S;
}

struct CCache {
  std::mutex mu;
  std::vector<std::pair<const fpe_tree*, CSched>> entries;
};
CCache& ccache() {
  static CCache c;
  return c;
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

bool compose_levels_ok(const fpe_tree* t, int32_t dq, int64_t* launches) {
  const CSched* S = csched_for(t, dq);
  if (launches) *launches = (int64_t)S->launches.size();
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
  // the schedule lives as long as the tree's cache entry, so the copies read
  // live memory whenever they run
  const void* src[9] = {S->groups.data(), S->gpars.data(), S->rounds.data(), S->ents.data(), S->cols.data(),
                        S->own.data(),    S->vpars.data(), S->vch.data(),    S->bent.data()};
  hipError_t e = hipSuccess;
  for (int k = 0; k < 9 && e == hipSuccess; ++k)
    if (S->bytes[k]) e = hipMemcpyAsync(base + S->off[k], src[k], S->bytes[k], hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition: ") + hipGetErrorString(e));
  GLists Ls{(const GGroup*)(base + S->off[0]), (const GParent*)(base + S->off[1]),
            (const GRound*)(base + S->off[2]), (const GEntry*)(base + S->off[3]),
            (const GCol*)(base + S->off[4]),   (const GOwn*)(base + S->off[5]),
            (const int32_t*)(base + S->off[8])};
  const CParent* vpars = (const CParent*)(base + S->off[6]);
  const CChild* vch = (const CChild*)(base + S->off[7]);
  CBases B{(uint32_t*)(base + S->off_arena), q, out, dev_view(t).coef_rows, S->arena_words, (int64_t)dq + 1,
           S->lmax, (int64_t)t->nodes.size()};
  for (const Launch& L : S->launches) {
    const int n = L.end - L.begin;
    if (L.mfma) {
      GLists Lg = Ls;
      Lg.groups += L.begin;
      const size_t lds = (size_t)16 * L.ntp + (size_t)4 * L.hp;
      hipLaunchKernelGGL(k_cm_mfma, dim3((unsigned)t->batch, n), dim3(64 * L.waves), lds, st, Lg, B, L.ntp, L.hp);
    } else {
      const int64_t gx = (t->batch * L.max_lout + 255) / 256;
      hipLaunchKernelGGL(k_cm_valu, dim3((unsigned)gx, n), dim3(256), 0, st, vpars + L.begin, vch, B, t->batch);
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
