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
// in the columns (output blocks) of up to four tiles; its four wavefronts
// share the tiles' work evenly.
// Their products are taken in rounds, one per power q^d: the power is the
// Toeplitz operand shared by every value of the group that multiplies it,
// and each value's factor sits in its own blocks of the h operand, so the
// small products of the lower levels fill the tiles as well as the large ones
// at the top.  Values beyond four tiles (4096 coefficients) or the exactness
// bound, and the short values of the lowest levels (at most 64
// coefficients: too little work to pay for a workgroup's staging) go to a
// VALU schoolbook kernel (a thread per output coefficient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "fpe_internal.h"

namespace fpe {

namespace {

typedef int8_t i8x16 __attribute__((ext_vector_type(16)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxTiles = 4;             // tiles (32 x 32 outputs) of one workgroup
constexpr int kWaves = 4;                // wavefronts of one workgroup
constexpr int kCols = 32 * kMaxTiles;    // output blocks of 32 coefficients per workgroup
constexpr int kObufTile = 32 * 33;       // 64-bit sums of one tile in LDS (rows padded to 33)
constexpr int32_t kValuMaxOut = 64;      // values this short go to the VALU kernel (latency-bound either way)
constexpr int kGroups = 7;               // digit pairs (s, a) grouped by s + a
constexpr int kMaxLaunchY = 65535;
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
  int32_t hblocks;          // 32-byte blocks of each h digit plane (block 0: zeros)
  int32_t b_begin;          // hblocks records: the entry of each block (-1: zeros)
  int32_t pe_begin;         // one record per value of the group: its entry in this round (-1: none)
  int32_t tbase, ntp;       // LDS byte offset of the 4 t digit planes, bytes per plane
  int32_t hbase;            // LDS byte offset of the 4 h digit planes (32 hblocks bytes each)
  int32_t pad;
};
struct GEntry {    // one factor: its blocks start at block hblk (>= 1) of the h planes
  CRef h;
  int32_t lh;
  int32_t hblk;
};
struct GOwn {      // column m of a group: its value (-1: none) and the value's first column
  int32_t parent, base;
};
struct GSeg {      // blocks r in [r_lo, r_hi] of one round for one tile
  int32_t tile, round, r_lo, r_hi;
};
// A group's records are contiguous in each list; the kernel copies them to
// LDS (at mbase) before anything else.
struct GGroup {
  int32_t p_begin, p_end, rd_begin, rd_end, e_begin, e_end, b_begin, b_end, pe_begin, pe_end;
  int32_t own_begin;
  int32_t ntiles;
  int32_t obase;                               // LDS byte offset of the tiles' sums
  int32_t mbase;                               // LDS byte offset of the copied records
  int32_t seg_begin[kWaves], seg_end[kWaves];  // the segments of each wavefront
  int32_t s_begin, s_end;                      // all of the group's segments
};
struct GLists {
  const GGroup* groups;
  const GParent* pars;
  const GRound* rounds;
  const GEntry* ents;
  const GOwn* own;
  const int32_t* bent;
  const int32_t* pent;
  const GSeg* segs;
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

// The 16 Toeplitz bytes of this lane for one digit plane, from the five
// aligned words d (its window starts e bytes into d[0]).
__device__ __forceinline__ i8x16 toeplitz_bytes(const uint32_t d[5], uint32_t e) {
  const u32x4 v = {__builtin_amdgcn_alignbyte(d[1], d[0], e), __builtin_amdgcn_alignbyte(d[2], d[1], e),
                   __builtin_amdgcn_alignbyte(d[3], d[2], e), __builtin_amdgcn_alignbyte(d[4], d[3], e)};
  return __builtin_bit_cast(i8x16, v);
}

__device__ __forceinline__ void copy_words(void* dst, const void* src, int bytes) {
  for (int i = threadIdx.x; i < bytes / 4; i += blockDim.x) ((uint32_t*)dst)[i] = ((const uint32_t*)src)[i];
}
__host__ __device__ constexpr int al16(int v) { return (v + 15) & ~15; }

// A workgroup copies its group's records to LDS, stages every round's
// operands in LDS at once, then each wavefront runs its own list of segments
// (the host splits the group's (tile, round, block) work evenly over the
// four wavefronts), adding the partial sums of each tile it touched into the
// tiles' 64-bit sums in LDS.
//
// LDS per round: 4 digit planes of the Toeplitz operand, where byte y of
// plane s is digit s of trev[y] = t[X0 - y] (zero outside t): the lane's 16
// bytes for block r start at byte s0 - 32 r (s0 = X0 - u + 16 hh) and are
// cut from five aligned words; then 4 digit planes of h in 32-byte blocks
// (block 0 zeros, read by the lanes whose block falls outside their factor),
// each plane as two halves (bytes 0..15 of every block, then 16..31) so the
// 16-byte reads of consecutive lanes are consecutive.  The tiles' sums are
// 32 x 33 words per tile (row-major, padded), residues < p added by at most
// four wavefronts.  Each block step loads and cuts one Toeplitz plane at a
// time, so a plane's loads are in flight while the previous plane's products
// run; three wavefronts per SIMD hide the rest.
__global__ __launch_bounds__(256, 3) void k_cm_mfma(GLists Ls, CBases B) {
  extern __shared__ __align__(16) uint8_t lds[];
  const GGroup G = Ls.groups[blockIdx.y];
  const int64_t inst = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int u = lane & 31, hh = lane >> 5;
  const int npar = G.p_end - G.p_begin;
  // the group's records
  uint8_t* mp = lds + G.mbase;
  GRound* Rl = (GRound*)mp;
  mp += al16((G.rd_end - G.rd_begin) * (int)sizeof(GRound));
  GEntry* El = (GEntry*)mp;
  mp += al16((G.e_end - G.e_begin) * (int)sizeof(GEntry));
  GParent* Pl = (GParent*)mp;
  mp += al16(npar * (int)sizeof(GParent));
  GOwn* Ol = (GOwn*)mp;
  mp += al16(kCols * (int)sizeof(GOwn));
  int32_t* Bl = (int32_t*)mp;
  mp += al16((G.b_end - G.b_begin) * 4);
  int32_t* PEl = (int32_t*)mp;
  mp += al16((G.pe_end - G.pe_begin) * 4);
  GSeg* Sl = (GSeg*)mp;
  mp += al16((G.s_end - G.s_begin) * (int)sizeof(GSeg));
  uint32_t* Cl = (uint32_t*)mp;
  copy_words(Rl, Ls.rounds + G.rd_begin, (G.rd_end - G.rd_begin) * (int)sizeof(GRound));
  copy_words(El, Ls.ents + G.e_begin, (G.e_end - G.e_begin) * (int)sizeof(GEntry));
  copy_words(Pl, Ls.pars + G.p_begin, npar * (int)sizeof(GParent));
  copy_words(Ol, Ls.own + G.own_begin, kCols * (int)sizeof(GOwn));
  copy_words(Bl, Ls.bent + G.b_begin, (G.b_end - G.b_begin) * 4);
  copy_words(PEl, Ls.pent + G.pe_begin, (G.pe_end - G.pe_begin) * 4);
  copy_words(Sl, Ls.segs + G.s_begin, (G.s_end - G.s_begin) * (int)sizeof(GSeg));
  uint64_t* obuf = (uint64_t*)(lds + G.obase);
  for (int i = tid; i < G.ntiles * kObufTile; i += blockDim.x) obuf[i] = 0u;
  __syncthreads();
  // the values' constants: issued now, in flight with the staging loads
  for (int j = tid; j < npar; j += blockDim.x) {
    const int cn = Pl[j].coef_node;
    Cl[j] = cn >= 0 ? B.coef[inst * B.n_nodes + cn] : 0u;
  }

  for (int rl = 0; rl < G.rd_end - G.rd_begin; ++rl) {
    const GRound& R = Rl[rl];
    const uint32_t* tv = cptr(B, R.t, inst);
    const int lt = R.lt;
    const int X0 = 32 * ((lt + 30) >> 5) + 31;
    uint32_t* tp = (uint32_t*)(lds + R.tbase);
    const int ntw = R.ntp >> 2;
    for (int w = tid; w < ntw; w += blockDim.x) {
      uint32_t pk[4], d[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = X0 - 4 * w - b;
        pk[b] = digit_word((i >= 0 && i < lt) ? tv[i] : 0u);
      }
      transpose4(pk, d);
#pragma unroll
      for (int s = 0; s < 4; ++s) tp[s * ntw + w] = d[s];
    }
    uint32_t* hp = (uint32_t*)(lds + R.hbase);
    const int hb = R.hblocks, hwords = 8 * hb;
    for (int W = tid; W < hwords; W += blockDim.x) {
      uint32_t pk[4] = {0u, 0u, 0u, 0u}, d[4];
      const int blk = W >> 3, wi = W & 7;
      const int ei = Bl[R.b_begin - G.b_begin + blk];
      if (ei >= 0) {
        const GEntry& E = El[ei - G.e_begin];
        const uint32_t* hv = cptr(B, E.h, inst);
        const int i0 = 32 * (blk - E.hblk) + 4 * wi;
#pragma unroll
        for (int b = 0; b < 4; ++b) pk[b] = digit_word(i0 + b < E.lh ? hv[i0 + b] : 0u);
      }
      transpose4(pk, d);
      const int dst = (wi >> 2) * 4 * hb + 4 * blk + (wi & 3);
#pragma unroll
      for (int s = 0; s < 4; ++s) hp[s * hwords + dst] = d[s];
    }
  }
  __syncthreads();

  i32x16 acc[kGroups];
#pragma unroll
  for (int g = 0; g < kGroups; ++g) acc[g] = i32x16{};
  auto flush = [&](int tile) {
    constexpr int kShift[kGroups] = {0, 8, 16, 24, 1, 9, 17};   // 8 g mod 31
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int row = 8 * (rr >> 2) + 4 * hh + (rr & 3);
      int64_t v = 0;
#pragma unroll
      for (int g = 0; g < kGroups; ++g) v += (int64_t)acc[g][rr] * (int64_t(1) << kShift[g]);
      // |v| < 2^31 (2^24 + 2^17 + 2^16 + 2^9 + 2^8 + 3) < 2^56, added as a
      // two's-complement 64-bit word: each wavefront's share of the tiles is
      // contiguous in tile order, so it flushes a tile at most once and a
      // tile's sum has at most kWaves terms, |sum| < 2^58 (reduced once, in
      // the output pass)
      atomicAdd((unsigned long long*)&obuf[tile * kObufTile + row * 33 + u], (unsigned long long)v);
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) acc[g] = i32x16{};
  };
  int cur = -1;
  for (int sg = G.seg_begin[wave]; sg < G.seg_end[wave]; ++sg) {
    const GSeg S = Sl[sg - G.s_begin];
    if (S.tile != cur) {
      if (cur >= 0) flush(cur);
      cur = S.tile;
    }
    const GRound& R = Rl[S.round - G.rd_begin];
    // this lane's output block, its value's factor in this round
    const int m = 32 * S.tile + u;
    const GOwn o = Ol[m];
    int hblk = 0, J = 0, jb0 = 0;
    if (o.parent >= 0) {
      const int ei = PEl[R.pe_begin - G.pe_begin + o.parent];
      if (ei >= 0) {
        hblk = El[ei - G.e_begin].hblk;
        J = (El[ei - G.e_begin].lh + 31) >> 5;
        jb0 = m - o.base;
      }
    }
    // this lane's row u of the Toeplitz operand holds k = 16 hh + j (byte
    // j): t[32 r + u - k] = trev[s0 - 32 r + j]
    const int X0 = 32 * ((R.lt + 30) >> 5) + 31;
    const int s0 = X0 - u + 16 * hh;
    const uint32_t e = s0 & 3;
    const int ntw = R.ntp >> 2;
    const uint32_t* tp = (const uint32_t*)(lds + R.tbase) + (s0 >> 2);
    const uint8_t* hp = lds + R.hbase + 16 * hh * R.hblocks;
    const int hpb = 32 * R.hblocks;
    for (int r = S.r_lo; r <= S.r_hi; ++r) {
      const int jb = jb0 - r;
      const int off = 16 * ((unsigned)jb < (unsigned)J ? hblk + jb : 0);
      u32x4 h[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) h[s] = *(const u32x4*)(hp + s * hpb + off);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        uint32_t w[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) w[k] = tp[a * ntw - 8 * r + k];
        const i8x16 A = toeplitz_bytes(w, e);
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc[a + s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, __builtin_bit_cast(i8x16, h[s]), acc[a + s], 0, 0, 0);
      }
    }
  }
  if (cur >= 0) flush(cur);
  __syncthreads();
  for (int idx = tid; idx < G.ntiles * 1024; idx += blockDim.x) {
    const int tile = idx >> 10, col = (idx >> 5) & 31, row = idx & 31;
    const int m = 32 * tile + col;
    const GOwn o = Ol[m];
    if (o.parent < 0) continue;
    const GParent& P = Pl[o.parent];
    const int n = 32 * (m - o.base) + row;
    if (n >= P.lout) continue;
    // the signed sum plus 2^28 p (> 2^58) is non-negative and below 2^60
    uint64_t v = (uint64_t)((int64_t)obuf[tile * kObufTile + row * 33 + col] + ((int64_t)kP31 << 28));
    if (n == 0) v += Cl[o.parent];
    optr(B, P.out, inst)[n] = reduce31(v);
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
  int32_t lds;          // dynamic LDS bytes (mfma)
  int32_t max_lout;
};
// The schedule's lists in one pinned host buffer, copied to the workspace by
// one asynchronous copy per call; freed once the last copy from it is done.
struct PinnedLists {
  uint8_t* p = nullptr;
  std::vector<uint8_t> pageable;   // if pinned memory is unavailable
  hipEvent_t done = nullptr;       // recorded after each copy from p
  PinnedLists() = default;
  PinnedLists(const PinnedLists&) = delete;
  PinnedLists& operator=(const PinnedLists&) = delete;
  ~PinnedLists() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (p) (void)hipHostFree(p);
  }
  uint8_t* data() { return p ? p : pageable.data(); }
};

struct CSched {
  int32_t dq = 0;
  std::vector<GGroup> groups;
  std::vector<GParent> gpars;
  std::vector<GRound> rounds;
  std::vector<GEntry> ents;
  std::vector<GOwn> own;
  std::vector<int32_t> bent, pent;
  std::vector<GSeg> segs;
  std::vector<CParent> vpars;
  std::vector<CChild> vch;
  std::vector<Launch> launches;
  int64_t arena_words = 0, out_len = 0, lmax = 0;
  size_t lds_limit = 0;
  size_t off[10] = {}, bytes[10] = {};   // device copies of the ten lists, then the arena
  size_t off_arena = 0;
  std::shared_ptr<PinnedLists> lists;
  std::string err;
};

inline size_t al256(size_t v) { return (v + 255) & ~size_t(255); }
inline int32_t rmax_of(int32_t lt) { return (lt + 30) >> 5; }
// bytes of one Toeplitz digit plane: up to the fifth word of the last window
// (byte X0 + 35), rounded up to 16
inline int32_t ntp_of(int32_t lt) {
  const int32_t X0 = 32 * rmax_of(lt) + 31;
  return (4 * ((X0 + 16) / 4 + 5) + 15) & ~15;
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
// LDS bytes of a group's copied records.
int32_t meta_bytes(int32_t rounds, int32_t ents, int32_t pars, int32_t bents, int32_t pents, int32_t segs) {
  return al16(rounds * (int)sizeof(GRound)) + al16(ents * (int)sizeof(GEntry)) + al16(pars * (int)sizeof(GParent)) +
         al16(kCols * (int)sizeof(GOwn)) + al16(bents * 4) + al16(pents * 4) + al16(segs * (int)sizeof(GSeg)) +
         al16(pars * 4);
}
// LDS of a group: every round's t and h planes, the tiles' sums, the records.
size_t group_lds(const std::vector<const Value*>& vals) {
  size_t bytes = 0;
  int32_t nb = 0, nr = 0, ne = 0, nbe = 0;
  for (const Value* v : vals) nb += (v->lout + 31) >> 5;
  for (auto& kv : rounds_of(vals)) {
    int32_t blocks = 1;
    for (auto& e : kv.second) blocks += (e.second->lh + 31) >> 5;
    bytes += 4 * (size_t)ntp_of(kv.second.front().second->lt) + 4 * 32 * (size_t)blocks;
    ++nr;
    ne += (int32_t)kv.second.size();
    nbe += blocks;
  }
  const int32_t np = (int32_t)vals.size(), nt = (nb + 31) >> 5;
  // segments: at most one per tile and round, plus one per cut between shares
  return ((bytes + 15) & ~size_t(15)) + (size_t)nt * kObufTile * 8 +
         meta_bytes(nr, ne, np, nbe, nr * np, nr * nt + kWaves);
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
  // rounds, their LDS planes, and the work of each tile (a list of (round,
  // r_lo, r_hi) per tile)
  std::vector<std::vector<GSeg>> work(G.ntiles);
  int32_t lds = 0;
  G.e_begin = (int32_t)S.ents.size();
  G.b_begin = (int32_t)S.bent.size();
  G.pe_begin = (int32_t)S.pent.size();
  struct Col {
    int32_t base, J;
  };
  for (auto& kv : rounds_of(vals)) {
    GRound R{};
    const Prod* p0 = kv.second.front().second;
    R.t = p0->t;
    R.lt = p0->lt;
    R.b_begin = (int32_t)S.bent.size();
    R.pe_begin = (int32_t)S.pent.size();
    R.ntp = ntp_of(R.lt);
    R.tbase = lds;
    lds += 4 * R.ntp;
    const int32_t rmax = rmax_of(R.lt);
    std::vector<Col> col(kCols, Col{0, 0});
    std::vector<int32_t> pe(vals.size(), -1);
    int32_t blocks = 1;
    S.bent.push_back(-1);
    for (auto& e : kv.second) {
      const int32_t j = e.first;
      const int32_t J = (e.second->lh + 31) >> 5;
      for (int32_t k = 0; k < J; ++k) S.bent.push_back((int32_t)S.ents.size());
      pe[j] = (int32_t)S.ents.size();
      S.ents.push_back(GEntry{e.second->h, e.second->lh, blocks});
      const int32_t nbj = (vals[j]->lout + 31) >> 5;
      for (int32_t m = base[j]; m < base[j] + nbj; ++m) col[m] = Col{base[j], J};
      blocks += J;
    }
    S.pent.insert(S.pent.end(), pe.begin(), pe.end());
    R.hblocks = blocks;
    R.hbase = lds;
    lds += 4 * 32 * blocks;
    const int32_t rd = (int32_t)S.rounds.size();
    for (int32_t w = 0; w < G.ntiles; ++w) {
      int32_t lo = 1 << 30, hi = -1;
      for (int32_t m = 32 * w; m < 32 * w + 32; ++m) {
        if (col[m].J == 0) continue;
        lo = std::min(lo, std::max(0, m - col[m].base - col[m].J + 1));
        hi = std::max(hi, std::min(rmax, m - col[m].base));
      }
      if (lo <= hi) work[w].push_back(GSeg{w, rd, lo, hi});
    }
    S.rounds.push_back(R);
  }
  G.rd_end = (int32_t)S.rounds.size();
  G.e_end = (int32_t)S.ents.size();
  G.b_end = (int32_t)S.bent.size();
  G.pe_end = (int32_t)S.pent.size();
  G.obase = (lds + 15) & ~15;
  G.mbase = G.obase + G.ntiles * kObufTile * 8;
  // the tiles' work, tile by tile, cut into kWaves contiguous shares of
  // (nearly) equal numbers of blocks
  int64_t total = 0;
  for (auto& wl : work)
    for (auto& sg : wl) total += sg.r_hi - sg.r_lo + 1;
  auto bound = [&](int32_t k) { return total * k / kWaves; };   // first block of share k
  int64_t pos = 0;
  int32_t wv = 0;
  G.seg_begin[0] = (int32_t)S.segs.size();
  for (auto& wl : work)
    for (const GSeg& sg : wl)
      for (int32_t lo = sg.r_lo; lo <= sg.r_hi;) {
        while (wv + 1 < kWaves && pos >= bound(wv + 1)) {
          G.seg_end[wv] = (int32_t)S.segs.size();
          G.seg_begin[++wv] = (int32_t)S.segs.size();
        }
        const int64_t lim = wv + 1 < kWaves ? bound(wv + 1) : INT64_MAX;
        const int32_t len = (int32_t)std::min<int64_t>(sg.r_hi - lo + 1, lim - pos);
        S.segs.push_back(GSeg{sg.tile, sg.round, lo, lo + len - 1});
        lo += len;
        pos += len;
      }
  G.seg_end[wv] = (int32_t)S.segs.size();
  for (int32_t k = wv + 1; k < kWaves; ++k) G.seg_begin[k] = G.seg_end[k] = (int32_t)S.segs.size();
  G.s_begin = G.seg_begin[0];
  G.s_end = (int32_t)S.segs.size();
  lds = G.mbase + meta_bytes(G.rd_end - G.rd_begin, G.e_end - G.e_begin, G.p_end - G.p_begin, G.b_end - G.b_begin,
                             G.pe_end - G.pe_begin, G.s_end - G.s_begin);
  S.groups.push_back(G);
  L.lds = std::max(L.lds, lds);
}

// One dependency depth: its values packed into groups (matrix cores) or
// left to the VALU kernel.
void add_depth(CSched& S, const std::vector<Value>& vals) {
  std::vector<const Value*> mf, va;
  for (const Value& v : vals) {
    int64_t sum_min = 0;
    for (const Prod& p : v.prods) sum_min += std::min(p.lt, p.lh);
    bool ok = v.lout > kValuMaxOut && v.lout <= kCols * 32 && sum_min < kExactLimit;
    if (ok) ok = group_lds({&v}) <= S.lds_limit;
    (ok ? mf : va).push_back(&v);
  }
  Launch L{1, (int32_t)S.groups.size(), 0, 0, 0};
  std::vector<const Value*> cur;
  int32_t blocks = 0;
  auto flush = [&]() {
    if (cur.empty()) return;
    if ((int32_t)S.groups.size() - L.begin == kMaxLaunchY) {
      L.end = (int32_t)S.groups.size();
      S.launches.push_back(L);
      L = Launch{1, (int32_t)S.groups.size(), 0, 0, 0};
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
      if (blocks + nb > kCols || group_lds(trial) > S.lds_limit) flush();
    }
    cur.push_back(v);
    blocks += nb;
  }
  flush();
  L.end = (int32_t)S.groups.size();
  if (L.end > L.begin) S.launches.push_back(L);
  for (size_t b = 0; b < va.size(); b += kMaxLaunchY) {
    Launch V{0, (int32_t)S.vpars.size(), 0, 0, 0};
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

// LDS a workgroup may allocate on the current device (64 KB if unknown).
size_t lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  return (size_t)v;
}

CSched build_csched(const fpe_tree* t, int32_t dq) {
  CSched S;
  S.dq = dq;
  S.lds_limit = lds_limit();
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
  const size_t sizes[10] = {S.groups.size() * sizeof(GGroup), S.gpars.size() * sizeof(GParent),
                            S.rounds.size() * sizeof(GRound), S.ents.size() * sizeof(GEntry),
                            S.own.size() * sizeof(GOwn),      S.bent.size() * sizeof(int32_t),
                            S.pent.size() * sizeof(int32_t),  S.segs.size() * sizeof(GSeg),
                            S.vpars.size() * sizeof(CParent), S.vch.size() * sizeof(CChild)};
  size_t o = 0;
  for (int k = 0; k < 10; ++k) {
    S.off[k] = o;
    S.bytes[k] = sizes[k];
    o = al256(o + sizes[k]);
  }
  S.off_arena = o;
  S.lists = std::make_shared<PinnedLists>();
  PinnedLists& H = *S.lists;
  if (hipHostMalloc((void**)&H.p, std::max<size_t>(o, 256), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&H.done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (H.p) (void)hipHostFree(H.p);
    H.p = nullptr;
    H.done = nullptr;
    H.pageable.assign(std::max<size_t>(o, 256), 0);
  }
  const void* src[10] = {S.groups.data(), S.gpars.data(), S.rounds.data(), S.ents.data(), S.own.data(),
                         S.bent.data(),   S.pent.data(),  S.segs.data(),  S.vpars.data(), S.vch.data()};
  std::memset(H.data(), 0, o);
  for (int k = 0; k < 10; ++k)
    if (S.bytes[k]) std::memcpy(H.data() + S.off[k], src[k], S.bytes[k]);
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
  // the lists stay alive until this copy has run (their buffer waits for
  // the event before it is freed)
  hipError_t e = hipMemcpyAsync(base, S->lists->data(), S->off_arena, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && S->lists->done) e = hipEventRecord(S->lists->done, st);
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition: ") + hipGetErrorString(e));
  GLists Ls{(const GGroup*)(base + S->off[0]), (const GParent*)(base + S->off[1]),
            (const GRound*)(base + S->off[2]), (const GEntry*)(base + S->off[3]),
            (const GOwn*)(base + S->off[4]),   (const int32_t*)(base + S->off[5]),
            (const int32_t*)(base + S->off[6]), (const GSeg*)(base + S->off[7])};
  const CParent* vpars = (const CParent*)(base + S->off[8]);
  const CChild* vch = (const CChild*)(base + S->off[9]);
  CBases B{(uint32_t*)(base + S->off_arena), q, out, dev_view(t).coef_rows, S->arena_words, (int64_t)dq + 1,
           S->lmax, (int64_t)t->nodes.size()};
  for (const Launch& L : S->launches) {
    const int n = L.end - L.begin;
    if (L.mfma) {
      GLists Lg = Ls;
      Lg.groups += L.begin;
      if (L.lds > 64 * 1024) {   // raise the kernel's dynamic LDS limit once per larger size
        static std::mutex mu;
        static int32_t set_to = 64 * 1024;
        std::lock_guard<std::mutex> lk(mu);
        if (L.lds > set_to) {
          e = hipFuncSetAttribute((const void*)k_cm_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, L.lds);
          if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition LDS: ") + hipGetErrorString(e));
          set_to = L.lds;
        }
      }
      hipLaunchKernelGGL(k_cm_mfma, dim3((unsigned)t->batch, n), dim3(64 * kWaves), (size_t)L.lds, st, Lg, B);
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
