// Internal layout shared by the host compiler (compile.cpp) and the HIP
// kernels (walk.hip, compose.hip, server.cpp).  Not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/fpe.h"

namespace fpe {

constexpr uint64_t kP61 = (uint64_t(1) << 61) - 1;
constexpr uint64_t kP31 = (uint64_t(1) << 31) - 1;

// The walk of Section 2.1, re-expressed as a stack program.  Node i of the
// tree (root excluded) is one op; the accumulators of the nodes whose
// subtree is being walked form a stack (top = the most recently opened).
// With the fused form u(P) = c(P) + sum_C u(C) x^{d(C)}, each op is one
// fused multiply-add at a stack position known when the tree is compiled:
//
//   LEAF_ADD   leaf N, not the first child:   top      = a * X + top
//   NODE_OPEN  inner N, first child of P:     top      = top * X + b   (b = c(P))
//   LEAF_OPEN  leaf N, first child of P:      push       a * X + b     (a = c(N), b = c(P))
//   NODE_ADD   inner N, not the first child:  below    = top * X + below; pop
//   END        root R:                        y = (children ? top : a) * X_R
//
// X is the power x_var^pdeg of the node, read from the per-point power table.
enum OpKind : uint32_t { kLeafAdd = 0, kNodeOpen = 1, kLeafOpen = 2, kNodeAdd = 3, kEnd = 4 };

// info word: bits 0-2 kind, bit 3 root-without-children (END), bit 4 root has
// a power (END), bits 5-7 the kind as flags (leaf / first child / end) for a
// two-test dispatch, bits 8-15 power-table index (kOffTable = on the fly),
// bits 16-19 variable, bits 20-24 the stack depth L before the op (so a flat
// loop can address the accumulators with compile-time indices), bits 25-31 a
// second table index (kNoPair if none): the power is then the product of the
// two entries.  deg holds the partial degree (for on-the-fly powers).
constexpr uint32_t kOffTable = 255;
constexpr uint32_t kNoPair = 127;
constexpr uint32_t kThirdBit = 1u << 19;   // in deg: the power has a third factor (index in bits 0-7)
constexpr uint32_t kEndLeafRoot = 1u << 3;
constexpr uint32_t kEndHasPow = 1u << 4;
constexpr uint32_t kBitLeaf = 1u << 5;
constexpr uint32_t kBitFirst = 1u << 6;
constexpr uint32_t kBitEnd = 1u << 7;

__host__ __device__ inline uint32_t op_kind(uint32_t info) { return info & 7u; }
__host__ __device__ inline uint32_t op_pidx(uint32_t info) { return (info >> 8) & 255u; }
__host__ __device__ inline uint32_t op_var(uint32_t info) { return (info >> 16) & 15u; }
__host__ __device__ inline uint32_t op_level(uint32_t info) { return (info >> 20) & 31u; }
__host__ __device__ inline uint32_t op_pidx2(uint32_t info) { return (info >> 25) & 127u; }

// The dispatch code of an op, in the top 12 bits of its deg field (the
// partial degree itself, < 2^20, uses the low 20 bits): bits 0-3 the stack
// depth L, bits 4-5 the kind (LEAF_ADD, NODE_OPEN, LEAF_OPEN, NODE_ADD),
// bits 6-8 where its power comes from (0-3: register entry 0-3, 4: an entry
// of the LDS tier, held in the private table by kernels without the tier,
// 5: a product of two or three entries, or computed on the fly, 6: an entry
// beyond the tier, in the private table).  Tier and private entries have
// classes of their own so that a walk can read each with a plain LDS or
// private load (with one class for both, the compiler selects the address
// and issues a flat load).  LEAF_ADD at depth 0
// cannot occur, so codes with L = 0 and kind 0 mark the root (END).
constexpr int kRegPowers = 4;   // table entries kept in registers
constexpr int kLdsPowers = 4;   // the next entries, kept in LDS (see walk_core.h)
// The double-float walk's tier is deeper: its records (OpF32) carry dispatch
// codes of their own, with the class boundary at entry 11.
constexpr int kLdsPowersF32 = 7;
enum PowClass : uint32_t { kPowMem = 4, kPowOther = 5, kPowPriv = 6 };
constexpr uint32_t make_code(uint32_t level, uint32_t kind, uint32_t pclass) {
  return (level & 15u) | (kind << 4) | (pclass << 6);
}
__host__ __device__ inline uint32_t op_code(uint32_t deg) { return deg >> 20; }
// The dispatch code of an op from its info word (whose level field holds the
// stack depth before the op), for a walk whose LDS tier holds `tier` entries.
__host__ __device__ inline uint32_t dispatch_code(uint32_t info, int tier = kLdsPowers) {
  const uint32_t p = op_pidx(info), p2 = op_pidx2(info), kind = op_kind(info);
  uint32_t pc = kPowOther;
  if (p2 == kNoPair && p < (uint32_t)kRegPowers) pc = p;
  else if (p2 == kNoPair && p != kOffTable) pc = p < (uint32_t)(kRegPowers + tier) ? kPowMem : kPowPriv;
  if (kind == kEnd) return make_code(0, 0, (info & kEndHasPow) ? pc : kPowOther);
  const uint32_t lvl = op_level(info);
  return make_code(lvl < 15u ? lvl : 15u, kind, pc);
}
__host__ __device__ inline uint32_t op_deg(uint32_t deg) { return deg & 0xFFFFFu; }

struct alignas(32) OpF64 {   // FP64 / double-double / mod-p walks
  uint64_t a;                // c(N) or c(P): FP64 bits or residue
  uint64_t b;                // c(P) for LEAF_OPEN
  uint32_t info;
  uint32_t deg;
  uint64_t pad;
};
static_assert(sizeof(OpF64) == 32, "OpF64 is one 32-byte scalar load");

struct alignas(32) OpF32 {   // double-float walk: constants pre-split on the host
  float ah, al;              // a = ah + al (FP64 constant rounded to 48 bits)
  float bh, bl;
  uint32_t info;
  uint32_t deg;
  float bk2;                 // kK2 * |bh| rounded up: the bound term of an exact b
  float pad;
};
static_assert(sizeof(OpF32) == 32, "OpF32 is one 32-byte scalar load");
// zero records after each op array: the walk reads op records in pairs, up to
// three records past END
constexpr int kOpTail = 3;

// A run record (plain FP64 walk of chain-like trees): b consecutive steps
// top = top * X0 + c at depth 1, X0 the first register power, with the
// coefficients c at runc[a .. a + b).  A Hörner step by x^(k d0) (d0 the
// degree of table entry 0, k <= kRunMaxGap) is k such steps, the first k - 1
// with c = 0 (exact in real arithmetic: (t x^d0 + 0) x^d0 = t x^(2 d0)).
// Its dispatch code lies outside the switch's range.
constexpr uint32_t kRunCode = 0x800;
constexpr int kRunMaxGap = 4;
constexpr int kRunMinOps = 8;
// The double-float walk's runs (OpF32 run records: the stream offset and the
// step count as the bits of ah and al): each step top = top * X0 + b as two
// 64-bit words of runc, the floats (b.h, b.l) and (b's bound term, 0).  Its
// runs take no gaps (the k - 1 inserted steps of a gap k would have b = 0 and
// no bound term): measured on MI355X, the extra compensated steps cost more
// than the dispatch they save, while gap-free runs do exactly the steps of
// the walk without runs, so the bits do not change.
constexpr int kRunWordsF32 = 2;
constexpr int kRunMaxGapF32 = 1;

// Power chain (fast exponentiation, Section 2.2): table[dst] = x_var (LOAD)
// or table[s1] * table[s2] (MUL), in order.  Entries 0..n_used-1 are the ones
// the walk reads, sorted by how often it reads them.
enum ChainKind : uint32_t { kChainLoad = 0, kChainMul = 1 };
// A MUL step's kind also carries its entry's variable (bits 4-7) and whether
// the entry's degree is odd (bit 1), for the interval walk, which takes the
// range of x^d from the bounds of |lo|^d and |hi|^d; LOAD steps stay 0.
constexpr uint32_t kChainOdd = 2;
__host__ __device__ inline bool chain_is_mul(uint32_t kind) { return (kind & 1u) != 0; }
__host__ __device__ inline uint32_t chain_var(uint32_t kind) { return kind >> 4; }
struct ChainStep {
  uint8_t kind, dst, s1, s2;
};

// Kernel-side view of an uploaded tree (built on the host from the device
// base pointer; passed by value as a kernel argument).
struct DevTree {
  const OpF64* ops64;
  const OpF64* ops64r;         // the FP64 chain walk's program: ops64 with runs (see kRunCode)
  const OpF32* ops32r;         // the double-float chain walk's program: ops32 with runs
  const uint64_t* runc;        // the runs' coefficients (FP64 bits; double-float: see kRunWordsF32)
  const uint64_t* runc64;      // a compensated tree's FP64 run coefficients (its double-double fallback)
  const uint64_t* tc;          // per node: its coefficient (FP64 bits or residue; 0 for junctions)
  const int32_t* te;           // per node: its monomial's exponents (nvars each)
  const OpF32* ops32;
  const ChainStep* chain;
  const uint32_t* coef_rows;   // composition: batch x n_nodes residues (node order)
  int32_t n_ops;               // including END
  int32_t n_chain;
  int32_t n_table;
  int32_t nvars;
  int32_t depth;               // max stack depth of the walk
  int32_t n_nodes;
  int32_t n_offtable;          // walk steps whose power is computed on the fly
  float bound_scale;           // double-float walk: factor on the final error bound
  int64_t batch;
  // double-float walk: the absolute part of the error bound is
  // abs_scale * prod_j max(1, |x_j|)^deg_max[j] (see df32_abs_bound)
  double abs_scale;
  int32_t deg_max[8];
};

// Work-table entry of a fused (served) launch: one request.  Its points are
// cut into 64-point blocks; prefix[r] is the first block of request r in the
// launch, so a workgroup finds its request by a binary search over prefix.
struct WorkItem {
  DevTree tree;
  const double* pts[8];
  double* out;
  float* cond;
  int32_t* list;       // F32C: fallback indices (request workspace)
  int64_t npts;
  double tol;
  int32_t domain;
  int32_t pad;
};

// Device-side description of one fused launch (fixed addresses, so that the
// launch can be replayed from a HIP graph with new contents each batch).
struct WorkTable {
  int32_t n_items;
  int32_t pad;
  int64_t total_blocks;
  // followed in memory by: WorkItem items[kMaxServe]; int64_t prefix[kMaxServe + 1];
  //                         int64_t counters[kMaxServe]
};

}  // namespace fpe

// The host tree object behind the opaque C handle.
struct fpe_tree {
  int32_t nvars = 1;
  int32_t domain = 0;
  uint64_t modulus = 0;
  int64_t batch = 1;
  int64_t n_terms = 0;
  std::vector<fpe_node> nodes;
  std::vector<int32_t> exps;            // n_nodes x nvars
  std::vector<uint64_t> coef_rows;      // batch x n_nodes (mod p), node order
  std::vector<uint32_t> coef_rows32;    // the same as 32-bit residues (composition mod 2^31 - 1)
  // program
  std::vector<fpe::OpF64> ops64;
  std::vector<fpe::OpF32> ops32;
  std::vector<fpe::OpF64> ops64r;       // derived by layout(): ops64 with runs (FP64, depth <= 2), else empty
  std::vector<fpe::OpF32> ops32r;       // derived by layout(): ops32 with runs (F32C, depth <= 2), else empty
  std::vector<uint64_t> runc;           // the runs' coefficients
  std::vector<uint64_t> runc64;         // F32C trees: the FP64 runs' coefficients (ops64r, double-double fallback)
  std::vector<uint64_t> term_c;         // FP64 / mod 2^61-1 trees: each node's coefficient (few-point path)
  std::vector<fpe::ChainStep> chain;
  std::vector<int32_t> table_var, table_deg;   // per table entry
  int32_t n_table = 0;
  int32_t n_powers = 0;
  int32_t depth = 0;
  int32_t max_slot = 0;
  int32_t max_lh = 0;
  int32_t n_offtable = 0;
  int32_t n_pairs = 0;
  int32_t n_kind[5] = {};   // walk ops by OpKind
  // derived from the node array by layout(): the largest exponent of each
  // variable and the compensated walk's absolute bound scale
  int32_t deg_max[8] = {};
  double abs_scale = 0;
  // device image
  void* dev = nullptr;
  size_t off_ops64 = 0, off_ops32 = 0, off_chain = 0, off_coef = 0, off_ops64r = 0, off_ops32r = 0, off_runc = 0,
         off_runc64 = 0, dev_bytes = 0;
  size_t off_term_c = 0, off_term_e = 0;
};

namespace fpe {
// Factor on the double-float walk's final error bound that covers the FP32
// evaluation of the bound over n steps (at most (1 + 4.001 u)^n, u = 2^-24),
// with 2^-20 to spare for the final test's own roundings; rounded up.
inline float df32_bound_scale(int64_t n_steps) {
  const double g = std::exp((double)n_steps * 4.001 * std::ldexp(1.0, -24)) * (1.0 + std::ldexp(1.0, -20));
  float f = (float)g;
  if ((double)f < g) f = std::nextafter(f, INFINITY);
  return f;
}
// Scale of the absolute part of the double-float walk's error bound, for a
// tree of n_steps walk steps whose coefficients have 1-norm c1: every step
// may lose up to 2^-147 to roundings in the subnormal range and to the split
// of its constants, plus 2^-148 |a| to a power below the normal range (|a| the
// multiplicand); carried up the tree, the powers scale these by at most
// prod_j max(1, |x_j|)^deg_max[j], and |a| times those powers by at most c1
// times it.  2^-145 (1 + c1) per step leaves a factor 2 of margin; rounded up.
inline double df32_abs_scale(int64_t n_steps, double c1) {
  return (double)n_steps * std::ldexp(1.0, -145) * (1.0 + c1) * (1.0 + std::ldexp(1.0, -30));
}
void set_error(const std::string& msg);
fpe_status fail(fpe_status st, const std::string& msg);
DevTree dev_view(const fpe_tree* t);
// Launchers (walk.hip).
fpe_status launch_eval(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                       const fpe_eval_opts* opts, void* stream);
size_t eval_workspace_bytes(const fpe_tree* t, int64_t npts);
fpe_status launch_compose(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out,
                          void* ws, size_t ws_bytes, void* stream);
size_t compose_workspace_bytes(const fpe_tree* t, int32_t dq);
size_t compose_workspace_bytes_ex(const fpe_tree* t, int32_t dq, int32_t product);
fpe_status launch_compose_ex(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                             size_t ws_bytes, int32_t product, void* stream);
// the composition walk op by op with batched launches (ntt.hip); products
// whose shorter operand has at least ntt_min coefficients use transforms
size_t compose_ops_workspace_bytes(const fpe_tree* t, int32_t dq, int32_t ntt_min);
fpe_status launch_compose_ops(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                              size_t ws_bytes, int32_t ntt_min, void* stream);
// the composition walk level by level, large products on the matrix cores
// (compose_mfma.hip); its schedule is cached per tree and dq
size_t compose_levels_workspace_bytes(const fpe_tree* t, int32_t dq);
bool compose_levels_ok(const fpe_tree* t, int32_t dq, int64_t* launches);
fpe_status launch_compose_levels(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, void* ws,
                                 size_t ws_bytes, void* stream);
void compose_levels_forget(const fpe_tree* t);
fpe_status launch_bigint(const fpe_tree* t, const uint32_t* x, int32_t lx, int64_t batch, uint32_t* out,
                         int32_t lout, void* ws, size_t ws_bytes, void* stream);
size_t bigint_workspace_bytes(const fpe_tree* t, int32_t lout, int64_t batch);
// evaluation at one big point (bigpoint.hip); its schedule is cached per tree
int64_t bigpoint_out_limbs(const fpe_tree* t, int32_t lx);
size_t bigpoint_workspace_bytes(const fpe_tree* t, int32_t lx);
fpe_status launch_bigpoint(const fpe_tree* t, const uint32_t* x, int32_t lx, uint32_t* out, int64_t lout, void* ws,
                           size_t ws_bytes, void* stream);
void bigpoint_forget(const fpe_tree* t);
// composition over the natural numbers at one big point, by Kronecker
// substitution into the big-point walk (compose_bigint.hip)
constexpr int kComposeBigMaxQ = 64;          // coefficients of q, passed as kernel arguments
constexpr int64_t kBigPointMaxLimbs = 1 << 14;   // the largest transform of the big-point walk
struct ComposeBigPlan {
  int32_t lc = 0;       // limbs per coefficient slot (0: unsupported)
  int64_t ly = 0;       // limbs of the point y = q(2^(16 lc))
  int64_t lz = 0;       // limbs of p(y) as the big-point walk writes it
  int64_t nout = 0;     // (deg p * dq + 1) * lc
  size_t off_y = 0, off_z = 0, bytes = 0;   // workspace: walk's, y, p(y)
};
ComposeBigPlan compose_bigint_plan(const fpe_tree* t, const uint64_t* q, int32_t dq);
fpe_status launch_compose_bigint(const fpe_tree* t, const uint64_t* q, int32_t dq, uint32_t* out, int64_t lout,
                                 void* ws, size_t ws_bytes, void* stream);
constexpr int kMaxDepth = 15;   // stack depth the kernels hold (the code's 4-bit level field)
constexpr int kBigMaxLimbs = 1 << 16;   // big-integer values: columns of 2^16 limb products fit in 64 bits
constexpr int kMaxTable = 48;   // power-table entries held per point (composition)
constexpr int kTableCap = 16;   // smallest table size the compiler tries
constexpr int kTableCapMulti = 32;   // largest table of the kernels with several points per lane
constexpr int kMaxServe = 256;  // requests per fused launch
constexpr int kServeGrid = 16384;  // fixed grid of the fused kernels (workgroups)
// Fused served launch (walk.hip).
struct ServeKernels {
  const void* zero;       // k_serve_zero(WorkTable*)
  const void* walk8;      // k_serve_walk<8>(WorkTable*)
  const void* walk16;     // k_serve_walk<kMaxDepth>(WorkTable*)
  const void* fallback8;  // k_serve_fallback<8>(WorkTable*)
  const void* fallback16;
  size_t walk_lds;        // dynamic LDS of the walk kernels (the power tables' LDS tier)
  size_t fallback_lds;    // and of the fallback kernels
};
ServeKernels serve_kernels();
size_t work_table_bytes();
__host__ __device__ inline WorkItem* table_items(WorkTable* t) { return (WorkItem*)((char*)t + 256); }
__host__ __device__ inline int64_t* table_prefix(WorkTable* t) {
  return (int64_t*)(table_items(t) + kMaxServe);
}
__host__ __device__ inline int64_t* table_counters(WorkTable* t) { return table_prefix(t) + kMaxServe + 1; }

// One pointwise launch (walk.hip picks the shape; the eval_*.hip files hold
// the kernels).
// Workgroups (one wavefront each) for n points at ppl points per lane.
inline int64_t blocks_for(int64_t n, int ppl) { return (n + 64 * ppl - 1) / (64 * ppl); }

struct KernelLaunch {
  DevTree tr;
  const void* pts[8];
  int64_t npts;
  int64_t nblocks;   // fixed grid of the fallback kernels (the walks size theirs from their PPL)
  hipStream_t stream;
  int ppl;           // requested points per lane (the launchers pick a kernel at most this wide)
  bool offt;
};
struct F32COut;
void launch_f64(const KernelLaunch& L, double* out);
// The few-point path (eval_terms.hip): one workgroup per point, the terms
// over its lanes, a wavefront reduction.  domain FPE_F64 or FPE_MODP.
void launch_terms(const KernelLaunch& L, int32_t domain, void* out);
// Whether a tree has the few-point path's data, and whether the library takes
// that path for npts points.
bool terms_eligible(const fpe_tree* t);
bool terms_preferred(const fpe_tree* t, int64_t npts);
void launch_m61(const KernelLaunch& L, uint64_t* out);
void launch_iv(const KernelLaunch& L, double* out);
void launch_df32(const KernelLaunch& L, const F32COut& o);
void launch_fallback(const KernelLaunch& L, const int32_t* list, const int64_t* count, double* out);
}  // namespace fpe
