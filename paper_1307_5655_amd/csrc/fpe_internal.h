// Internal layout shared by the host compiler (compile.cpp) and the HIP
// kernels (walk.hip, compose.hip, server.cpp).  Not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

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
// a power (END), bits 8-15 power-table index (kOffTable = on the fly),
// bits 16-19 variable.  deg holds the partial degree (for on-the-fly powers).
constexpr uint32_t kOffTable = 255;
constexpr uint32_t kEndLeafRoot = 1u << 3;
constexpr uint32_t kEndHasPow = 1u << 4;

__host__ __device__ inline uint32_t op_kind(uint32_t info) { return info & 7u; }
__host__ __device__ inline uint32_t op_pidx(uint32_t info) { return (info >> 8) & 255u; }
__host__ __device__ inline uint32_t op_var(uint32_t info) { return (info >> 16) & 15u; }

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
  float aabs;                // |a| rounded up, for the condition sum
  float babs;
};
static_assert(sizeof(OpF32) == 32, "OpF32 is one 32-byte scalar load");

// Power chain (fast exponentiation, Section 2.2): table[dst] = x_var (LOAD)
// or table[s1] * table[s2] (MUL), in order.  Entries 0..n_used-1 are the ones
// the walk reads, sorted by how often it reads them.
enum ChainKind : uint32_t { kChainLoad = 0, kChainMul = 1 };
struct ChainStep {
  uint8_t kind, dst, s1, s2;
};

// Kernel-side view of an uploaded tree (built on the host from the device
// base pointer; passed by value as a kernel argument).
struct DevTree {
  const OpF64* ops64;
  const OpF32* ops32;
  const ChainStep* chain;
  const uint32_t* coef_rows;   // composition: batch x n_nodes residues (node order)
  int32_t n_ops;               // including END
  int32_t n_chain;
  int32_t n_table;
  int32_t nvars;
  int32_t depth;               // max stack depth of the walk
  int32_t n_nodes;
  int64_t batch;
};

// Work-table entry of a fused (served) launch: one block of points of one
// request.
struct WorkItem {
  DevTree tree;
  const double* pts[8];
  double* out;
  float* cond;
  uint32_t* flags;     // fallback bitmask of this request (32 points / word)
  int64_t begin;       // first point of this block
  int64_t npts;        // points of the whole request
  double tol;
  int32_t domain;
  int32_t pad;
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
  // program
  std::vector<fpe::OpF64> ops64;
  std::vector<fpe::OpF32> ops32;
  std::vector<fpe::ChainStep> chain;
  std::vector<int32_t> table_var, table_deg;   // per table entry
  int32_t n_table = 0;
  int32_t n_powers = 0;
  int32_t depth = 0;
  int32_t max_slot = 0;
  int32_t max_lh = 0;
  int32_t n_offtable = 0;
  // device image
  void* dev = nullptr;
  size_t off_ops64 = 0, off_ops32 = 0, off_chain = 0, off_coef = 0, dev_bytes = 0;
};

namespace fpe {
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
// Fused served launch (walk.hip): items in device memory.
fpe_status launch_work_table(const WorkItem* items_dev, int32_t n_items, int32_t n_f32c,
                             int64_t* fallback_counter, void* stream);
constexpr int kMaxDepth = 16;   // stack depth the kernels hold
constexpr int kMaxTable = 48;   // power-table entries held per point
constexpr int kServeBlockPts = 256;
}  // namespace fpe
