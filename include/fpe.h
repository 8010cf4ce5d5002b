/* fpe.h — fast polynomial evaluation through evaluation trees on MI355X (gfx950).
 *
 * C-ABI of libfpe.so.  The library compiles a polynomial p under a function
 * scheme f into an evaluation tree (G. Moroz, "Fast polynomial evaluation and
 * composition", Section 1: Definition of evaluation tree; Section 1.1:
 * Definition of function scheme), lays the tree out as a flat, topologically
 * ordered node array, and runs the coefficient walk of Section 2.1 on the GPU
 * at very many points at once, in
 *   - plain FP64,
 *   - compensated FP32 (double-float arithmetic with error-free TwoProd and
 *     TwoSum, a running error bound, and an FP64 re-evaluation of every point
 *     whose bound exceeds the requested tolerance), or
 *   - exact arithmetic modulo the Mersenne prime 2^61 - 1,
 * and composes p(q(x)) over Z/(2^31 - 1) through the same tree.
 *
 * Conventions
 *  - Every function returns an fpe_status (0 = OK, < 0 = error) and never
 *    throws or aborts across the ABI; fpe_last_error() gives a message for the
 *    last failing call on the calling thread.
 *  - "device" pointers are HIP device memory (for example torch tensors on a
 *    ROCm build, passed as data_ptr()).  The caller owns every point, output,
 *    workspace and q buffer.  The library owns the host side of a tree; the
 *    device image of a tree lives in a caller-owned device buffer handed to
 *    fpe_tree_upload.
 *  - "stream" is a hipStream_t (NULL = the default stream).  Calls that take
 *    a stream are asynchronous on it and make no hidden synchronisation.
 *  - Validation errors are reported synchronously.  A device error surfaces as
 *    FPE_EDEVICE at the next call that checks the stream.
 */
#ifndef FPE_H
#define FPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FPE_OK = 0,
  FPE_EINVAL = -1,        /* invalid argument (shape, scheme, duplicate term, residue >= p, ...) */
  FPE_ENOMEM = -2,        /* host allocation failed, or a caller buffer is too small */
  FPE_EDEVICE = -3,       /* a HIP call failed */
  FPE_EBUDGET = -4,       /* the server's HBM budget cannot hold the request */
  FPE_EUNSUPPORTED = -5,  /* valid, but outside what the kernels support (see each call) */
  FPE_EBUSY = -6          /* the server has no free slot right now (retry later) */
} fpe_status;

/* Message for the last failing call on this thread; valid until the next call. */
const char* fpe_last_error(void);

/* Library version, e.g. "fpe 1.0 gfx950". */
const char* fpe_version(void);

typedef enum {
  FPE_F64 = 0,   /* plain FP64 walk, one fused multiply-add per node (Section 2.1) */
  FPE_F32C = 1,  /* compensated FP32 (double-float) walk + FP64 fallback */
  FPE_MODP = 2,  /* exact walk in Z/pZ, p = 2^61 - 1 for evaluation, 2^31 - 1 for composition */
  FPE_IVAL = 3,  /* interval walk (the abstract's interval coefficient type): FP64 bounds
                    rounded outward, enclosing the tree's interval evaluation over a box */
  FPE_BIGINT = 4 /* exact evaluation over the natural numbers at big-integer points
                    (the workload of the Benchmarks section, Figure 1): fpe_eval_bigint */
} fpe_domain;

/* Function schemes (Section 1.1 and 1.2).  The argument of f is the degree n
 * of the sub-polynomial being split as p = a x^{f(n)} + b, and 0 < f(n) <= n. */
typedef enum {
  FPE_DIRECT = 0,          /* D(n) = n                                      */
  FPE_HORNER = 1,          /* H(n) = 1                                      */
  FPE_ESTRIN = 2,          /* E(n) = 2^floor(log2 n)                        */
  FPE_BALANCED = 3,        /* B(n) = ceil(n / 2)  (Section 1.2, on the degree) */
  FPE_BALANCED_FLOOR = 4,  /* max(1, floor(n / 2)): the literal formula, for comparison */
  FPE_THRESHOLD = 5,       /* E(n) if n > threshold, else H(n) (Section 1.1, Remark) */
  FPE_TABLE = 6            /* user scheme: f(n) = table[n], each entry validated in [1, n] */
} fpe_scheme_kind;

typedef struct {
  int32_t kind;            /* fpe_scheme_kind */
  int32_t threshold;       /* FPE_THRESHOLD only */
  const int32_t* table;    /* FPE_TABLE only: host array, table[n] for 1 <= n < table_len */
  int32_t table_len;
} fpe_scheme;

/* One node of the compiled tree, in the order <_t of Section 1: decreasing
 * lexicographic order of the monomials, index 0 is the biggest, the root is
 * last, and every child has a lower index than its parent.  Each non-root
 * node's partial degree d(N) = exp(N) - exp(parent(N)) has exactly one
 * nonzero variable (var, pdeg); the root's partial degree is its own monomial
 * (var, pdeg), pdeg = 0 if p has a constant term.  Junction nodes (flag
 * FPE_NODE_JUNCTION, coefficient 0) are added only for sparse multivariate
 * input whose nested coefficient polynomial has no constant term. */
typedef struct {
  union { double f; uint64_t u; } coef;  /* FP64 value, or residue (row 0 for a batch) */
  int32_t pdeg;         /* partial degree in variable var */
  uint8_t var;          /* 0-based variable index, x1 outermost */
  uint8_t slot;         /* accumulator slot of the walk (Section 1.3, safe reading) */
  uint8_t lazy_height;  /* lh(N) exactly as defined in Section 1.3 */
  uint8_t flags;        /* FPE_NODE_* */
  int32_t parent;       /* index of the parent, -1 for the root */
  int32_t sub_begin;    /* the subtree of node i is [sub_begin, i]; its children lie in it */
} fpe_node;

#define FPE_NODE_LEAF 1u
#define FPE_NODE_FIRST_CHILD 2u   /* C_1 of its parent (the biggest child) */
#define FPE_NODE_JUNCTION 4u
#define FPE_NODE_ROOT 8u

typedef struct fpe_tree fpe_tree;

/* Compile p = sum_t coeffs[t] * prod_j x_j^exps[t*nvars + j] under scheme f.
 *   nvars   1..8
 *   nterms  >= 1 terms; exponents >= 0 and < 2^20; no monomial twice.
 *           Terms with a zero coefficient are dropped (all zero: FPE_EINVAL).
 *   coeffs  host array: double[nterms] for FPE_F64 / FPE_F32C / FPE_IVAL (finite;
 *           FPE_IVAL takes them as exact point coefficients), uint64_t[nterms]
 *           for FPE_BIGINT (univariate; any value), or
 *           uint64_t[batch * nterms] residues < modulus for FPE_MODP (row r
 *           holds instance r; all rows share the exponents; the tree shape is
 *           taken from the union of nonzero positions).
 *   batch   1 for evaluation; the number of instances for fpe_compose.
 *   modulus FPE_MODP only: 2^61 - 1 (evaluation) or 2^31 - 1 (composition).
 * On success *out owns a new tree (free with fpe_tree_free). */
fpe_status fpe_compile(int32_t nvars, int64_t nterms, const int32_t* exps, const void* coeffs,
                       int64_t batch, int32_t domain, uint64_t modulus, const fpe_scheme* f,
                       fpe_tree** out);

void fpe_tree_free(fpe_tree* t);

/* Read-only view of the node array (valid while the tree lives). */
fpe_status fpe_tree_nodes(const fpe_tree* t, const fpe_node** nodes, int64_t* n, int32_t* max_slot);

/* Walk statistics (stack depth of the walk, size of the per-point power table,
 * length of the power chain, number of distinct partial degrees, steps by
 * kind) and what the tree was compiled for (domain, modulus, batch). */
typedef struct {
  int64_t n_nodes;
  int64_t n_terms;         /* nonzero input terms (n_nodes minus junctions) */
  int32_t nvars;
  int32_t max_slot;        /* largest safe slot */
  int32_t max_lazy_height; /* largest lh(N) by the definition of Section 1.3 */
  int32_t walk_depth;      /* accumulators live at once in the GPU walk */
  int32_t n_powers;        /* distinct (variable, partial degree) pairs */
  int32_t n_table;         /* powers held per point in the table (incl. chain temporaries) */
  int32_t n_chain;         /* steps of the power chain (Section 2.2, fast exponentiation) */
  int32_t n_offtable;      /* walk steps whose power is computed on the fly */
  int32_t n_pair_ops;      /* walk steps whose power is the product of two table entries */
  int32_t n_ops_kind[5];   /* walk steps by kind: LEAF_ADD (a X + top), NODE_OPEN (top X + b),
                              LEAF_OPEN (push a X + b), NODE_ADD (below += top X; pop), END */
  int32_t domain;          /* fpe_domain the tree was compiled for */
  uint64_t modulus;        /* FPE_MODP: the modulus, else 0 */
  int64_t batch;           /* instances (composition), else 1 */
} fpe_tree_info;

fpe_status fpe_tree_get_info(const fpe_tree* t, fpe_tree_info* info);

/* Exponent vector of node i (nvars entries, the node's monomial). */
fpe_status fpe_tree_node_exps(const fpe_tree* t, int64_t i, int32_t* exps_out);

/* Device image: its size, and its upload into a caller-owned device buffer of
 * at least that many bytes (256-byte aligned).  The tree records the buffer;
 * the buffer must outlive every evaluation that uses it.  Asynchronous on
 * stream: the host copy is staged so the call may return before the copy. */
size_t fpe_tree_device_bytes(const fpe_tree* t);
fpe_status fpe_tree_upload(fpe_tree* t, void* dev_buf, size_t bytes, void* stream);

/* Serialise the host tree (node array, program, coefficients) into a byte
 * buffer and back, for reloading resident trees; *bytes in/out. */
fpe_status fpe_tree_serialize(const fpe_tree* t, void* buf, size_t* bytes);
fpe_status fpe_tree_deserialize(const void* buf, size_t bytes, fpe_tree** out);

typedef struct {
  double tol;               /* FPE_F32C: relative tolerance; points whose running error
                               bound exceeds tol*|y| are re-evaluated in FP64.  <= 0 means 1e-12. */
  int32_t force;            /* FPE_F32C: 0 = by bound, 1 = re-evaluate every point, 2 = never */
  int32_t points_per_lane;  /* 0 = library default */
  float* cond_out;          /* optional device float[npts]: ptilde(|x|)/|y| (FPE_F32C) */
  uint32_t* flags_out;      /* optional device uint32[ceil(npts/32)]: fallback bitmask (FPE_F32C) */
  void* workspace;          /* FPE_F32C: device buffer of fpe_workspace_bytes() bytes */
  size_t workspace_bytes;
  int64_t* nfallback_out;   /* optional device int64: number of re-evaluated points (FPE_F32C) */
  void* ev_walk_begin;      /* optional hipEvent_t recorded on the stream right before the walk kernel */
  void* ev_walk_end;        /* optional hipEvent_t recorded right after it (before any fallback) */
  double* bound_out;        /* optional device double[npts] (FPE_F32C): the error bound of the
                               compensated walk that the fallback test compared with tol*|y|
                               (its running relative terms plus its absolute part); a point
                               not re-evaluated has |y - p(x)| <= bound_out[i] */
  int32_t path;             /* FPE_F64 / FPE_MODP: 0 = the tree walk, 1 = the library's choice
                               by its cost model, 2 = the term-parallel few-point path (see
                               fpe_evaluate) */
} fpe_eval_opts;

/* Workspace needed by fpe_evaluate for npts points (0 unless FPE_F32C). */
size_t fpe_workspace_bytes(const fpe_tree* t, int64_t npts);

/* Evaluate the uploaded tree at npts points: the coefficient walk of
 * Section 2.1 (each step one multiplication and one addition, in the fused
 * form u(P) = c(P) + sum_C u(C) x^{d(C)}), with the distinct powers x^d
 * precomputed per point by fast exponentiation (Section 2.2, Table 1); the
 * value is that of the evaluation tree (Section 1, Definition), which every
 * function scheme makes equal to p(x) in exact arithmetic.
 *   pts  host array of nvars device pointers, each to npts values (SoA):
 *        double for FPE_F64 / FPE_F32C, uint64_t residues < p for FPE_MODP;
 *        for FPE_IVAL each points to double[2 * npts], interval i of that
 *        variable as (lo, hi) at [2i], [2i + 1], lo <= hi.
 *   out  device array of npts doubles (FPE_F64, FPE_F32C) or uint64_t (FPE_MODP);
 *        FPE_IVAL: double[2 * npts], (lo, hi) per point.  [lo, hi] contains the
 *        interval evaluation of the tree over the box (exact interval sums and
 *        products, each power x^d taken as its exact range over the interval),
 *        hence p(x) for every x in the box; every bound is rounded outward.
 *        A bound that overflows is returned as [-inf, +inf].
 *   opts may be NULL for FPE_F64 / FPE_MODP / FPE_IVAL.
 * Few points, big trees (FPE_F64, FPE_MODP with 2^61 - 1): with opts->path =
 * 2 (or 1, when the library's cost model prefers it) one workgroup per point
 * evaluates the polynomial's terms in parallel, c * prod_j x_j^{e_j} with
 * powers by fast exponentiation, and sums them by a wavefront reduction (DPP)
 * and across the workgroup: the direct scheme's evaluation of the same
 * polynomial (Section 1), exact modulo p, and in FP64 within the same
 * 1e-13 * p~(|x|) as the walk but not bit-identical to it.  The default (0)
 * is the tree walk.
 * Errors: FPE_EINVAL (not uploaded, npts < 0, NULL pointers, path not 0-2),
 * FPE_ENOMEM (workspace too small), FPE_EUNSUPPORTED (walk deeper than the
 * kernels hold, path 2 for another domain), FPE_EDEVICE. */
fpe_status fpe_evaluate(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                        const fpe_eval_opts* opts, void* stream);

/* The path fpe_evaluate takes with opts->path = 1 for npts points: 1 = the
 * tree walk, 2 = the term-parallel few-point path (0 for a NULL tree).  The
 * cost model (calibrated on MI355X): the walk runs one chain of dispatched
 * steps per lane, about 100 ns a step in FP64 and 200 ns mod p (lanes in
 * parallel up to ~2.6e5 points); the term path costs npts x nodes x (2 bit
 * lengths of each variable's largest exponent + 2) operations of about 4
 * FP64 lane-operations each (20 mod p) at 3.9e13 per second, plus 5 us; the
 * terms are taken below half the walk's estimate. */
int32_t fpe_eval_path(const fpe_tree* t, int64_t npts);

/* Allocation-free evaluation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as fpe_evaluate, except
 * that FPE_F32C takes its scratch (the fallback counter and the list of
 * flagged point indices, 256 + 4 * FPE_NOALLOC_MAX_POINTS bytes) from a
 * static device array of the library instead of opts->workspace (ignored).
 * The array is zeroed where needed by the call itself (a kernel, no memset);
 * each GPU holds its own copy until the process ends, looked up on the first
 * call made with that device current.  The call allocates nothing (no
 * hipMalloc, no library allocator).  Calls on one GPU share its array, so
 * calls that overlap on one GPU (different streams, or several host
 * threads) race and must be serialised by the caller.
 * Errors: as fpe_evaluate; FPE_EINVAL if npts > FPE_NOALLOC_MAX_POINTS. */
#define FPE_NOALLOC_MAX_POINTS (1 << 22)
fpe_status fpe_evaluate_noalloc(const fpe_tree* t, const void* const* pts, int64_t npts, void* out,
                                const fpe_eval_opts* opts, void* stream);

/* Composition over Z/(2^31 - 1) (the title problem; Section 1.2: the
 * divide-and-conquer schemes suit elements whose size grows linearly with
 * each multiplication, such as polynomials): the coefficient walk of
 * Section 2.1 with polynomial values, the powers q^d by the tree's
 * multiplication chain (Section 2.2).  For every instance r of the batch
 * compiled into t (univariate, FPE_MODP, modulus 2^31 - 1),
 * out[r] = p_r(q_r(x)).
 *   q    device uint32[batch * (dq + 1)], coefficient j of instance r at r*(dq+1)+j, < p
 *   out  device uint32[batch * (deg_p * dq + 1)], coefficients by exponent
 *   workspace  device buffer of fpe_compose_workspace_bytes() bytes */
size_t fpe_compose_workspace_bytes(const fpe_tree* t, int32_t dq);

/* How the polynomial products of a composition are computed.
 *   FPE_PRODUCT_FUSED       one wavefront walks one instance, every product a
 *                           schoolbook convolution (outputs up to 4096 coefficients)
 *   FPE_PRODUCT_SCHOOLBOOK  the walk op by op, each op one launch over all
 *                           instances, products by batched schoolbook kernels
 *   FPE_PRODUCT_NTT         the same walk with every product whose shorter
 *                           operand has at least 64 coefficients computed
 *                           exactly by number-theoretic transforms modulo three
 *                           primes below 2^31 and Garner's recombination
 *                           (subquadratic products, up to 2^14 coefficients)
 *   FPE_PRODUCT_MFMA        the tree walked by levels (every value whose operands
 *                           exist, for all instances, in one launch; Section 1's
 *                           definition u(N) = c(N) + sum_C u(C) q^d(C), powers by
 *                           the chain of Section 2.2), each value of 65 to 4096
 *                           output coefficients an exact integer matrix product
 *                           on the matrix cores (balanced 8-bit digits of the
 *                           centred residues, Toeplitz blocks, 32x32x32 int8
 *                           MFMA), shorter and longer ones on a schoolbook kernel
 *   FPE_PRODUCT_AUTO        deg_p * dq + 1 <= 4096: MFMA when the level walk
 *                           takes at most 64 launches (divide-and-conquer
 *                           trees), else FUSED; beyond 4096: NTT
 * All give the same residues. */
typedef enum { FPE_PRODUCT_AUTO = 0, FPE_PRODUCT_FUSED = 1, FPE_PRODUCT_SCHOOLBOOK = 2,
               FPE_PRODUCT_NTT = 3, FPE_PRODUCT_MFMA = 4 } fpe_product;
size_t fpe_compose_ex_workspace_bytes(const fpe_tree* t, int32_t dq, int32_t product);
/* fpe_compose with a chosen product method (fpe_compose is FPE_PRODUCT_AUTO).
 * Errors: as fpe_compose; FPE_EUNSUPPORTED if a transform would exceed 2^14
 * coefficients or the batch exceeds 65535 instances (op-by-op methods). */
fpe_status fpe_compose_ex(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out, int32_t product,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Exact evaluation over the natural numbers at big-integer points (the
 * workload of the paper's Benchmarks section, Figure 1): for every point r of
 * the batch, out[r] = p(x_r), with the tree (univariate, FPE_BIGINT, uint64
 * coefficients) walked with big-integer values.
 *   x    device uint32[batch * lx]: point r's limbs at r*lx, 16 bits per word
 *        (values < 2^16), least significant first
 *   out  device uint32[batch * lout]: p(x_r)'s 16-bit limbs, least significant
 *        first, zero-padded; lout >= fpe_bigint_out_limbs(t, lx) (which is 0 if
 *        more than 2^16 limbs would be needed: unsupported)
 *   workspace  device buffer of fpe_bigint_workspace_bytes(t, lout, batch)
 *        bytes, 256-byte aligned
 * One wavefront walks one point; products are schoolbook over 16-bit limbs.
 * Errors: FPE_EINVAL (not a FPE_BIGINT tree, lout too small, NULL), FPE_ENOMEM
 * (workspace), FPE_EUNSUPPORTED (powers outside the table, lout > 2^16). */
int32_t fpe_bigint_out_limbs(const fpe_tree* t, int32_t lx);
size_t fpe_bigint_workspace_bytes(const fpe_tree* t, int32_t lout, int64_t batch);
fpe_status fpe_eval_bigint(const fpe_tree* t, const uint32_t* x, int32_t lx, int64_t batch, uint32_t* out,
                           int32_t lout, void* workspace, size_t workspace_bytes, void* stream);
/* Exact evaluation at ONE big natural number x (the setting of the Benchmarks
 * section, Figure 1: one polynomial, one large point).  The tree (univariate,
 * FPE_BIGINT, uint64 coefficients) is walked level by level from its
 * definition (Section 1): u(N) = c(N) + sum_C u(C) x^{d(C)}, p(x) = u(R) x^{d(R)};
 * the nodes of one height are independent (the divide-and-conquer
 * parallelism of Section 2.3) and run as batched launches, the powers x^d
 * first, by the tree's chain (Section 2.2).  Products of big integers are
 * exact convolutions of 16-bit limbs by number-theoretic transforms (two
 * primes below 2^31, Garner's recombination) or schoolbook when an operand
 * has fewer than 64 limbs; sums are normalised by a parallel carry-lookahead.
 *   x    device uint32[lx]: the point's 16-bit limbs (values < 2^16), least
 *        significant first
 *   out  device uint32[lout]: p(x)'s limbs, zero-padded;
 *        lout >= fpe_bigpoint_out_limbs(t, lx) (0: a product would exceed 2^14
 *        limbs, unsupported)
 *   workspace  device buffer of fpe_bigpoint_workspace_bytes(t, lx) bytes,
 *        256-byte aligned; its first 4 bytes are the overflow flag that
 *        fpe_bigint_status reads
 * The schedule (which products and sums each level runs) is built on the host
 * at the first call for a tree and point length and kept with the tree.
 * Errors: FPE_EINVAL, FPE_ENOMEM (workspace), FPE_EUNSUPPORTED. */
int64_t fpe_bigpoint_out_limbs(const fpe_tree* t, int32_t lx);
size_t fpe_bigpoint_workspace_bytes(const fpe_tree* t, int32_t lx);
fpe_status fpe_eval_bigpoint(const fpe_tree* t, const uint32_t* x, int32_t lx, uint32_t* out, int64_t lout,
                             void* workspace, size_t workspace_bytes, void* stream);
/* Composition over the natural numbers at one big point: the coefficients of
 * p(q(X)), the title problem with integer elements, whose size grows with the
 * degree (Section 1.2).  p is the tree (univariate, FPE_BIGINT, uint64
 * coefficients >= 0), q has uint64 coefficients >= 0.  By Kronecker
 * substitution: every coefficient of p(q(X)) is at most p(q(1)), so with
 * slots of lc 16-bit limbs, 2^(16 lc) > p(q(1)), the natural number
 * p(q(2^(16 lc))) holds the coefficient of X^k in its limbs
 * [k lc, (k + 1) lc); q(2^(16 lc)) is q's coefficients one per slot, and p at
 * that point is fpe_eval_bigpoint's level walk (Figure 1's setting: one big
 * point, the tree's scheme deciding the products).
 *   q    HOST uint64[dq + 1], q[0] + q[1] X + ..., 0 <= dq < 64; read during
 *        the call
 *   out  device uint32[lout]: coefficient k (k = 0 .. deg p * dq) as lc
 *        16-bit limbs (values < 2^16, least significant first) at
 *        out[k lc .. (k + 1) lc), zero beyond; lout >=
 *        fpe_compose_bigint_out_limbs(t, q, dq) = (deg p * dq + 1) lc
 *   workspace  device buffer of fpe_compose_bigint_workspace_bytes(t, q, dq)
 *        bytes, 256-byte aligned; its first 4 bytes are the overflow flag
 *        that fpe_bigint_status reads
 * fpe_compose_bigint_coef_limbs returns lc, or 0 when unsupported: dq >= 64,
 * or a product of the walk longer than 2^14 limbs (the point and p(point)
 * must fit the big-point walk).
 * Errors: FPE_EINVAL (not a FPE_BIGINT tree, lout too small, NULL, dq < 0),
 * FPE_ENOMEM (workspace), FPE_EUNSUPPORTED. */
int32_t fpe_compose_bigint_coef_limbs(const fpe_tree* t, const uint64_t* q, int32_t dq);
int64_t fpe_compose_bigint_out_limbs(const fpe_tree* t, const uint64_t* q, int32_t dq);
size_t fpe_compose_bigint_workspace_bytes(const fpe_tree* t, const uint64_t* q, int32_t dq);
fpe_status fpe_compose_bigint(const fpe_tree* t, const uint64_t* q, int32_t dq, uint32_t* out, int64_t lout,
                              void* workspace, size_t workspace_bytes, void* stream);
/* Waits for stream, then reads the overflow flag that the last fpe_eval_bigint,
 * fpe_eval_bigpoint or fpe_compose_bigint on this workspace wrote (a value
 * needed more than lout limbs, which the
 * host's lout bound rules out; a device-side check).  FPE_OK, or FPE_ENOMEM
 * if the result was truncated.  This call synchronises; fpe_eval_bigint does not. */
fpe_status fpe_bigint_status(const void* workspace, void* stream);
fpe_status fpe_compose(const fpe_tree* t, const uint32_t* q, int32_t dq, uint32_t* out,
                       void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a persistent request loop with continuous batching (the walk of
 * Section 2.1 run for many requests at once; the trees are compiled once and
 * stay resident, the "subsequent fast evaluation" of Section 1).
 *
 * Requests of uneven size are admitted in arrival order while the bytes they
 * use fit the HBM budget and an in-flight slot is free.  Admitted FPE_F64 /
 * FPE_F32C evaluate requests are packed into one fused launch (a work table
 * of (tree, point range) blocks) replayed through a HIP graph; FPE_MODP
 * evaluate requests, FPE_F64 requests that take the term-parallel path (few
 * points on big trees: request path 2, or 1 where the cost model picks it)
 * and compose requests of the batch run beside it as their own launches.  Each batch runs on one of two streams of the server (default
 * priority), so a batch overlaps the tail of the one before it; requests
 * arriving while batches run join the next one.  Each point's result depends
 * only on its own walk, so a request's output is the same bits alone
 * (fpe_evaluate with the request's path / fpe_compose) and in any mix.  Latency is measured from
 * submit to the host observing completion.
 *
 * Device memory: the server takes one caller-owned device buffer (for
 * example a torch uint8 tensor) of fpe_server_workspace_bytes(hbm_budget)
 * bytes for its work tables and the per-request scratch (fallback lists,
 * composition workspaces), and allocates no device memory itself.
 * Ordering: before each batch the server's streams wait for the work the
 * caller enqueued on `stream` (given at creation) up to that moment, so
 * inputs written there before submit are seen; outputs are complete once
 * poll reports the ticket done or wait returns.
 * ---------------------------------------------------------------------- */
typedef struct fpe_server fpe_server;

typedef enum { FPE_REQ_EVALUATE = 0, FPE_REQ_COMPOSE = 1 } fpe_request_kind;

typedef struct {
  const fpe_tree* tree;     /* uploaded; FPE_F64, FPE_F32C or FPE_MODP (2^61 - 1) for evaluate,
                               FPE_MODP 2^31 - 1 (a batch of p) for compose */
  const void* pts[8];       /* evaluate: nvars device pointers (SoA), double or uint64 residues */
  int64_t npts;             /* evaluate: points */
  void* out;                /* evaluate: device double[npts] / uint64[npts];
                               compose: device uint32[batch * (deg_p * dq + 1)] */
  float* cond_out;          /* optional device float[npts] (FPE_F32C) */
  double tol;               /* FPE_F32C tolerance (<= 0: 1e-12) */
  int32_t domain;           /* the tree's domain */
  int32_t kind;             /* fpe_request_kind */
  const uint32_t* q;        /* compose: device uint32[batch * (dq + 1)] */
  int32_t dq;               /* compose: degree of q (>= 1) */
  int32_t path;             /* evaluate, FPE_F64 / FPE_MODP: as fpe_eval_opts.path (0 = the tree
                               walk, 1 = the cost model's choice, 2 = the term-parallel path);
                               0 for FPE_F32C.  A request on the term path runs as its own
                               launch beside the fused walk. */
} fpe_request;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t batches;
  double p50_ms, p99_ms, mean_ms;   /* submit -> completion latency (quantiles within 0.5 %) */
  double term_evals;                /* sum of nonzero terms x points over completed evaluate requests */
  double busy_s;                    /* wall time with at least one batch on the GPU */
  double fallback_frac;             /* re-evaluated points / points (FPE_F32C requests) */
  int64_t hbm_in_use;               /* bytes counted against the budget by admitted requests */
  int64_t compose_instances;        /* instances of completed compose requests */
} fpe_stats;

/* Device bytes the server needs for a given budget: its work tables and the
 * pool that per-request scratch comes from. */
size_t fpe_server_workspace_bytes(size_t hbm_budget);

/* workspace: caller-owned device buffer of fpe_server_workspace_bytes(hbm_budget)
 *   bytes, 256-byte aligned, which must outlive the server.
 * hbm_budget: bytes admitted requests may use at once.  A request counts its
 *   points (8 B per variable and point), output, condition output, fallback
 *   list (4 B per point, FPE_F32C), composition workspace and tree image.
 * max_inflight: requests admitted at once (at most 256).
 * stream: the caller's stream whose prior work every batch waits for (NULL =
 *   the default stream).
 * Errors: FPE_EINVAL, FPE_ENOMEM (workspace too small), FPE_EDEVICE. */
fpe_status fpe_server_create(void* workspace, size_t workspace_bytes, size_t hbm_budget, int32_t max_inflight,
                             void* stream, fpe_server** out);
/* Non-blocking.  FPE_EBUDGET if the request alone exceeds the budget. */
fpe_status fpe_server_submit(fpe_server* s, const fpe_request* r, uint64_t* ticket);
/* *done = 1 once the request has completed (its outputs are written);
 * completed requests keep no state, so any earlier ticket no longer pending
 * reports done.  FPE_EINVAL for a ticket never issued. */
fpe_status fpe_server_poll(fpe_server* s, uint64_t ticket, int32_t* done);
fpe_status fpe_server_wait(fpe_server* s, uint64_t ticket);
fpe_status fpe_server_drain(fpe_server* s);
fpe_status fpe_server_stats(fpe_server* s, fpe_stats* st);
/* Drains, then releases the server (not the caller's workspace). */
void fpe_server_destroy(fpe_server* s);

#ifdef __cplusplus
}
#endif
#endif /* FPE_H */
