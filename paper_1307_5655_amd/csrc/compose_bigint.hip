// Composition over the natural numbers at one big point: p(q(X)) for p with
// uint64 coefficients (an FPE_BIGINT tree) and q with uint64 coefficients,
// the title problem over the integers, whose elements grow with the degree
// as in Section 1.2.
//
// Kronecker substitution: every coefficient of p(q(X)) is at most the sum of
// all of them, p(q(1)) < 2^B with B = bitlen(sum c_m) + deg p bitlen(q(1)),
// so with slots of lc >= B / 16 limbs the natural number p(q(2^(16 lc))) holds
// the coefficient of X^k in limbs [k lc, (k + 1) lc), no two slots
// overlapping.  The point y = q(2^(16 lc)) is q's coefficients placed one per
// slot; p(y) is the level walk at one big point (bigpoint.hip: the tree's
// levels as batched launches, products by number-theoretic transforms), so
// the schemes' differences are those of Figure 1's setting; the slots are
// then the output.
#include <hip/hip_runtime.h>

#include <string>

#include "fpe_internal.h"

namespace fpe {

namespace {

struct QCoefs {
  uint64_t c[kComposeBigMaxQ];
};

// y[i] for i < ly: limb i mod lc of coefficient i / lc (four limbs each)
__global__ void k_pack_slots(QCoefs q, int32_t dq, int32_t lc, uint32_t* y, int64_t ly) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ly; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = i / lc, t = i - j * lc;
    y[i] = j <= dq && t < 4 ? (uint32_t)((q.c[j] >> (16 * t)) & 0xFFFFu) : 0u;
  }
}

// out[i] = z[i] below nz, zero from there to nout
__global__ void k_copy_slots(const uint32_t* z, int64_t nz, uint32_t* out, int64_t nout) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nout; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = i < nz ? z[i] : 0u;
}

int bitlen128(unsigned __int128 v) {
  int n = 0;
  while (v) {
    ++n;
    v >>= 1;
  }
  return n;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

ComposeBigPlan compose_bigint_plan(const fpe_tree* t, const uint64_t* q, int32_t dq) {
  ComposeBigPlan P{};
  if (!t || t->domain != FPE_BIGINT || !q || dq < 0 || dq >= kComposeBigMaxQ) return P;
  unsigned __int128 sp = 0, q1 = 0;
  for (uint64_t c : t->coef_rows) sp += c;
  for (int32_t j = 0; j <= dq; ++j) q1 += q[j];
  const int64_t dp = t->deg_max[0];
  const int64_t bits = bitlen128(sp) + dp * bitlen128(q1);
  const int64_t lc = std::max<int64_t>(4, (bits + 15) / 16);
  const int64_t ly = (int64_t)dq * lc + 4;
  if (ly > kBigPointMaxLimbs) return P;   // no product of such a point fits a transform
  const int64_t lz = bigpoint_out_limbs(t, (int32_t)ly);
  if (lz <= 0) return P;
  P.lc = (int32_t)lc;
  P.ly = ly;
  P.lz = lz;
  P.nout = (dp * dq + 1) * lc;
  P.off_y = align256(bigpoint_workspace_bytes(t, (int32_t)ly));
  P.off_z = P.off_y + align256((size_t)ly * sizeof(uint32_t));
  P.bytes = P.off_z + align256((size_t)lz * sizeof(uint32_t));
  return P;
}

fpe_status launch_compose_bigint(const fpe_tree* t, const uint64_t* q, int32_t dq, uint32_t* out, int64_t lout,
                                 void* ws, size_t ws_bytes, void* stream) {
  const ComposeBigPlan P = compose_bigint_plan(t, q, dq);
  if (P.lc == 0)
    return fail(FPE_EUNSUPPORTED, "composition at one big point: q longer than 64 coefficients or values "
                                  "beyond the big-point walk's 2^14-limb products");
  if (lout < P.nout) return fail(FPE_EINVAL, "lout smaller than (deg p * dq + 1) * fpe_compose_bigint_coef_limbs()");
  if (!ws || ws_bytes < P.bytes) return fail(FPE_ENOMEM, "workspace smaller than fpe_compose_bigint_workspace_bytes()");
  if (((uintptr_t)ws) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  QCoefs qc{};
  for (int32_t j = 0; j <= dq; ++j) qc.c[j] = q[j];
  uint32_t* y = (uint32_t*)((char*)ws + P.off_y);
  uint32_t* z = (uint32_t*)((char*)ws + P.off_z);
  const unsigned gy = (unsigned)std::min<int64_t>((P.ly + 255) / 256, 1024);
  hipLaunchKernelGGL(k_pack_slots, dim3(gy), dim3(256), 0, st, qc, dq, P.lc, y, P.ly);
  // the big-point walk's workspace is the first part of ours: its overflow
  // flag is the first word, as fpe_bigint_status expects
  const fpe_status s = launch_bigpoint(t, y, (int32_t)P.ly, z, P.lz, ws, P.off_y, stream);
  if (s != FPE_OK) return s;
  const unsigned go = (unsigned)std::min<int64_t>((lout + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy_slots, dim3(go), dim3(256), 0, st, z, std::min(P.lz, P.nout), out, lout);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FPE_EDEVICE, std::string("composition at a big point: ") + hipGetErrorString(e));
  return FPE_OK;
}

}  // namespace fpe
