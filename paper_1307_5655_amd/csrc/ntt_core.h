// Residue arithmetic of the number-theoretic transforms (shared by the
// composition products and the big-integer products): three primes below
// 2^31 with large power-of-two roots of unity, Montgomery multiplication
// (R = 2^32), and the twiddle tables (Montgomery form) of transforms of up to
// kNttMax points.  Included by one translation unit each; everything has
// internal linkage.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpe {
namespace {

constexpr int kNttLogMax = 14;
constexpr int kNttMax = 1 << kNttLogMax;   // largest transform length (LDS: 4 bytes per word, 64 KB)
constexpr int kNttThreads = 1024;

struct NttPrime {
  uint32_t p, pinv, r2, g;   // pinv = -p^-1 mod 2^32, r2 = 2^64 mod p, g a generator
};
constexpr uint32_t neg_inv32(uint32_t p) {
  uint32_t x = p;   // Newton's iteration for p^-1 mod 2^32 (p odd)
  for (int i = 0; i < 5; ++i) x *= 2u - p * x;
  return 0u - x;
}
constexpr uint32_t r2_mod(uint32_t p) {
  const uint64_t r = ((uint64_t)1 << 32) % p;
  return (uint32_t)((r * r) % p);
}
constexpr NttPrime make_prime(uint32_t p, uint32_t g) { return NttPrime{p, neg_inv32(p), r2_mod(p), g}; }
constexpr NttPrime kPrimes[3] = {make_prime(2113929217u, 5u), make_prime(2013265921u, 31u),
                                 make_prime(1811939329u, 13u)};

__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  const uint64_t t = (uint64_t)a * b;
  const uint32_t m = (uint32_t)t * pinv;
  const uint32_t r = (uint32_t)((t + (uint64_t)m * p) >> 32);
  return r >= p ? r - p : r;
}
__device__ __forceinline__ uint32_t madd(uint32_t a, uint32_t b, uint32_t p) {
  const uint32_t s = a + b;
  return s >= p ? s - p : s;
}
__device__ __forceinline__ uint32_t msub(uint32_t a, uint32_t b, uint32_t p) { return a >= b ? a - b : a + p - b; }

uint64_t host_pow(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = (uint64_t)((unsigned __int128)r * b % m);
    b = (uint64_t)((unsigned __int128)b * b % m);
    e >>= 1;
  }
  return r;
}

// Twiddle tables of one prime: tw[k] = w^k and tw[kNttMax / 2 + k] = w^-k
// (k < kNttMax / 2) in Montgomery form, w a primitive kNttMax-th root.
__global__ void k_twiddles(uint32_t* tw, uint32_t w, uint32_t winv, int prime) {
  const NttPrime P = kPrimes[prime];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNttMax / 2) return;
  uint32_t acc = mmul(1u, P.r2, P.p, P.pinv), acci = acc;
  uint32_t b = mmul(w, P.r2, P.p, P.pinv), bi = mmul(winv, P.r2, P.p, P.pinv);
  for (int e = k; e; e >>= 1) {
    if (e & 1) {
      acc = mmul(acc, b, P.p, P.pinv);
      acci = mmul(acci, bi, P.p, P.pinv);
    }
    b = mmul(b, b, P.p, P.pinv);
    bi = mmul(bi, bi, P.p, P.pinv);
  }
  tw[k] = acc;
  tw[kNttMax / 2 + k] = acci;
}

struct Scales {
  uint32_t s[3];   // n^-1 R^2 mod p for each prime
};
Scales scales_for(int n) {
  Scales sc{};
  for (int k = 0; k < 3; ++k) {
    const uint64_t p = kPrimes[k].p;
    const uint64_t ninv = host_pow((uint64_t)n, p - 2, p);
    sc.s[k] = (uint32_t)((unsigned __int128)ninv * kPrimes[k].r2 % p);
  }
  return sc;
}

// Fills the twiddle tables of the first nprimes primes (kNttMax words each).
void launch_twiddles(uint32_t* tw, int nprimes, hipStream_t st) {
  for (int k = 0; k < nprimes; ++k) {
    const uint64_t p = kPrimes[k].p;
    const uint64_t w = host_pow(kPrimes[k].g, (p - 1) / kNttMax, p);
    const uint64_t wi = host_pow(w, p - 2, p);
    hipLaunchKernelGGL(k_twiddles, dim3(kNttMax / 2 / 256), dim3(256), 0, st, tw + (size_t)k * kNttMax,
                       (uint32_t)w, (uint32_t)wi, k);
  }
}

}  // namespace
}  // namespace fpe
