// Goldilocks field arithmetic, p = 2^64 - 2^32 + 1, for gfx950 VALU and the host.
//
// No Montgomery form: a 128-bit product x = hi*2^64 + lo with hi = hh*2^32 + hl
// reduces through 2^64 = 2^32 - 1 (mod p) and 2^96 = -1 (mod p) to
//   x = lo - hh + hl*(2^32 - 1)   (mod p),
// one subtraction and one addition with carry fix-ups. Products are built from
// four 32x32->64 multiply-adds (v_mad_u64_u32 is full rate on gfx950).
//
// Two kinds of values appear:
//   canonical   in [0, p): every public input and output, and the NTT data;
//   relaxed     in [0, 2^64): Poseidon state between rounds (reduced at the end).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GL_HD __host__ __device__ __forceinline__

namespace gl {

constexpr uint64_t P = 0xffffffff00000001ull;
constexpr uint64_t EPS = 0xffffffffull;  // 2^64 mod p

// 64x64 -> 128 product from 32-bit halves.
GL_HD void mul_wide(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi) {
  uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint64_t t = (uint64_t)a0 * b0;
  uint64_t u = (uint64_t)a1 * b0 + (t >> 32);
  uint64_t v = (uint64_t)a0 * b1 + (uint32_t)u;
  hi = (uint64_t)a1 * b1 + (u >> 32) + (v >> 32);
  lo = (v << 32) | (uint32_t)t;
}

#ifdef __HIP_DEVICE_COMPILE__
// c + a * (2^32 - 1) modulo 2^64 as one v_mad_u64_u32 (written out because the
// compiler splits a multiply-add whose sum is also compared into two instructions).
__device__ __forceinline__ uint64_t mad_eps(uint32_t a, uint64_t c) {
  uint64_t d;
  asm("v_mad_u64_u32 %0, vcc, %1, -1, %2" : "=&v"(d) : "v"(a), "v"(c) : "vcc");
  return d;
}
#endif

// Reduce hi*2^64 + lo (any 128-bit value) to a relaxed value in [0, 2^64).
GL_HD uint64_t reduce128(uint64_t lo, uint64_t hi) {
  const uint32_t hh = (uint32_t)(hi >> 32), hl = (uint32_t)hi;
#ifdef __HIP_DEVICE_COMPILE__
  // r = lo - hh + b*2^64, s = r + hl*(2^32-1) - c*2^64, so x = s + (c - b)*(2^32-1).
  // If c and not b, s < 2^64 - 2^33 + 2 has room for 2^32-1; if b and not c,
  // s >= r >= 2^64 - 2^32 + 1, so subtracting 2^32-1 stays non-negative.
  unsigned b1, b;
  const uint32_t r0 = __builtin_subc((uint32_t)lo, hh, 0u, &b1);
  const uint32_t r1 = __builtin_subc((uint32_t)(lo >> 32), 0u, b1, &b);
  const uint64_t r = ((uint64_t)r1 << 32) | r0;
  const uint64_t s = mad_eps(hl, r);
  const bool c = s < r;
  return s + (c ? EPS : 0) - (b ? EPS : 0);
#else
  uint64_t t0;
  if (__builtin_sub_overflow(lo, (uint64_t)hh, &t0)) t0 -= EPS;  // borrowed 2^64 = EPS; t0 >= 2^64 - 2^32 here
  const uint64_t t1 = (uint64_t)hl * EPS;                         // hl * (2^32 - 1)
  uint64_t t2;
  if (__builtin_add_overflow(t0, t1, &t2)) t2 += EPS;            // carried 2^64; cannot carry again
  return t2;
#endif
}

GL_HD uint64_t canon(uint64_t x) { return x >= P ? x - P : x; }

// x * 2^K (0 < K < 64), relaxed: the 128-bit product is a pair of shifts.
template <int K>
GL_HD uint64_t mul_pow2(uint64_t x) {
  return reduce128(x << K, x >> (64 - K));
}

// relaxed * relaxed -> relaxed
GL_HD uint64_t mul_r(uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  mul_wide(a, b, lo, hi);
  return reduce128(lo, hi);
}

// canonical results
GL_HD uint64_t mul(uint64_t a, uint64_t b) { return canon(mul_r(a, b)); }

GL_HD uint64_t add(uint64_t a, uint64_t b) {  // a, b canonical
  // a + b < 2p: subtract p (add 2^64 - p = EPS modulo 2^64) when the sum carried
  // out of 64 bits or is at least p; written without branches
  const uint64_t s = a + b, t = s + EPS;
  return (s < a) | (s >= P) ? t : s;
}

GL_HD uint64_t sub(uint64_t a, uint64_t b) {  // a, b canonical
  // a - b + p = d - 2^64 + p = d - EPS when the subtraction borrowed; the borrow
  // is taken from the carry chain rather than from a second comparison
  unsigned b1, bw;
  const uint32_t d0 = __builtin_subc((uint32_t)a, (uint32_t)b, 0u, &b1);
  const uint32_t d1 = __builtin_subc((uint32_t)(a >> 32), (uint32_t)(b >> 32), b1, &bw);
  const uint64_t d = ((uint64_t)d1 << 32) | d0;
  return d - (bw ? EPS : 0);
}

// relaxed a + canonical b -> relaxed
GL_HD uint64_t add_r(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  if (s < b) s += EPS;               // a + b - 2^64 < p - 1, so no second carry
  return s;
}

GL_HD uint64_t pow(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mul(r, a);
    a = mul(a, a);
    e >>= 1;
  }
  return r;
}

GL_HD uint64_t inv(uint64_t a) { return pow(a, P - 2); }

// w_{2^k} = 7^((p-1)/2^k): 7 generates the multiplicative group.
inline uint64_t root_of_unity(uint32_t log_n) { return pow(7, (P - 1) >> log_n); }

}  // namespace gl
