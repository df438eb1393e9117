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
// Single gfx950 instructions whose carry or borrow is a lane mask in an SGPR pair,
// so a carry feeds the next instruction (or a select) directly instead of being
// turned into a 0/1 value first. One instruction per statement lets the compiler
// schedule them and insert the wait states between them.
namespace isa {
__device__ __forceinline__ uint64_t mad(uint32_t a, uint32_t b, uint64_t c, uint64_t &co) {
  uint64_t d;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=&v"(d), "=s"(co) : "v"(a), "v"(b), "v"(c));
  return d;
}
__device__ __forceinline__ uint64_t mad_eps(uint32_t a, uint64_t c, uint64_t &co) {  // c + a * (2^32 - 1)
  uint64_t d;
  asm("v_mad_u64_u32 %0, %1, %2, -1, %3" : "=&v"(d), "=s"(co) : "v"(a), "v"(c));
  return d;
}
__device__ __forceinline__ uint32_t add_co(uint32_t a, uint32_t b, uint64_t &co) {
  uint32_t d;
  asm("v_add_co_u32_e64 %0, %1, %2, %3" : "=v"(d), "=s"(co) : "v"(a), "v"(b));
  return d;
}
__device__ __forceinline__ uint32_t addc(uint32_t a, uint32_t b, uint64_t ci, uint64_t &co) {
  uint32_t d;
  asm("v_addc_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(d), "=s"(co) : "v"(a), "v"(b), "s"(ci));
  return d;
}
__device__ __forceinline__ uint32_t addc0(uint32_t a, uint64_t ci) {  // a + carry; no carry out possible here
  uint32_t d;
  uint64_t co;
  asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(d), "=s"(co) : "v"(a), "s"(ci));
  return d;
}
__device__ __forceinline__ uint32_t sub_co(uint32_t a, uint32_t b, uint64_t &bo) {
  uint32_t d;
  asm("v_sub_co_u32_e64 %0, %1, %2, %3" : "=v"(d), "=s"(bo) : "v"(a), "v"(b));
  return d;
}
__device__ __forceinline__ uint32_t subb(uint32_t a, uint32_t b, uint64_t bi, uint64_t &bo) {
  uint32_t d;
  asm("v_subb_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(d), "=s"(bo) : "v"(a), "v"(b), "s"(bi));
  return d;
}
__device__ __forceinline__ uint32_t addc0_co(uint32_t a, uint64_t ci, uint64_t &co) {  // a + carry, carry out
  uint32_t d;
  asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(d), "=s"(co) : "v"(a), "s"(ci));
  return d;
}
__device__ __forceinline__ uint32_t subb0(uint32_t a, uint64_t bi, uint64_t &bo) {  // a - borrow
  uint32_t d;
  asm("v_subb_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(d), "=s"(bo) : "v"(a), "s"(bi));
  return d;
}
template <int IF1>
__device__ __forceinline__ uint32_t sel0(uint64_t m) {  // m ? IF1 : 0 (IF1 an inline constant)
  uint32_t d;
  asm("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(d) : "i"(IF1), "s"(m));
  return d;
}
template <int IF1>
__device__ __forceinline__ uint32_t sel(uint64_t m, uint32_t if0) {  // m ? IF1 : if0
  uint32_t d;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(d) : "v"(if0), "i"(IF1), "s"(m));
  return d;
}

// d + (2^32 - 1) * (up - down) for lane masks up, down, where the callers
// guarantee that the result lies in [0, 2^64). The two corrections cancel where
// both masks are set; otherwise one 64-bit addend, 2^32 - 1 or -(2^32 - 1), made
// with three selects after two scalar mask operations.
__device__ __forceinline__ uint64_t fix_eps(uint32_t d0, uint32_t d1, uint64_t up, uint64_t down) {
  const uint64_t pos = up & ~down, neg = down & ~up;
  const uint32_t f1 = sel0<-1>(neg);
  const uint32_t f0 = sel<-1>(pos, 0u - f1);  // neg: 1 = -(2^32 - 1) mod 2^32, from a plain subtraction
  uint64_t r;  // one 64-bit add (the compiler would add the high word separately)
  asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(r) : "v"((((uint64_t)d1) << 32) | d0), "v"((((uint64_t)f1) << 32) | f0));
  return r;
}
}  // namespace isa

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
  // s + c*2^64 = lo + hl*(2^32-1); d - b*2^64 = s - hh; the value is
  // d + (c - b)*(2^32-1). If c and not b, s < 2^64 - 2^33 + 1 leaves room for
  // 2^32-1; if b and not c, d >= 2^64 - 2^32, so subtracting 2^32-1 stays >= 0.
  uint64_t c, x, b;
  const uint64_t s = isa::mad_eps(hl, lo, c);
  const uint32_t d0 = isa::sub_co((uint32_t)s, hh, x);
  const uint32_t d1 = isa::subb0((uint32_t)(s >> 32), x, b);
  return isa::fix_eps(d0, d1, c, b);
#else
  uint64_t t0;
  if (__builtin_sub_overflow(lo, (uint64_t)hh, &t0)) t0 -= EPS;  // borrowed 2^64 = EPS; t0 >= 2^64 - 2^32 here
  const uint64_t t1 = (uint64_t)hl * EPS;                         // hl * (2^32 - 1)
  uint64_t t2;
  if (__builtin_add_overflow(t0, t1, &t2)) t2 += EPS;            // carried 2^64; cannot carry again
  return t2;
#endif
}

GL_HD uint64_t canon(uint64_t x) {
#ifdef __HIP_DEVICE_COMPILE__
  // x - p = x + (2^32 - 1) modulo 2^64 where x >= p, with the compare's mask as the
  // borrow into the low word and the carry into the high word (which then wraps)
  uint64_t bb;
  const uint64_t m = __builtin_amdgcn_uicmpl(P - 1, x, 36 /* unsigned less than */);
  const uint32_t r0 = isa::subb0((uint32_t)x, m, bb);
  const uint32_t r1 = isa::addc0((uint32_t)(x >> 32), m & ~bb);
  return ((uint64_t)r1 << 32) | r0;
#else
  return x >= P ? x - P : x;
#endif
}

// x * 2^K (0 < K < 64), relaxed: the 128-bit product is a pair of shifts.
template <int K>
GL_HD uint64_t mul_pow2(uint64_t x) {
  return reduce128(x << K, x >> (64 - K));
}

// relaxed * relaxed -> relaxed
GL_HD uint64_t mul_r(uint64_t a, uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  // The four partial products, the middle two summed with the carry c (weight
  // 2^96); the 128-bit product is L + 2^64*H + 2^96*c with L = p00 + 2^32*m.lo
  // and H = p11 + m.hi + carry, assembled by one add-with-carry chain (H cannot
  // overflow: p11 <= 2^64 - 2^33 + 1). Then, with 2^64 = 2^32-1 and 2^96 = -1,
  // the value is L + H.lo*(2^32-1) - H.hi - c, reduced as in reduce128 with c as
  // the first subtraction's borrow in.
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint64_t c, k1, k2, c2, x, bw;
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t m = isa::mad(a0, b1, (uint64_t)a1 * b0, c);
  const uint64_t p11 = (uint64_t)a1 * b1;
  const uint32_t t1 = isa::add_co((uint32_t)(p00 >> 32), (uint32_t)m, k1);
  const uint32_t t2 = isa::addc((uint32_t)p11, (uint32_t)(m >> 32), k1, k2);
  const uint32_t t3 = isa::addc0((uint32_t)(p11 >> 32), k2);
  const uint64_t s = isa::mad_eps(t2, (((uint64_t)t1) << 32) | (uint32_t)p00, c2);
  const uint32_t d0 = isa::subb((uint32_t)s, t3, c, x);
  const uint32_t d1 = isa::subb0((uint32_t)(s >> 32), x, bw);
  return isa::fix_eps(d0, d1, c2, bw);
#else
  uint64_t lo, hi;
  mul_wide(a, b, lo, hi);
  return reduce128(lo, hi);
#endif
}

// relaxed * relaxed -> relaxed with a shorter dependent chain than mul_r (more
// instructions, fewer of them waiting on a carry written by the one before), for
// code bound by one permutation's latency rather than by issue throughput.
GL_HD uint64_t mul_r_lat(uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  mul_wide(a, b, lo, hi);
#ifdef __HIP_DEVICE_COMPILE__
  // lo - hh + hl*(2^32-1) as in reduce128, with the borrow and the carry turned
  // into 0/1 values and 64-bit additions
  const uint32_t hh = (uint32_t)(hi >> 32), hl = (uint32_t)hi;
  unsigned b1, bw;
  const uint32_t r0 = __builtin_subc((uint32_t)lo, hh, 0u, &b1);
  const uint32_t r1 = __builtin_subc((uint32_t)(lo >> 32), 0u, b1, &bw);
  const uint64_t r = ((uint64_t)r1 << 32) | r0;
  const uint64_t s = mad_eps(hl, r);
  const bool c = s < r;
  return s + (c ? EPS : 0) - (bw ? EPS : 0);
#else
  return reduce128(lo, hi);
#endif
}

// canonical results
GL_HD uint64_t mul(uint64_t a, uint64_t b) { return canon(mul_r(a, b)); }

GL_HD uint64_t add(uint64_t a, uint64_t b) {  // a, b canonical
  // a + b < 2p: subtract p (add 2^64 - p = EPS modulo 2^64) when the sum carried
  // out of 64 bits or is at least p
#ifdef __HIP_DEVICE_COMPILE__
  // the sum on the carry chain; then + m * (2^32 - 1) for the mask m = carry | (s >= p)
  // as a subtract-with-borrow on the low word and an add-with-carry on the high word
  // (the high word wraps exactly when s >= p, giving s - p)
  uint64_t c, c1, bb, m;
  const uint32_t s0 = isa::add_co((uint32_t)a, (uint32_t)b, c1);
  const uint32_t s1 = isa::addc((uint32_t)(a >> 32), (uint32_t)(b >> 32), c1, c);
  const uint64_t sum = ((uint64_t)s1 << 32) | s0;
  m = c | (uint64_t)__builtin_amdgcn_uicmpl(P - 1, sum, 36 /* unsigned less than */);
  const uint32_t r0 = isa::subb0(s0, m, bb);
  const uint32_t r1 = isa::addc0(s1, m & ~bb);
  return ((uint64_t)r1 << 32) | r0;
#else
  const uint64_t s = a + b, t = s + EPS;
  return ((s < a) | (s >= P)) ? t : s;
#endif
}

GL_HD uint64_t sub(uint64_t a, uint64_t b) {  // a, b canonical
  // a - b + p = d - 2^64 + p = d - EPS when the subtraction borrowed; the borrow
  // is taken from the carry chain rather than from a second comparison
#ifdef __HIP_DEVICE_COMPILE__
  // d - EPS = d + p (mod 2^64): low word + bw with carry k, high word + (2^32 - 1) * bw + k,
  // i.e. minus (bw and not k)
  uint64_t b1, bw, k, unused;
  const uint32_t d0 = isa::sub_co((uint32_t)a, (uint32_t)b, b1);
  const uint32_t d1 = isa::subb((uint32_t)(a >> 32), (uint32_t)(b >> 32), b1, bw);
  const uint32_t r0 = isa::addc0_co(d0, bw, k);
  const uint32_t r1 = isa::subb0(d1, bw & ~k, unused);
  return ((uint64_t)r1 << 32) | r0;
#else
  unsigned b1, bw;
  const uint32_t d0 = __builtin_subc((uint32_t)a, (uint32_t)b, 0u, &b1);
  const uint32_t d1 = __builtin_subc((uint32_t)(a >> 32), (uint32_t)(b >> 32), b1, &bw);
  const uint64_t d = ((uint64_t)d1 << 32) | d0;
  return d - (bw ? EPS : 0);
#endif
}

// relaxed a + canonical b -> relaxed
GL_HD uint64_t add_r(uint64_t a, uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  // the sum on the carry chain, then + c * (2^32 - 1) for its carry c out of bit 64 as
  // a subtract-with-borrow on the low word and an add-with-carry on the high word; with
  // a carry the sum is a + b - 2^64 < p - 1, whose high word is at most 2^32 - 2
  uint64_t c1, c, bb;
  const uint32_t s0 = isa::add_co((uint32_t)a, (uint32_t)b, c1);
  const uint32_t s1 = isa::addc((uint32_t)(a >> 32), (uint32_t)(b >> 32), c1, c);
  const uint32_t r0 = isa::subb0(s0, c, bb);
  const uint32_t r1 = isa::addc0(s1, c & ~bb);
  return ((uint64_t)r1 << 32) | r0;
#else
  uint64_t s = a + b;
  if (s < b) s += EPS;               // a + b - 2^64 < p - 1, so no second carry
  return s;
#endif
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
