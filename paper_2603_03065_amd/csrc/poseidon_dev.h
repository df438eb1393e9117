// Device routines of the width-12 Poseidon permutation, shared by the
// single-trace kernels (poseidon.hip) and the batch kernels (batch.hip).
//
// Round r: add round constants to all 12 lanes, x^7 on all lanes (r < 4 or
// r >= 26) or on lane 0 only, then multiply by the circulant MDS matrix
// M[i][j] = a[(j - i) mod 12] with small entries a[j] in [1, 255].
//
// The state is kept relaxed in [0, 2^64) between rounds and reduced to [0, p)
// only when written out. The matrix product uses the entries' smallness: each
// state word is split into 32-bit halves and every output accumulates
//   lo = sum_j a * s_j.lo,  hi = sum_j a * s_j.hi   (each < 12 * 255 * 2^32 < 2^44)
// with one v_mad_u64_u32 per term; lo + hi * 2^32 (< 2^77) is then folded with
// 2^64 = 2^32 - 1 (mod p). The round constants are wave-uniform scalar loads;
// the 12 matrix entries are kernel arguments (SGPRs).
#pragma once
#include "internal.h"

namespace v3db {
namespace pos {

struct Circ {
  uint32_t a[WIDTH];
};

// x^7; LAT selects the multiplication with the shorter dependent chain
template <bool LAT = false>
__device__ __forceinline__ uint64_t sbox(uint64_t x) {
  auto mul = [](uint64_t a, uint64_t b) { return LAT ? gl::mul_r_lat(a, b) : gl::mul_r(a, b); };
  const uint64_t x2 = mul(x, x);
  const uint64_t x3 = mul(x2, x);
  const uint64_t x4 = mul(x2, x2);
  return mul(x3, x4);
}

// lo + hi * 2^32 for lo, hi < 2^46, to a relaxed value: with hi = hh*2^32 + hl,
// the sum is lo + hh*2^64 + hl*2^32 = (hh*(2^32-1) + lo) + hl*2^32 (mod p); the
// first part t is one multiply-add below 2^47, the second adds hl to its high word,
// and a carry c out of bit 64 is worth 2^32 - 1 again. The sum is then below 2^47, so
// adding c*(2^32 - 1) cannot overflow; it is done on the two words with the carry
// masks: low word t.lo - c (borrowing b only when t.lo = 0), high word + (c and not b).
__device__ __forceinline__ uint64_t fold(uint64_t lo, uint64_t hi) {
  const uint64_t t = (uint64_t)(uint32_t)(hi >> 32) * gl::EPS + lo;
#ifdef __HIP_DEVICE_COMPILE__
  uint64_t c, b;
  const uint32_t rh = gl::isa::add_co((uint32_t)(t >> 32), (uint32_t)hi, c);
  const uint32_t r0 = gl::isa::subb0((uint32_t)t, c, b);
  const uint32_t r1 = gl::isa::addc0(rh, c & ~b);
  return ((uint64_t)r1 << 32) | r0;
#else
  const uint32_t th = (uint32_t)(t >> 32);
  const uint32_t rh = th + (uint32_t)hi;
  const uint64_t r = ((uint64_t)rh << 32) | (uint32_t)t;
  return r + (rh < th ? gl::EPS : 0);
#endif
}

// c + a * x, and acc += a * x, each as one v_mad_u64_u32 (the carry out is unused).
__device__ __forceinline__ uint64_t mad_start(uint32_t a, uint32_t x, uint64_t c) {
  uint64_t d;
  asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=&v"(d) : "v"(a), "v"(x), "s"(c) : "vcc");
  return d;
}
__device__ __forceinline__ void mad_acc(uint64_t &acc, uint32_t a, uint32_t x) {
  asm("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(acc) : "v"(a), "v"(x) : "vcc");
}

// state <- M * state + rc_next. The next round's constants enter as the initial
// values of the two accumulators (their low and high 32-bit halves), so the
// constant addition costs nothing. All sums stay below 2^44.
__device__ __forceinline__ void mds_ark(uint64_t s[WIDTH], const uint32_t a[WIDTH],
                                        const uint64_t *__restrict__ rc_next) {
  uint32_t lo[WIDTH], hi[WIDTH];
#pragma unroll
  for (int j = 0; j < WIDTH; j++) {
    lo[j] = (uint32_t)s[j];
    hi[j] = (uint32_t)(s[j] >> 32);
  }
#pragma unroll
  for (int i = 0; i < WIDTH; i++) {
    const uint64_t rc = rc_next[i];
    // one chain per accumulator with the constant as the first multiply-add's
    // addend, written as single instructions so the sum is not re-associated into
    // several chains joined by additions
    uint64_t al = mad_start(a[(1 - i + WIDTH) % WIDTH], lo[1], (uint32_t)rc);
    uint64_t ah = mad_start(a[(1 - i + WIDTH) % WIDTH], hi[1], rc >> 32);
#pragma unroll
    for (int jj = 2; jj <= WIDTH; jj++) {
      const int j = jj % WIDTH;  // word 0 (a partial round's only S-box output) last
      const uint32_t c = a[(j - i + WIDTH) % WIDTH];
      mad_acc(al, c, lo[j]);
      mad_acc(ah, c, hi[j]);
    }
    s[i] = fold(al, ah);
  }
}

// The matrix entries as per-lane registers: with the multiplier in a VGPR, the
// accumulator's initial value (a round constant in SGPRs) can be the
// multiply-add's scalar operand.
__device__ __forceinline__ void circ_to_vgprs(const Circ &c, uint32_t a[WIDTH]) {
#pragma unroll
  for (int i = 0; i < WIDTH; i++) asm volatile("v_mov_b32 %0, %1" : "=v"(a[i]) : "s"(c.a[i]));
}

// rc: 31 rows of 12 (the 30 rounds' constants, then a row of zeros so the last
// round's linear layer can take "next constants" like every other round).
__device__ __forceinline__ void permute(uint64_t s[WIDTH], const uint64_t *__restrict__ rc, const uint32_t a[WIDTH]) {
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = gl::add_r(s[i], rc[i]);
#pragma unroll 1
  for (int r = 0; r < FULL_HALF; r++) {
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);
    mds_ark(s, a, rc + (r + 1) * WIDTH);
  }
#pragma unroll 2
  for (int r = FULL_HALF; r < ROUNDS - FULL_HALF; r++) {
    s[0] = sbox(s[0]);
    mds_ark(s, a, rc + (r + 1) * WIDTH);
  }
#pragma unroll 1
  for (int r = ROUNDS - FULL_HALF; r < ROUNDS; r++) {
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);
    mds_ark(s, a, rc + (r + 1) * WIDTH);
  }
}

// Leaf digest of row k of a column-major matrix with n_rows rows: the rate-8
// overwrite sponge over columns 0..n_cols-1 (lane k reads column c at row k, so a
// wave's loads are 64 consecutive words of one column). Writes 4 canonical words.
__device__ __forceinline__ void leaf_digest(const uint64_t *__restrict__ mat, uint32_t n_cols, uint64_t n_rows,
                                            uint64_t k, uint64_t *__restrict__ out, const uint64_t *__restrict__ rc,
                                            const uint32_t a[WIDTH]) {
  uint64_t s[WIDTH];
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = 0;
  for (uint32_t q = 0; q < n_cols; q += RATE) {
    const uint32_t len = (n_cols - q) < RATE ? (n_cols - q) : RATE;
    const uint64_t *base = mat + uint64_t(q) * n_rows + k;
#pragma unroll
    for (int i = 0; i < RATE; i++)
      if (i < (int)len) s[i] = base[uint64_t(i) * n_rows];
    permute(s, rc, a);
  }
#pragma unroll
  for (int i = 0; i < DIGEST; i++) out[i] = gl::canon(s[i]);
}

// Node k of a level = Compress(below[2k], below[2k+1]).
__device__ __forceinline__ void merkle_node(const uint64_t *__restrict__ below, uint64_t k, uint64_t *__restrict__ out,
                                            const uint64_t *__restrict__ rc, const uint32_t a[WIDTH]) {
  uint64_t s[WIDTH];
  const uint64_t *src = below + k * (2 * DIGEST);
#pragma unroll
  for (int i = 0; i < 2 * DIGEST; i++) s[i] = src[i];
#pragma unroll
  for (int i = 2 * DIGEST; i < WIDTH; i++) s[i] = 0;
  permute(s, rc, a);
#pragma unroll
  for (int i = 0; i < DIGEST; i++) out[i] = gl::canon(s[i]);
}

// Permutation by a group of 16 lanes, lane g < 12 holding state word g (lanes
// 12..15 follow lane 0 and are discarded). Each round applies the S-box on the
// lane's own word (full rounds) or on lane 0 (partial rounds); then every lane
// receives the 12 words by 64-bit row broadcasts (DPP row_newbcast: a group is
// one 16-lane row) and forms its own row of the matrix product. The dependent chain per permutation is a fraction of the
// one-permutation-per-lane form, which is what the upper tree levels (too few
// nodes to fill the device) and long sequential sponges are bound by. All 64
// lanes of the wave must be active when this is called.
constexpr int WIDE_GROUP = 16;
constexpr int WIDE_THREADS = 64;  // one wave: 4 permutations
constexpr int WIDE_PER_BLOCK = WIDE_THREADS / WIDE_GROUP;

// lane J of each 16-lane row, at every lane of the row (v_mov_b64_dpp row_newbcast:J).
// Every lane has a source, so no previous value of the destination is kept and the
// compiler needs no zeroing move before it.
template <int J>
__device__ __forceinline__ uint64_t row_bcast(uint64_t v) {
  return (uint64_t)__builtin_amdgcn_mov_dpp((long)v, 0x150 + J, 0xf, 0xf, true);
}

template <int J>
__device__ __forceinline__ void mds_term(uint64_t s, const uint32_t m[WIDTH], uint64_t &al, uint64_t &ah) {
  const uint64_t v = row_bcast<J>(s);
  al += (uint64_t)m[J] * (uint32_t)v;
  ah += (uint64_t)m[J] * (uint32_t)(v >> 32);
}

__device__ __forceinline__ uint64_t wide_permute(uint64_t s, int g, const uint64_t *__restrict__ rc,
                                                 const uint32_t *__restrict__ circ_rows) {
  const int gi = g < WIDTH ? g : 0;
  uint32_t m[WIDTH];  // this lane's row of the matrix
#pragma unroll
  for (int j = 0; j < WIDTH; j++) m[j] = circ_rows[gi * WIDTH + j];
  s = gl::add_r(s, rc[gi]);
  uint64_t rcn = rc[WIDTH + gi];
#pragma unroll 1
  for (int r = 0; r < ROUNDS; r++) {
    const uint64_t rc_next = rcn;
    if (r + 1 < ROUNDS) rcn = rc[(r + 2) * WIDTH + gi];
    const bool full = r < FULL_HALF || r >= ROUNDS - FULL_HALF;
    if (full) {
      s = sbox<true>(s);
    } else {
      // x^7 of word 0 with two lanes: every lane forms x^2, lane 1 then x^4 while the
      // others form x^3, and x^3 * x^4 (three dependent products instead of four)
      const uint64_t x = row_bcast<0>(s);
      const uint64_t x2 = gl::mul_r_lat(x, x);
      const uint64_t y = gl::mul_r_lat(x2, g == 1 ? x2 : x);
      const uint64_t x7 = gl::mul_r_lat(y, row_bcast<1>(y));
      if (g == 0) s = x7;
    }
    uint64_t al = (uint32_t)rc_next, ah = rc_next >> 32;
    mds_term<0>(s, m, al, ah);
    mds_term<1>(s, m, al, ah);
    mds_term<2>(s, m, al, ah);
    mds_term<3>(s, m, al, ah);
    mds_term<4>(s, m, al, ah);
    mds_term<5>(s, m, al, ah);
    mds_term<6>(s, m, al, ah);
    mds_term<7>(s, m, al, ah);
    mds_term<8>(s, m, al, ah);
    mds_term<9>(s, m, al, ah);
    mds_term<10>(s, m, al, ah);
    mds_term<11>(s, m, al, ah);
    s = fold(al, ah);
  }
  return s;
}

// Rate-8 overwrite sponge over a sequence of len words by a group of 16 lanes
// (wide_permute); elem(x) gives word x and is called only by live lanes g < 8.
// Lane g < 12 returns state word g.
template <class Elem>
__device__ __forceinline__ uint64_t wide_sponge(uint64_t len, bool live, Elem elem, int g,
                                                const uint64_t *__restrict__ rc,
                                                const uint32_t *__restrict__ circ_rows) {
  uint64_t s = 0;
  for (uint64_t c0 = 0; c0 < len; c0 += RATE) {
    if (live && g < RATE && c0 + g < len) s = elem(c0 + g);
    s = wide_permute(s, g, rc, circ_rows);
  }
  return s;
}

inline Circ circ_of(const v3db_ctx *ctx) {
  Circ c;
  for (int i = 0; i < WIDTH; i++) c.a[i] = ctx->pos.circ[i];
  return c;
}

// Permutation by 32 lanes (two 16-lane rows), for work bound by one permutation's
// latency (a long sponge, a query's authentication path, the top levels of a
// tree): a single wave then issues every instruction of the chain in turn, so
// what counts is the number of instructions per lane per round. Both rows hold
// the state (lane g < 12 of each row holds word g). Per round:
//   * S-box: every lane forms x^2, the even row x^3 and the odd row x^4, the two
//     are exchanged with v_permlane16_swap and multiplied (three products per
//     lane instead of the four of x^7 on one lane; in partial rounds x is word 0
//     broadcast over the row and only lane 0 keeps the result);
//   * matrix product: the even row forms, for every output, the terms of words
//     0..5 and the odd row those of words 6..11 (moved to its lanes 0..5 by a row
//     shift), six broadcasts and twelve multiply-adds per lane instead of twelve
//     and twenty-four; the two halves are added across the rows with
//     v_permlane16_swap and folded as in wide_permute.
// Used where few permutations run at once; with many, the 16-lane form does less
// work in all. All 64 lanes of the wave must be active.
constexpr int PAIR_GROUP = 32;
constexpr int PAIR_THREADS = 64;  // one wave: 2 permutations
constexpr int PAIR_PER_BLOCK = PAIR_THREADS / PAIR_GROUP;

// v on the even row and v on the odd row of this lane's row pair, at every lane
__device__ __forceinline__ void rows_both(uint64_t v, uint64_t &even, uint64_t &odd) {
  const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)v, (uint32_t)v, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(v >> 32), (uint32_t)(v >> 32), false, false);
  even = ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0];
  odd = ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1];
}

// lane i of each row receives lane i + 6 of the row (DPP row_shl:6; lanes 10..15 have
// no source and read 0 under bound_ctrl)
__device__ __forceinline__ uint64_t row_shl6(uint64_t v) {
  return (uint64_t)__builtin_amdgcn_mov_dpp((long)v, 0x106, 0xf, 0xf, true);
}

template <int J>
__device__ __forceinline__ void pair_term(uint64_t src, const uint32_t m[6], uint64_t &al, uint64_t &ah) {
  const uint64_t v = row_bcast<J>(src);
  al += (uint64_t)m[J] * (uint32_t)v;
  ah += (uint64_t)m[J] * (uint32_t)(v >> 32);
}

__device__ __forceinline__ uint64_t pair_permute(uint64_t s, int q, const uint64_t *__restrict__ rc,
                                                 const uint32_t *__restrict__ circ_rows) {
  const int g = q & 15, odd = q >> 4;
  const int gi = g < WIDTH ? g : 0;
  uint32_t m[6];  // this lane's half row of the matrix: entries 6 odd .. 6 odd + 5 of row gi
#pragma unroll
  for (int j = 0; j < 6; j++) m[j] = circ_rows[gi * WIDTH + 6 * odd + j];
  s = gl::add_r(s, rc[gi]);
  uint64_t rcn = rc[WIDTH + gi];
#pragma unroll 1
  for (int r = 0; r < ROUNDS; r++) {
    const uint64_t rc_next = rcn;
    if (r + 1 < ROUNDS) rcn = rc[(r + 2) * WIDTH + gi];
    const bool full = r < FULL_HALF || r >= ROUNDS - FULL_HALF;
    const uint64_t x = full ? s : row_bcast<0>(s);
    const uint64_t x2 = gl::mul_r_lat(x, x);
    const uint64_t y = gl::mul_r_lat(x2, odd ? x2 : x);
    uint64_t y_even, y_odd;
    rows_both(y, y_even, y_odd);
    const uint64_t x7 = gl::mul_r_lat(y_even, y_odd);
    s = (full || g == 0) ? x7 : s;
    const uint64_t t = row_shl6(s);
    const uint64_t src = odd ? t : s;
    uint64_t al = odd ? 0 : (uint32_t)rc_next, ah = odd ? 0 : rc_next >> 32;
    pair_term<0>(src, m, al, ah);
    pair_term<1>(src, m, al, ah);
    pair_term<2>(src, m, al, ah);
    pair_term<3>(src, m, al, ah);
    pair_term<4>(src, m, al, ah);
    pair_term<5>(src, m, al, ah);
    uint64_t al_e, al_o, ah_e, ah_o;
    rows_both(al, al_e, al_o);
    rows_both(ah, ah_e, ah_o);
    s = fold(al_e + al_o, ah_e + ah_o);
  }
  return s;
}

// Rate-8 overwrite sponge over len words by a group of 32 lanes (pair_permute);
// elem(x) gives word x and is called only by live lanes with q % 16 < 8. Lane
// q % 16 < 12 returns state word q % 16.
template <class Elem>
__device__ __forceinline__ uint64_t pair_sponge(uint64_t len, bool live, Elem elem, int q,
                                                const uint64_t *__restrict__ rc,
                                                const uint32_t *__restrict__ circ_rows) {
  const int g = q & 15;
  uint64_t s = 0;
  for (uint64_t c0 = 0; c0 < len; c0 += RATE) {
    if (live && g < RATE && c0 + g < len) s = elem(c0 + g);
    s = pair_permute(s, q, rc, circ_rows);
  }
  return s;
}

}  // namespace pos
}  // namespace v3db
