// Device routines of the coset low-degree extension, shared by the
// single-trace kernels (ntt.hip) and the multi-trace batch kernels (batch.hip).
//
// For a column a of n = 2^L values (a_i = P(w_n^i)), the extension to N = B*n
// points is LDE[k] = P(s * w_N^k) = sum_j c_j (s w_N^k)^j with c = iNTT_n(a).
// It runs as LDS-tiled passes of a four-step factorisation, n = n1*n2:
//
//   pass 1  (interpolation, first half)   j = j1*n2 + j2, k = k1 + n1*k2
//           Y[k1][j2] = w_n^(-j2 k1) * sum_j1 a[j1 n2 + j2] w_n1^(-j1 k1)
//   pass 2  per residue k1: c'[k2] = sum_j2 Y[k1][j2] w_n2^(-j2 k2)   (= n c[k1 + n1 k2])
//           then a blowup-B extension of that residue sequence with shift s^n1,
//           for every e < W = B*n2 (e = r + B*m1: coset r, point m1):
//           Z[k1][e] = n^-1 s^k1 w_N^(k1 e) * sum_k2 c'[k2] (s^n1)^k2 w_W^(k2 e)
//   pass 3  per column e of Z: LDE[e + W m2] = sum_k1 Z[k1][e] w_n1^(k1 m2)
//
// (LDE[e + B n2 m2] = sum_k1 w_n1^(k1 m2) s^k1 w_N^(k1 e) sum_k2 c[k1+n1 k2]
//  (s^n1)^k2 w_(B n2)^(k2 e) follows from j = k1 + n1 k2 and k = e + B n2 m2.)
//
// Pass 2's first half (the size-n2 inverse transforms and the scaling by n^-1 s^k1)
// runs as a kernel of its own, pass 2i, over tiles of up to 16 rows of Y, writing the
// scaled coefficients back over Y; pass 2 proper then starts from them.
//
// Each pass moves tiles of T adjacent columns/rows so global accesses are runs
// of T*8 bytes and does its sub-transforms in LDS with radix-8 register
// butterflies (decimation in frequency: natural order in, bit-reversed out;
// decimation in time: the reverse), applying the twiddles on the way out.
// Pass 1 writes Y (n words per column) to scratch. Pass 2 writes Z (N words per
// column, rows of W contiguous words): in natural layout over the output
// column itself, since pass 3 then reads and writes the same words and runs in
// place; in bit-reversed layout to scratch, a chunk of columns at a time. Pass 3
// writes natural order in runs of T words, bit-reversed order in whole rows.
#pragma once
#include "internal.h"

#include <type_traits>

namespace v3db {
namespace lde {

constexpr int LDE_THREADS = 512;
constexpr int TILE_ELEMS = 8192;         // T * M per tile
constexpr int MAX_PER_THREAD = TILE_ELEMS / LDE_THREADS;

__device__ __forceinline__ uint32_t brev(uint32_t x, int bits) {
  return bits ? (__brev(x) >> (32 - bits)) : 0u;
}

// Global-to-LDS copy of a tile of `total` <= TILE_ELEMS words (element e read by
// src(e), stored by dst(e, v)) by a block of LDE_THREADS threads: each thread first
// requests all its words, then stores them, so a wave keeps every load in flight at
// once rather than waiting for each before issuing the next. Every input tile the
// plans make fits (passes 1 and 3: T * n1 <= 8192; pass 2: T * n2 <= 8192).
template <class Src, class Dst>
__device__ __forceinline__ void stage_tile(int total, Src src, Dst dst) {
  uint64_t v[MAX_PER_THREAD];
#pragma unroll
  for (int m = 0; m < MAX_PER_THREAD; m++) {
    const int e = threadIdx.x + m * LDE_THREADS;
    if (e < total) v[m] = src(e);
  }
#pragma unroll
  for (int m = 0; m < MAX_PER_THREAD; m++) {
    const int e = threadIdx.x + m * LDE_THREADS;
    if (e < total) dst(e, v[m]);
  }
}

// Elements per thread whose table loads an output loop issues before using any.
constexpr int OUT_BATCH = 8;

// Position of word w of a tile row in LDS. Rows are 2^k words; the XOR of two
// right shifts is an invertible linear map on k-bit indices, chosen so that the
// access patterns of the passes (runs of consecutive words, the strided words
// of each radix-8 butterfly, and bit-reversed reads) spread a half-wave over
// distinct banks (at most 2 lanes per 8-byte bank slot). Linear over XOR:
// swz(a ^ b) = swz(a) ^ swz(b).
__device__ __forceinline__ int swz(int w) { return w ^ (w >> 3) ^ (w >> 8); }

// w^e for e < 2^26 from the two-level table (w = w_{2^26} or its inverse).
__device__ __forceinline__ uint64_t tw_pow(const uint64_t *__restrict__ lo, const uint64_t *__restrict__ hi,
                                           uint32_t e) {
  return gl::mul(hi[e >> TW_HALF], lo[e & ((1u << TW_HALF) - 1)]);
}

// The internal twiddles of a radix-8 butterfly are powers of w_8 = 7^((p-1)/8)
// = -2^24 (so w_8^2 = 2^48, w_8^3 = -2^72; inverse: 2^72, -2^48, 2^24). The
// product (u - w) * w_8^k is formed with the sign folded into the subtraction
// ((w - u) * 2^m for -2^m) and the power of two as shifts where that is cheaper
// than a multiplication (2^24, 2^48); 2^72 = 2^40 - 2^8 (mod p) takes the
// general product.
constexpr uint64_t TWO_72 = 1099511627520ull;

template <int K, bool INV>
__device__ __forceinline__ uint64_t sub_w8(uint64_t u, uint64_t w) {
  if (K == 0) return gl::sub(u, w);
  if (!INV) {
    if (K == 1) return gl::canon(gl::mul_pow2<24>(gl::sub(w, u)));
    if (K == 2) return gl::canon(gl::mul_pow2<48>(gl::sub(u, w)));
    return gl::mul(gl::sub(w, u), TWO_72);
  }
  if (K == 1) return gl::mul(gl::sub(u, w), TWO_72);
  if (K == 2) return gl::canon(gl::mul_pow2<48>(gl::sub(w, u)));
  return gl::canon(gl::mul_pow2<24>(gl::sub(u, w)));
}

// Size-R transform in registers (R = 2, 4, 8) by radix-2 decimation-in-frequency
// stages: natural order in, bit-reversed order out.
template <int R, bool INV>
__device__ __forceinline__ void reg_dif(uint64_t v[R]) {
#pragma unroll
  for (int h = R / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int b = 0; b < R; b += 2 * h)
#pragma unroll
      for (int i = 0; i < h; i++) {
        const uint64_t u = v[b + i], w = v[b + i + h];
        v[b + i] = gl::add(u, w);
        switch (i * (8 / (2 * h))) {
          case 0: v[b + i + h] = sub_w8<0, INV>(u, w); break;
          case 1: v[b + i + h] = sub_w8<1, INV>(u, w); break;
          case 2: v[b + i + h] = sub_w8<2, INV>(u, w); break;
          default: v[b + i + h] = sub_w8<3, INV>(u, w); break;
        }
      }
}

template <int R>
__device__ __forceinline__ int brev_r(int j) {
  return R == 8 ? ((j & 1) << 2 | (j & 2) | (j >> 2)) : R == 4 ? ((j & 1) << 1 | (j >> 1)) : j;
}

// Butterfly twiddle rows of the radix-8 passes: for sub-block size S = 2^logS
// (3 <= logS <= 12), row i < S/8 holds w_S^(i * bitrev3(j)), j = 0..7, so a
// butterfly reads its seven twiddles as one 64-byte row. Rows of all sizes are
// concatenated, smallest S first.
__host__ __device__ constexpr int bfly_row0(int logS) { return (1 << (logS - 3)) - 1; }
constexpr int BFLY_ROWS = (1 << (DFT_LOG_MAX - 2)) - 1;  // rows for logS = 3..12

// One radix-R pass of a decimation-in-frequency transform over T rows of
// 2^logM words in LDS (row stride rs): sub-blocks of 2^logS words, each
// butterfly takes the R words i + j*2^logS/R, transforms them, and multiplies
// output slot j (frequency bitrev(j)) by w_S^(i * bitrev(j)) (radix 8 with
// logS > 3 only: for the other passes i is always 0).
template <int R, bool INV, bool TW>
__device__ __forceinline__ void dif_pass(uint64_t *sh, int T, int logM, int rs, int logS,
                                         const uint64_t *__restrict__ bfly) {
  constexpr int LR = R == 8 ? 3 : R == 4 ? 2 : 1;
  const int logStride = logS - LR;
  const int per_row = 1 << (logM - LR);
  const int nb = T * per_row;
  const uint64_t *rows = bfly + 8 * bfly_row0(TW ? logS : 3);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int t = b >> (logM - LR);
    const int q = b & (per_row - 1);
    const int i = q & ((1 << logStride) - 1);
    // word (q >> logStride) << logS | i | j << logStride of row t; the three parts
    // have disjoint bits, so its swizzled position is the XOR of theirs
    uint64_t *row = sh + t * rs;
    const int wb = swz(((q >> logStride) << logS) + i);
    uint64_t v[R];
#pragma unroll
    for (int j = 0; j < R; j++) v[j] = row[wb ^ swz(j << logStride)];
    // the twiddle row is requested together with the inputs, so its latency overlaps
    // the butterfly instead of following it
    uint64_t tw[8];
    if (TW) {
      const ulonglong2 *trow = reinterpret_cast<const ulonglong2 *>(rows + 8 * i);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const ulonglong2 x = trow[k];
        tw[2 * k] = x.x, tw[2 * k + 1] = x.y;
      }
    }
    reg_dif<R, INV>(v);
    if (TW) {
#pragma unroll
      for (int j = 1; j < R; j++) v[j] = gl::mul(v[j], tw[j]);
    }
#pragma unroll
    for (int j = 0; j < R; j++) row[wb ^ swz(j << logStride)] = v[j];
  }
}

// Whole transforms over the rows: radix-8 passes, then one radix-4 or radix-2
// pass for the remaining bits. Each pass ends with a barrier.
// Passes from sub-block size 2^logS0 down (logS0 < logM when the earlier passes
// were done another way). With leave_tail, the last pass (radix 2, 4, or an untwiddled
// radix 8, on sub-blocks of R consecutive words) is not run but left to the caller's
// reader (tail_read), and its radix R is returned (0 when every pass ran).
template <bool INV>
__device__ __forceinline__ int dif_rows_from(uint64_t *sh, int T, int logM, int logS0, int rs,
                                             const uint64_t *__restrict__ bfly, bool leave_tail = false) {
  int logS = logS0;
  for (; logS >= 3; logS -= 3) {
    if (logS > 3) dif_pass<8, INV, true>(sh, T, logM, rs, logS, bfly);
    else if (leave_tail) return 8;
    else dif_pass<8, INV, false>(sh, T, logM, rs, logS, bfly);
    __syncthreads();
  }
  if (logS == 2) {
    if (leave_tail) return 4;
    dif_pass<4, INV, false>(sh, T, logM, rs, 2, bfly);
    __syncthreads();
  } else if (logS == 1) {
    if (leave_tail) return 2;
    dif_pass<2, INV, false>(sh, T, logM, rs, 1, bfly);
    __syncthreads();
  }
  return 0;
}

template <bool INV>
__device__ __forceinline__ int dif_rows(uint64_t *sh, int T, int logM, int rs, const uint64_t *__restrict__ bfly,
                                        bool leave_tail = false) {
  return dif_rows_from<INV>(sh, T, logM, logM, rs, bfly, leave_tail);
}

// The last pass of a row transform (left by dif_rows_from) done by its reader: the R
// words at positions p0 .. p0 + R - 1 of the row (p0 a multiple of R), transformed in
// registers. Slot j then holds position p0 + j, i.e. for p0 = brev(f0) (f0 < M/R,
// M = 2^logM) frequency f0 + brev_R(j) M/R. The pass has no twiddles in either direction.
template <int R, bool INV>
__device__ __forceinline__ void tail_read(const uint64_t *row, int p0, uint64_t v[R]) {
  const int w = swz(p0);  // swz(p0 + j) = swz(p0) ^ j for j < 8 when R divides p0
#pragma unroll
  for (int j = 0; j < R; j++) v[j] = row[w ^ j];
  reg_dif<R, INV>(v);
}


// Output loop of a pass whose row transforms left their last pass (radix R) to it. Group
// g of the tile is (row t, first frequency f0 < M/R) = coords(g); its outputs are the
// frequencies f0 + brev_R(j) M/R, each through val(t, f, v) (its twiddle or scale) and
// put(t, f, v). Each thread takes OUT_BATCH/R groups per trip and forms every value
// before the first store (groups past the end redo the last one and store nothing).
template <int R, bool INV, class Coords, class Val, class Put>
__device__ __forceinline__ void tail_out(const uint64_t *sh, int rs, int groups, int logM, Coords coords, Val val,
                                         Put put) {
  constexpr int G = OUT_BATCH / R, LR = R == 8 ? 3 : R == 4 ? 2 : 1;
  for (int g0 = threadIdx.x; g0 < groups; g0 += G * LDE_THREADS) {
    uint64_t r[G][R];
#pragma unroll
    for (int u = 0; u < G; u++) {
      int t, f0;
      coords(min(g0 + u * LDE_THREADS, groups - 1), t, f0);
      uint64_t v[R];
      tail_read<R, INV>(sh + t * rs, (int)brev(f0, logM), v);
#pragma unroll
      for (int j = 0; j < R; j++) r[u][j] = val(t, f0 + (brev_r<R>(j) << (logM - LR)), v[j]);
    }
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int g = g0 + u * LDE_THREADS;
      if (g < groups) {
        int t, f0;
        coords(g, t, f0);
#pragma unroll
        for (int j = 0; j < R; j++) put(t, f0 + (brev_r<R>(j) << (logM - LR)), r[u][j]);
      }
    }
  }
}

// tail_out for the radix the row transforms left (2, 4 or 8; false when none was left).
template <bool INV, class Coords, class Val, class Put>
__device__ __forceinline__ bool tail_out_any(int R, const uint64_t *sh, int rs, int rows, int logM, Coords coords,
                                             Val val, Put put) {
  switch (R) {
    case 2: tail_out<2, INV>(sh, rs, rows << (logM - 1), logM, coords, val, put); return true;
    case 4: tail_out<4, INV>(sh, rs, rows << (logM - 2), logM, coords, val, put); return true;
    case 8: tail_out<8, INV>(sh, rs, rows << (logM - 3), logM, coords, val, put); return true;
    default: return false;
  }
}

// One trace's LDE as the passes see it. Column c of the trace is trace + c*n,
// of Y (pass 1 output) y + c*n, of the output lde + c*N, and the Z rows of
// column c start at z + zc*zstride where zc is the column (natural layout:
// z = lde, zstride = N, Z is written over the output column and pass 3 runs in
// place) or its index within the current chunk (bit-reversed layout: z is scratch).
struct LdeTask {
  const uint64_t *trace;
  uint64_t *y;
  uint64_t *z;
  uint64_t *lde;
  const uint64_t *twist;  // [B][n2]: (shift^n1 w_{B n2}^r)^i
  const uint64_t *scale;  // [n1]: n^-1 shift^k1
  const uint64_t *ztw;    // [n1][W]: w_N^(k1 e), or null (then from the two-level table)
  uint64_t zstride;
  int L, b, L1, L2;       // log n, log blowup, log n1, log n2 (n = n1 n2)
  int logT1, logT2, logT3;
  int logT2i;             // log2 rows per tile of the separate inverse part of pass 2
  int bitrev;
};

__device__ __forceinline__ int lde_tiles1(const LdeTask &t) { return (1 << t.L2) >> t.logT1; }
__device__ __forceinline__ int lde_tiles2(const LdeTask &t) { return (1 << t.L1) >> t.logT2; }
__device__ __forceinline__ int lde_tiles2i(const LdeTask &t) { return (1 << t.L1) >> t.logT2i; }
__device__ __forceinline__ int lde_tiles3(const LdeTask &t) { return (1 << (t.L2 + t.b)) >> t.logT3; }

// The first radix-8 pass of a row transform (sub-blocks of the whole row, 2^logM words)
// with its inputs read straight from global memory: word w of row t is src(t, w). The
// butterflies are numbered with t fastest, so with T >= 16 rows the lanes of a
// half-wave read 16 consecutive words (the rows are adjacent columns of a matrix).
template <bool INV, class Src>
__device__ __forceinline__ void first_pass_global(uint64_t *sh, int T, int logT, int logM, int rs,
                                                  const uint64_t *__restrict__ bfly, Src src) {
  const int logStride = logM - 3;
  const int nb = T << logStride;
  const uint64_t *rows = bfly + 8 * bfly_row0(logM);
  for (int b = threadIdx.x; b < nb; b += LDE_THREADS) {
    const int t = b & (T - 1), i = b >> logT;
    uint64_t v[8], w[8];
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = src(t, i + (j << logStride));
    const ulonglong2 *trow = reinterpret_cast<const ulonglong2 *>(rows + 8 * i);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const ulonglong2 x = trow[k];
      w[2 * k] = x.x, w[2 * k + 1] = x.y;
    }
    reg_dif<8, INV>(v);
    uint64_t *row = sh + t * rs;
    const int wb = swz(i);
    row[wb] = v[0];
#pragma unroll
    for (int j = 1; j < 8; j++) row[wb ^ swz(j << logStride)] = gl::mul(v[j], w[j]);
  }
}

// Pass 1, tile = T consecutive j2 of column col.
__device__ __forceinline__ void lde_pass1_tile(const LdeTask &s, const Twiddles &tw, uint64_t *sh, int col, int tile) {
  const int n1 = 1 << s.L1, n2 = 1 << s.L2, T = 1 << s.logT1, rs = n1 + 1;
  const size_t n = size_t(1) << s.L;
  const uint64_t *a = s.trace + size_t(col) * n;
  uint64_t *y = s.y + size_t(col) * n;
  const int j2_0 = tile << s.logT1;
  const int total = T * n1;
  int tail;
  if (s.L1 >= 4) {
    // the first radix-8 pass reads the trace straight from global memory
    first_pass_global<true>(sh, T, s.logT1, s.L1, rs, tw.bfly_inv,
                            [&](int t, int w) { return a[size_t(w) * n2 + j2_0 + t]; });
    __syncthreads();
    tail = dif_rows_from<true>(sh, T, s.L1, s.L1 - 3, rs, tw.bfly_inv, true);
  } else {
    stage_tile(
        total, [&](int e) { return a[size_t(e >> s.logT1) * n2 + j2_0 + (e & (T - 1))]; },
        [&](int e, uint64_t v) { sh[(e & (T - 1)) * rs + swz(e >> s.logT1)] = v; });
    __syncthreads();
    tail = dif_rows<true>(sh, T, s.L1, rs, tw.bfly_inv, true);
  }
  const int shl = TW_LOG - s.L;
  constexpr uint32_t lo_mask = (1u << TW_HALF) - 1;
  // w_n^(-j2 k1) = hi[x >> TW_HALF] * lo[x & lo_mask] with x = (j2 k1 mod n) << shl.
  // Every lane requests the table words of all its elements before the first product
  // (lanes past the end read the last element instead and store nothing), and every
  // product is formed unconditionally, so no load is left outstanding on any path.
  auto twiddled = [&](int t, int k1, uint64_t v) {
    const uint32_t ex = (uint32_t)((uint64_t(j2_0 + t) * k1) & (n - 1));
    const uint32_t x = ex << shl;
    const uint64_t w = gl::mul(tw.inv_hi[x >> TW_HALF], tw.inv_lo[x & lo_mask]);
    return ex ? gl::mul(v, w) : v;
  };
  // the transforms' last pass done here: group g = (row t, first frequency k1 < n1/R)
  if (tail_out_any<true>(
          tail, sh, rs, T, s.L1,
          [&](int g, int &t, int &k1) { t = g & (T - 1), k1 = g >> s.logT1; }, twiddled,
          [&](int t, int k1, uint64_t v) { y[size_t(k1) * n2 + j2_0 + t] = v; }))
    return;
  for (int e0 = threadIdx.x; e0 < total; e0 += OUT_BATCH * LDE_THREADS) {
    uint64_t r[OUT_BATCH];
#pragma unroll
    for (int u = 0; u < OUT_BATCH; u++) {
      const int e = min(e0 + u * LDE_THREADS, total - 1);
      const int t = e & (T - 1), k1 = e >> s.logT1;
      r[u] = twiddled(t, k1, sh[t * rs + swz(brev(k1, s.L1))]);
    }
#pragma unroll
    for (int u = 0; u < OUT_BATCH; u++) {
      const int e = e0 + u * LDE_THREADS;
      if (e < total) y[size_t(e >> s.logT1) * n2 + j2_0 + (e & (T - 1))] = r[u];
    }
  }
}

// Pass 2's expansion of a residue sequence to the B = 2^b cosets: input i (element e of
// the tile, row t) times twist[r][i] lands in coset r = bitrev_b(j) at slot j of the
// first zero-padded radix-B butterfly. The B table words of an input are requested
// together; inputs past the end read the last one and store nothing.
template <int B>
__device__ __forceinline__ void twist_stage(const LdeTask &s, uint64_t *sh, int rs, int n_in, int total_in,
                                            const uint64_t c[MAX_PER_THREAD]) {
  const int n2 = 1 << s.L2;
#pragma unroll
  for (int m = 0; m < MAX_PER_THREAD; m++) {
    if (m < n_in) {
      const int e0 = threadIdx.x + m * LDE_THREADS;
      const int e = min(e0, total_in - 1);
      const int t = e >> s.L2, i = e & (n2 - 1);
      uint64_t tv[B];
#pragma unroll
      for (int j = 0; j < B; j++) tv[j] = s.twist[(brev(j, s.b) << s.L2) + i];
      uint64_t r[B];
#pragma unroll
      for (int j = 0; j < B; j++) r[j] = gl::mul(c[m], tv[j]);
      if (e0 < total_in) {
        const int wi = swz(i);
#pragma unroll
        for (int j = 0; j < B; j++) sh[t * rs + (wi ^ swz(j << s.L2))] = r[j];
      }
    }
  }
}

// Pass 2's inverse part on its own, tile = T2i consecutive rows k1 of Y (column col):
// row k1 is transformed back, giving n*c[k1 + n1*k2] in bit-reversed positions, and
// written over itself in natural order k2, times n^-1 s^k1. A tile holds up to 8192
// words, so every thread has butterflies (inside pass 2 a tile has only the T2 rows
// its W-point outputs leave room for: T2*n2 = 8192/B inputs).
__device__ __forceinline__ void lde_pass2i_tile(const LdeTask &s, const Twiddles &tw, uint64_t *sh, int col,
                                                int tile) {
  const int n2 = 1 << s.L2, T = 1 << s.logT2i, rs = n2 + 1;
  const size_t n = size_t(1) << s.L;
  uint64_t *y = s.y + size_t(col) * n;
  const int k1_0 = tile << s.logT2i;
  const int total = T << s.L2;
  stage_tile(
      total, [&](int e) { return y[size_t(k1_0 + (e >> s.L2)) * n2 + (e & (n2 - 1))]; },
      [&](int e, uint64_t v) { sh[(e >> s.L2) * rs + swz(e & (n2 - 1))] = v; });
  __syncthreads();
  const int tail = dif_rows<true>(sh, T, s.L2, rs, tw.bfly_inv, true);
  // the transforms' last pass done here: group g = (row t, first frequency i < n2/R)
  {
    const int lg = s.L2 - (tail == 8 ? 3 : tail == 4 ? 2 : 1);
    if (tail_out_any<true>(
            tail, sh, rs, T, s.L2, [&](int g, int &t, int &i) { t = g >> lg, i = g & ((1 << lg) - 1); },
            [&](int t, int i, uint64_t v) { return gl::mul(v, s.scale[k1_0 + t]); },
            [&](int t, int i, uint64_t v) { y[size_t(k1_0 + t) * n2 + i] = v; }))
      return;
  }
  for (int e0 = threadIdx.x; e0 < total; e0 += OUT_BATCH * LDE_THREADS) {
    uint64_t r[OUT_BATCH];
#pragma unroll
    for (int u = 0; u < OUT_BATCH; u++) {
      const int e = min(e0 + u * LDE_THREADS, total - 1);
      const int t = e >> s.L2, i = e & (n2 - 1);
      r[u] = gl::mul(sh[t * rs + swz(brev(i, s.L2))], s.scale[k1_0 + t]);
    }
#pragma unroll
    for (int u = 0; u < OUT_BATCH; u++) {
      const int e = e0 + u * LDE_THREADS;
      if (e < total) y[size_t(k1_0 + (e >> s.L2)) * n2 + (e & (n2 - 1))] = r[u];
    }
  }
}

// Pass 2, tile = T consecutive residues k1 (rows of Y) of column col; W = B*n2.
// Row k1 of Y holds n^-1 s^k1 c' in natural order (written by lde_pass2i_tile); it is
// expanded to the W-point zero-padded transform: its first radix-B
// decimation-in-frequency pass has a single nonzero input per butterfly, so output
// slot j of butterfly i is the input times the twist (s^n1 w_W^r)^i, r = bitrev(j).
// The remaining passes run on the B cosets together; row k1 of Z gets
// Z[k1][e] = w_N^(k1 e) * (result at e).
__device__ __forceinline__ void lde_pass2_tile(const LdeTask &s, const Twiddles &tw, uint64_t *sh, int col, int zcol,
                                               int tile) {
  const int n2 = 1 << s.L2, T = 1 << s.logT2;
  const int LW = s.L2 + s.b, W = 1 << LW, rs = W + 1;
  const size_t n = size_t(1) << s.L, N = size_t(1) << (s.L + s.b);
  const int logN = s.L + s.b;
  const uint64_t *y = s.y + size_t(col) * n;
  uint64_t *zc = s.z + size_t(zcol) * s.zstride;
  const int k1_0 = tile << s.logT2;
  const int total_in = T << s.L2;
  // this thread's inputs m < n_in (the same count for the whole block): n^-1 s^k1 c'
  const int n_in = (total_in + LDE_THREADS - 1) / LDE_THREADS;
  uint64_t c[MAX_PER_THREAD];
#pragma unroll
  for (int m = 0; m < MAX_PER_THREAD; m++) {
    if (m < n_in) {
      const int e = min(threadIdx.x + m * LDE_THREADS, total_in - 1);
      c[m] = y[size_t(k1_0 + (e >> s.L2)) * n2 + (e & (n2 - 1))];
    }
  }
  switch (s.b) {
    case 0: twist_stage<1>(s, sh, rs, n_in, total_in, c); break;
    case 1: twist_stage<2>(s, sh, rs, n_in, total_in, c); break;
    case 2: twist_stage<4>(s, sh, rs, n_in, total_in, c); break;
    case 3: twist_stage<8>(s, sh, rs, n_in, total_in, c); break;
    default: twist_stage<16>(s, sh, rs, n_in, total_in, c); break;
  }
  __syncthreads();
  const int tail = dif_rows_from<false>(sh, T, LW, s.L2, rs, tw.bfly_fwd, true);
  const int total_out = T << LW;
  const int shl = TW_LOG - logN;
  constexpr uint32_t lo_mask = (1u << TW_HALF) - 1;
  // w_N^(k1 e) for each element (one ztw word, or two words of the two-level table),
  // requested for a batch of elements before the first product; lanes past the end read
  // the last element and store nothing, and every product is formed unconditionally
  auto out_loops = [&](auto use_ztw) {
    constexpr bool Z = decltype(use_ztw)::value;
    auto twiddled = [&](int t, int f, uint64_t v) {
      if constexpr (Z) {
        return gl::mul(v, s.ztw[(size_t(k1_0 + t) << LW) + f]);
      } else {
        const uint32_t ex = (uint32_t)((uint64_t(k1_0 + t) * f) & (N - 1));
        const uint32_t x = ex << shl;
        const uint64_t w = gl::mul(tw.fwd_hi[x >> TW_HALF], tw.fwd_lo[x & lo_mask]);
        return ex ? gl::mul(v, w) : v;
      }
    };
    // the transforms' last pass done here: group g = (row t, first frequency f < W/R)
    const int lg = LW - (tail == 8 ? 3 : tail == 4 ? 2 : 1);
    if (tail_out_any<false>(
            tail, sh, rs, T, LW, [&](int g, int &t, int &f) { t = g >> lg, f = g & ((1 << lg) - 1); }, twiddled,
            [&](int t, int f, uint64_t v) { zc[(size_t(k1_0 + t) << LW) + f] = v; }))
      return;
    for (int e0 = threadIdx.x; e0 < total_out; e0 += OUT_BATCH * LDE_THREADS) {
      uint64_t r[OUT_BATCH];
#pragma unroll
      for (int u = 0; u < OUT_BATCH; u++) {
        const int e = min(e0 + u * LDE_THREADS, total_out - 1);
        const int t = e >> LW, f = e & (W - 1);
        r[u] = twiddled(t, f, sh[t * rs + swz(brev(f, LW))]);
      }
#pragma unroll
      for (int u = 0; u < OUT_BATCH; u++) {
        const int e = e0 + u * LDE_THREADS;
        if (e < total_out) zc[(size_t(k1_0 + (e >> LW)) << LW) + (e & (W - 1))] = r[u];
      }
    }
  };
  if (s.ztw) out_loops(std::true_type{});
  else out_loops(std::false_type{});
}

// Pass 3, tile = T consecutive columns e of Z (of column col). In natural
// layout the words it reads, Z[k1][e] at k1*W + e, are exactly the words it
// writes, LDE[e + W*m2], so it can run in place.
// The last pass of a row transform (radix R on sub-blocks of R consecutive words, no
// twiddles) with its outputs written straight to global memory: position w of row t
// (frequency bitrev(w)) goes to dst(t, w, value). Butterflies numbered with t fastest.
template <int R, bool INV, class Dst>
__device__ __forceinline__ void last_pass_global(const uint64_t *sh, int T, int logT, int logM, int rs, Dst dst) {
  constexpr int LR = R == 8 ? 3 : R == 4 ? 2 : 1;
  const int nb = T << (logM - LR);
  for (int b = threadIdx.x; b < nb; b += LDE_THREADS) {
    const int t = b & (T - 1), q = b >> logT;
    const uint64_t *row = sh + t * rs;
    const int wb = swz(q << LR);
    uint64_t v[R];
#pragma unroll
    for (int j = 0; j < R; j++) v[j] = row[wb ^ swz(j)];
    reg_dif<R, INV>(v);
#pragma unroll
    for (int j = 0; j < R; j++) dst(t, (q << LR) + j, v[j]);
  }
}

__device__ __forceinline__ void lde_pass3_tile(const LdeTask &s, const Twiddles &tw, uint64_t *sh, int col, int zcol,
                                               int tile) {
  const int n1 = 1 << s.L1, T = 1 << s.logT3, rs = n1 + 1;
  const int LW = s.L2 + s.b, W = 1 << LW;
  const size_t N = size_t(1) << (s.L + s.b);
  const uint64_t *zc = s.z + size_t(zcol) * s.zstride;
  uint64_t *out = s.lde + size_t(col) * N;
  const int e0 = tile << s.logT3;
  const int total = T * n1;
  if (!s.bitrev && s.L1 >= 4) {
    // natural layout, at least two passes: the first reads Z straight from global
    // memory and the last writes the output straight to it, saving a round trip
    // through LDS and a barrier at each end. Z is the output column itself (the tile's
    // words are read before the first barrier and written after the last one).
    first_pass_global<false>(sh, T, s.logT3, s.L1, rs, tw.bfly_fwd,
                             [&](int t, int w) { return zc[(size_t(w) << LW) + e0 + t]; });
    __syncthreads();
    const int last = s.L1 % 3 == 0 ? 3 : s.L1 % 3;  // log2 of the last pass's radix
    for (int logS = s.L1 - 3; logS > last; logS -= 3) {
      dif_pass<8, false, true>(sh, T, s.L1, rs, logS, tw.bfly_fwd);
      __syncthreads();
    }
    auto dst = [&](int t, int w, uint64_t v) { out[size_t(e0 + t) + size_t(W) * brev(w, s.L1)] = v; };
    if (last == 3) last_pass_global<8, false>(sh, T, s.logT3, s.L1, rs, dst);
    else if (last == 2) last_pass_global<4, false>(sh, T, s.logT3, s.L1, rs, dst);
    else last_pass_global<2, false>(sh, T, s.logT3, s.L1, rs, dst);
    return;
  }
  int tail;
  if (s.bitrev && s.L1 >= 4) {
    // the first radix-8 pass reads Z straight from global memory, as in natural layout
    first_pass_global<false>(sh, T, s.logT3, s.L1, rs, tw.bfly_fwd,
                             [&](int t, int w) { return zc[(size_t(w) << LW) + e0 + t]; });
    __syncthreads();
    tail = dif_rows_from<false>(sh, T, s.L1, s.L1 - 3, rs, tw.bfly_fwd, true);
  } else {
    stage_tile(
        total, [&](int e) { return zc[(size_t(e >> s.logT3) << LW) + e0 + (e & (T - 1))]; },
        [&](int e, uint64_t v) { sh[(e & (T - 1)) * rs + swz(e >> s.logT3)] = v; });
    __syncthreads();
    // bit-reversed layout: the last radix-2 pass is left to the writer, which stores each
    // butterfly's two outputs (positions 2q and 2q + 1, adjacent in the output row) together
    tail = dif_rows<false>(sh, T, s.L1, rs, tw.bfly_fwd, s.bitrev != 0);
  }
  if (!s.bitrev) {
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e & (T - 1), m2 = e >> s.logT3;
      out[size_t(e0 + t) + size_t(W) * m2] = sh[t * rs + swz(brev(m2, s.L1))];
    }
  } else if (tail) {
    // the last pass done here: each group's R outputs are adjacent in the output row
    auto put = [&](auto RT) {
      constexpr int R = decltype(RT)::value, LR = R == 8 ? 3 : R == 4 ? 2 : 1;
      const int lg = s.L1 - LR;
      for (int g = threadIdx.x; g < (total >> LR); g += blockDim.x) {
        const int t = g >> lg, q = g & ((1 << lg) - 1);
        uint64_t v[R];
        tail_read<R, false>(sh + t * rs, q * R, v);
        ulonglong2 *o = reinterpret_cast<ulonglong2 *>(out + size_t(brev(e0 + t, LW)) * n1 + q * R);
#pragma unroll
        for (int j = 0; j < R / 2; j++) o[j] = make_ulonglong2(v[2 * j], v[2 * j + 1]);
      }
    };
    if (tail == 2) put(std::integral_constant<int, 2>{});
    else if (tail == 4) put(std::integral_constant<int, 4>{});
    else put(std::integral_constant<int, 8>{});
  } else {
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e >> s.L1, p = e & (n1 - 1);
      out[size_t(brev(e0 + t, LW)) * n1 + p] = sh[t * rs + swz(p)];
    }
  }
}

}  // namespace lde

// The task of one trace with this plan (ntt.hip). z is the Z scratch for
// bit-reversed layout (ignored in natural layout, where Z is built in lde).
lde::LdeTask lde_task(const LdePlan &plan, const uint64_t *trace, uint64_t *y, uint64_t *z, uint64_t *lde,
                      v3db_layout layout);

namespace lde {

// LDS words a pass needs for its tile.
__host__ __device__ inline size_t lde_lds_words(int pass, int L1, int L2, int b, int logT) {
  if (pass == 2) return (size_t(1) << logT) * ((size_t(1) << (L2 + b)) + 1);
  if (pass == 4) return (size_t(1) << logT) * ((size_t(1) << L2) + 1);  // pass 2's inverse part
  return (size_t(1) << logT) * ((size_t(1) << L1) + 1);
}

}  // namespace lde
}  // namespace v3db
