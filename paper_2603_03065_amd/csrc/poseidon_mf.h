// Width-12 Poseidon with the matrix product on the int8 matrix cores, for
// kernels that hash many independent inputs (leaf rows, tree nodes, records).
//
// A wave holds 64 permutations. Lane l (h = l / 32, c = l % 32) keeps words
// 6h .. 6h+5 of permutations c and c + 32, so each lane still holds 12 state
// words. S-boxes run on those words as before; the partial rounds' single S-box
// (word 0, held by the lanes with h = 0 for both permutations) is moved so that
// every lane computes one: permutation c + 32's word goes to lane c + 32 and
// back with v_permlane32_swap.
//
// The linear layer y_i = sum_j a[(j-i) mod 12] s_j is exact over the integers
// before the reduction, and it is computed limb by limb: with b_jk byte k of s_j,
//   y_i = sum_k 2^(8k) sum_j C_ij b_jk.
// v_mfma_i32_32x32x32_i8 (signed bytes, int32 sums) works on two limbs k = 2p, 2p + 1
// of the 32 permutations of one half of the wave:
//   * B column = one permutation; a lane supplies the K slots of its half
//     (16h .. 16h+15), slot 4q + 2w + l holding b'_jk, k = 2p + l, of its word
//     jj = 2q + w, with b' = b - 128 (the byte XOR 0x80 read as signed); slots 12..15
//     are unused (zero in A, so whatever their register holds adds nothing);
//   * both factors shifted by 128 fit a signed byte (C - 128 for an entry C <= 255):
//     (C - 128)(b - 128) = C b - 128 b' - 128 C, so with the A row of output i
//     and limb l holding C_ij - 128 in the slots of limb l (zero in those of the other),
//       D_ik = sum_j C_ij b_jk - 128 S_k - 128 R,  S_k = sum_j b'_jk, R = sum_j C_ij
//     (R the same for every row of a circulant); two more rows of A, -128 in all the
//     slots of limb 0 resp. 1, give -128 S_k in the same product;
//   * D row 8(e/4) + 4h + e%4 of column c lands in lane 32h + c, element e: the
//     host puts output i = 6h + ii, limb l in the row of element e = 6l + ii, and
//     -128 S of limbs 0 and 1 in the rows of elements 12 and 13 of both halves, so each
//     lane receives exactly the outputs for the words it holds, both limbs, and S.
// One v_perm packs two limbs of two words, and a round takes 24 of them for eight limbs
// of twelve words, and 8 matrix products (one per limb pair and half of the wave).
// Each output accumulates lo = K + rc.lo + sum_{k<4} 2^(8k) (D_ik + 128 S_k) and hi
// likewise over k >= 4, K = 128 R (2^24 + 2^16 + 2^8 + 1): a limb pair's two sums are
// first joined in 32 bits (|D| < 2^18), then added with one 64-bit multiply-add; the
// 128 S terms, the same for all outputs of a permutation, are summed the same way once
// (with negated weights) and added to each output's lo and hi. Both are then exact,
// non-negative and below
// 2^46, and fold(lo, hi) gives the relaxed output exactly as in the VALU form. The
// start values K + next round's constant come from a small table.
#pragma once
#include "poseidon_dev.h"

namespace v3db {
namespace pos {

typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef int mf_v16i __attribute__((ext_vector_type(16)));

struct MfLane {
  mf_v4i A;  // this lane's 16 bytes of the matrix
  int mult[4];  // 1, -1, 2^16, -2^16 read from the table: each term stays one v_mad_i64_i32
  int h, c;
};

__device__ __forceinline__ MfLane mf_lane(const uint64_t *__restrict__ tab) {
  MfLane L;
  const int l = threadIdx.x & 63;
  L.h = l >> 5;
  L.c = l & 31;
  const uint32_t *am = reinterpret_cast<const uint32_t *>(tab + MF_AMAT) + l * 4;
#pragma unroll
  for (int q = 0; q < 4; q++) L.A[q] = (int)am[q];
  const int *m = reinterpret_cast<const int *>(tab + MF_MULT);
#pragma unroll
  for (int q = 0; q < 4; q++) L.mult[q] = m[q];
  return L;
}

// v_permlane32_swap on 64-bit values: a of lanes 32..63 and b of lanes 0..31 trade
// places (lane l + 32's a with lane l's b); a of lanes 0..31 and b of lanes 32..63 stay.
__device__ __forceinline__ void mf_swap(uint64_t &a, uint64_t &b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
  a = ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0];
  b = ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1];
}

// The permutation of the wave's 64 states (layout above). rc: the round-constant
// rows (row 0 added first); tab: the table above. All 64 lanes must be active.
__device__ __forceinline__ void permute_mf(uint64_t S[2][6], const MfLane &L, const uint64_t *__restrict__ rc,
                                           const uint64_t *__restrict__ tab) {
  const int h = L.h;
#pragma unroll
  for (int u = 0; u < 2; u++)
#pragma unroll
    for (int jj = 0; jj < 6; jj++) S[u][jj] = gl::add_r(S[u][jj], rc[6 * h + jj]);
#pragma unroll 1
  for (int r0 = 0; r0 < ROUNDS; r0++) {
    // the round number as a scalar: the round test and the table row stay off the VALU
    const int r = __builtin_amdgcn_readfirstlane(r0);
    const bool full = r < FULL_HALF || r >= ROUNDS - FULL_HALF;
    if (full) {
#pragma unroll
      for (int u = 0; u < 2; u++)
#pragma unroll
        for (int jj = 0; jj < 6; jj++) S[u][jj] = sbox(S[u][jj]);
    } else {
      // word 0 of permutation c + 32 (lane c's S[1][0]) trades places with the word lane
      // c + 32 keeps in S[0][0] (word 6 of permutation c), so every lane's S[0][0] is a
      // word 0; after the S-box the same exchange returns each value to where it was
      mf_swap(S[0][0], S[1][0]);
      S[0][0] = sbox(S[0][0]);
      mf_swap(S[0][0], S[1][0]);
    }
    const uint64_t *kr = tab + MF_RCK + size_t(r + 1) * WIDTH * 2 + 12u * (uint32_t)h;
    uint32_t dw[2][6][2];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
      for (int jj = 0; jj < 6; jj++) {
        dw[u][jj][0] = (uint32_t)S[u][jj] ^ 0x80808080u;
        dw[u][jj][1] = (uint32_t)(S[u][jj] >> 32) ^ 0x80808080u;
      }
    int64_t lo[2][6], hi[2][6], sum[2];
#pragma unroll
    for (int ii = 0; ii < 6; ii++) {
      lo[0][ii] = lo[1][ii] = (int64_t)kr[2 * ii];
      hi[0][ii] = hi[1][ii] = (int64_t)kr[2 * ii + 1];
    }
#pragma unroll
    for (int p = 0; p < 4; p++) {
      const uint32_t kk = (2 * p) & 3, half = p >> 1;
      // bytes kk and kk + 1 (limbs 2p, 2p + 1) of two words: v_perm selectors 0-3 pick
      // from the second source, 4-7 from the first
      const uint32_t sel = kk | ((kk + 1) << 8) | ((kk + 4) << 16) | ((kk + 5) << 24);
      mf_v4i B[2];
#pragma unroll
      for (int u = 0; u < 2; u++) {
        B[u][0] = (int)__builtin_amdgcn_perm(dw[u][1][half], dw[u][0][half], sel);
        B[u][1] = (int)__builtin_amdgcn_perm(dw[u][3][half], dw[u][2][half], sel);
        B[u][2] = (int)__builtin_amdgcn_perm(dw[u][5][half], dw[u][4][half], sel);
        // K slots 12..15 meet zero entries of A: the register is left as it is (an empty
        // asm statement defines it), which saves a move per operand
        int pad;
        asm volatile("" : "=v"(pad));
        B[u][3] = pad;
      }
      mf_v16i D[2];
#pragma unroll
      for (int u = 0; u < 2; u++) D[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(L.A, B[u], (mf_v16i){}, 0, 0, 0);
      // both products issued before either is read: the matrix core runs the second
      // while the first is recombined
      __builtin_amdgcn_sched_barrier(0);
      // the two limbs first added in 32 bits (|D| < 2^18, so D_2p + 2^8 D_2p+1 fits),
      // then one 64-bit multiply-add per word and limb pair
#pragma unroll
      for (int u = 0; u < 2; u++) {
#pragma unroll
        for (int ii = 0; ii < 6; ii++) {
          const int32_t pr = (int32_t)(((uint32_t)D[u][6 + ii] << 8) + (uint32_t)D[u][ii]);
          const int64_t t = (int64_t)pr * (int64_t)L.mult[(2 * p) & 3];
          if (p < 2) lo[u][ii] += t;
          else hi[u][ii] += t;
        }
        // -128 S of the pair (|128 S| < 2^18), weighted by minus the pair's weight
        const int32_t ps = (int32_t)(((uint32_t)D[u][13] << 8) + (uint32_t)D[u][12]);
        const int64_t t = (int64_t)ps * (int64_t)L.mult[((2 * p) & 3) + 1];
        sum[u] = (p & 1) ? sum[u] + t : t;
      }
      // 128 times the byte sums of limbs 0..3 (after p = 1) or 4..7 (after p = 3),
      // added to every output's lo or hi
      if (p & 1) {
#pragma unroll
        for (int u = 0; u < 2; u++)
#pragma unroll
          for (int ii = 0; ii < 6; ii++) {
            if (p < 2) lo[u][ii] += sum[u];
            else hi[u][ii] += sum[u];
          }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
      for (int ii = 0; ii < 6; ii++) S[u][ii] = fold((uint64_t)lo[u][ii], (uint64_t)hi[u][ii]);
  }
}

// Rate-8 overwrite sponge over len elements for the wave's 64 inputs: elem(u, x)
// gives element x of input c + 32u (called only for x < len, and only by lanes
// whose input exists when `live(u)`; others absorb zeros). Leaves the state in S.
template <typename Elem, typename Live>
__device__ __forceinline__ void sponge_mf(uint64_t S[2][6], uint64_t len, Elem elem, Live live, const MfLane &L,
                                          const uint64_t *__restrict__ rc, const uint64_t *__restrict__ tab) {
#pragma unroll
  for (int u = 0; u < 2; u++)
#pragma unroll
    for (int jj = 0; jj < 6; jj++) S[u][jj] = 0;
  for (uint64_t q = 0; q < len; q += RATE) {
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
      for (int jj = 0; jj < 6; jj++) {
        const int j = 6 * L.h + jj;
        if (j < RATE && q + j < len) S[u][jj] = live(u) ? elem(u, q + j) : 0;
      }
    permute_mf(S, L, rc, tab);
  }
}

// Write the digests (words 0..3, held by the lanes with h = 0) of the wave's
// inputs base + c + 32u that are below count, canonical, to out[input * 4 + w]
// (and to out2 as well unless it is null).
__device__ __forceinline__ void store_digests_mf(const uint64_t S[2][6], const MfLane &L, uint64_t base,
                                                 uint64_t count, uint64_t *__restrict__ out,
                                                 uint64_t *__restrict__ out2 = nullptr) {
  if (L.h != 0) return;
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const uint64_t k = base + L.c + 32 * u;
    if (k < count) {
#pragma unroll
      for (int w = 0; w < DIGEST; w++) {
        const uint64_t v = gl::canon(S[u][w]);
        out[k * DIGEST + w] = v;
        if (out2) out2[k * DIGEST + w] = v;
      }
    }
  }
}

// Leaf digests of rows base .. base+63 of a column-major matrix with n_rows rows: the
// rate-8 overwrite sponge of sponge_mf with the loads written out. A lane with h = 0
// absorbs columns q + 0..5 of each chunk, a lane with h = 1 columns q + 6, q + 7; word jj
// of a chunk is at (column) * n_rows + row, a uniform offset from the lane's base pointer,
// and whether the column exists is a uniform test (the branch on h is the only divergence).
__device__ __forceinline__ void leaf_digests_mf(const uint64_t *__restrict__ mat, uint32_t n_cols, uint64_t n_rows,
                                                uint64_t base, uint64_t *__restrict__ out, const MfLane &L,
                                                const uint64_t *__restrict__ rc, const uint64_t *__restrict__ tab,
                                                uint64_t *__restrict__ out2 = nullptr) {
  uint64_t S[2][6];
#pragma unroll
  for (int u = 0; u < 2; u++)
#pragma unroll
    for (int jj = 0; jj < 6; jj++) S[u][jj] = 0;
  // the lane's row and column pointer are formed anew from the lane index in every chunk
  // and for the store (the index hidden from the compiler, which would otherwise keep the
  // 64-bit values live across the permutations and, at 128 VGPRs, spill them)
  for (uint32_t q = 0; q < n_cols; q += RATE) {
    uint32_t lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const uint64_t row = base + (lane & 31);
    const bool live0 = row < n_rows, live1 = row + 32 < n_rows;
    const uint64_t *pq = mat + uint64_t(6 * (lane >> 5) + q) * n_rows + row;  // column q + 6h
    if (L.h == 0) {
#pragma unroll
      for (int jj = 0; jj < 6; jj++)
        if (q + jj < n_cols) {
          const uint64_t *w = pq + uint64_t(jj) * n_rows;
          S[0][jj] = live0 ? w[0] : 0;
          S[1][jj] = live1 ? w[32] : 0;
        }
    } else {
#pragma unroll
      for (int jj = 0; jj < 2; jj++)
        if (q + 6 + jj < n_cols) {
          const uint64_t *w = pq + uint64_t(jj) * n_rows;
          S[0][jj] = live0 ? w[0] : 0;
          S[1][jj] = live1 ? w[32] : 0;
        }
    }
    permute_mf(S, L, rc, tab);
  }
  store_digests_mf(S, L, base, n_rows, out, out2);
}

// Nodes base .. base+63 of a level: node k = Compress(below[2k], below[2k+1]).
__device__ __forceinline__ void merkle_nodes_mf(const uint64_t *__restrict__ below, uint64_t count, uint64_t base,
                                                uint64_t *__restrict__ out, const MfLane &L,
                                                const uint64_t *__restrict__ rc, const uint64_t *__restrict__ tab,
                                                uint64_t *__restrict__ out2 = nullptr) {
  uint64_t S[2][6];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const uint64_t k = base + L.c + 32 * u;
#pragma unroll
    for (int jj = 0; jj < 6; jj++) {
      const int j = 6 * L.h + jj;
      S[u][jj] = (j < 2 * DIGEST && k < count) ? below[k * 2 * DIGEST + j] : 0;
    }
  }
  permute_mf(S, L, rc, tab);
  store_digests_mf(S, L, base, count, out, out2);
}

}  // namespace pos
}  // namespace v3db
