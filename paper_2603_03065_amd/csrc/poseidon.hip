// Width-12 Poseidon on gfx950 VALU: one permutation per lane, state in VGPRs.
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
#include "internal.h"

namespace v3db {

namespace {

constexpr int THREADS = 256;

struct Circ {
  uint32_t a[WIDTH];
};

__device__ __forceinline__ uint64_t sbox(uint64_t x) {
  const uint64_t x2 = gl::mul_r(x, x);
  const uint64_t x3 = gl::mul_r(x2, x);
  const uint64_t x4 = gl::mul_r(x2, x2);
  return gl::mul_r(x3, x4);
}

// lo + hi * 2^32 for lo, hi < 2^46, to a relaxed value: with hi = hh*2^32 + hl,
// the sum is lo + hh*2^64 + hl*2^32 = (hh*(2^32-1) + lo) + hl*2^32 (mod p); the
// first part is one multiply-add below 2^47, the second adds hl to its high word
// and a carry out of bit 64 is worth 2^32 - 1 again.
__device__ __forceinline__ uint64_t fold(uint64_t lo, uint64_t hi) {
  const uint64_t t = (uint64_t)(uint32_t)(hi >> 32) * gl::EPS + lo;
  const uint32_t th = (uint32_t)(t >> 32);
  const uint32_t rh = th + (uint32_t)hi;
  uint64_t r = ((uint64_t)rh << 32) | (uint32_t)t;
  if (rh < th) r += gl::EPS;
  return r;
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
    uint64_t al = (uint32_t)rc, ah = rc >> 32;
#pragma unroll
    for (int j = 0; j < WIDTH; j++) {
      const uint32_t c = a[(j - i + WIDTH) % WIDTH];
      al += (uint64_t)c * lo[j];
      ah += (uint64_t)c * hi[j];
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
#pragma unroll 1
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

__global__ void __launch_bounds__(THREADS) k_permute(uint64_t *__restrict__ states, size_t count,
                                                     const uint64_t *__restrict__ rc, Circ c) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  uint32_t a[WIDTH];
  circ_to_vgprs(c, a);
  uint64_t s[WIDTH];
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = states[k * WIDTH + i];
  permute(s, rc, a);
#pragma unroll
  for (int i = 0; i < WIDTH; i++) states[k * WIDTH + i] = gl::canon(s[i]);
}

// Leaf k = sponge over row k of a column-major matrix (lane k reads column c at
// row k: a wave's loads are 64 consecutive words of one column).
__global__ void __launch_bounds__(THREADS) k_leaf_hash(const uint64_t *__restrict__ mat, uint32_t n_cols,
                                                       uint64_t n_rows, uint64_t *__restrict__ dig,
                                                       const uint64_t *__restrict__ rc, Circ c) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_rows) return;
  uint32_t a[WIDTH];
  circ_to_vgprs(c, a);
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
  uint64_t *d = dig + k * DIGEST;
#pragma unroll
  for (int i = 0; i < DIGEST; i++) d[i] = gl::canon(s[i]);
}

// One Merkle level: node k = Compress(below[2k], below[2k+1]).
__global__ void __launch_bounds__(THREADS) k_merkle_level(const uint64_t *__restrict__ below,
                                                          uint64_t *__restrict__ above, uint64_t count,
                                                          const uint64_t *__restrict__ rc, Circ c) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  uint32_t a[WIDTH];
  circ_to_vgprs(c, a);
  uint64_t s[WIDTH];
  const uint64_t *src = below + k * (2 * DIGEST);
#pragma unroll
  for (int i = 0; i < 2 * DIGEST; i++) s[i] = src[i];
#pragma unroll
  for (int i = 2 * DIGEST; i < WIDTH; i++) s[i] = 0;
  permute(s, rc, a);
  uint64_t *d = above + k * DIGEST;
#pragma unroll
  for (int i = 0; i < DIGEST; i++) d[i] = gl::canon(s[i]);
}

Circ circ_of(const v3db_ctx *ctx) {
  Circ c;
  for (int i = 0; i < WIDTH; i++) c.a[i] = ctx->pos.circ[i];
  return c;
}

inline unsigned blocks_for(uint64_t n) { return (unsigned)((n + THREADS - 1) / THREADS); }

}  // namespace

v3db_status enqueue_permute(v3db_ctx *ctx, uint64_t *states, size_t count, hipStream_t stream) {
  if (count == 0) return V3DB_OK;
  hipLaunchKernelGGL(k_permute, dim3(blocks_for(count)), dim3(THREADS), 0, stream, states, count, ctx->d_pos,
                     circ_of(ctx));
  return hip_check(hipGetLastError(), "permute launch");
}

v3db_status enqueue_leaf_hash(v3db_ctx *ctx, const uint64_t *mat, uint32_t n_cols, uint32_t log_leaves,
                              uint64_t *digests, hipStream_t stream) {
  const uint64_t n = uint64_t(1) << log_leaves;
  hipLaunchKernelGGL(k_leaf_hash, dim3(blocks_for(n)), dim3(THREADS), 0, stream, mat, n_cols, n, digests,
                     ctx->d_pos, circ_of(ctx));
  return hip_check(hipGetLastError(), "leaf hash launch");
}

v3db_status enqueue_merkle_levels(v3db_ctx *ctx, uint64_t *tree, uint32_t log_leaves, uint32_t cap_height,
                                  uint64_t *cap, hipStream_t stream) {
  const Circ c = circ_of(ctx);
  uint64_t off = 0, cnt = uint64_t(1) << log_leaves;
  for (uint32_t lvl = log_leaves; lvl > cap_height; lvl--) {
    const uint64_t above = cnt / 2;
    hipLaunchKernelGGL(k_merkle_level, dim3(blocks_for(above)), dim3(THREADS), 0, stream, tree + off * DIGEST,
                       tree + (off + cnt) * DIGEST, above, ctx->d_pos, c);
    off += cnt;
    cnt = above;
  }
  v3db_status st = hip_check(hipGetLastError(), "merkle level launch");
  if (st != V3DB_OK) return st;
  if (cap != tree + off * DIGEST)
    st = hip_check(hipMemcpyAsync(cap, tree + off * DIGEST, cnt * DIGEST * 8, hipMemcpyDeviceToDevice, stream),
                   "cap copy");
  return st;
}

}  // namespace v3db
