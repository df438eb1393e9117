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

// lo + hi * 2^32 with lo, hi < 2^44, reduced to [0, 2^64).
__device__ __forceinline__ uint64_t fold(uint64_t lo, uint64_t hi) {
  const uint64_t s = lo + (hi << 32);
  const uint32_t k = (uint32_t)(hi >> 32) + (s < lo ? 1u : 0u);  // multiples of 2^64
  const uint64_t kk = ((uint64_t)k << 32) - k;                    // k * (2^64 mod p)
  uint64_t r = s + kk;
  if (r < kk) r += gl::EPS;
  return r;
}

__device__ __forceinline__ void mds(uint64_t s[WIDTH], const Circ &c) {
  uint64_t out[WIDTH];
#pragma unroll
  for (int i = 0; i < WIDTH; i++) {
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < WIDTH; j++) {
      const uint32_t a = c.a[(j - i + WIDTH) % WIDTH];
      lo += (uint64_t)a * (uint32_t)s[j];
      hi += (uint64_t)a * (uint32_t)(s[j] >> 32);
    }
    out[i] = fold(lo, hi);
  }
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = out[i];
}

__device__ __forceinline__ void full_round(uint64_t s[WIDTH], const uint64_t *__restrict__ rc, const Circ &c) {
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = sbox(gl::add_r(s[i], rc[i]));
  mds(s, c);
}

__device__ __forceinline__ void partial_round(uint64_t s[WIDTH], const uint64_t *__restrict__ rc, const Circ &c) {
  s[0] = sbox(gl::add_r(s[0], rc[0]));
#pragma unroll
  for (int i = 1; i < WIDTH; i++) s[i] = gl::add_r(s[i], rc[i]);
  mds(s, c);
}

__device__ __forceinline__ void permute(uint64_t s[WIDTH], const uint64_t *__restrict__ rc, const Circ &c) {
#pragma unroll 1
  for (int r = 0; r < FULL_HALF; r++) full_round(s, rc + r * WIDTH, c);
#pragma unroll 1
  for (int r = FULL_HALF; r < ROUNDS - FULL_HALF; r++) partial_round(s, rc + r * WIDTH, c);
#pragma unroll 1
  for (int r = ROUNDS - FULL_HALF; r < ROUNDS; r++) full_round(s, rc + r * WIDTH, c);
}

__global__ void __launch_bounds__(THREADS) k_permute(uint64_t *__restrict__ states, size_t count,
                                                     const uint64_t *__restrict__ rc, Circ c) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  uint64_t s[WIDTH];
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = states[k * WIDTH + i];
  permute(s, rc, c);
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
  uint64_t s[WIDTH];
#pragma unroll
  for (int i = 0; i < WIDTH; i++) s[i] = 0;
  for (uint32_t q = 0; q < n_cols; q += RATE) {
    const uint32_t len = (n_cols - q) < RATE ? (n_cols - q) : RATE;
    const uint64_t *base = mat + uint64_t(q) * n_rows + k;
#pragma unroll
    for (int i = 0; i < RATE; i++)
      if (i < (int)len) s[i] = base[uint64_t(i) * n_rows];
    permute(s, rc, c);
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
  uint64_t s[WIDTH];
  const uint64_t *src = below + k * (2 * DIGEST);
#pragma unroll
  for (int i = 0; i < 2 * DIGEST; i++) s[i] = src[i];
#pragma unroll
  for (int i = 2 * DIGEST; i < WIDTH; i++) s[i] = 0;
  permute(s, rc, c);
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
