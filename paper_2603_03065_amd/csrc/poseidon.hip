// Poseidon kernels for single calls: permutation of state arrays, leaf hashing
// of a matrix, and one Merkle level per launch (routines in poseidon_dev.h).
#include "poseidon_mf.h"

namespace v3db {

namespace {

using namespace pos;

constexpr int THREADS = 256;

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

__global__ void __launch_bounds__(THREADS) k_leaf_hash(const uint64_t *__restrict__ mat, uint32_t n_cols,
                                                       uint64_t n_rows, uint64_t *__restrict__ dig,
                                                       const uint64_t *__restrict__ rc, Circ c) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_rows) return;
  uint32_t a[WIDTH];
  circ_to_vgprs(c, a);
  leaf_digest(mat, n_cols, n_rows, k, dig + k * DIGEST, rc, a);
}

__global__ void __launch_bounds__(THREADS) k_merkle_level(const uint64_t *__restrict__ below,
                                                          uint64_t *__restrict__ above, uint64_t count,
                                                          const uint64_t *__restrict__ rc, Circ c) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  uint32_t a[WIDTH];
  circ_to_vgprs(c, a);
  merkle_node(below, k, above + k * DIGEST, rc, a);
}

// The same two kernels with the matrix-core linear layer: each wave covers 64
// consecutive rows (nodes), a block of THREADS threads covers THREADS of them. The
// leaf kernel is held to 128 VGPRs (four waves per SIMD): left alone it takes 141 and
// runs three, which measured slower.
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_leaf_hash_mf(const uint64_t *__restrict__ mat, uint32_t n_cols,
                                                          uint64_t n_rows, uint64_t *__restrict__ dig,
                                                          const uint64_t *__restrict__ rc,
                                                          const uint64_t *__restrict__ tab) {
  const uint64_t base = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
  if (base >= n_rows) return;  // whole waves only
  const MfLane L = mf_lane(tab);
  leaf_digests_mf(mat, n_cols, n_rows, base, dig, L, rc, tab);
}

__global__ void __launch_bounds__(THREADS) k_merkle_level_mf(const uint64_t *__restrict__ below,
                                                             uint64_t *__restrict__ above, uint64_t count,
                                                             const uint64_t *__restrict__ rc,
                                                             const uint64_t *__restrict__ tab) {
  const uint64_t base = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
  if (base >= count) return;
  const MfLane L = mf_lane(tab);
  merkle_nodes_mf(below, count, base, above, L, rc, tab);
}

// One level with very few nodes: 32 lanes per node (pair_permute).
__global__ void __launch_bounds__(PAIR_THREADS) k_merkle_level_pair(const uint64_t *__restrict__ below,
                                                                    uint64_t *__restrict__ above, uint64_t count,
                                                                    const uint64_t *__restrict__ rc,
                                                                    const uint32_t *__restrict__ circ_rows) {
  const int q = threadIdx.x % PAIR_GROUP, grp = threadIdx.x / PAIR_GROUP, g = q & 15;
  const uint64_t k = uint64_t(blockIdx.x) * PAIR_PER_BLOCK + grp;
  const bool live = k < count;
  uint64_t s = 0;
  if (live && g < 2 * DIGEST) s = below[k * 2 * DIGEST + g];
  s = pair_permute(s, q, rc, circ_rows);
  if (live && q < DIGEST) above[k * DIGEST + q] = gl::canon(s);
}

// One level with few nodes: 16 lanes per node (wide_permute).
__global__ void __launch_bounds__(WIDE_THREADS) k_merkle_level_wide(const uint64_t *__restrict__ below,
                                                                    uint64_t *__restrict__ above, uint64_t count,
                                                                    const uint64_t *__restrict__ rc,
                                                                    const uint32_t *__restrict__ circ_rows) {
  const int g = threadIdx.x % WIDE_GROUP, grp = threadIdx.x / WIDE_GROUP;
  const uint64_t k = uint64_t(blockIdx.x) * WIDE_PER_BLOCK + grp;
  const bool live = k < count;
  uint64_t s = 0;
  if (live && g < 2 * DIGEST) s = below[k * 2 * DIGEST + g];
  s = wide_permute(s, g, rc, circ_rows);
  if (live && g < DIGEST) above[k * DIGEST + g] = gl::canon(s);
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
  if (ctx->mf)
    hipLaunchKernelGGL(k_leaf_hash_mf, dim3(blocks_for(n)), dim3(THREADS), 0, stream, mat, n_cols, n, digests,
                       ctx->d_pos, ctx->d_mf);
  else
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
    if (above <= MERKLE_PAIR_MAX_NODES)
      hipLaunchKernelGGL(k_merkle_level_pair, dim3((unsigned)((above + PAIR_PER_BLOCK - 1) / PAIR_PER_BLOCK)),
                         dim3(PAIR_THREADS), 0, stream, tree + off * DIGEST, tree + (off + cnt) * DIGEST, above,
                         ctx->d_pos, ctx->d_circ_rows);
    else if (above <= MERKLE_WIDE_MAX_NODES)
      hipLaunchKernelGGL(k_merkle_level_wide, dim3((unsigned)((above + WIDE_PER_BLOCK - 1) / WIDE_PER_BLOCK)),
                         dim3(WIDE_THREADS), 0, stream, tree + off * DIGEST, tree + (off + cnt) * DIGEST, above,
                         ctx->d_pos, ctx->d_circ_rows);
    else if (ctx->mf)
      hipLaunchKernelGGL(k_merkle_level_mf, dim3(blocks_for(above)), dim3(THREADS), 0, stream, tree + off * DIGEST,
                         tree + (off + cnt) * DIGEST, above, ctx->d_pos, ctx->d_mf);
    else
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
