// FRI commit phase over a codeword on a coset: per round, the Merkle tree whose
// leaf k hashes the pair (f(x_k), f(-x_k)) = (f[k], f[k + N/2]) (the batched leaf-hash
// and Merkle kernels of the trace commitment, reading the codeword as a two-column
// matrix [2][N/2]), then the arity-2 fold with the round's challenge beta:
//   f'[k] = (f[k] + f[k + N/2]) / 2 + beta (f[k] - f[k + N/2]) / (2 x_k),
// on the squared coset (shift s^2, N/2 points, natural order).
#include <vector>

#include "lde_dev.h"

namespace v3db {

namespace {

constexpr int FOLD_THREADS = 256;

// v / 2 mod p for canonical v: an odd v becomes (v + p) / 2 = (v - 1) / 2 + (p + 1) / 2.
__device__ __forceinline__ uint64_t halve(uint64_t v) {
  return (v >> 1) + ((v & 1) ? (gl::P >> 1) + 1 : 0);
}

// t = beta / s_r; x_k^-1 = s_r^-1 w_{N_r}^-k from the two-level table of w_{2^26}^-1.
__global__ void __launch_bounds__(FOLD_THREADS)
    k_fri_fold(const uint64_t *__restrict__ f, uint64_t half, uint32_t log_nr, uint64_t t, uint64_t *__restrict__ out,
               Twiddles tw) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < half; k += stride) {
    const uint64_t a = f[k], b = f[k + half];
    const uint64_t wk = lde::tw_pow(tw.inv_lo, tw.inv_hi, (uint32_t)(k << (TW_LOG - log_nr)));
    const uint64_t odd = gl::mul(gl::sub(a, b), gl::mul(t, wk));
    out[k] = halve(gl::add(gl::add(a, b), odd));
  }
}

}  // namespace

size_t fri_tree_digests(uint32_t log_n, uint32_t rounds, uint32_t cap_height) {
  size_t d = 0;
  for (uint32_t r = 0; r < rounds; r++) d += (size_t(1) << (log_n - r)) - (size_t(1) << cap_height);
  return d;
}

// The fold chain first (each fold reads the previous round's codeword only), then every
// round's tree in one batch: one leaf-hashing launch over the pair leaves of all rounds
// and one launch per tree depth over all rounds that still have it, all on the caller's
// stream.
v3db_status enqueue_fri_commit(v3db_ctx *ctx, const uint64_t *codeword, uint32_t log_n, uint64_t shift,
                               const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *folded,
                               uint64_t *trees, uint64_t *caps, uint64_t *scratch_tree, hipStream_t stream) {
  std::vector<TreeJob> tj(rounds);
  const uint64_t *f = codeword;
  uint64_t *next = folded, *tree = trees ? trees : scratch_tree;
  uint64_t s_r = shift % gl::P;
  for (uint32_t r = 0; r < rounds; r++) {
    const uint32_t log_nr = log_n - r;
    const uint64_t half = uint64_t(1) << (log_nr - 1);
    // leaf k = Hash(f_r[k], f_r[k + N_r/2]): the codeword read as the matrix [2][N_r/2]
    tj[r] = TreeJob{f, tree, caps + size_t(r) * (DIGEST << cap_height), 2, log_nr - 1, cap_height};
    const uint64_t tr = gl::mul(betas[r] % gl::P, gl::inv(s_r));
    const unsigned blocks = (unsigned)std::min<uint64_t>((half + FOLD_THREADS - 1) / FOLD_THREADS, 8192);
    hipLaunchKernelGGL(k_fri_fold, dim3(blocks), dim3(FOLD_THREADS), 0, stream, f, half, log_nr, tr, next, ctx->tw);
    v3db_status st = hip_check(hipGetLastError(), "fri fold launch");
    if (st != V3DB_OK) return st;
    tree += ((uint64_t(2) * half) - (uint64_t(1) << cap_height)) * DIGEST;
    f = next;
    next += half;
    s_r = gl::mul(s_r, s_r);
  }
  return enqueue_tree_batch(ctx, tj.data(), rounds, stream);
}

}  // namespace v3db
