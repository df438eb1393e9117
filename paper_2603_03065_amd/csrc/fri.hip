// FRI commit phase over a codeword on a coset: per round, the Merkle tree whose
// leaf k hashes the pair (f(x_k), f(-x_k)) = (f[k], f[k + N/2]) (the leaf-hash and
// Merkle kernels of the trace commitment, reading the codeword as a two-column
// matrix [2][N/2]), then the arity-2 fold with the round's challenge beta:
//   f'[k] = (f[k] + f[k + N/2]) / 2 + beta (f[k] - f[k + N/2]) / (2 x_k),
// on the squared coset (shift s^2, N/2 points, natural order).
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

// The fold chain runs on the caller's stream; round r's tree only reads f_r, so it
// runs on side stream r mod FRI_STREAMS once f_r is ready (an event recorded after
// the fold that produced it) and overlaps the later folds and trees; the caller's
// stream waits for every side stream before anything enqueued after this call.
v3db_status enqueue_fri_commit(v3db_ctx *ctx, const uint64_t *codeword, uint32_t log_n, uint64_t shift,
                               const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *folded,
                               uint64_t *trees, uint64_t *caps, uint64_t *scratch_tree, hipStream_t stream) {
  constexpr int NS = v3db_ctx::FRI_STREAMS;
  hipError_t e = hipSuccess;
  for (int i = 0; i < NS && e == hipSuccess; i++) {
    if (!ctx->fri_streams[i]) e = hipStreamCreateWithFlags(&ctx->fri_streams[i], hipStreamNonBlocking);
    if (e == hipSuccess && !ctx->fri_done[i]) e = hipEventCreateWithFlags(&ctx->fri_done[i], hipEventDisableTiming);
  }
  for (uint32_t r = 0; r < rounds && e == hipSuccess; r++)
    if (!ctx->fri_ready[r]) e = hipEventCreateWithFlags(&ctx->fri_ready[r], hipEventDisableTiming);
  if (e != hipSuccess) return hip_check(e, "fri streams");
  const int used = rounds < (uint32_t)NS ? (int)rounds : NS;
  const uint64_t *f = codeword;
  uint64_t *next = folded, *tree = trees ? trees : scratch_tree;
  uint64_t s_r = shift % gl::P;
  v3db_status st = hip_check(hipEventRecord(ctx->fri_ready[0], stream), "fri fork");
  for (uint32_t r = 0; r < rounds && st == V3DB_OK; r++) {
    const uint32_t log_nr = log_n - r;
    const uint64_t half = uint64_t(1) << (log_nr - 1);
    hipStream_t side = ctx->fri_streams[r % NS];
    st = hip_check(hipStreamWaitEvent(side, ctx->fri_ready[r], 0), "fri wait");
    if (st == V3DB_OK) st = enqueue_leaf_hash(ctx, f, 2, log_nr - 1, tree, side);
    if (st == V3DB_OK)
      st = enqueue_merkle_levels(ctx, tree, log_nr - 1, cap_height, caps + size_t(r) * (DIGEST << cap_height), side);
    if (st != V3DB_OK) break;
    const uint64_t tr = gl::mul(betas[r] % gl::P, gl::inv(s_r));
    const unsigned blocks = (unsigned)std::min<uint64_t>((half + FOLD_THREADS - 1) / FOLD_THREADS, 8192);
    hipLaunchKernelGGL(k_fri_fold, dim3(blocks), dim3(FOLD_THREADS), 0, stream, f, half, log_nr, tr, next, ctx->tw);
    st = hip_check(hipGetLastError(), "fri fold launch");
    if (st == V3DB_OK && r + 1 < rounds) st = hip_check(hipEventRecord(ctx->fri_ready[r + 1], stream), "fri ready");
    tree += ((uint64_t(2) * half) - (uint64_t(1) << cap_height)) * DIGEST;
    f = next;
    next += half;
    s_r = gl::mul(s_r, s_r);
  }
  // join every side stream that received work, also after an error
  for (int i = 0; i < used; i++) {
    hipError_t j = hipEventRecord(ctx->fri_done[i], ctx->fri_streams[i]);
    if (j == hipSuccess) j = hipStreamWaitEvent(stream, ctx->fri_done[i], 0);
    if (st == V3DB_OK && j != hipSuccess) st = hip_check(j, "fri join");
  }
  return st;
}

}  // namespace v3db
