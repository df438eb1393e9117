// Openings of committed traces (audit on demand): gather the rows and Merkle
// authentication paths of challenged leaves from the resident LDE and tree, and
// the verifier's check of such openings against a cap (MerkleOpen, batched).
#include "poseidon_dev.h"

namespace v3db {

namespace {

constexpr int GATHER_THREADS = 256;

// Item i < n_q * n_cols: element (q, c) of the rows; after that, word w of the
// sibling at level l of query q's path (level 0 = the leaves).
__global__ void __launch_bounds__(GATHER_THREADS)
    k_open_gather(const uint64_t *__restrict__ lde, uint32_t n_cols, uint32_t log_leaves,
                  const uint64_t *__restrict__ tree, uint32_t depth, const uint64_t *__restrict__ idx, uint64_t n_q,
                  uint64_t *__restrict__ rows, uint64_t *__restrict__ paths) {
  const uint64_t N = uint64_t(1) << log_leaves, mask = N - 1;
  const uint64_t n_rows = n_q * n_cols, n_path = n_q * depth * DIGEST;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_rows + n_path; i += stride) {
    if (i < n_rows) {
      const uint64_t q = i / n_cols, c = i - q * n_cols;
      rows[i] = lde[c * N + (idx[q] & mask)];
    } else {
      const uint64_t j = i - n_rows;
      const uint64_t q = j / (uint64_t(depth) * DIGEST), r = j - q * depth * DIGEST;
      const uint32_t l = (uint32_t)(r / DIGEST), w = (uint32_t)(r % DIGEST);
      const uint64_t sib = ((idx[q] & mask) >> l) ^ 1;
      const uint64_t off = (uint64_t(2) << log_leaves) - (uint64_t(2) << (log_leaves - l));  // level l
      paths[j] = tree[(off + sib) * DIGEST + w];
    }
  }
}

// One query per group of 16 lanes (wide_permute) or, for few queries, of 32 lanes
// (pair_permute: the chains are then latency-bound): the row's sponge, then one
// compression per path level with the running node on the side the index bit
// gives, then the comparison with the cap entry above the leaf. In the 32-lane
// form both rows of a group hold the state; the even row's lanes write the shared
// values.
template <bool PAIR>
__global__ void __launch_bounds__(64)
    k_verify(const uint64_t *__restrict__ rows, uint32_t n_cols, uint32_t log_leaves, uint32_t cap_height,
             const uint64_t *__restrict__ idx, uint64_t n_q, const uint64_t *__restrict__ paths,
             const uint64_t *__restrict__ cap, uint32_t *__restrict__ ok, const uint64_t *__restrict__ rc,
             const uint32_t *__restrict__ circ_rows) {
  using namespace pos;
  constexpr int GROUP = PAIR ? PAIR_GROUP : WIDE_GROUP, PER_BLOCK = 64 / GROUP;
  __shared__ uint64_t node[PER_BLOCK][DIGEST];
  __shared__ uint32_t match[PER_BLOCK][DIGEST];
  const int q = threadIdx.x % GROUP, grp = threadIdx.x / GROUP, g = q & 15;
  const uint64_t qi = uint64_t(blockIdx.x) * PER_BLOCK + grp;
  const bool live = qi < n_q;
  const uint64_t index = live ? (idx[qi] & ((uint64_t(1) << log_leaves) - 1)) : 0;
  const uint32_t depth = log_leaves - cap_height;
  auto perm = [&](uint64_t x) { return PAIR ? pair_permute(x, q, rc, circ_rows) : wide_permute(x, g, rc, circ_rows); };
  // leaf: overwrite sponge over the row, 8 elements per permutation
  uint64_t s = 0;
  for (uint32_t c0 = 0; c0 < n_cols; c0 += RATE) {
    if (g < RATE && c0 + g < n_cols) s = live ? rows[qi * n_cols + c0 + g] : 0;
    s = perm(s);
  }
  for (uint32_t l = 0; l < depth; l++) {
    if (q < DIGEST) node[grp][q] = s;
    __syncthreads();
    const uint64_t *sib = paths + (qi * depth + l) * DIGEST;
    const bool right = (index >> l) & 1;  // the running node is the right child
    if (g < DIGEST) s = right ? (live ? sib[g] : 0) : node[grp][g];
    else if (g < 2 * DIGEST) s = right ? node[grp][g - DIGEST] : (live ? sib[g - DIGEST] : 0);
    else s = 0;
    __syncthreads();
    s = perm(s);
  }
  const uint64_t ci = index >> depth;
  if (q < DIGEST) match[grp][q] = live && gl::canon(s) == cap[ci * DIGEST + q];
  __syncthreads();
  if (live && q == 0) ok[qi] = match[grp][0] & match[grp][1] & match[grp][2] & match[grp][3];
}

unsigned grid_for(uint64_t items, int threads) {
  const uint64_t b = (items + threads - 1) / threads;
  return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

}  // namespace

v3db_status enqueue_open(v3db_ctx *, const uint64_t *lde, uint32_t n_cols, uint32_t log_leaves, const uint64_t *tree,
                         uint32_t cap_height, const uint64_t *idx, size_t n_q, uint64_t *rows, uint64_t *paths,
                         hipStream_t stream) {
  if (n_q == 0) return V3DB_OK;
  const uint32_t depth = log_leaves - cap_height;
  const uint64_t items = uint64_t(n_q) * n_cols + uint64_t(n_q) * depth * DIGEST;
  hipLaunchKernelGGL(k_open_gather, dim3(grid_for(items, GATHER_THREADS)), dim3(GATHER_THREADS), 0, stream, lde,
                     n_cols, log_leaves, tree, depth, idx, (uint64_t)n_q, rows, paths);
  return hip_check(hipGetLastError(), "open launch");
}

v3db_status enqueue_verify(v3db_ctx *ctx, const uint64_t *rows, uint32_t n_cols, uint32_t log_leaves,
                           uint32_t cap_height, const uint64_t *idx, size_t n_q, const uint64_t *paths,
                           const uint64_t *cap, uint32_t *ok, hipStream_t stream) {
  if (n_q == 0) return V3DB_OK;
  if (n_q <= MERKLE_PAIR_MAX_NODES) {
    const unsigned blocks = (unsigned)((n_q + pos::PAIR_PER_BLOCK - 1) / pos::PAIR_PER_BLOCK);
    hipLaunchKernelGGL(k_verify<true>, dim3(blocks), dim3(64), 0, stream, rows, n_cols, log_leaves, cap_height, idx,
                       (uint64_t)n_q, paths, cap, ok, ctx->d_pos, ctx->d_circ_rows);
  } else {
    const unsigned blocks = (unsigned)((n_q + pos::WIDE_PER_BLOCK - 1) / pos::WIDE_PER_BLOCK);
    hipLaunchKernelGGL(k_verify<false>, dim3(blocks), dim3(64), 0, stream, rows, n_cols, log_leaves, cap_height, idx,
                       (uint64_t)n_q, paths, cap, ok, ctx->d_pos, ctx->d_circ_rows);
  }
  return hip_check(hipGetLastError(), "verify launch");
}

}  // namespace v3db
