// Snapshot commitment of a fixed-shape IVF-PQ layout (Sec. 4.3 "Snapshot
// Commitments"): every slot record hashed, one Merkle tree per inverted list
// (the lists are consecutive leaf ranges, so the list roots are the level of a
// single tree at height log2(n_list)), each centroid hashed with its list root,
// a Merkle tree over those digests, and a digest of the PQ codebooks. The
// codebook digest is one long sequential sponge; it runs on a side stream,
// forked from and joined back into the caller's stream, beside the rest.
#include "poseidon_mf.h"

namespace v3db {

namespace {

using namespace pos;

constexpr int LEAF_THREADS = 256;

// hash_{i,j} = Hash(i, j, f, item, v^(0..M-1)) of record t = i * n + j.
__global__ void __launch_bounds__(LEAF_THREADS)
    k_snap_leaf(const uint64_t *__restrict__ flag, const uint64_t *__restrict__ item,
                const uint64_t *__restrict__ codes, uint32_t m, uint32_t log_slots, uint64_t n_rec,
                uint64_t *__restrict__ digests, const uint64_t *__restrict__ rc, Circ c) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_rec) return;
  uint32_t a[WIDTH];
  circ_to_vgprs(c, a);
  const uint64_t i = t >> log_slots, j = t & ((uint64_t(1) << log_slots) - 1);
  const uint32_t len = 4 + m;
  uint64_t s[WIDTH];
#pragma unroll
  for (int w = 0; w < WIDTH; w++) s[w] = 0;
  for (uint32_t c0 = 0; c0 < len; c0 += RATE) {
#pragma unroll
    for (int q = 0; q < RATE; q++) {
      const uint32_t x = c0 + q;
      if (x < len) s[q] = x == 0 ? i : x == 1 ? j : x == 2 ? flag[t] : x == 3 ? item[t] : codes[uint64_t(x - 4) * n_rec + t];
    }
    permute(s, rc, a);
  }
#pragma unroll
  for (int w = 0; w < DIGEST; w++) digests[t * DIGEST + w] = gl::canon(s[w]);
}

// The same with the matrix-core linear layer: each wave covers 64 consecutive records.
__global__ void __launch_bounds__(LEAF_THREADS)
    k_snap_leaf_mf(const uint64_t *__restrict__ flag, const uint64_t *__restrict__ item,
                   const uint64_t *__restrict__ codes, uint32_t m, uint32_t log_slots, uint64_t n_rec,
                   uint64_t *__restrict__ digests, const uint64_t *__restrict__ rc, const uint64_t *__restrict__ tab) {
  const uint64_t base = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
  if (base >= n_rec) return;  // whole waves only
  const MfLane L = mf_lane(tab);
  const uint64_t mask = (uint64_t(1) << log_slots) - 1;
  auto elem = [&](int u, uint64_t x) -> uint64_t {
    const uint64_t t = base + L.c + 32 * u;
    return x == 0 ? t >> log_slots : x == 1 ? t & mask : x == 2 ? flag[t] : x == 3 ? item[t] : codes[(x - 4) * n_rec + t];
  };
  uint64_t S[2][6];
  sponge_mf(S, 4 + uint64_t(m), elem, [&](int u) { return base + L.c + 32 * u < n_rec; }, L, rc, tab);
  store_digests_mf(S, L, base, n_rec, digests);
}

// hash_i = Hash(i, mu_i[0..D-1], root_i), 32 lanes per list (few lists: latency-bound).
__global__ void __launch_bounds__(PAIR_THREADS)
    k_snap_centroid(const uint64_t *__restrict__ centroids, uint32_t dim, const uint64_t *__restrict__ roots,
                    uint64_t n_list, uint64_t *__restrict__ hashes, const uint64_t *__restrict__ rc,
                    const uint32_t *__restrict__ circ_rows) {
  const int q = threadIdx.x % PAIR_GROUP, grp = threadIdx.x / PAIR_GROUP;
  const uint64_t i = uint64_t(blockIdx.x) * PAIR_PER_BLOCK + grp;
  const bool live = i < n_list;
  const uint64_t *mu = centroids + i * dim;
  const uint64_t *root = roots + i * DIGEST;
  auto elem = [&](uint64_t x) -> uint64_t { return x == 0 ? i : x <= dim ? mu[x - 1] : root[x - 1 - dim]; };
  const uint64_t s = pair_sponge(1 + uint64_t(dim) + DIGEST, live, elem, q, rc, circ_rows);
  if (live && q < DIGEST) hashes[i * DIGEST + q] = gl::canon(s);
}

// root_cb = Hash(codebooks, canonical flattening of len words): one group of 32 lanes.
__global__ void __launch_bounds__(PAIR_THREADS)
    k_snap_codebook(const uint64_t *__restrict__ codebooks, uint64_t len, uint64_t *__restrict__ root_cb,
                    const uint64_t *__restrict__ rc, const uint32_t *__restrict__ circ_rows) {
  const int q = threadIdx.x % PAIR_GROUP, grp = threadIdx.x / PAIR_GROUP;
  const bool live = grp == 0;
  auto elem = [&](uint64_t x) -> uint64_t { return codebooks[x]; };
  const uint64_t s = pair_sponge(len, live, elem, q, rc, circ_rows);
  if (live && q < DIGEST) root_cb[q] = gl::canon(s);
}

}  // namespace

size_t snapshot_scratch_words(uint32_t log_lists, uint32_t log_slots) {
  const size_t n_list = size_t(1) << log_lists, N = n_list << log_slots;
  // record tree (leaves up to the list roots), list roots, list digests and their tree
  return ((2 * N - n_list) + n_list + (2 * n_list - 1)) * DIGEST;
}

v3db_status enqueue_snapshot(v3db_ctx *ctx, uint32_t log_lists, uint32_t log_slots, uint32_t m, uint32_t dim,
                             uint32_t k, const uint64_t *flag, const uint64_t *item, const uint64_t *codes,
                             const uint64_t *centroids, const uint64_t *codebooks, uint64_t *list_roots,
                             uint64_t *root_mk, uint64_t *root_cb, uint64_t *scratch, hipStream_t stream) {
  const uint64_t n_list = uint64_t(1) << log_lists, N = n_list << log_slots;
  uint64_t *tree = scratch;                             // [2N - n_list][4]
  uint64_t *roots = tree + (2 * N - n_list) * DIGEST;  // [n_list][4]
  uint64_t *top = roots + n_list * DIGEST;              // [2 n_list - 1][4]
  if (!list_roots) list_roots = roots;
  // the codebook digest on the side stream, joined back at the end
  if (!ctx->side_stream) {
    v3db_status st = hip_check(hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking), "side stream");
    if (st == V3DB_OK) st = hip_check(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming), "fork event");
    if (st == V3DB_OK) st = hip_check(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming), "join event");
    if (st != V3DB_OK) return st;
  }
  hipError_t e = hipEventRecord(ctx->fork_ev, stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side_stream, ctx->fork_ev, 0);
  if (e != hipSuccess) return hip_check(e, "snapshot fork");
  hipLaunchKernelGGL(k_snap_codebook, dim3(1), dim3(PAIR_THREADS), 0, ctx->side_stream, codebooks,
                     uint64_t(k) * dim, root_cb, ctx->d_pos, ctx->d_circ_rows);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(ctx->join_ev, ctx->side_stream);
  if (e != hipSuccess) return hip_check(e, "snapshot codebook digest");
  const unsigned leaf_blocks = (unsigned)((N + LEAF_THREADS - 1) / LEAF_THREADS);
  if (ctx->mf)
    hipLaunchKernelGGL(k_snap_leaf_mf, dim3(leaf_blocks), dim3(LEAF_THREADS), 0, stream, flag, item, codes, m,
                       log_slots, N, tree, ctx->d_pos, ctx->d_mf);
  else
    hipLaunchKernelGGL(k_snap_leaf, dim3(leaf_blocks), dim3(LEAF_THREADS), 0, stream, flag, item, codes, m,
                       log_slots, N, tree, ctx->d_pos, circ_of(ctx));
  v3db_status st = hip_check(hipGetLastError(), "snapshot leaves");
  // list roots = the level of the record tree at height log2(n_list)
  if (st == V3DB_OK) st = enqueue_merkle_levels(ctx, tree, log_lists + log_slots, log_lists, list_roots, stream);
  if (st == V3DB_OK) {
    hipLaunchKernelGGL(k_snap_centroid, dim3((unsigned)((n_list + PAIR_PER_BLOCK - 1) / PAIR_PER_BLOCK)),
                       dim3(PAIR_THREADS), 0, stream, centroids, dim, list_roots, n_list, top, ctx->d_pos,
                       ctx->d_circ_rows);
    st = hip_check(hipGetLastError(), "snapshot centroid digests");
  }
  if (st == V3DB_OK) st = enqueue_merkle_levels(ctx, top, log_lists, 0, root_mk, stream);
  // join even after an error, so the side stream's work is ordered before anything later on stream
  e = hipStreamWaitEvent(stream, ctx->join_ev, 0);
  if (st == V3DB_OK) st = hip_check(e, "snapshot join");
  return st;
}

}  // namespace v3db
