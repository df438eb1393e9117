// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/v3db.h"
#include "gl.h"

namespace v3db {

constexpr int WIDTH = 12, RATE = 8, DIGEST = 4, ROUNDS = 30, FULL_HALF = 4;
// Device Poseidon table: (ROUNDS + 1) x WIDTH round-constant words, then WIDTH x WIDTH
// 32-bit matrix entries (half as many 64-bit words).
// Tree levels of at most this many nodes use 16 lanes per node (shorter latency).
constexpr uint64_t MERKLE_WIDE_MAX_NODES = uint64_t(1) << 15;
// ... and levels of at most this many, latency-bound, 32 lanes per node.
constexpr uint64_t MERKLE_PAIR_MAX_NODES = uint64_t(1) << 11;
constexpr size_t POS_TABLE_WORDS = (ROUNDS + 1) * WIDTH + WIDTH * WIDTH / 2;
// Table of the matrix-core linear layer (poseidon_mf.h), in 64-bit words: the int8
// matrix as 16 bytes per lane, the four limb weights as int32, then (ROUNDS + 1) x WIDTH
// pairs {lo, hi} of accumulator start values (row r + 1 used by round r).
constexpr size_t MF_AMAT = 0, MF_MULT = 128, MF_RCK = 130;
constexpr size_t MF_TABLE_WORDS = MF_RCK + size_t(ROUNDS + 1) * WIDTH * 2;
constexpr int TW_LOG = 26;        // largest transform, 2^26 points
constexpr int TW_HALF = 13;       // two-level twiddle table: 2^13 x 2^13
constexpr int DFT_LOG_MAX = 12;   // largest in-LDS sub-transform, 4096 points

// Round constants and MDS first row, as the kernels consume them.
struct PoseidonTables {
  uint64_t rc[ROUNDS][WIDTH];
  uint32_t circ[WIDTH];
};

// Device twiddle tables, built once per context.
struct Twiddles {
  uint64_t *fwd_lo, *fwd_hi;   // w^i and w^(2^13 i), w = w_{2^26}, i < 2^13
  uint64_t *inv_lo, *inv_hi;   // same for w^-1
  uint64_t *bfly_fwd, *bfly_inv; // radix-8 butterfly twiddle rows, forward and inverse (lde_dev.h)
};

// Schedule of the LDE passes for one (log_rows, log_blowup): the split
// n = n1 * n2 (n2 = 2^L2), caps on each pass's log2 tile height, and how many
// columns go through passes 2 and 3 together in the single-trace path.
struct LdeSchedule {
  uint32_t L2, cap1, cap2, cap3, chunk;
  double us;  // measured time of the tuning shape (0 = default, untimed)
};

// Per-shape LDE tables: see ntt.hip.
struct LdePlan {
  uint32_t log_rows, log_blowup, L1, L2;
  uint32_t logT1, logT2, logT3;  // log2 tile heights of passes 1, 2 and 3
  uint32_t logT2i;               // log2 rows per tile of pass 2's inverse part (run as its own kernel)
  uint32_t chunk;                // columns per pass-2/3 round (single-trace path)
  uint64_t shift;
  uint64_t *d_twist;  // [B][n2]: (shift^n1 * w_{B n2}^r)^j
  uint64_t *d_scale;  // [n1]: n^-1 * shift^k1
  uint64_t *d_ztw;    // [n1][B n2]: w_N^(k1 e) for N <= 2^ZTW_MAX_LOG, else null
};

// Largest extension (log2 rows) whose pass-2 twiddles w_N^(k1 e) are kept as a
// full table (8 N bytes per shape) instead of two lookups and a product.
constexpr uint32_t ZTW_MAX_LOG = 23;

struct ScratchBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct BatchGraph;
struct EagerTable;

}  // namespace v3db

struct v3db_ctx {
  int device = 0;
  uint64_t seed = 0;
  size_t budget = 0;       // 0 = unlimited
  size_t allocated = 0;    // bytes currently held by this context
  uint32_t mds_attempts = 0;
  v3db::PoseidonTables pos{};
  uint64_t *d_pos = nullptr;         // POS_TABLE_WORDS: round constants (ROUNDS + 1 rows, last zero),
                                    // then the matrix rows M[i][j] as 32-bit words
  const uint32_t *d_circ_rows = nullptr;  // inside d_pos
  uint64_t *d_mf = nullptr;          // MF_TABLE_WORDS: the matrix-core linear layer's table
  bool mf = false;                   // hash kernels use the matrix-core linear layer
  v3db::Twiddles tw{};
  std::map<std::tuple<uint32_t, uint32_t, uint64_t>, v3db::LdePlan> plans;
  std::map<std::pair<uint32_t, uint32_t>, v3db::LdeSchedule> tuned;  // autotuned schedules
  std::map<void *, v3db::ScratchBuf> scratch;  // per stream
  // phase timing (v3db_profile_*): event pairs per phase, recycled through a pool
  bool profiling = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
  std::vector<hipEvent_t> event_pool;
  // batched commits: captured launch sequences per (shapes, stream)
  bool batching = true;
  size_t batch_group_bytes = size_t(32) << 30;
  std::vector<v3db::BatchGraph *> graphs;
  uint64_t graph_clock = 0;
  // shape lists seen once (a graph is captured at the second sighting) and, per
  // stream, the job and range table of batches launched without a graph
  std::vector<std::vector<uint64_t>> seen_keys;
  std::vector<v3db::EagerTable *> eager_tables;
  hipStream_t capture_stream = nullptr;
  hipStream_t side_stream = nullptr;  // snapshot codebook digest, forked from and joined into the caller's stream
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // batches of Merkle trees over resident matrices (enqueue_tree_batch): the job and
  // range table on the device, its pinned staging copy, and events marking when the
  // staging copy has been read and when the last batch's kernels have read the table
  void *tree_table_d = nullptr, *tree_table_h = nullptr;
  size_t tree_table_bytes = 0;
  hipEvent_t tree_table_staged = nullptr, tree_table_done = nullptr;
  std::mutex mu;
};

namespace v3db {

// Error reporting (thread-local message).
v3db_status set_error(v3db_status st, const std::string &msg);
void clear_error();
v3db_status hip_check(hipError_t e, const char *what);

// Context-owned device memory, counted against the budget.
v3db_status ctx_alloc(v3db_ctx *ctx, void **ptr, size_t bytes, const char *what);
void ctx_free(v3db_ctx *ctx, void *ptr, size_t bytes);
// Per-stream scratch of at least `bytes` (grown as needed).
v3db_status ctx_scratch(v3db_ctx *ctx, hipStream_t stream, size_t bytes, void **out);

// Host-side constant derivation (constants.cpp).
uint64_t splitmix64(uint64_t seed, uint64_t i);
bool derive_poseidon(uint64_t seed, PoseidonTables &out, uint32_t &attempts);
bool circulant_is_mds(const uint32_t circ[WIDTH]);
// The matrix-core linear layer's table; false if an entry exceeds 255 (C - 128 would
// not fit a signed byte), in which case the hash kernels keep the VALU form.
bool build_mf_table(const PoseidonTables &t, uint64_t out[MF_TABLE_WORDS]);

// Tables (ntt.hip).
v3db_status build_twiddles(v3db_ctx *ctx);
// raise the LDS limit of the tiled LDE kernels on the current device (context creation)
v3db_status set_lde_kernel_attributes();
v3db_status set_batch_kernel_attributes();
void free_twiddles(v3db_ctx *ctx);
v3db_status get_plan(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint64_t shift, const LdePlan **out);

// Enqueue an LDE (ntt.hip). Arguments already validated.
// Columns that go through passes 2 and 3 together (their Z stays cache-resident):
// the default, and the most a schedule may use (bit-reversed scratch is sized for it).
constexpr uint32_t LDE_CHUNK_COLS = 8;
constexpr uint32_t LDE_MAX_CHUNK_COLS = 16;
LdeSchedule default_schedule(uint32_t log_rows, uint32_t log_blowup);
void drop_plans(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup);  // frees their tables
bool schedule_valid(const LdeSchedule &s, uint32_t log_rows, uint32_t log_blowup);
v3db_status autotune_lde(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint32_t n_cols, v3db_layout layout,
                         LdeSchedule *out);
// Scratch of one v3db_lde call: Y (n words per column), plus Z for one chunk of
// columns in bit-reversed layout (natural layout builds Z in the output).
size_t lde_scratch_bytes(uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup, v3db_layout layout);
v3db_status enqueue_lde(v3db_ctx *ctx, const uint64_t *trace, uint32_t n_cols, uint32_t log_rows,
                        uint32_t log_blowup, uint64_t shift, v3db_layout layout, uint64_t *lde,
                        uint64_t *scratch, hipStream_t stream);

// The no-alloc entry point's static scratch: its address on `device` (noalloc.hip),
// looked up once per device with that device current.
v3db_status noalloc_setup(int device);

// Phase timing: returns an event recorded on `stream` (or nullptr when not profiling).
hipEvent_t prof_mark(v3db_ctx *ctx, hipStream_t stream);
void prof_interval(v3db_ctx *ctx, int phase, hipEvent_t a, hipEvent_t b);

// Batched commits (batch.hip). scratch (nullable) replaces the context's
// per-stream scratch; it must hold v3db_commit_batch_scratch_bytes(jobs).
void free_batch_graphs(v3db_ctx *ctx);
// One Merkle tree of a batch: leaf k hashes row k of mat ([n_cols][2^log_leaves],
// column-major); the levels go to tree (leaves first, 2^(log_leaves+1) - 2^cap_height
// digests) and the 2^cap_height cap nodes to cap.
struct TreeJob {
  const uint64_t *mat;
  uint64_t *tree, *cap;
  uint32_t n_cols, log_leaves, cap_height;
};
// Every tree of jobs[0..n) at once: one leaf-hashing launch over all their rows, then one
// launch per tree depth over all the trees that still have that depth (batch.hip).
v3db_status enqueue_tree_batch(v3db_ctx *ctx, const TreeJob *jobs, size_t n, hipStream_t stream);
void free_tree_batch(v3db_ctx *ctx);
size_t fri_tree_digests(uint32_t log_n, uint32_t rounds, uint32_t cap_height);
v3db_status enqueue_fri_commit(v3db_ctx *ctx, const uint64_t *codeword, uint32_t log_n, uint64_t shift,
                               const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *folded,
                               uint64_t *trees, uint64_t *caps, uint64_t *scratch_tree, hipStream_t stream);
size_t grand_product_scratch_words(uint64_t n);
v3db_status enqueue_grand_product(v3db_ctx *ctx, const uint64_t *cols, uint32_t width, uint64_t n, uint64_t alpha,
                                  uint64_t beta, uint64_t *z, uint64_t *total, uint64_t *scratch, hipStream_t stream);
size_t snapshot_scratch_words(uint32_t log_lists, uint32_t log_slots);
v3db_status enqueue_snapshot(v3db_ctx *ctx, uint32_t log_lists, uint32_t log_slots, uint32_t m, uint32_t dim,
                             uint32_t k, const uint64_t *flag, const uint64_t *item, const uint64_t *codes,
                             const uint64_t *centroids, const uint64_t *codebooks, uint64_t *list_roots,
                             uint64_t *root_mk, uint64_t *root_cb, uint64_t *scratch, hipStream_t stream);
v3db_status enqueue_open(v3db_ctx *ctx, const uint64_t *lde, uint32_t n_cols, uint32_t log_leaves, const uint64_t *tree,
                         uint32_t cap_height, const uint64_t *idx, size_t n_q, uint64_t *rows, uint64_t *paths,
                         hipStream_t stream);
v3db_status enqueue_verify(v3db_ctx *ctx, const uint64_t *rows, uint32_t n_cols, uint32_t log_leaves,
                           uint32_t cap_height, const uint64_t *idx, size_t n_q, const uint64_t *paths,
                           const uint64_t *cap, uint32_t *ok, hipStream_t stream);
v3db_status commit_batch_impl(v3db_ctx *ctx, const v3db_commit_job *jobs, size_t n_jobs, hipStream_t stream,
                              void *scratch, size_t scratch_bytes);

// Poseidon work (poseidon.hip).
v3db_status enqueue_permute(v3db_ctx *ctx, uint64_t *states, size_t count, hipStream_t stream);
v3db_status enqueue_leaf_hash(v3db_ctx *ctx, const uint64_t *mat, uint32_t n_cols, uint32_t log_leaves,
                              uint64_t *digests, hipStream_t stream);
v3db_status enqueue_merkle_levels(v3db_ctx *ctx, uint64_t *tree, uint32_t log_leaves, uint32_t cap_height,
                                  uint64_t *cap, hipStream_t stream);

}  // namespace v3db
