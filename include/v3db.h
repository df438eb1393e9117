/*
 * v3db: trace commitment on AMD Instinct MI355X (gfx950).
 *
 * The commitment phase of proof generation in V3DB (arXiv 2603.03065): trace
 * columns are interpolated and extended onto a coset of a larger power-of-two
 * domain (the "FFT-based polynomial operations over a power-of-two evaluation
 * domain" of §2.1, paragraph "Gate counts and proving time (binning effect)"),
 * each extended row is hashed with Poseidon, and the row digests are committed
 * with a Merkle tree whose top levels form a cap (Hash = Poseidon and
 * commitments = Merkle trees over a fixed-length canonical sequence of field
 * elements, §4.3 "Snapshot Commitments"; authentication paths fold by the bits of
 * the leaf index, §4.4 "Snapshot-Binding Circuit").
 *
 * The paper names these pieces but not their parameters (its prover runs the
 * default configuration of its proof backend, §5 "Evaluation environment"). This
 * library fixes them as follows:
 *   field    Goldilocks, p = 2^64 - 2^32 + 1; roots w_{2^k} = 7^((p-1)/2^k)
 *   LDE      c = iNTT_n(a) (a_i = P(w_n^i)); LDE[k] = P(shift * w_N^k), N = n << log_blowup
 *   hash     width-12 Poseidon, S-box x^7, rounds 4 full + 22 partial + 4 full,
 *            each round = add round constants (all lanes), S-box, multiply by a
 *            12x12 circulant MDS matrix M[i][j] = a[(j - i) mod 12]
 *   constants  SplitMix64 stream with the context's seed: accepted outputs z < p
 *            fill the 360 round constants round-major; then a[j] = 1 + (z mod 255)
 *            for the next 12 outputs, redrawn until every square submatrix of M
 *            is nonsingular mod p
 *   sponge   zero state; each chunk of up to 8 row elements (columns in order)
 *            overwrites lanes 0..k-1, then permute; digest = lanes 0..3
 *   node     Compress(L, R) = permute(L || R || 0,0,0,0) lanes 0..3
 *   tree     leaves = digests of the stored rows; left child = even index
 *
 * Conventions for every call:
 *   - All data pointers are device pointers unless stated otherwise. Field
 *     elements are uint64 and must be canonical (< p); outputs are canonical.
 *   - Matrices are column-major: column c of an R-row matrix is elements
 *     [c*R, (c+1)*R). Digests are [count][4] row-major.
 *   - The caller owns every buffer. Calls validate arguments on the host, enqueue
 *     work on `stream` (a hipStream_t; NULL = the default stream) and return;
 *     buffers must stay alive until the stream reaches that point.
 *   - A context is used from one host thread at a time; a server owns its context
 *     while it runs (it calls it from its scheduler thread). Scratch is kept per
 *     stream, so calls on different streams may overlap.
 *   - Errors are returned as v3db_status; v3db_last_error() gives a message for
 *     the last failing call on the calling thread. No exception crosses the ABI.
 */
#ifndef V3DB_H
#define V3DB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct v3db_ctx v3db_ctx;
typedef struct v3db_server v3db_server;
typedef void *v3db_stream; /* a hipStream_t */

typedef enum {
  V3DB_OK = 0,
  V3DB_ERR_INVALID_ARG = 1,   /* NULL pointer, zero columns, cap_height > log_leaves, shift 0 or >= p, ... */
  V3DB_ERR_UNSUPPORTED = 2,   /* sizes beyond the build limits below */
  V3DB_ERR_NONCANONICAL = 3,  /* an input element >= p (checked only when validation is on) */
  V3DB_ERR_OUT_OF_MEMORY = 4, /* device allocation failed or the context's HBM budget would be exceeded */
  V3DB_ERR_DEVICE = 5,        /* a HIP runtime error */
  V3DB_ERR_BUSY = 6           /* server: request queue full */
} v3db_status;

typedef enum { V3DB_LAYOUT_NATURAL = 0, V3DB_LAYOUT_BITREV = 1 } v3db_layout;

/* Build limits. */
#define V3DB_MAX_LOG_ROWS 24    /* trace rows per column: 2^0 .. 2^24 */
#define V3DB_MAX_LOG_BLOWUP 4   /* blowup 2^0 .. 2^4 */
#define V3DB_MAX_LOG_LDE 26     /* log_rows + log_blowup <= 26 */
#define V3DB_MAX_COLS 65535

/* Create a context on HIP device `device`: derives the Poseidon constants from
 * `poseidon_seed` (as described above; the project's seed is 260303065), builds
 * the twiddle tables and uploads both (they stay resident until destroy).
 * `hbm_budget_bytes` caps the device memory the context itself may allocate for
 * scratch and pooled buffers (0 = no cap). On success *out owns the context. */
v3db_status v3db_ctx_create(int device, uint64_t poseidon_seed, size_t hbm_budget_bytes, v3db_ctx **out);
void v3db_ctx_destroy(v3db_ctx *ctx);

/* Message for the last non-OK status returned on this thread ("" if none). The
 * string stays valid until the next call on this thread. */
const char *v3db_last_error(void);

/* Sixteen hex digits identifying the sources this library was built from (a SHA-256
 * prefix over the HIP/C++ sources and this header, fixed at build time), so a loader can
 * refuse a library built from other sources than it was given. Static string; no
 * device work, no context needed. */
const char *v3db_build_digest(void);

/* Host copies of the derived Poseidon constants: rc [30][12], circ [12] (first
 * row of the circulant) and the number of 12-value draws the MDS search took.
 * Any output pointer may be NULL. */
v3db_status v3db_poseidon_constants(const v3db_ctx *ctx, uint64_t *rc_out, uint64_t *circ_out,
                                    uint32_t *attempts_out);

/* Which form the context's bulk hashing kernels (leaf rows, tree levels of more
 * than 2^15 nodes, batch phases, snapshot records) use for the permutation's
 * linear layer (the circulant product of the hash fixed above); both give
 * identical results, the arithmetic being exact.
 *   1  int8 matrix cores (the default: each circulant entry C, 1..255, is held
 *      as the signed byte C - 128);
 *   0  VALU multiply-adds: the environment variable V3DB_POSEIDON_VALU was set
 *      to a non-zero value when the context was made;
 *  -1  ctx is NULL.
 * The single-permutation call, openings, tree tops and the FRI fold are the same
 * either way. */
int v3db_ctx_hash_path(const v3db_ctx *ctx);

/* Host only (no device, no context): the constants a context created with
 * `poseidon_seed` uses, as in v3db_poseidon_constants. Takes about a second the
 * first time per seed in a process (the exhaustive submatrix check). Returns
 * UNSUPPORTED if no draw passes within 1000 attempts. */
v3db_status v3db_derive_poseidon_constants(uint64_t poseidon_seed, uint64_t *rc_out, uint64_t *circ_out,
                                           uint32_t *attempts_out);

/* Coset low-degree extension.
 * d_trace [n_cols][2^log_rows] -> d_lde [n_cols][2^(log_rows+log_blowup)].
 * Column by column: c = iNTT(a), then LDE[k] = sum_j c_j (shift * w_N^k)^j.
 * layout NATURAL stores out[k] = LDE[k]; BITREV stores out[k] = LDE[rev(k)],
 * rev reversing log2(N) bits. d_trace and d_lde must not overlap. The context's
 * scratch (at most 2^(log_rows+log_blowup+3) * min(n_cols, 8) bytes, pooled) is used.
 * Errors: INVALID_ARG (NULL, n_cols == 0, shift == 0 or >= p, bad layout),
 * UNSUPPORTED (beyond the limits above), OUT_OF_MEMORY, DEVICE. */
v3db_status v3db_lde(v3db_ctx *ctx, const uint64_t *d_trace, uint32_t n_cols, uint32_t log_rows,
                     uint32_t log_blowup, uint64_t shift, v3db_layout layout, uint64_t *d_lde,
                     v3db_stream stream);

/* Poseidon permutation in place on `count` states, row-major [count][12].
 * Inputs canonical; outputs canonical. count == 0 is a no-op. */
v3db_status v3db_poseidon_permute(v3db_ctx *ctx, uint64_t *d_states, size_t count, v3db_stream stream);

/* Merkle commitment of the rows of a column-major matrix.
 * Leaves: digest of row k of d_mat [n_cols][2^log_leaves] (elements d_mat[c][k],
 * c = 0..n_cols-1, by the sponge above). Levels are built up to height
 * cap_height; the cap is the 2^cap_height nodes of that level.
 * d_tree (nullable) receives every level, leaves first:
 *   [2^L][4], [2^(L-1)][4], ..., [2^h][4]   ((2^(L+1) - 2^h) digests in all).
 * d_cap receives [2^h][4] (device memory). When d_tree is NULL, scratch from the
 * context holds the levels.
 * Errors: INVALID_ARG (NULL d_mat/d_cap, n_cols == 0, cap_height > log_leaves),
 * UNSUPPORTED (log_leaves > 26), OUT_OF_MEMORY, DEVICE. */
v3db_status v3db_merkle_commit(v3db_ctx *ctx, const uint64_t *d_mat, uint32_t n_cols, uint32_t log_leaves,
                               uint32_t cap_height, uint64_t *d_tree, uint64_t *d_cap, v3db_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): v3db_merkle_commit with d_tree NULL,
 * the tree levels held in a static device array of V3DB_NOALLOC_SCRATCH_BYTES instead of
 * the context's pooled scratch. Nothing is allocated and nothing is freed by the call;
 * the array exists on each device the library runs on until the process ends, and its
 * device address is looked up once per device at v3db_ctx_create. It holds at most
 * 2^20 leaves ((2^(log_leaves+1) - 2^cap_height) * 32 bytes <= 64 MiB). Every call on a
 * device shares that device's array: calls that overlap on one device (on other streams
 * or from other threads) race and must be ordered by the caller; the array keeps the
 * last call's levels. No input validation pass runs (V3DB_VALIDATE is not honoured).
 * d_mat [n_cols][2^log_leaves] device, column-major; d_cap [2^cap_height][4] device.
 * Errors: INVALID_ARG (NULL ctx/d_mat/d_cap, n_cols == 0, cap_height > log_leaves),
 * UNSUPPORTED (beyond the build limits or the static scratch), DEVICE. */
#define V3DB_NOALLOC_SCRATCH_BYTES (64u << 20)
v3db_status v3db_merkle_commit_noalloc(v3db_ctx *ctx, const uint64_t *d_mat, uint32_t n_cols, uint32_t log_leaves,
                                       uint32_t cap_height, uint64_t *d_cap, v3db_stream stream);

/* One commit job: LDE of the trace, leaf hashing, Merkle tree up to the cap. */
typedef struct {
  const uint64_t *d_trace; /* [n_cols][2^log_rows], device */
  uint32_t n_cols, log_rows, log_blowup, cap_height;
  uint64_t shift;
  v3db_layout layout;
  uint64_t *d_lde;  /* [n_cols][2^(log_rows+log_blowup)] or NULL: pooled scratch, released after the call's work */
  uint64_t *d_tree; /* whole tree as in v3db_merkle_commit, or NULL: only the cap is kept */
  uint64_t *d_cap;  /* [2^cap_height][4], device; required */
} v3db_commit_job;

/* Commit many independent traces of different shapes: the proof backend answers
 * challenges on demand (§3.1, paragraph "Proving backend (online/audit)"), so many
 * proofs, hence many trace commitments (comm = MerkleTree over Hash = Poseidon of
 * the extended rows, §4.3 "Snapshot Commitments"), are in flight at once.
 * Natural-layout jobs are committed together, phase by phase: every phase (each
 * extension pass, leaf hashing, each tree depth) runs as one launch over the work of
 * all jobs, so small traces share the GPU. A list of shapes seen for the first time
 * (per stream) is launched directly; from its second call on, its launch sequence is
 * captured once as a HIP graph and replayed, and only a small table of buffer
 * pointers is uploaded per call. Bit-reversed jobs are committed one at a time.
 * Scratch for NULL d_lde/d_tree comes from the context (per stream) and counts
 * against its HBM budget. Results are identical to committing each job alone.
 * jobs is a host array of n_jobs descriptors (read during the call only); every
 * buffer in it is the caller's and must stay alive until the stream reaches this
 * point. Errors: as v3db_lde / v3db_merkle_commit for any job (checked before
 * anything is enqueued), OUT_OF_MEMORY if the scratch does not fit. */
v3db_status v3db_commit_batch(v3db_ctx *ctx, const v3db_commit_job *jobs, size_t n_jobs, v3db_stream stream);

/* Phase timing. While enabled, commit calls record HIP events on their stream
 * around each phase: V3DB_PHASE_LDE (all extension passes), V3DB_PHASE_LEAF
 * (row hashing) and V3DB_PHASE_MERKLE (tree levels and cap) for traces
 * committed one at a time, V3DB_PHASE_BATCH around each batched group.
 * v3db_profile_read waits for the recorded events, adds each phase's elapsed
 * milliseconds and count of timed intervals into ms_out[4] / count_out[4] (either may be NULL)
 * and forgets them. Enabling or disabling also forgets pending records. */
#define V3DB_PHASES 4
#define V3DB_PHASE_LDE 0
#define V3DB_PHASE_LEAF 1
#define V3DB_PHASE_MERKLE 2
#define V3DB_PHASE_BATCH 3  /* a whole batched group (all its phases) */
v3db_status v3db_profile_enable(v3db_ctx *ctx, int on);
v3db_status v3db_profile_read(v3db_ctx *ctx, double *ms_out, uint64_t *count_out);

/* Context options.
 * V3DB_OPT_BATCHING (default 1): 0 commits every job of v3db_commit_batch one at a
 *   time with the single-trace kernels (one launch sequence per trace) instead of
 *   the batched phase launches; results are identical either way.
 * V3DB_OPT_BATCH_GROUP_BYTES (default 32 GiB): natural-layout jobs are batched in
 *   groups whose scratch (Y, plus LDE and tree when not given) stays below this. */
typedef enum { V3DB_OPT_BATCHING = 0, V3DB_OPT_BATCH_GROUP_BYTES = 1 } v3db_option;
v3db_status v3db_set_option(v3db_ctx *ctx, v3db_option opt, uint64_t value);

/* ---------------------------------------------------------------- openings
 * Audit on demand: after a commitment the prover answers challenged leaf indices
 * with the committed rows and their Merkle authentication paths, and the verifier
 * recomputes the cap entry from each (MerkleOpen, Sec. 4.4: walk from the leaf to
 * the top, taking the node as left or right child by the bits of the index).
 *
 * v3db_open_batch gathers, for each of n_queries indices idx[q] (device array,
 * each < 2^log_leaves):
 *   d_rows  [n_queries][n_cols]: row idx[q] of the stored matrix d_mat
 *           (column-major [n_cols][1 << log_leaves], the LDE as committed);
 *   d_paths [n_queries][log_leaves - cap_height][4]: for level l = 0 (leaves) ..
 *           log_leaves - cap_height - 1, the sibling of the node above leaf idx[q]
 *           at that level, read from d_tree (the stored tree of v3db_merkle_commit
 *           or v3db_commit_batch: [(2 << log_leaves) - (1 << cap_height)][4]).
 * All pointers are device memory owned by the caller; d_paths may be NULL when
 * log_leaves == cap_height. An index >= 2^log_leaves is a caller error: with
 * V3DB_VALIDATE=1 it fails with INVALID_ARG before anything is enqueued,
 * otherwise the index is taken modulo 2^log_leaves (nothing is read out of
 * bounds). n_queries == 0 does nothing. Errors: INVALID_ARG (NULL pointer,
 * n_cols == 0, cap_height > log_leaves), UNSUPPORTED (log_leaves > 26 or
 * n_cols > 65535), DEVICE. */
v3db_status v3db_open_batch(v3db_ctx *ctx, const uint64_t *d_mat, uint32_t n_cols, uint32_t log_leaves,
                            const uint64_t *d_tree, uint32_t cap_height, const uint64_t *d_idx, size_t n_queries,
                            uint64_t *d_rows, uint64_t *d_paths, v3db_stream stream);

/* The verifier's side, batched: d_ok[q] = 1 if hashing row q (the rate-8 sponge of
 * the commitment) and compressing up its path (layouts as v3db_open_batch) gives
 * entry idx[q] >> (log_leaves - cap_height) of d_cap ([1 << cap_height][4]),
 * else 0. Rows and paths may be any 64-bit words (a non-canonical word is treated
 * as its residue, so a tampered opening fails only if it changes the value mod p);
 * indices as v3db_open_batch. Errors as v3db_open_batch. */
v3db_status v3db_verify_batch(v3db_ctx *ctx, const uint64_t *d_rows, uint32_t n_cols, uint32_t log_leaves,
                              uint32_t cap_height, const uint64_t *d_idx, size_t n_queries, const uint64_t *d_paths,
                              const uint64_t *d_cap, uint32_t *d_ok, v3db_stream stream);

/* ---------------------------------------------------------------- snapshot commitment
 * The commitment comm = (root_mk, root_cb) of a fixed-shape IVF-PQ snapshot
 * (Sec. 4.3 "Snapshot Commitments"): n_list = 2^log_lists inverted lists of
 * n = 2^log_slots slots; record t = i*n + j (list i, slot j) has a validity flag,
 * a payload and M PQ codes; each list has a D-dimensional centroid; the codebooks
 * hold M x K vectors of D/M coordinates.
 *   hash_{i,j} = Hash(i, j, flag_t, item_t, codes_t^(0), ..., codes_t^(M-1))
 *   root_i     = MerkleTree(hash_{i,0}, ..., hash_{i,n-1})
 *   hash_i     = Hash(i, centroid_i[0..D-1], root_i)
 *   root_mk    = MerkleTree(hash_0, ..., hash_{n_list-1})
 *   root_cb    = Hash(C_{0,0}, ..., C_{0,K-1}, C_{1,0}, ..., C_{M-1,K-1})
 * Hash is the rate-8 overwrite sponge of the trace commitment (4-word digest),
 * MerkleTree the same binary tree of Compress, down to one root. All arrays are
 * device memory in the caller's ownership (u64 words, canonical field elements): */
typedef struct {
  uint32_t log_lists, log_slots;   /* n_list = 2^log_lists, n = 2^log_slots; sum <= 26 */
  uint32_t m;                      /* PQ codes per record, >= 1 */
  uint32_t dim;                    /* D, centroid dimension, a multiple of m */
  uint32_t k;                      /* codebook size K, >= 1 */
  const uint64_t *d_flag;          /* [N] validity flags, N = n_list * n, record order */
  const uint64_t *d_item;          /* [N] payloads */
  const uint64_t *d_codes;         /* [m][N] codes, one array per sub-quantizer */
  const uint64_t *d_centroids;     /* [n_list][dim] */
  const uint64_t *d_codebooks;     /* [m][k][dim/m], the canonical flattening */
} v3db_snapshot;

/* Enqueue the commitment on the stream: d_root_mk [4] and d_root_cb [4] receive
 * the two roots, d_list_roots [n_list][4] (nullable) the list roots. The
 * codebook digest is a sequential chain of K*D/8 permutations; it runs on an
 * internal stream that waits for the caller's stream at the call and is waited
 * for by it before anything enqueued later, so stream order is kept. Scratch:
 * (3 n_list - 1 + 2N - n_list) digests from the context. Errors: INVALID_ARG (NULL
 * pointer, m = 0, k = 0, dim not a multiple of m), UNSUPPORTED (log_lists +
 * log_slots > 26, m > 65535, k * dim >= 2^32), NONCANONICAL (with V3DB_VALIDATE=1),
 * OUT_OF_MEMORY, DEVICE. */
v3db_status v3db_snapshot_commit(v3db_ctx *ctx, const v3db_snapshot *snap, uint64_t *d_list_roots,
                                 uint64_t *d_root_mk, uint64_t *d_root_cb, v3db_stream stream);

/* ---------------------------------------------------------------- multiset equality
 * The grand product behind a multiset-equality check (Sec. 4.5 "Gadgets and Cost
 * Model": tuple compression with a challenge beta, then SetEq compares
 * prod (alpha - x_i) of two sequences). For the n rows of a column-major table
 * d_cols [width][n] (row i = (x_{0,i}, ..., x_{width-1,i}), canonical words):
 *   c_i = sum_k x_{k,i} beta^k,   z_i = prod_{j <= i} (alpha - c_j)  (mod p).
 * d_z [n] (nullable) receives the running products, d_total [1] the last one
 * (1 when n = 0); alpha and beta are reduced mod p. Scratch: 2 words per 4096 rows
 * from the context. Errors: INVALID_ARG (NULL pointer, width = 0), UNSUPPORTED
 * (width > 65535 or n >= 2^40), NONCANONICAL (V3DB_VALIDATE=1), DEVICE. */
v3db_status v3db_grand_product(v3db_ctx *ctx, const uint64_t *d_cols, uint32_t width, uint64_t n, uint64_t alpha,
                               uint64_t beta, uint64_t *d_z, uint64_t *d_total, v3db_stream stream);

/* ---------------------------------------------------------------- FRI commit phase
 * The low-degree test of the proving backend (Sec. 5 para. "Evaluation environment":
 * the backend's default FRI parameters), commit phase with arity 2. Round
 * r = 0..rounds-1 holds the codeword f_r of N_r = 2^(log_n - r) values on the coset
 * { s_r w_{N_r}^k } (s_0 = shift, s_{r+1} = s_r^2, natural order; f_0 = d_codeword):
 *   commit:  leaf k < N_r/2 = Hash(f_r[k], f_r[k + N_r/2]) (the points x and -x), a
 *            Merkle tree of those leaves up to cap_height, cap r -> d_caps[r]
 *   fold:    f_{r+1}[k] = (f_r[k] + f_r[k + N_r/2])/2 + beta_r (f_r[k] - f_r[k + N_r/2])/(2 x_k)
 * betas: host array [rounds], the challenges (reduced mod p).
 * d_folded: device [2^log_n - 2^(log_n - rounds)] receives f_1 .. f_rounds concatenated.
 * d_trees:  device, nullable, receives the rounds' trees concatenated (round r:
 *           [N_r - 2^cap_height][4], leaves first); when NULL a context scratch tree
 *           is used per round. d_caps: device [rounds][2^cap_height][4].
 * Errors: INVALID_ARG (NULL pointer, rounds = 0, rounds + cap_height > log_n,
 * shift = 0 mod p), UNSUPPORTED (log_n > 26), NONCANONICAL (V3DB_VALIDATE=1),
 * OUT_OF_MEMORY, DEVICE. */
v3db_status v3db_fri_commit(v3db_ctx *ctx, const uint64_t *d_codeword, uint32_t log_n, uint64_t shift,
                            const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *d_folded,
                            uint64_t *d_trees, uint64_t *d_caps, v3db_stream stream);

/* ---------------------------------------------------------------- schedules
 * How the extension of one shape (log_rows, log_blowup) is cut into kernels. The
 * size-n transforms (the FFT-based polynomial operations of Sec. 2.1 para. "Gate
 * counts and proving time") are computed four-step, n = n1 * n2, a choice of this
 * library: pass 1 runs inverse size-n1 sub-transforms in tiles of 2^t1 columns,
 * pass 2i the inverse size-n2 transforms in tiles of up to 16 rows, pass 2 the
 * forward size-(B n2) transforms in tiles of 2^t2 rows, pass 3 the forward size-n1
 * transforms in tiles of 2^t3 columns; the single-trace path runs passes 2 and 3
 * over chunk_cols columns at a time. A schedule never changes
 * results, only speed. Every context starts with a default schedule for each shape;
 * v3db_autotune_lde times candidates on the device and installs the fastest.
 *   split_log   log2 n2: n1 = 2^(log_rows - split_log) <= 4096, n2 <= 4096,
 *               split_log + log_blowup <= 14
 *   tile_cap[k] upper bound on log2 of pass k+1's tile height, 0..4 (the height is
 *               also bounded by LDS: 2^t * M <= 8192 words for transform length M)
 *   chunk_cols  1..16
 *   time_us     the extension's measured time when the schedule was tuned (0 if
 *               never timed); informational. */
typedef struct {
  uint32_t log_rows, log_blowup;
  uint32_t split_log;
  uint32_t tile_cap[3];
  uint32_t chunk_cols;
  double time_us;
} v3db_schedule;

/* Time candidate schedules for one shape and install the fastest in the context
 * (coordinate search from the current default: the split, each pass's tile cap,
 * the column chunk). Runs an LDE of n_cols synthetic columns in the given layout
 * several times per candidate on a private stream, allocating its buffers from the
 * context budget for the duration of the call; blocks until done. The context's
 * cached tables and batched graphs for the shape are dropped. out may be NULL.
 * Errors: INVALID_ARG / UNSUPPORTED for shapes v3db_lde rejects, OUT_OF_MEMORY,
 * HIP. Must not overlap any other call on the context (it waits for the device). */
v3db_status v3db_autotune_lde(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint32_t n_cols,
                              v3db_layout layout, v3db_schedule *out);

/* The schedule the context uses for a shape (the default one if none was set). */
v3db_status v3db_get_schedule(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, v3db_schedule *out);

/* Install a schedule for (s->log_rows, s->log_blowup); INVALID_ARG if it breaks
 * the bounds above. Drops the shape's cached tables and the batched graphs, so
 * it waits for the device first. */
v3db_status v3db_set_schedule(v3db_ctx *ctx, const v3db_schedule *s);

/* Save every installed (set or tuned) schedule as text, one line per shape:
 *   "v3db-schedule <log_rows> <log_blowup> <split_log> <cap1> <cap2> <cap3> <chunk> <time_us>"
 * and load such a file back (lines that do not start with "v3db-schedule" are
 * ignored; a malformed or out-of-bounds schedule line fails the load with
 * INVALID_ARG, leaving the schedules installed before it in place). The count of
 * schedules written / read goes to *count (may be NULL). IO errors: INVALID_ARG. */
v3db_status v3db_schedules_save(v3db_ctx *ctx, const char *path, size_t *count);
v3db_status v3db_schedules_load(v3db_ctx *ctx, const char *path, size_t *count);

/* Device bytes of scratch a batch of jobs needs beyond the caller's buffers. */
size_t v3db_commit_batch_scratch_bytes(const v3db_commit_job *jobs, size_t n_jobs);

/* ---------------------------------------------------------------- serving
 * An audit-on-demand commit server (§3.1, paragraph "Proving backend (online/audit)":
 * proofs are produced when a returned result is challenged, so commitment work
 * arrives as requests at any time; each request is one trace commitment as in §4.3).
 * Requests (host traces) arrive at any time; a scheduler thread admits them in
 * arrival order whenever a slot (a stream) and enough of the server's HBM budget are
 * free, as many as fit into one batch, and runs each batch on its slot stream: trace
 * upload, one v3db_commit_batch, cap download. Batches on different slots overlap on
 * the device; a request that arrives while others run is admitted as soon as a slot
 * and memory free up. All request buffers (trace, LDE, tree, cap) and batch scratch
 * live in one device arena of the budget's size, reserved at creation and kept
 * resident; a request is admitted when its buffers fit in the arena.
 * Requests carry host traces and receive host caps (v3db_request) rather than device
 * job descriptors: the server owns where a request's device buffers live (its arena,
 * which is what admission by HBM budget manages), and a request's latency runs from its
 * arrival to its cap on the host, the trace upload included. */
typedef struct {
  uint32_t slots;             /* batches in flight at once (streams), >= 1 */
  uint32_t max_batch;         /* requests per batch, 0 = no limit */
  uint32_t max_queue;         /* queued requests before submit returns BUSY, 0 = no limit */
  size_t hbm_budget_bytes;    /* device memory for request buffers: trace, LDE, tree, Y scratch */
  double sim_ns_per_element;  /* > 0: no device work, each batch "runs" for this many ns per
                                 LDE element (tests of the scheduler without a GPU; ctx may be NULL) */
} v3db_server_cfg;

#define V3DB_REQ_FAIL_INJECT 1u /* test hook: the request fails at admission, others are unaffected */

typedef struct {
  const uint64_t *h_trace;    /* host [n_cols][2^log_rows], canonical; pinned memory lets the upload
                                 overlap; must stay valid until the request is done */
  uint32_t n_cols, log_rows, log_blowup, cap_height;
  uint64_t shift;
  uint64_t *h_cap;            /* host [2^cap_height][4], written when the request is done */
  double t_arrive;            /* arrival stamp on v3db_clock(); < 0 means "now" */
  uint32_t flags;
} v3db_request;

typedef struct {
  double t_arrive, t_admit, t_done; /* v3db_clock() seconds; latency = t_done - t_arrive */
  uint32_t batch_size;              /* requests in the batch it ran in */
  uint32_t slot;
  /* device time of its batch (trace upload to cap download) in seconds since the server
   * was created, from events on the slot's stream; -1 when not measured (simulated
   * executor, failed batch) */
  double t_dev_start, t_dev_end;
} v3db_request_timing;

typedef struct {
  uint64_t submitted, completed, failed, batches;
  size_t hbm_in_use, hbm_peak;      /* bytes of admitted requests now / at most */
  size_t pool_bytes;                /* device memory held by the server (its arena: the budget) */
} v3db_server_stats;

/* Seconds on a monotonic clock (the one request stamps use). */
double v3db_clock(void);
/* ctx may be NULL only when cfg->sim_ns_per_element > 0. Errors: INVALID_ARG. */
v3db_status v3db_server_create(v3db_ctx *ctx, const v3db_server_cfg *cfg, v3db_server **out);
/* Queue a request; *ticket identifies it. Errors: INVALID_ARG / UNSUPPORTED (as for a
 * commit job), OUT_OF_MEMORY (its buffers alone exceed the budget), BUSY (queue full). */
v3db_status v3db_server_submit(v3db_server *srv, const v3db_request *req, uint64_t *ticket);
/* *done = 1 once the request finished (its h_cap written, or an error in *status);
 * a finished ticket is forgotten after this call reports it. */
v3db_status v3db_server_poll(v3db_server *srv, uint64_t ticket, int *done, v3db_status *status,
                             v3db_request_timing *timing);
/* Block until every request submitted so far has finished. */
v3db_status v3db_server_drain(v3db_server *srv);
v3db_status v3db_server_stats_get(v3db_server *srv, v3db_server_stats *out);
/* Drains, stops the scheduler and frees the pool. */
void v3db_server_destroy(v3db_server *srv);

#ifdef __cplusplus
}
#endif
#endif
