/*
 * Reference oracle for the trace-commitment phase: coset low-degree extension
 * (LDE) of trace columns over the Goldilocks field, Poseidon row hashing, and a
 * Merkle tree with a cap.
 *
 * TEST INFRASTRUCTURE ONLY. This plain, slow CPU implementation exists to check
 * the GPU library. Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it. It shares no code, header, table or constant generator
 * with the GPU library.
 *
 * The paper ("V3DB", arXiv 2603.03065) names the pieces but not their parameters:
 *   - FFT-based polynomial operations over a power-of-two evaluation domain
 *     (§2.1, paragraph "Gate counts and proving time (binning effect)"; §5.2,
 *     paragraph "Metrics");
 *   - Hash = Poseidon and commitments are Merkle trees over a fixed-length
 *     canonical sequence of field elements (§4.3 "Snapshot Commitments");
 *   - MerkleOpen recomputes a root from a leaf and its sibling path by the bits
 *     of the leaf index (§4.4 "Snapshot-Binding Circuit");
 *   - the prover runs the default configuration of its proof backend (§5,
 *     paragraph "Evaluation environment").
 * The concrete parameters below are this project's fixed reading of that
 * unspecified default: the Goldilocks field p = 2^64 - 2^32 + 1, generator 7,
 * blowup 2^log_blowup on the coset s*<w_N>, width-12 x^7 Poseidon with 4 + 22 + 4
 * rounds, rate-8 overwrite sponge, 4-element digests, and round constants and a
 * circulant MDS matrix drawn from SplitMix64 with a stated seed.
 *
 * All values are uint64 in [0, p). Matrices are column-major: column c of a
 * matrix with R rows occupies elements [c*R, (c+1)*R).
 */
#ifndef V3DB_ORACLE_H
#define V3DB_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_P 0xffffffff00000001ULL
#define OR_WIDTH 12
#define OR_RATE 8
#define OR_DIGEST 4
#define OR_ROUNDS 30
#define OR_FULL_HALF 4

/* ---- field ---- */
uint64_t or_add(uint64_t a, uint64_t b);
uint64_t or_sub(uint64_t a, uint64_t b);
uint64_t or_mul(uint64_t a, uint64_t b);
uint64_t or_pow(uint64_t a, uint64_t e);
uint64_t or_inv(uint64_t a);                 /* a != 0 */
uint64_t or_root_of_unity(uint32_t log_n);   /* 7^((p-1)/2^log_n), log_n <= 32 */

/* ---- SplitMix64 (Steele, Lea, Flood 2014): output i of the stream with seed s ---- */
uint64_t or_splitmix64(uint64_t seed, uint64_t i);

/* ---- NTT: textbook iterative radix-2, natural order in and out ----
 * forward: X[k] = sum_j x[j] w^(jk), w = w_n; inverse: x[j] = n^-1 sum_k X[k] w^(-jk). */
void or_ntt(uint64_t *a, uint32_t log_n, int inverse);

/* ---- LDE ----
 * trace [n_cols][2^log_rows] -> lde [n_cols][2^(log_rows+log_blowup)].
 * c = iNTT(a); LDE[k] = sum_j c_j (shift * w_N^k)^j; layout 0 = natural
 * (out[k] = LDE[k]); layout 1 = bit-reversed (out[k] = LDE[rev_{log N}(k)]).
 * Returns 0 on success, -1 on invalid arguments. */
int or_lde(const uint64_t *trace, uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup,
           uint64_t shift, int layout, uint64_t *lde);
/* Interpolation only: coefficients c (natural order) of each column, [n_cols][2^log_rows]. */
int or_interpolate(const uint64_t *trace, uint32_t n_cols, uint32_t log_rows, uint64_t *coeffs);

/* Horner evaluation: out[c][i] = sum_j coeffs[c][j] * x[i]^j for each column c
 * of coeffs [n_cols][n] and each of the n_points points. */
void or_eval_columns(const uint64_t *coeffs, uint32_t n_cols, uint64_t n, const uint64_t *x,
                     uint32_t n_points, uint64_t *out);

/* ---- Poseidon (t = 12, x^7) ---- */
typedef struct {
  uint64_t seed;
  uint64_t rc[OR_ROUNDS][OR_WIDTH];   /* round constants, r-major */
  uint64_t circ[OR_WIDTH];            /* first row a_0..a_11 of the circulant: M[i][j] = a_{(j-i) mod 12} */
  uint64_t mds[OR_WIDTH][OR_WIDTH];   /* the full matrix, for reference */
  uint32_t mds_attempts;              /* number of 12-value draws until the matrix passed */
  uint64_t stream_next;               /* first stream index not consumed */
} or_poseidon_params;

/* Derive constants from seed. Returns 0, or -1 if no MDS draw passed. */
int or_poseidon_params_init(uint64_t seed, or_poseidon_params *out);
/* Number of singular square submatrices (all sizes 1..12) of a 12x12 matrix
 * over F_p. Every submatrix determinant is computed by Laplace expansion along
 * its first row, built up from all minors one size smaller. */
uint64_t or_singular_minor_count(const uint64_t m[OR_WIDTH][OR_WIDTH]);
/* Determinant of the full 12x12 matrix by the same expansion. */
uint64_t or_det12(const uint64_t m[OR_WIDTH][OR_WIDTH]);

void or_poseidon_permute(const or_poseidon_params *pp, uint64_t state[OR_WIDTH]);
void or_poseidon_permute_batch(const or_poseidon_params *pp, uint64_t *states, size_t count);

/* Sponge over one row of len elements: zero state, overwrite lanes 0..k-1 with
 * each chunk of up to 8 elements in order, permute after each chunk. The full
 * final state is returned; the digest is lanes 0..3. len = 0 gives the
 * all-zero state (no permutation). */
void or_sponge_state(const or_poseidon_params *pp, const uint64_t *row, uint32_t len,
                     uint64_t state[OR_WIDTH]);
/* Compress(L, R) = permute(L || R || 0^4); full state returned, digest lanes 0..3. */
void or_compress_state(const or_poseidon_params *pp, const uint64_t l[OR_DIGEST],
                       const uint64_t r[OR_DIGEST], uint64_t state[OR_WIDTH]);

/* ---- Merkle ----
 * Leaves: digest of each stored row of mat [n_cols][2^log_leaves] (row k = mat[c][k],
 * c = 0..n_cols-1). Tree levels from the leaves up to height cap_height:
 * tree = [2^L][4], [2^(L-1)][4], ..., [2^h][4] (nullable). cap = [2^h][4].
 * Returns 0, or -1 on invalid arguments. */
int or_merkle_commit(const or_poseidon_params *pp, const uint64_t *mat, uint32_t n_cols,
                     uint32_t log_leaves, uint32_t cap_height, uint64_t *tree, uint64_t *cap);
/* Leaf digests only: [2^log_leaves][4]. */
int or_leaf_digests(const or_poseidon_params *pp, const uint64_t *mat, uint32_t n_cols,
                    uint32_t log_leaves, uint64_t *digests);
/* Authentication path of leaf `index` in a stored tree: siblings from the leaf
 * level up to (excluding) the cap level: [(L - h)][4]. */
int or_merkle_path(const uint64_t *tree, uint32_t log_leaves, uint32_t cap_height, uint64_t index,
                   uint64_t *path);
/* MerkleOpen: fold a leaf digest with its path by the bits of index; returns the
 * cap node reached in node_out[4] and its index in the cap via *cap_index. */
void or_merkle_open(const or_poseidon_params *pp, const uint64_t leaf[OR_DIGEST], uint64_t index,
                    const uint64_t *path, uint32_t path_len, uint64_t node_out[OR_DIGEST],
                    uint64_t *cap_index);

/* Whole commit: LDE then leaf hashing then Merkle to the cap. lde, tree nullable.
 * Returns 0, or -1 on invalid arguments. */
int or_commit(const or_poseidon_params *pp, const uint64_t *trace, uint32_t n_cols,
              uint32_t log_rows, uint32_t log_blowup, uint64_t shift, int layout,
              uint32_t cap_height, uint64_t *lde, uint64_t *tree, uint64_t *cap);

/* ---- Snapshot commitment (Sec. 4.3 "Snapshot Commitments") ----
 * A fixed-shape IVF-PQ snapshot: n_list = 2^log_lists inverted lists of n = 2^log_slots
 * slots; slot (i, j) is record t = i*n + j with validity flag flag[t], payload item[t]
 * and M PQ codes codes[m*N + t] (N = n_list*n); centroid i is centroids[i*D .. i*D+D-1];
 * the codebooks C_{m,k} (m < M, k < K, each of D/M coordinates) are given in their
 * canonical flattening codebooks[(m*K + k)*(D/M) + c].
 *   hash_{i,j} = Hash(i, j, f_ij, item_ij, v_ij^(0), ..., v_ij^(M-1))
 *   root_i     = MerkleTree(hash_{i,0}, ..., hash_{i,n-1})
 *   hash_i     = Hash(i, mu_i[0..D-1], root_i)
 *   root_mk    = MerkleTree(hash_0, ..., hash_{n_list-1})
 *   root_cb    = Hash(C_{0,0}, ..., C_{M-1,K-1})
 * Hash is the rate-8 overwrite sponge (digest = lanes 0..3), MerkleTree the binary tree
 * of Compress to a single root. list_roots [n_list][4] and list_hashes [n_list][4] are
 * nullable outputs. Returns 0, or -1 on invalid arguments (M = 0, D not a multiple of M,
 * K = 0, log_lists + log_slots > 30). */
int or_snapshot_commit(const or_poseidon_params *pp, uint32_t log_lists, uint32_t log_slots, uint32_t m,
                       uint32_t dim, uint32_t k, const uint64_t *flag, const uint64_t *item,
                       const uint64_t *codes, const uint64_t *centroids, const uint64_t *codebooks,
                       uint64_t *list_roots, uint64_t *list_hashes, uint64_t root_mk[OR_DIGEST],
                       uint64_t root_cb[OR_DIGEST]);

/* ---- Multiset equality (Sec. 4.5 "Gadgets and Cost Model": tuple compression and SetEq) ----
 * Rows of a column-major table cols [width][n] (row i = (x_{0,i}, ..., x_{width-1,i})):
 *   c_i = Compress(row i; beta) = sum_k x_{k,i} beta^k   (Horner)
 *   z_i = prod_{j <= i} (alpha - c_j)
 * z [n] is nullable; *total receives z_{n-1} (1 when n = 0). Returns 0, or -1 on
 * invalid arguments (width = 0). */
int or_grand_product(const uint64_t *cols, uint32_t width, uint64_t n, uint64_t alpha, uint64_t beta,
                     uint64_t *z, uint64_t *total);

/* ---- FRI commit phase: the low-degree test of the paper's proving backend, which
 * Sec. 5 para. "Evaluation environment" runs with its default FRI parameters; the
 * arity-2 folding and pair-leaf commitment below are the standard commit phase ----
 * Round r = 0..rounds-1 holds the codeword f_r of length N_r = 2^(log_n - r) on the
 * coset D_r = { s_r w_{N_r}^k }, s_0 = shift, s_{r+1} = s_r^2, natural order.
 *   commit:  leaf k < N_r/2 = Hash(f_r[k], f_r[k + N_r/2]) (the two points x, -x of D_r);
 *            a Merkle tree of those N_r/2 leaves up to cap_height; caps [rounds][2^h][4]
 *   fold:    f_{r+1}[k] = (f_r[k] + f_r[k + N_r/2]) / 2
 *                         + beta_r (f_r[k] - f_r[k + N_r/2]) / (2 x_k),   x_k = s_r w_{N_r}^k
 * folded receives f_1, ..., f_rounds concatenated (2^log_n - 2^(log_n - rounds) words);
 * trees (nullable) the rounds' trees concatenated, each [N_r - 2^h][4].
 * Returns 0, or -1 on invalid arguments (rounds = 0, rounds + cap_height > log_n, shift = 0 mod p). */
int or_fri_commit(const or_poseidon_params *pp, const uint64_t *codeword, uint32_t log_n, uint64_t shift,
                  const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *folded, uint64_t *trees,
                  uint64_t *caps);

/* Threads used by the parallel loops (OpenMP); 0 leaves the default. Returns the count in use. */
int or_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
