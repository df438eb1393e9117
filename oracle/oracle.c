/*
 * Reference oracle for the trace-commitment phase (LDE + Poseidon + Merkle cap).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow and written to be checked by eye. Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code with the GPU library. Field arithmetic is the plain
 * definition: a 128-bit product reduced with the '%' operator, no special-form
 * reduction. The passages followed are listed in oracle.h.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ field */

uint64_t or_add(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a + b) % OR_P); }
uint64_t or_sub(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a + OR_P - (b % OR_P)) % OR_P); }
uint64_t or_mul(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) % OR_P); }

uint64_t or_pow(uint64_t a, uint64_t e) {
  uint64_t r = 1, b = a % OR_P;
  while (e) {
    if (e & 1) r = or_mul(r, b);
    b = or_mul(b, b);
    e >>= 1;
  }
  return r;
}

/* Fermat: a^(p-2) = a^-1 for a != 0. */
uint64_t or_inv(uint64_t a) { return or_pow(a, OR_P - 2); }

/* 7 generates the multiplicative group; (p-1) = 2^32 * 3 * 5 * 17 * 257 * 65537,
 * so 7^((p-1)/2^k) has order exactly 2^k. */
uint64_t or_root_of_unity(uint32_t log_n) {
  if (log_n > 32) return 0;
  return or_pow(7, (OR_P - 1) >> log_n);
}

/* --------------------------------------------------------------- SplitMix64 */

/* Output i (0-based) of SplitMix64 started at `seed`: the state advances by the
 * golden-ratio increment before each output, then the 64-bit finaliser mixes it. */
uint64_t or_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* -------------------------------------------------------------------- NTT */

static uint64_t bit_reverse(uint64_t x, uint32_t bits) {
  uint64_t r = 0;
  for (uint32_t b = 0; b < bits; b++) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

void or_ntt(uint64_t *a, uint32_t log_n, int inverse) {
  uint64_t n = 1ULL << log_n;
  /* bit-reversal permutation, then Cooley-Tukey decimation-in-time stages */
  for (uint64_t i = 0; i < n; i++) {
    uint64_t j = bit_reverse(i, log_n);
    if (i < j) {
      uint64_t t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
  for (uint32_t s = 1; s <= log_n; s++) {
    uint64_t len = 1ULL << s, half = len >> 1;
    uint64_t wlen = or_root_of_unity(s);
    if (inverse) wlen = or_inv(wlen);
    for (uint64_t i = 0; i < n; i += len) {
      uint64_t w = 1;
      for (uint64_t j = 0; j < half; j++) {
        uint64_t u = a[i + j];
        uint64_t v = or_mul(a[i + j + half], w);
        a[i + j] = or_add(u, v);
        a[i + j + half] = or_sub(u, v);
        w = or_mul(w, wlen);
      }
    }
  }
  if (inverse) {
    uint64_t ninv = or_inv(n % OR_P);
    for (uint64_t i = 0; i < n; i++) a[i] = or_mul(a[i], ninv);
  }
}

/* -------------------------------------------------------------------- LDE */

static int lde_args_ok(const void *in, uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup,
                       uint64_t shift, const void *out) {
  if (!in || !out || n_cols == 0) return 0;
  if (log_rows + log_blowup > 32) return 0;
  if (shift == 0 || shift >= OR_P) return 0;
  return 1;
}

int or_interpolate(const uint64_t *trace, uint32_t n_cols, uint32_t log_rows, uint64_t *coeffs) {
  if (!trace || !coeffs || n_cols == 0 || log_rows > 32) return -1;
  uint64_t n = 1ULL << log_rows;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < (int64_t)n_cols; c++) {
    memcpy(coeffs + (uint64_t)c * n, trace + (uint64_t)c * n, n * sizeof(uint64_t));
    or_ntt(coeffs + (uint64_t)c * n, log_rows, 1);
  }
  return 0;
}

int or_lde(const uint64_t *trace, uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup,
           uint64_t shift, int layout, uint64_t *lde) {
  if (!lde_args_ok(trace, n_cols, log_rows, log_blowup, shift, lde)) return -1;
  if (layout != 0 && layout != 1) return -1;
  uint32_t log_N = log_rows + log_blowup;
  uint64_t n = 1ULL << log_rows, N = 1ULL << log_N;
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < (int64_t)n_cols; c++) {
    const uint64_t *a = trace + (uint64_t)c * n;
    uint64_t *out = lde + (uint64_t)c * N;
    uint64_t *buf = (uint64_t *)calloc(N, sizeof(uint64_t));
    if (!buf) {
      failed = 1;
      continue;
    }
    /* interpolate: coefficients of the degree < n polynomial through (w_n^i, a_i) */
    memcpy(buf, a, n * sizeof(uint64_t));
    or_ntt(buf, log_rows, 1);
    /* c_j * s^j, zero-padded to N: P(s x) has these coefficients */
    uint64_t sj = 1;
    for (uint64_t j = 0; j < n; j++) {
      buf[j] = or_mul(buf[j], sj);
      sj = or_mul(sj, shift);
    }
    /* evaluate on <w_N>: LDE[k] = P(s w_N^k) */
    or_ntt(buf, log_N, 0);
    if (layout == 0) {
      memcpy(out, buf, N * sizeof(uint64_t));
    } else {
      for (uint64_t k = 0; k < N; k++) out[k] = buf[bit_reverse(k, log_N)];
    }
    free(buf);
  }
  return failed ? -1 : 0;
}

void or_eval_columns(const uint64_t *coeffs, uint32_t n_cols, uint64_t n, const uint64_t *x,
                     uint32_t n_points, uint64_t *out) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int64_t c = 0; c < (int64_t)n_cols; c++) {
    for (int64_t i = 0; i < (int64_t)n_points; i++) {
      const uint64_t *cf = coeffs + (uint64_t)c * n;
      uint64_t acc = 0;
      for (uint64_t j = n; j-- > 0;) acc = or_add(or_mul(acc, x[i]), cf[j]);
      out[(uint64_t)c * n_points + (uint64_t)i] = acc;
    }
  }
}

/* --------------------------------------------------------------- Poseidon */

/* Index of each 12-bit mask among the masks of the same popcount, in increasing order. */
static void subset_ranks(uint32_t rank[1 << OR_WIDTH], uint32_t count[OR_WIDTH + 1]) {
  memset(count, 0, sizeof(uint32_t) * (OR_WIDTH + 1));
  for (uint32_t m = 0; m < (1u << OR_WIDTH); m++) {
    uint32_t k = (uint32_t)__builtin_popcount(m);
    rank[m] = count[k]++;
  }
}

/* All square minors by Laplace expansion along the first row of each submatrix.
 * det(R, C) = sum_t (-1)^t m[r0][c_t] det(R \ {r0}, C \ {c_t}), r0 = min R,
 * c_0 < c_1 < ... the columns of C. Minors of size k are kept in a table indexed
 * by (rank of R, rank of C) among the k-subsets. If det12 is not NULL, the full
 * determinant is stored there. Returns the number of zero minors. */
static uint64_t all_minors(const uint64_t m[OR_WIDTH][OR_WIDTH], uint64_t *det12) {
  static uint32_t rank[1 << OR_WIDTH];
  uint32_t count[OR_WIDTH + 1];
  subset_ranks(rank, count);
  /* masks of each popcount, in increasing order */
  uint32_t *masks[OR_WIDTH + 1];
  uint32_t filled[OR_WIDTH + 1] = {0};
  for (uint32_t k = 0; k <= OR_WIDTH; k++) masks[k] = (uint32_t *)malloc(sizeof(uint32_t) * count[k]);
  for (uint32_t msk = 0; msk < (1u << OR_WIDTH); msk++) {
    uint32_t k = (uint32_t)__builtin_popcount(msk);
    masks[k][filled[k]++] = msk;
  }
  uint64_t zeros = 0;
  uint64_t *prev = NULL;
  uint32_t prev_n = 0;
  for (uint32_t k = 1; k <= OR_WIDTH; k++) {
    uint32_t nk = count[k];
    uint64_t *cur = (uint64_t *)malloc((size_t)nk * nk * sizeof(uint64_t));
    for (uint32_t ri = 0; ri < nk; ri++) {
      uint32_t R = masks[k][ri];
      uint32_t r0 = (uint32_t)__builtin_ctz(R);
      uint32_t Rp = R & ~(1u << r0);
      for (uint32_t ci = 0; ci < nk; ci++) {
        uint32_t C = masks[k][ci];
        uint64_t det = 0;
        if (k == 1) {
          det = m[r0][__builtin_ctz(C)] % OR_P;
        } else {
          uint32_t t = 0;
          for (uint32_t c = 0; c < OR_WIDTH; c++) {
            if (!(C & (1u << c))) continue;
            uint32_t Cp = C & ~(1u << c);
            uint64_t term = or_mul(m[r0][c], prev[(size_t)rank[Rp] * prev_n + rank[Cp]]);
            det = (t & 1) ? or_sub(det, term) : or_add(det, term);
            t++;
          }
        }
        cur[(size_t)ri * nk + ci] = det;
        if (det == 0) zeros++;
      }
    }
    free(prev);
    prev = cur;
    prev_n = nk;
  }
  if (det12) *det12 = prev[0];
  free(prev);
  for (uint32_t k = 0; k <= OR_WIDTH; k++) free(masks[k]);
  return zeros;
}

uint64_t or_singular_minor_count(const uint64_t m[OR_WIDTH][OR_WIDTH]) { return all_minors(m, NULL); }

uint64_t or_det12(const uint64_t m[OR_WIDTH][OR_WIDTH]) {
  uint64_t d = 0;
  all_minors(m, &d);
  return d;
}

int or_poseidon_params_init(uint64_t seed, or_poseidon_params *pp) {
  memset(pp, 0, sizeof(*pp));
  pp->seed = seed;
  uint64_t i = 0;
  /* round constants: accepted stream values (z < p), round-major, lane-minor */
  for (int r = 0; r < OR_ROUNDS; r++) {
    for (int j = 0; j < OR_WIDTH; j++) {
      uint64_t z;
      do {
        z = or_splitmix64(seed, i++);
      } while (z >= OR_P);
      pp->rc[r][j] = z;
    }
  }
  /* circulant MDS: a_j = 1 + (z mod 255) from the next 12 stream values; redraw
   * all twelve until every square submatrix is nonsingular */
  for (uint32_t attempt = 1; attempt <= 1000; attempt++) {
    for (int j = 0; j < OR_WIDTH; j++) pp->circ[j] = 1 + or_splitmix64(seed, i++) % 255;
    for (int r = 0; r < OR_WIDTH; r++)
      for (int c = 0; c < OR_WIDTH; c++) pp->mds[r][c] = pp->circ[(c - r + OR_WIDTH) % OR_WIDTH];
    if (or_singular_minor_count((const uint64_t(*)[OR_WIDTH])pp->mds) == 0) {
      pp->mds_attempts = attempt;
      pp->stream_next = i;
      return 0;
    }
  }
  return -1;
}

/* One permutation: for r = 0..29, add round constants to all lanes, apply x^7
 * to all lanes (full rounds: r < 4 or r >= 26) or to lane 0 (partial rounds),
 * then multiply the state by the MDS matrix. */
void or_poseidon_permute(const or_poseidon_params *pp, uint64_t s[OR_WIDTH]) {
  for (int r = 0; r < OR_ROUNDS; r++) {
    int full = (r < OR_FULL_HALF) || (r >= OR_ROUNDS - OR_FULL_HALF);
    for (int i = 0; i < OR_WIDTH; i++) s[i] = or_add(s[i], pp->rc[r][i]);
    for (int i = 0; i < (full ? OR_WIDTH : 1); i++) s[i] = or_pow(s[i], 7);
    uint64_t t[OR_WIDTH];
    for (int i = 0; i < OR_WIDTH; i++) {
      /* (M s)_i = sum_j M[i][j] s_j mod p. The entries are 1 + (z mod 255) <= 255, so
       * the twelve products sum to less than 12 * 2^8 * 2^64 < 2^76: the sum is exact in
       * 128 bits and is reduced once. */
      u128 acc = 0;
      for (int j = 0; j < OR_WIDTH; j++) acc += (u128)pp->mds[i][j] * s[j];
      t[i] = (uint64_t)(acc % OR_P);
    }
    memcpy(s, t, sizeof(t));
  }
}

void or_poseidon_permute_batch(const or_poseidon_params *pp, uint64_t *states, size_t count) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) or_poseidon_permute(pp, states + (size_t)i * OR_WIDTH);
}

void or_sponge_state(const or_poseidon_params *pp, const uint64_t *row, uint32_t len,
                     uint64_t state[OR_WIDTH]) {
  memset(state, 0, sizeof(uint64_t) * OR_WIDTH);
  for (uint32_t q = 0; q < len; q += OR_RATE) {
    uint32_t chunk = (len - q < OR_RATE) ? (len - q) : OR_RATE;
    for (uint32_t i = 0; i < chunk; i++) state[i] = row[q + i];
    or_poseidon_permute(pp, state);
  }
}

void or_compress_state(const or_poseidon_params *pp, const uint64_t l[OR_DIGEST],
                       const uint64_t r[OR_DIGEST], uint64_t state[OR_WIDTH]) {
  memset(state, 0, sizeof(uint64_t) * OR_WIDTH);
  for (int i = 0; i < OR_DIGEST; i++) {
    state[i] = l[i];
    state[OR_DIGEST + i] = r[i];
  }
  or_poseidon_permute(pp, state);
}

/* ----------------------------------------------------------------- Merkle */

int or_leaf_digests(const or_poseidon_params *pp, const uint64_t *mat, uint32_t n_cols,
                    uint32_t log_leaves, uint64_t *digests) {
  if (!pp || !mat || !digests || n_cols == 0 || log_leaves > 40) return -1;
  uint64_t nl = 1ULL << log_leaves;
#pragma omp parallel
  {
    uint64_t *row = (uint64_t *)malloc(sizeof(uint64_t) * n_cols);
#pragma omp for schedule(static)
    for (int64_t k = 0; k < (int64_t)nl; k++) {
      for (uint32_t c = 0; c < n_cols; c++) row[c] = mat[(uint64_t)c * nl + (uint64_t)k];
      uint64_t st[OR_WIDTH];
      or_sponge_state(pp, row, n_cols, st);
      memcpy(digests + (uint64_t)k * OR_DIGEST, st, sizeof(uint64_t) * OR_DIGEST);
    }
    free(row);
  }
  return 0;
}

/* Build levels above `below` (2^(lvl+1) nodes) into `above` (2^lvl nodes). */
static void merkle_level(const or_poseidon_params *pp, const uint64_t *below, uint64_t *above,
                         uint64_t count_above) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < (int64_t)count_above; k++) {
    uint64_t st[OR_WIDTH];
    or_compress_state(pp, below + (uint64_t)(2 * k) * OR_DIGEST, below + (uint64_t)(2 * k + 1) * OR_DIGEST, st);
    memcpy(above + (uint64_t)k * OR_DIGEST, st, sizeof(uint64_t) * OR_DIGEST);
  }
}

int or_merkle_commit(const or_poseidon_params *pp, const uint64_t *mat, uint32_t n_cols,
                     uint32_t log_leaves, uint32_t cap_height, uint64_t *tree, uint64_t *cap) {
  if (!pp || !mat || !cap || n_cols == 0 || cap_height > log_leaves || log_leaves > 40) return -1;
  uint64_t nl = 1ULL << log_leaves;
  /* whole tree in one buffer: level L (leaves) first, then L-1, ..., h */
  uint64_t total = 2 * nl - (1ULL << cap_height);
  uint64_t *t = tree ? tree : (uint64_t *)malloc(sizeof(uint64_t) * OR_DIGEST * total);
  if (!t) return -1;
  or_leaf_digests(pp, mat, n_cols, log_leaves, t);
  uint64_t off = 0, cnt = nl;
  for (uint32_t lvl = log_leaves; lvl > cap_height; lvl--) {
    merkle_level(pp, t + off * OR_DIGEST, t + (off + cnt) * OR_DIGEST, cnt / 2);
    off += cnt;
    cnt /= 2;
  }
  memcpy(cap, t + off * OR_DIGEST, sizeof(uint64_t) * OR_DIGEST * cnt);
  if (!tree) free(t);
  return 0;
}

int or_merkle_path(const uint64_t *tree, uint32_t log_leaves, uint32_t cap_height, uint64_t index,
                   uint64_t *path) {
  if (!tree || cap_height > log_leaves || index >= (1ULL << log_leaves)) return -1;
  if (!path && log_leaves > cap_height) return -1;
  uint64_t off = 0, cnt = 1ULL << log_leaves;
  for (uint32_t lvl = log_leaves, d = 0; lvl > cap_height; lvl--, d++) {
    uint64_t sib = index ^ 1;
    memcpy(path + (uint64_t)d * OR_DIGEST, tree + (off + sib) * OR_DIGEST, sizeof(uint64_t) * OR_DIGEST);
    off += cnt;
    cnt /= 2;
    index >>= 1;
  }
  return 0;
}

void or_merkle_open(const or_poseidon_params *pp, const uint64_t leaf[OR_DIGEST], uint64_t index,
                    const uint64_t *path, uint32_t path_len, uint64_t node_out[OR_DIGEST],
                    uint64_t *cap_index) {
  uint64_t cur[OR_DIGEST], st[OR_WIDTH];
  memcpy(cur, leaf, sizeof(cur));
  for (uint32_t d = 0; d < path_len; d++) {
    const uint64_t *sib = path + (uint64_t)d * OR_DIGEST;
    /* bit d of the index: 0 means the current node is the left child */
    if ((index >> d) & 1)
      or_compress_state(pp, sib, cur, st);
    else
      or_compress_state(pp, cur, sib, st);
    memcpy(cur, st, sizeof(cur));
  }
  memcpy(node_out, cur, sizeof(cur));
  *cap_index = index >> path_len;
}

int or_commit(const or_poseidon_params *pp, const uint64_t *trace, uint32_t n_cols,
              uint32_t log_rows, uint32_t log_blowup, uint64_t shift, int layout,
              uint32_t cap_height, uint64_t *lde, uint64_t *tree, uint64_t *cap) {
  if (!pp || !trace || !cap || n_cols == 0) return -1;
  uint32_t log_N = log_rows + log_blowup;
  if (cap_height > log_N) return -1;
  uint64_t N = 1ULL << log_N;
  uint64_t *l = lde ? lde : (uint64_t *)malloc(sizeof(uint64_t) * N * n_cols);
  if (!l) return -1;
  int rc = or_lde(trace, n_cols, log_rows, log_blowup, shift, layout, l);
  if (rc == 0) rc = or_merkle_commit(pp, l, n_cols, log_N, cap_height, tree, cap);
  if (!lde) free(l);
  return rc;
}

/* MerkleTree over 2^log_leaves given digests: pairs compressed level by level down
 * to one root. */
static void merkle_root_of(const or_poseidon_params *pp, const uint64_t *leaves, uint32_t log_leaves,
                           uint64_t root[OR_DIGEST]) {
  uint64_t cnt = 1ULL << log_leaves;
  uint64_t *cur = (uint64_t *)malloc(sizeof(uint64_t) * OR_DIGEST * cnt);
  memcpy(cur, leaves, sizeof(uint64_t) * OR_DIGEST * cnt);
  while (cnt > 1) {
    for (uint64_t k = 0; k < cnt / 2; k++) {
      uint64_t st[OR_WIDTH];
      or_compress_state(pp, cur + 2 * k * OR_DIGEST, cur + (2 * k + 1) * OR_DIGEST, st);
      memcpy(cur + k * OR_DIGEST, st, sizeof(uint64_t) * OR_DIGEST);
    }
    cnt /= 2;
  }
  memcpy(root, cur, sizeof(uint64_t) * OR_DIGEST);
  free(cur);
}

int or_snapshot_commit(const or_poseidon_params *pp, uint32_t log_lists, uint32_t log_slots, uint32_t m,
                       uint32_t dim, uint32_t k, const uint64_t *flag, const uint64_t *item,
                       const uint64_t *codes, const uint64_t *centroids, const uint64_t *codebooks,
                       uint64_t *list_roots, uint64_t *list_hashes, uint64_t root_mk[OR_DIGEST],
                       uint64_t root_cb[OR_DIGEST]) {
  if (!pp || !flag || !item || !codes || !centroids || !codebooks || !root_mk || !root_cb) return -1;
  if (m == 0 || k == 0 || dim % m != 0 || log_lists + log_slots > 30) return -1;
  const uint64_t n_list = 1ULL << log_lists, n = 1ULL << log_slots, N = n_list * n;
  /* leaf digests hash_{i,j}, record order (list-major) */
  uint64_t *leaf = (uint64_t *)malloc(sizeof(uint64_t) * OR_DIGEST * N);
  uint64_t *roots = (uint64_t *)malloc(sizeof(uint64_t) * OR_DIGEST * n_list);
  uint64_t *hashes = (uint64_t *)malloc(sizeof(uint64_t) * OR_DIGEST * n_list);
  if (!leaf || !roots || !hashes) {
    free(leaf), free(roots), free(hashes);
    return -1;
  }
#pragma omp parallel
  {
    uint64_t *seq = (uint64_t *)malloc(sizeof(uint64_t) * (4 + m));
#pragma omp for schedule(static)
    for (int64_t t = 0; t < (int64_t)N; t++) {
      uint64_t st[OR_WIDTH];
      seq[0] = (uint64_t)t >> log_slots;          /* i */
      seq[1] = (uint64_t)t & (n - 1);             /* j */
      seq[2] = flag[t];
      seq[3] = item[t];
      for (uint32_t mm = 0; mm < m; mm++) seq[4 + mm] = codes[(uint64_t)mm * N + t];
      or_sponge_state(pp, seq, 4 + m, st);
      memcpy(leaf + (uint64_t)t * OR_DIGEST, st, sizeof(uint64_t) * OR_DIGEST);
    }
    free(seq);
  }
  /* list roots, then each centroid bound to its list root */
#pragma omp parallel
  {
    uint64_t *seq = (uint64_t *)malloc(sizeof(uint64_t) * (1 + dim + OR_DIGEST));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < (int64_t)n_list; i++) {
      uint64_t st[OR_WIDTH];
      merkle_root_of(pp, leaf + (uint64_t)i * n * OR_DIGEST, log_slots, roots + (uint64_t)i * OR_DIGEST);
      seq[0] = (uint64_t)i;
      memcpy(seq + 1, centroids + (uint64_t)i * dim, sizeof(uint64_t) * dim);
      memcpy(seq + 1 + dim, roots + (uint64_t)i * OR_DIGEST, sizeof(uint64_t) * OR_DIGEST);
      or_sponge_state(pp, seq, 1 + dim + OR_DIGEST, st);
      memcpy(hashes + (uint64_t)i * OR_DIGEST, st, sizeof(uint64_t) * OR_DIGEST);
    }
    free(seq);
  }
  merkle_root_of(pp, hashes, log_lists, root_mk);
  /* codebook digest over the canonical flattening (K*D elements) */
  {
    uint64_t st[OR_WIDTH];
    or_sponge_state(pp, codebooks, (uint32_t)((uint64_t)k * dim), st);
    memcpy(root_cb, st, sizeof(uint64_t) * OR_DIGEST);
  }
  if (list_roots) memcpy(list_roots, roots, sizeof(uint64_t) * OR_DIGEST * n_list);
  if (list_hashes) memcpy(list_hashes, hashes, sizeof(uint64_t) * OR_DIGEST * n_list);
  free(leaf), free(roots), free(hashes);
  return 0;
}

int or_grand_product(const uint64_t *cols, uint32_t width, uint64_t n, uint64_t alpha, uint64_t beta,
                     uint64_t *z, uint64_t *total) {
  if (width == 0 || !total || (n && !cols)) return -1;
  uint64_t acc = 1;
  for (uint64_t i = 0; i < n; i++) {
    /* Compress by Horner's rule from the last coordinate */
    uint64_t c = cols[(uint64_t)(width - 1) * n + i];
    for (int64_t k = (int64_t)width - 2; k >= 0; k--) c = or_add(or_mul(c, beta), cols[(uint64_t)k * n + i]);
    acc = or_mul(acc, or_sub(alpha, c));
    if (z) z[i] = acc;
  }
  *total = acc;
  return 0;
}

int or_fri_commit(const or_poseidon_params *pp, const uint64_t *codeword, uint32_t log_n, uint64_t shift,
                  const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *folded, uint64_t *trees,
                  uint64_t *caps) {
  if (!pp || !codeword || !folded || !caps || (rounds && !betas)) return -1;
  if (rounds == 0 || rounds > log_n || cap_height + rounds > log_n || shift % OR_P == 0) return -1;
  const uint64_t inv2 = or_inv(2);
  const uint64_t *f = codeword;
  uint64_t *next = folded, *tree_out = trees;
  uint64_t s_r = shift % OR_P;
  for (uint32_t r = 0; r < rounds; r++) {
    const uint32_t log_nr = log_n - r;
    const uint64_t nr = 1ULL << log_nr, half = nr / 2;
    /* commit: leaves are the pairs (f[k], f[k + N/2]); a matrix [2][N/2] hashed by rows */
    const uint64_t tree_words = (2 * half - (1ULL << cap_height)) * OR_DIGEST;
    uint64_t *t = tree_out ? tree_out : (uint64_t *)malloc(sizeof(uint64_t) * tree_words);
    if (!t) return -1;
    int rc = or_merkle_commit(pp, f, 2, log_nr - 1, cap_height, t, caps + (uint64_t)r * (OR_DIGEST << cap_height));
    if (!tree_out) free(t);
    if (rc != 0) return -1;
    if (tree_out) tree_out += tree_words;
    /* fold with beta_r */
    const uint64_t w = or_root_of_unity(log_nr), winv = or_inv(w), sinv = or_inv(s_r);
    const uint64_t beta = betas[r] % OR_P;
    uint64_t xinv = sinv; /* 1 / x_k for k = 0, then times w^-1 */
    for (uint64_t k = 0; k < half; k++) {
      const uint64_t a = f[k], b = f[k + half];
      const uint64_t even = or_mul(or_add(a, b), inv2);
      const uint64_t odd = or_mul(or_mul(or_sub(a, b), inv2), xinv);
      next[k] = or_add(even, or_mul(beta, odd));
      xinv = or_mul(xinv, winv);
    }
    f = next;
    next += half;
    s_r = or_mul(s_r, s_r);
  }
  return 0;
}

int or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
