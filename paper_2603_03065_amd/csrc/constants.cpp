// Poseidon constants derived from a seed (host side, once per context).
//
// Stream: SplitMix64 (Steele, Lea, Flood 2014), output i = finaliser(seed + (i+1) * golden gamma).
// Round constants: the first 360 outputs below p, round-major. MDS: a circulant
// whose first row is a_j = 1 + (z mod 255) over the next 12 outputs, redrawn
// until every square submatrix is nonsingular mod p.
#include <string.h>

#include <map>
#include <mutex>

#include "internal.h"

namespace v3db {

uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Nonsingularity of a k x k matrix over F_p by fraction-free Gaussian
// elimination: row_r <- pivot * row_r - a_r * row_pivot keeps the rank and
// needs no inverses.
static bool nonsingular(uint64_t m[WIDTH][WIDTH], int k) {
  for (int col = 0; col < k; col++) {
    int piv = -1;
    for (int r = col; r < k; r++)
      if (m[r][col] != 0) {
        piv = r;
        break;
      }
    if (piv < 0) return false;
    if (piv != col)
      for (int c = 0; c < k; c++) {
        uint64_t t = m[col][c];
        m[col][c] = m[piv][c];
        m[piv][c] = t;
      }
    const uint64_t pv = m[col][col];
    for (int r = col + 1; r < k; r++) {
      const uint64_t f = m[r][col];
      if (f == 0) continue;
      for (int c = col; c < k; c++) m[r][c] = gl::sub(gl::mul(m[r][c], pv), gl::mul(m[col][c], f));
    }
  }
  return true;
}

// A circulant satisfies M[i+s][j+s] = M[i][j] (indices mod 12), so the
// submatrix on (R, C) equals, up to a reordering of rows and columns, the one on
// (R - s, C - s). Shifting by min(R) leaves 0 in R: checking only row sets that
// contain row 0 covers every square submatrix.
bool circulant_is_mds(const uint32_t circ[WIDTH]) {
  uint64_t sub[WIDTH][WIDTH];
  int rows[WIDTH], cols[WIDTH];
  for (uint32_t R = 1; R < (1u << WIDTH); R += 2) {  // bit 0 set
    const int k = __builtin_popcount(R);
    int nr = 0;
    for (int i = 0; i < WIDTH; i++)
      if (R >> i & 1) rows[nr++] = i;
    for (uint32_t C = 1; C < (1u << WIDTH); C++) {
      if (__builtin_popcount(C) != k) continue;
      int nc = 0;
      for (int j = 0; j < WIDTH; j++)
        if (C >> j & 1) cols[nc++] = j;
      for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++) sub[a][b] = circ[(cols[b] - rows[a] + WIDTH) % WIDTH];
      if (!nonsingular(sub, k)) return false;
    }
  }
  return true;
}

bool derive_poseidon(uint64_t seed, PoseidonTables &out, uint32_t &attempts) {
  // The search costs ~1e8 field operations; cache results per seed for the process.
  static std::mutex mu;
  static std::map<uint64_t, std::pair<PoseidonTables, uint32_t>> cache;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(seed);
    if (it != cache.end()) {
      out = it->second.first;
      attempts = it->second.second;
      return true;
    }
  }
  PoseidonTables t;
  memset(&t, 0, sizeof(t));
  uint64_t i = 0;
  for (int r = 0; r < ROUNDS; r++)
    for (int j = 0; j < WIDTH; j++) {
      uint64_t z;
      do z = splitmix64(seed, i++);
      while (z >= gl::P);
      t.rc[r][j] = z;
    }
  for (uint32_t attempt = 1; attempt <= 1000; attempt++) {
    for (int j = 0; j < WIDTH; j++) t.circ[j] = 1 + (uint32_t)(splitmix64(seed, i++) % 255);
    if (circulant_is_mds(t.circ)) {
      out = t;
      attempts = attempt;
      std::lock_guard<std::mutex> g(mu);
      cache[seed] = {t, attempt};
      return true;
    }
  }
  return false;
}

// Matrix-core linear layer (poseidon_mf.h): one int8 matrix A (32 x 32) holding C - 128
// for each circulant entry C = a[(j - i) mod 12], applied to two byte limbs l = 0, 1 at
// once. Row of output i = 6h + ii (h = i / 6), limb l: 8 (e / 4) + 4h + e % 4 with
// e = 6l + ii, where the 32x32 output layout puts it in the lanes that hold words
// 6h .. 6h+5. Column of word j = 6h' + 2q + w, limb l: 16h' + 4q + 2w + l; the row of
// output i, limb l holds C - 128 in the columns of limb l, zero in those of the other
// limb. Rows for e = 12, 13 (24 + 4h and 25 + 4h, both halves h) hold -128 in every
// column of limb 0, resp. 1: minus 128 times the byte sum, which the kernel adds back
// to every output (with the weights -1 and -2^16 kept as the table's second and fourth
// limb weights). Columns 12..15 and 28..31 stay zero. Lane x holds row x % 32, columns
// 16 (x / 32) .. +15 as 16 bytes. The accumulator start values are
// K + (next round constant).lo and K + (next round constant).hi with
// K = 128 (sum_j a_j) (2^24 + 2^16 + 2^8 + 1).
bool build_mf_table(const PoseidonTables &t, uint64_t out[MF_TABLE_WORDS]) {
  memset(out, 0, MF_TABLE_WORDS * sizeof(uint64_t));
  uint64_t R = 0;
  for (int j = 0; j < WIDTH; j++) {
    if (t.circ[j] > 255) return false;
    R += t.circ[j];
  }
  int8_t A[32][32] = {};
  for (int h = 0; h < 2; h++)
    for (int l = 0; l < 2; l++) {
      const int e = 12 + l, row = 8 * (e / 4) + 4 * h + e % 4;
      for (int j = 0; j < WIDTH; j++) {
        const int jj = j % 6;
        A[row][16 * (j / 6) + 4 * (jj / 2) + 2 * (jj % 2) + l] = -128;
      }
    }
  for (int i = 0; i < WIDTH; i++) {
    const int h = i / 6, ii = i % 6;
    for (int l = 0; l < 2; l++) {
      const int e = 6 * l + ii, row = 8 * (e / 4) + 4 * h + e % 4;
      for (int j = 0; j < WIDTH; j++) {
        const int C = (int)t.circ[(j - i + WIDTH) % WIDTH];
        const int jj = j % 6, col = 16 * (j / 6) + 4 * (jj / 2) + 2 * (jj % 2) + l;
        A[row][col] = (int8_t)(C - 128);
      }
    }
  }
  uint8_t *am = reinterpret_cast<uint8_t *>(out + MF_AMAT);
  for (int x = 0; x < 64; x++)
    for (int b = 0; b < 16; b++) am[x * 16 + b] = (uint8_t)A[x % 32][16 * (x / 32) + b];
  int32_t *mult = reinterpret_cast<int32_t *>(out + MF_MULT);
  mult[0] = 1;
  mult[1] = -1;
  mult[2] = 1 << 16;
  mult[3] = -(1 << 16);
  const uint64_t K = 128 * R * 0x01010101ull;
  for (int r = 0; r <= ROUNDS; r++)
    for (int i = 0; i < WIDTH; i++) {
      const uint64_t c = r < ROUNDS ? t.rc[r][i] : 0;
      out[MF_RCK + (size_t(r) * WIDTH + i) * 2] = K + (uint32_t)c;
      out[MF_RCK + (size_t(r) * WIDTH + i) * 2 + 1] = K + (c >> 32);
    }
  return true;
}

}  // namespace v3db
