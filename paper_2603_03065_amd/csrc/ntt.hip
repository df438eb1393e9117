// Coset low-degree extension on gfx950.
//
// For a column a of n = 2^L values (a_i = P(w_n^i)), the extension to N = B*n
// points is LDE[k] = P(s * w_N^k) = sum_j c_j (s w_N^k)^j with c = iNTT_n(a).
// It runs as three LDS-tiled passes of a four-step factorisation, n = n1*n2:
//
//   pass 1  (interpolation, first half)   j = j1*n2 + j2, k = k1 + n1*k2
//           Y[k1][j2] = w_n^(-j2 k1) * sum_j1 a[j1 n2 + j2] w_n1^(-j1 k1)
//   pass 2  per residue k1: c'[k2] = sum_j2 Y[k1][j2] w_n2^(-j2 k2)   (= n c[k1 + n1 k2])
//           then a blowup-B extension of that residue sequence with shift s^n1,
//           for every e < W = B*n2 (e = r + B*m1: coset r, point m1):
//           Z[k1][e] = n^-1 s^k1 w_N^(k1 e) * sum_k2 c'[k2] (s^n1)^k2 w_W^(k2 e)
//   pass 3  per column e of Z: LDE[e + W m2] = sum_k1 Z[k1][e] w_n1^(k1 m2)
//
// (LDE[e + B n2 m2] = sum_k1 w_n1^(k1 m2) s^k1 w_N^(k1 e) sum_k2 c[k1+n1 k2]
//  (s^n1)^k2 w_(B n2)^(k2 e) follows from j = k1 + n1 k2 and k = e + B n2 m2.)
//
// Each pass moves tiles of T adjacent columns/rows so global accesses are runs
// of T*8 bytes, does its sub-transforms in LDS (radix-2 decimation-in-frequency
// for natural -> bit-reversed, decimation-in-time for bit-reversed -> natural),
// and applies the twiddles on the way out. Pass 1 writes Y into the first n
// entries of the output column (free until pass 3); pass 2 writes Z (B*n per
// column, rows of W contiguous words) to scratch, a chunk of columns at a time;
// pass 3 reads runs of T words of Z and writes the output in natural order
// (runs of T) or bit-reversed order (contiguous rows).
#include "internal.h"

namespace v3db {

namespace {

constexpr int THREADS = 512;
constexpr int DFT_N = 1 << DFT_LOG_MAX;  // 4096
constexpr int TILE_ELEMS = 8192;         // T * M per tile
constexpr int MAX_PER_THREAD = TILE_ELEMS / THREADS;

__device__ __forceinline__ uint32_t brev(uint32_t x, int bits) {
  return bits ? (__brev(x) >> (32 - bits)) : 0u;
}

// w^e for e < 2^26 from the two-level table (w = w_{2^26} or its inverse).
__device__ __forceinline__ uint64_t tw_pow(const uint64_t *__restrict__ lo, const uint64_t *__restrict__ hi,
                                           uint32_t e) {
  return gl::mul(hi[e >> TW_HALF], lo[e & ((1u << TW_HALF) - 1)]);
}

// Powers of w_8 = 7^((p-1)/8) (forward) and of its inverse; all are +-2^(24 k),
// so with these compile-time operands the products need only half the partial
// products.
__device__ __forceinline__ uint64_t w8(int k, bool inv) {
  constexpr uint64_t F[4] = {1ull, 18446744069397807105ull, 281474976710656ull, 18446742969902956801ull};
  constexpr uint64_t I[4] = {1ull, 1099511627520ull, 18446462594437873665ull, 16777216ull};
  return inv ? I[k] : F[k];
}

// Size-R transform in registers (R = 2, 4, 8) by radix-2 stages.
// dif: natural order in, bit-reversed order out. dit: bit-reversed in, natural out.
template <int R, bool INV>
__device__ __forceinline__ void reg_dif(uint64_t v[R]) {
#pragma unroll
  for (int h = R / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int b = 0; b < R; b += 2 * h)
#pragma unroll
      for (int i = 0; i < h; i++) {
        const uint64_t u = v[b + i], w = v[b + i + h];
        v[b + i] = gl::add(u, w);
        const uint64_t d = gl::sub(u, w);
        v[b + i + h] = i ? gl::mul(d, w8(i * (8 / (2 * h)), INV)) : d;
      }
}

template <int R, bool INV>
__device__ __forceinline__ void reg_dit(uint64_t v[R]) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1)
#pragma unroll
    for (int b = 0; b < R; b += 2 * h)
#pragma unroll
      for (int i = 0; i < h; i++) {
        const uint64_t u = v[b + i];
        uint64_t w = v[b + i + h];
        if (i) w = gl::mul(w, w8(i * (8 / (2 * h)), INV));
        v[b + i] = gl::add(u, w);
        v[b + i + h] = gl::sub(u, w);
      }
}

template <int R>
__device__ __forceinline__ int brev_r(int j) {
  return R == 8 ? ((j & 1) << 2 | (j & 2) | (j >> 2)) : R == 4 ? ((j & 1) << 1 | (j >> 1)) : j;
}

// One radix-R pass of a decimation-in-frequency transform over T rows of
// 2^logM words in LDS (row stride rs): sub-blocks of 2^logS words, each
// butterfly takes the R words i + j*2^logS/R, transforms them, and multiplies
// output slot j (frequency bitrev(j)) by w_S^(i * bitrev(j)). tw = w_4096^t.
template <int R, bool INV>
__device__ __forceinline__ void dif_pass(uint64_t *sh, int T, int logM, int rs, int logS,
                                         const uint64_t *__restrict__ tw) {
  constexpr int LR = R == 8 ? 3 : R == 4 ? 2 : 1;
  const int logStride = logS - LR;
  const int per_row = 1 << (logM - LR);
  const int nb = T * per_row;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int t = b >> (logM - LR);
    const int q = b & (per_row - 1);
    const int i = q & ((1 << logStride) - 1);
    uint64_t *base = sh + t * rs + ((q >> logStride) << logS) + i;
    uint64_t v[R];
#pragma unroll
    for (int j = 0; j < R; j++) v[j] = base[j << logStride];
    reg_dif<R, INV>(v);
    if (i) {
#pragma unroll
      for (int j = 1; j < R; j++) v[j] = gl::mul(v[j], tw[(i * brev_r<R>(j)) << (DFT_LOG_MAX - logS)]);
    }
#pragma unroll
    for (int j = 0; j < R; j++) base[j << logStride] = v[j];
  }
}

// One radix-R pass of a decimation-in-time transform: combines R transformed
// sub-blocks of 2^logS/R words into one of 2^logS words.
template <int R, bool INV>
__device__ __forceinline__ void dit_pass(uint64_t *sh, int T, int logM, int rs, int logS,
                                         const uint64_t *__restrict__ tw) {
  constexpr int LR = R == 8 ? 3 : R == 4 ? 2 : 1;
  const int logStride = logS - LR;
  const int per_row = 1 << (logM - LR);
  const int nb = T * per_row;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int t = b >> (logM - LR);
    const int q = b & (per_row - 1);
    const int i = q & ((1 << logStride) - 1);
    uint64_t *base = sh + t * rs + ((q >> logStride) << logS) + i;
    uint64_t v[R];
#pragma unroll
    for (int j = 0; j < R; j++) v[j] = base[j << logStride];
    if (i) {
#pragma unroll
      for (int j = 1; j < R; j++) v[j] = gl::mul(v[j], tw[(i * brev_r<R>(j)) << (DFT_LOG_MAX - logS)]);
    }
    reg_dit<R, INV>(v);
#pragma unroll
    for (int j = 0; j < R; j++) base[j << logStride] = v[j];
  }
}

// Whole transforms over the rows: radix-8 passes, then one radix-4 or radix-2
// pass for the remaining bits. Each pass ends with a barrier.
// Passes from sub-block size 2^logS0 down (logS0 < logM when the earlier passes
// were done another way).
template <bool INV>
__device__ void dif_rows_from(uint64_t *sh, int T, int logM, int logS0, int rs, const uint64_t *__restrict__ tw) {
  int logS = logS0;
  for (; logS >= 3; logS -= 3) {
    dif_pass<8, INV>(sh, T, logM, rs, logS, tw);
    __syncthreads();
  }
  if (logS == 2) {
    dif_pass<4, INV>(sh, T, logM, rs, 2, tw);
    __syncthreads();
  } else if (logS == 1) {
    dif_pass<2, INV>(sh, T, logM, rs, 1, tw);
    __syncthreads();
  }
}

template <bool INV>
__device__ __forceinline__ void dif_rows(uint64_t *sh, int T, int logM, int rs, const uint64_t *__restrict__ tw) {
  dif_rows_from<INV>(sh, T, logM, logM, rs, tw);
}

template <bool INV>
__device__ void dit_rows(uint64_t *sh, int T, int logM, int rs, const uint64_t *__restrict__ tw) {
  int logS = logM % 3;
  if (logS == 2) {
    dit_pass<4, INV>(sh, T, logM, rs, 2, tw);
    __syncthreads();
  } else if (logS == 1) {
    dit_pass<2, INV>(sh, T, logM, rs, 1, tw);
    __syncthreads();
  }
  for (logS += 3; logS <= logM; logS += 3) {
    dit_pass<8, INV>(sh, T, logM, rs, logS, tw);
    __syncthreads();
  }
}

struct Shape {
  int L, b, L1, L2;   // log n, log blowup, log n1, log n2
  int logT1, logT2, logT3;
};

// Pass 1: tile = T consecutive j2 of one column.
__global__ void __launch_bounds__(THREADS) k_lde_pass1(const uint64_t *__restrict__ trace, uint64_t *__restrict__ lde,
                                                       Shape s, Twiddles tw) {
  extern __shared__ uint64_t sh[];
  const int n1 = 1 << s.L1, n2 = 1 << s.L2, T = 1 << s.logT1, rs = n1 + 1;
  const size_t n = size_t(1) << s.L, N = size_t(1) << (s.L + s.b);
  const uint64_t *a = trace + size_t(blockIdx.y) * n;
  uint64_t *y = lde + size_t(blockIdx.y) * N;
  const int j2_0 = blockIdx.x << s.logT1;
  const int total = T * n1;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int t = e & (T - 1), j1 = e >> s.logT1;
    sh[t * rs + j1] = a[size_t(j1) * n2 + j2_0 + t];
  }
  __syncthreads();
  dif_rows<true>(sh, T, s.L1, rs, tw.dft_inv);
  const int shl = TW_LOG - s.L;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int t = e & (T - 1), k1 = e >> s.logT1;
    const uint32_t j2 = j2_0 + t;
    uint64_t v = sh[t * rs + brev(k1, s.L1)];
    const uint32_t ex = (uint32_t)((uint64_t(j2) * k1) & (n - 1));
    if (ex) v = gl::mul(v, tw_pow(tw.inv_lo, tw.inv_hi, ex << shl));
    y[size_t(k1) * n2 + j2] = v;
  }
}

// Pass 2: tile = T consecutive residues k1 (rows of Y) of one column; W = B*n2.
// Row k1 of Y is transformed back (giving n*c[k1 + n1*k2] in bit-reversed
// positions), scaled by n^-1 s^k1 and expanded to the W-point zero-padded
// transform: its first radix-B decimation-in-frequency pass has a single
// nonzero input per butterfly, so output slot j of butterfly i is the input
// times the twist (s^n1 w_W^r)^i, r = bitrev(j). The remaining passes run on the
// B cosets together; row k1 of Z gets Z[k1][e] = w_N^(k1 e) * (result at e).
__global__ void __launch_bounds__(THREADS) k_lde_pass2(const uint64_t *__restrict__ lde, uint64_t *__restrict__ z,
                                                       int col0, Shape s, Twiddles tw,
                                                       const uint64_t *__restrict__ twist,
                                                       const uint64_t *__restrict__ scale) {
  extern __shared__ uint64_t sh[];
  const int n2 = 1 << s.L2, T = 1 << s.logT2, B = 1 << s.b;
  const int LW = s.L2 + s.b, W = 1 << LW, rs = W + 1;
  const size_t N = size_t(1) << (s.L + s.b);
  const int logN = s.L + s.b;
  const uint64_t *y = lde + size_t(col0 + blockIdx.y) * N;
  uint64_t *zc = z + size_t(blockIdx.y) * N;
  const int k1_0 = blockIdx.x << s.logT2;
  const int total_in = T << s.L2;
  for (int e = threadIdx.x; e < total_in; e += blockDim.x) {
    const int t = e >> s.L2, j = e & (n2 - 1);
    sh[t * rs + j] = y[size_t(k1_0 + t) * n2 + j];
  }
  __syncthreads();
  dif_rows<true>(sh, T, s.L2, rs, tw.dft_inv);
  uint64_t c[MAX_PER_THREAD];
#pragma unroll
  for (int m = 0; m < MAX_PER_THREAD; m++) {
    const int e = threadIdx.x + m * THREADS;
    if (e < total_in) {
      const int t = e >> s.L2, i = e & (n2 - 1);
      c[m] = gl::mul(sh[t * rs + brev(i, s.L2)], scale[k1_0 + t]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MAX_PER_THREAD; m++) {
    const int e = threadIdx.x + m * THREADS;
    if (e < total_in) {
      const int t = e >> s.L2, i = e & (n2 - 1);
      for (int j = 0; j < B; j++) sh[t * rs + i + (j << s.L2)] = gl::mul(c[m], twist[(brev(j, s.b) << s.L2) + i]);
    }
  }
  __syncthreads();
  dif_rows_from<false>(sh, T, LW, s.L2, rs, tw.dft_fwd);
  const int total_out = T << LW;
  const int shl = TW_LOG - logN;
  for (int e = threadIdx.x; e < total_out; e += blockDim.x) {
    const int t = e >> LW, f = e & (W - 1);
    const uint32_t k1 = k1_0 + t;
    uint64_t v = sh[t * rs + brev(f, LW)];
    const uint32_t ex = (uint32_t)((uint64_t(k1) * f) & (N - 1));
    if (ex) v = gl::mul(v, tw_pow(tw.fwd_lo, tw.fwd_hi, ex << shl));
    zc[(size_t(k1) << LW) + f] = v;
  }
}

// Pass 3: tile = T consecutive rows e of Z of one column.
template <bool BITREV>
__global__ void __launch_bounds__(THREADS) k_lde_pass3(const uint64_t *__restrict__ z, uint64_t *__restrict__ lde,
                                                       int col0, Shape s, Twiddles tw) {
  extern __shared__ uint64_t sh[];
  const int n1 = 1 << s.L1, n2 = 1 << s.L2, T = 1 << s.logT3, rs = n1 + 1, B = 1 << s.b;
  const size_t N = size_t(1) << (s.L + s.b);
  const uint64_t *zc = z + size_t(blockIdx.y) * N;
  uint64_t *out = lde + size_t(col0 + blockIdx.y) * N;
  const int e0 = blockIdx.x << s.logT3;
  const int total = T * n1;
  const int LW = s.L2 + s.b;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int t = e & (T - 1), k1 = e >> s.logT3;
    sh[t * rs + k1] = zc[(size_t(k1) << LW) + e0 + t];
  }
  __syncthreads();
  dif_rows<false>(sh, T, s.L1, rs, tw.dft_fwd);
  if (!BITREV) {
    const size_t stride = size_t(B) * n2;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e & (T - 1), m2 = e >> s.logT3;
      out[size_t(e0 + t) + stride * m2] = sh[t * rs + brev(m2, s.L1)];
    }
  } else {
    const int lr = s.L2 + s.b;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e >> s.L1, p = e & (n1 - 1);
      out[size_t(brev(e0 + t, lr)) * n1 + p] = sh[t * rs + p];
    }
  }
}

int tile_log(int logM, int other_log) {
  // T * M <= TILE_ELEMS, T <= 16, T <= size of the other dimension
  int lt = DFT_LOG_MAX + 1 - logM;  // log2(8192 / M)
  if (lt > 4) lt = 4;
  if (lt < 0) lt = 0;
  if (lt > other_log) lt = other_log;
  return lt;
}

}  // namespace

v3db_status build_twiddles(v3db_ctx *ctx) {
  const size_t half = size_t(1) << TW_HALF;
  std::vector<uint64_t> lo(half), hi(half), ilo(half), ihi(half), dfw(DFT_N), dinv(DFT_N);
  const uint64_t w = gl::root_of_unity(TW_LOG), wi = gl::inv(w);
  const uint64_t wstep = gl::pow(w, half), wistep = gl::pow(wi, half);
  uint64_t a = 1, b = 1, c = 1, d = 1;
  for (size_t i = 0; i < half; i++) {
    lo[i] = a, hi[i] = b, ilo[i] = c, ihi[i] = d;
    a = gl::mul(a, w), b = gl::mul(b, wstep), c = gl::mul(c, wi), d = gl::mul(d, wistep);
  }
  const uint64_t w4 = gl::root_of_unity(DFT_LOG_MAX), w4i = gl::inv(w4);
  a = 1, c = 1;
  for (int t = 0; t < DFT_N; t++) {
    dfw[t] = a, dinv[t] = c;
    a = gl::mul(a, w4), c = gl::mul(c, w4i);
  }
  uint64_t *buf = nullptr;
  const size_t total = 4 * half + 2 * DFT_N;
  v3db_status st = ctx_alloc(ctx, (void **)&buf, total * 8, "twiddle tables");
  if (st != V3DB_OK) return st;
  ctx->tw.fwd_lo = buf;
  ctx->tw.fwd_hi = buf + half;
  ctx->tw.inv_lo = buf + 2 * half;
  ctx->tw.inv_hi = buf + 3 * half;
  ctx->tw.dft_fwd = buf + 4 * half;
  ctx->tw.dft_inv = buf + 4 * half + DFT_N;
  std::vector<uint64_t> host(total);
  std::copy(lo.begin(), lo.end(), host.begin());
  std::copy(hi.begin(), hi.end(), host.begin() + half);
  std::copy(ilo.begin(), ilo.end(), host.begin() + 2 * half);
  std::copy(ihi.begin(), ihi.end(), host.begin() + 3 * half);
  std::copy(dfw.begin(), dfw.end(), host.begin() + 4 * half);
  std::copy(dinv.begin(), dinv.end(), host.begin() + 4 * half + DFT_N);
  return hip_check(hipMemcpy(buf, host.data(), total * 8, hipMemcpyHostToDevice), "upload twiddles");
}

void free_twiddles(v3db_ctx *ctx) {
  if (ctx->tw.fwd_lo) ctx_free(ctx, ctx->tw.fwd_lo, (4 * (size_t(1) << TW_HALF) + 2 * DFT_N) * 8);
  ctx->tw = Twiddles{};
  for (auto &kv : ctx->plans) {
    const LdePlan &p = kv.second;
    const size_t bytes = ((size_t(1) << (p.L2 + p.log_blowup)) + (size_t(1) << p.L1)) * 8;
    ctx_free(ctx, p.d_twist, bytes);
  }
  ctx->plans.clear();
}

v3db_status get_plan(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint64_t shift, const LdePlan **out) {
  auto key = std::make_tuple(log_rows, log_blowup, shift);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    *out = &it->second;
    return V3DB_OK;
  }
  LdePlan p{};
  p.log_rows = log_rows;
  p.log_blowup = log_blowup;
  p.shift = shift;
  // n2 = 2^L2 with B*n2 <= 2^14 (pass 2 holds B*n2 words per residue in LDS), n1 <= 2^12
  p.L2 = log_rows / 2;
  if (p.L2 + log_blowup > 14) p.L2 = 14 - log_blowup;
  p.L1 = log_rows - p.L2;
  const size_t n1 = size_t(1) << p.L1, n2 = size_t(1) << p.L2, B = size_t(1) << log_blowup;
  std::vector<uint64_t> host(B * n2 + n1);
  // twist[r][j] = (s^n1 * w_{B n2}^r)^j
  const uint64_t sn1 = gl::pow(shift, n1);
  const uint64_t wb = gl::root_of_unity(p.L2 + log_blowup);
  uint64_t wr = 1;
  for (size_t r = 0; r < B; r++) {
    const uint64_t base = gl::mul(sn1, wr);
    uint64_t v = 1;
    for (size_t j = 0; j < n2; j++) {
      host[r * n2 + j] = v;
      v = gl::mul(v, base);
    }
    wr = gl::mul(wr, wb);
  }
  // scale[k1] = n^-1 s^k1
  uint64_t v = gl::inv(uint64_t(1) << log_rows);
  for (size_t k = 0; k < n1; k++) {
    host[B * n2 + k] = v;
    v = gl::mul(v, shift);
  }
  uint64_t *buf = nullptr;
  v3db_status st = ctx_alloc(ctx, (void **)&buf, host.size() * 8, "LDE plan tables");
  if (st != V3DB_OK) return st;
  st = hip_check(hipMemcpy(buf, host.data(), host.size() * 8, hipMemcpyHostToDevice), "upload plan");
  if (st != V3DB_OK) {
    ctx_free(ctx, buf, host.size() * 8);
    return st;
  }
  p.d_twist = buf;
  p.d_scale = buf + B * n2;
  *out = &(ctx->plans[key] = p);
  return V3DB_OK;
}

size_t lde_scratch_bytes(uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup) {
  const uint32_t chunk = n_cols < LDE_CHUNK_COLS ? n_cols : LDE_CHUNK_COLS;
  return size_t(chunk) * (size_t(8) << (log_rows + log_blowup));
}

v3db_status enqueue_lde(v3db_ctx *ctx, const uint64_t *trace, uint32_t n_cols, uint32_t log_rows,
                        uint32_t log_blowup, uint64_t shift, v3db_layout layout, uint64_t *lde,
                        uint64_t *z, hipStream_t stream) {
  const LdePlan *plan = nullptr;
  v3db_status st = get_plan(ctx, log_rows, log_blowup, shift, &plan);
  if (st != V3DB_OK) return st;
  Shape s{};
  s.L = (int)log_rows;
  s.b = (int)log_blowup;
  s.L1 = (int)plan->L1;
  s.L2 = (int)plan->L2;
  s.logT1 = tile_log(s.L1, s.L2);
  s.logT2 = tile_log(s.L2 + s.b, s.L1);
  s.logT3 = tile_log(s.L1, s.L2 + s.b);
  const size_t N = size_t(1) << (s.L + s.b);
  (void)N;
  // z holds Z for a chunk of columns at a time (lde_scratch_bytes)
  const uint32_t chunk = n_cols < LDE_CHUNK_COLS ? n_cols : LDE_CHUNK_COLS;

  const size_t sh1 = size_t(1 << s.logT1) * ((1 << s.L1) + 1) * 8;
  const size_t sh2 = size_t(1 << s.logT2) * ((1 << (s.L2 + s.b)) + 1) * 8;
  const size_t sh3 = size_t(1 << s.logT3) * ((1 << s.L1) + 1) * 8;
  static bool attr_done = false;
  if (!attr_done) {
    const int maxsh = 160 * 1024;
    hipFuncSetAttribute((const void *)k_lde_pass1, hipFuncAttributeMaxDynamicSharedMemorySize, maxsh);
    hipFuncSetAttribute((const void *)k_lde_pass2, hipFuncAttributeMaxDynamicSharedMemorySize, maxsh);
    hipFuncSetAttribute((const void *)k_lde_pass3<false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxsh);
    hipFuncSetAttribute((const void *)k_lde_pass3<true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxsh);
    attr_done = true;
  }
  const Twiddles tw = ctx->tw;
  dim3 g1((1u << s.L2) >> s.logT1, n_cols);
  hipLaunchKernelGGL(k_lde_pass1, g1, dim3(THREADS), sh1, stream, trace, lde, s, tw);
  for (uint32_t c0 = 0; c0 < n_cols; c0 += chunk) {
    const uint32_t nc = (n_cols - c0) < chunk ? (n_cols - c0) : chunk;
    dim3 g2((1u << s.L1) >> s.logT2, nc);
    hipLaunchKernelGGL(k_lde_pass2, g2, dim3(THREADS), sh2, stream, lde, z, (int)c0, s, tw, plan->d_twist,
                       plan->d_scale);
    dim3 g3((1u << (s.L2 + s.b)) >> s.logT3, nc);
    if (layout == V3DB_LAYOUT_BITREV)
      hipLaunchKernelGGL(k_lde_pass3<true>, g3, dim3(THREADS), sh3, stream, z, lde, (int)c0, s, tw);
    else
      hipLaunchKernelGGL(k_lde_pass3<false>, g3, dim3(THREADS), sh3, stream, z, lde, (int)c0, s, tw);
  }
  return hip_check(hipGetLastError(), "LDE launch");
}

}  // namespace v3db
