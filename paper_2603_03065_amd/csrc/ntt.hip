// Coset low-degree extension of one trace: tables, plans and the pass kernels
// (1, 2i, 2, 3; the pass bodies and the transform engine are in lde_dev.h).
#include "lde_dev.h"

namespace v3db {

namespace {

using namespace lde;

// Tile of block x when tiles of 8 words per row leave each 128-byte line half used by
// one tile and half by the next: blocks are dealt to the eight XCDs in turn, so tiles
// 2i and 2i + 1 go to blocks 16q + r and 16q + 8 + r (same XCD r, dispatched 8 apart)
// and the second reads the line from that XCD's L2. Identity for other grids.
__device__ __forceinline__ int xcd_pair_tile(int x, int n, int logT) {
  if (logT != 3 || (n & 15)) return x;
  return (x & ~15) | ((x & 7) << 1) | ((x >> 3) & 1);
}

__global__ void __launch_bounds__(LDE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_lde_pass1(LdeTask s, Twiddles tw) {
  extern __shared__ uint64_t sh[];
  lde_pass1_tile(s, tw, sh, blockIdx.y, xcd_pair_tile(blockIdx.x, gridDim.x, s.logT1));
}

__global__ void __launch_bounds__(LDE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_lde_pass2i(LdeTask s, Twiddles tw) {
  extern __shared__ uint64_t sh[];
  lde_pass2i_tile(s, tw, sh, blockIdx.y, blockIdx.x);
}

__global__ void __launch_bounds__(LDE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_lde_pass2(LdeTask s, Twiddles tw, int col0) {
  extern __shared__ uint64_t sh[];
  const int col = col0 + blockIdx.y;
  lde_pass2_tile(s, tw, sh, col, s.bitrev ? (int)blockIdx.y : col, blockIdx.x);
}

__global__ void __launch_bounds__(LDE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_lde_pass3(LdeTask s, Twiddles tw, int col0) {
  extern __shared__ uint64_t sh[];
  const int col = col0 + blockIdx.y;
  lde_pass3_tile(s, tw, sh, col, s.bitrev ? (int)blockIdx.y : col, xcd_pair_tile(blockIdx.x, gridDim.x, s.logT3));
}

// log2 of the tile height: T * M <= 8192 words, T <= 2^cap, T <= the other dimension.
int tile_log(int logM, int other_log, int cap) {
  int lt = DFT_LOG_MAX + 1 - logM;
  if (lt > cap) lt = cap;
  if (lt < 0) lt = 0;
  if (lt > other_log) lt = other_log;
  return lt;
}

// ztw[k1 * W + e] = w_N^(k1 e mod N), from the two-level table of w_{2^26}.
__global__ void k_fill_ztw(uint64_t *__restrict__ ztw, int LW, int logN, Twiddles tw) {
  const size_t N = size_t(1) << logN;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += size_t(gridDim.x) * blockDim.x) {
    const uint64_t k1 = i >> LW, e = i & ((size_t(1) << LW) - 1);
    const uint32_t ex = (uint32_t)((k1 * e) & (N - 1));
    ztw[i] = tw_pow(tw.fwd_lo, tw.fwd_hi, ex << (TW_LOG - logN));
  }
}

__global__ void k_fill_pattern(uint64_t *__restrict__ x, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    x[i] = (i * 0x9E3779B97F4A7C15ull) >> 1;  // below 2^63 < p
}

}  // namespace

static size_t twiddle_words() { return 4 * (size_t(1) << TW_HALF) + 2 * 8 * size_t(BFLY_ROWS); }

v3db_status build_twiddles(v3db_ctx *ctx) {
  const size_t half = size_t(1) << TW_HALF;
  std::vector<uint64_t> host(twiddle_words());
  const uint64_t w = gl::root_of_unity(TW_LOG), wi = gl::inv(w);
  const uint64_t wstep = gl::pow(w, half), wistep = gl::pow(wi, half);
  uint64_t a = 1, b = 1, c = 1, d = 1;
  for (size_t i = 0; i < half; i++) {
    host[i] = a, host[half + i] = b, host[2 * half + i] = c, host[3 * half + i] = d;
    a = gl::mul(a, w), b = gl::mul(b, wstep), c = gl::mul(c, wi), d = gl::mul(d, wistep);
  }
  // butterfly rows: for S = 2^logS, row i holds w_S^(i * bitrev3(j)), j < 8
  uint64_t *bf = host.data() + 4 * half, *bi = bf + 8 * size_t(BFLY_ROWS);
  for (int logS = 3; logS <= DFT_LOG_MAX; logS++) {
    const uint64_t ws = gl::root_of_unity(logS), wsi = gl::inv(ws);
    for (int i = 0; i < (1 << (logS - 3)); i++) {
      const size_t row = 8 * size_t(bfly_row0(logS) + i);
      for (int j = 0; j < 8; j++) {
        const int r = ((j & 1) << 2) | (j & 2) | (j >> 2);
        bf[row + j] = gl::pow(ws, uint64_t(i) * r);
        bi[row + j] = gl::pow(wsi, uint64_t(i) * r);
      }
    }
  }
  uint64_t *buf = nullptr;
  v3db_status st = ctx_alloc(ctx, (void **)&buf, host.size() * 8, "twiddle tables");
  if (st != V3DB_OK) return st;
  ctx->tw.fwd_lo = buf;
  ctx->tw.fwd_hi = buf + half;
  ctx->tw.inv_lo = buf + 2 * half;
  ctx->tw.inv_hi = buf + 3 * half;
  ctx->tw.bfly_fwd = buf + 4 * half;
  ctx->tw.bfly_inv = buf + 4 * half + 8 * size_t(BFLY_ROWS);
  return hip_check(hipMemcpy(buf, host.data(), host.size() * 8, hipMemcpyHostToDevice), "upload twiddles");
}

static void free_plan(v3db_ctx *ctx, LdePlan &p);

void free_twiddles(v3db_ctx *ctx) {
  if (ctx->tw.fwd_lo) ctx_free(ctx, ctx->tw.fwd_lo, twiddle_words() * 8);
  ctx->tw = Twiddles{};
  for (auto &kv : ctx->plans) free_plan(ctx, kv.second);
  ctx->plans.clear();
}

LdeSchedule default_schedule(uint32_t log_rows, uint32_t log_blowup) {
  LdeSchedule s{};
  // n2 = 2^L2 with B*n2 <= 2^14 (pass 2 holds B*n2 words per residue in LDS), n1 <= 2^12
  s.L2 = log_rows / 2;
  if (s.L2 + log_blowup > 14) s.L2 = 14 - log_blowup;
  s.cap1 = s.cap2 = s.cap3 = 4;
  s.chunk = LDE_CHUNK_COLS;
  s.us = 0;
  return s;
}

bool schedule_valid(const LdeSchedule &s, uint32_t log_rows, uint32_t log_blowup) {
  if (s.L2 > log_rows || s.L2 + log_blowup > 14 || log_rows - s.L2 > (uint32_t)DFT_LOG_MAX) return false;
  if (s.L2 > (uint32_t)DFT_LOG_MAX) return false;
  if (s.cap1 > 4 || s.cap2 > 4 || s.cap3 > 4) return false;
  return s.chunk >= 1 && s.chunk <= LDE_MAX_CHUNK_COLS;
}

static v3db_status build_plan(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint64_t shift,
                              const LdeSchedule &sched, LdePlan &p) {
  p = LdePlan{};
  p.log_rows = log_rows;
  p.log_blowup = log_blowup;
  p.shift = shift;
  p.L2 = sched.L2;
  p.L1 = log_rows - p.L2;
  p.logT1 = tile_log(p.L1, p.L2, sched.cap1);
  p.logT2 = tile_log(p.L2 + log_blowup, p.L1, sched.cap2);
  p.logT3 = tile_log(p.L1, p.L2 + log_blowup, sched.cap3);
  p.logT2i = tile_log(p.L2, p.L1, 4);
  // the tile loaders hold one tile of input words per block in registers
  // (MAX_PER_THREAD per thread): passes 1, 2i and 3 read T * (row length) words and
  // pass 2 reads T * n2
  auto fits = [](uint32_t log_words) { return (size_t(1) << log_words) <= size_t(lde::TILE_ELEMS); };
  if (!fits(p.L1 + p.logT1) || !fits(p.L2 + p.logT2i) || !fits(p.L1 + p.logT3) || !fits(p.L2 + p.logT2))
    return set_error(V3DB_ERR_UNSUPPORTED, "LDE plan: an input tile exceeds 8192 words");
  p.chunk = sched.chunk;
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
  p.d_ztw = nullptr;
  const uint32_t logN = log_rows + log_blowup;
  if (logN <= ZTW_MAX_LOG) {
    const size_t N = size_t(1) << logN;
    st = ctx_alloc(ctx, (void **)&p.d_ztw, N * 8, "LDE twiddle table");
    if (st == V3DB_OK) {
      const unsigned blocks = (unsigned)std::min<size_t>((N + 255) / 256, 4096);
      hipLaunchKernelGGL(k_fill_ztw, dim3(blocks), dim3(256), 0, nullptr, p.d_ztw, (int)(p.L2 + log_blowup),
                         (int)logN, ctx->tw);
      st = hip_check(hipGetLastError(), "fill LDE twiddle table");
      if (st == V3DB_OK) st = hip_check(hipStreamSynchronize(nullptr), "fill LDE twiddle table");
    }
    if (st != V3DB_OK) {
      free_plan(ctx, p);
      return st;
    }
  }
  return V3DB_OK;
}

static void free_plan(v3db_ctx *ctx, LdePlan &p) {
  const size_t bytes = ((size_t(1) << (p.L2 + p.log_blowup)) + (size_t(1) << p.L1)) * 8;
  ctx_free(ctx, p.d_twist, bytes);
  if (p.d_ztw) ctx_free(ctx, p.d_ztw, (size_t(1) << (p.log_rows + p.log_blowup)) * 8);
  p.d_twist = p.d_scale = p.d_ztw = nullptr;
}

void drop_plans(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup) {
  for (auto it = ctx->plans.begin(); it != ctx->plans.end();) {
    if (std::get<0>(it->first) == log_rows && std::get<1>(it->first) == log_blowup) {
      free_plan(ctx, it->second);
      it = ctx->plans.erase(it);
    } else {
      ++it;
    }
  }
}

v3db_status get_plan(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint64_t shift, const LdePlan **out) {
  auto key = std::make_tuple(log_rows, log_blowup, shift);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    *out = &it->second;
    return V3DB_OK;
  }
  auto tk = ctx->tuned.find({log_rows, log_blowup});
  const LdeSchedule sched = tk != ctx->tuned.end() ? tk->second : default_schedule(log_rows, log_blowup);
  LdePlan p;
  v3db_status st = build_plan(ctx, log_rows, log_blowup, shift, sched, p);
  if (st != V3DB_OK) return st;
  *out = &(ctx->plans[key] = p);
  return V3DB_OK;
}

size_t lde_scratch_bytes(uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup, v3db_layout layout) {
  const size_t y = (size_t(n_cols) << log_rows) * 8;
  if (layout == V3DB_LAYOUT_NATURAL) return y;
  const uint32_t chunk = n_cols < LDE_MAX_CHUNK_COLS ? n_cols : LDE_MAX_CHUNK_COLS;
  return y + size_t(chunk) * (size_t(8) << (log_rows + log_blowup));
}

// Tiles above 64 KiB of LDS need the kernels' dynamic LDS limit raised to the CU's
// 160 KiB; set on the current device when a context is created.
v3db_status set_lde_kernel_attributes() {
  const int maxsh = 160 * 1024;
  for (const void *k : {(const void *)k_lde_pass1, (const void *)k_lde_pass2i, (const void *)k_lde_pass2,
                        (const void *)k_lde_pass3}) {
    const v3db_status st =
        hip_check(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, maxsh), "LDE kernel LDS limit");
    if (st != V3DB_OK) return st;
  }
  return V3DB_OK;
}

LdeTask lde_task(const LdePlan &plan, const uint64_t *trace, uint64_t *y, uint64_t *z, uint64_t *lde,
                  v3db_layout layout) {
  LdeTask s{};
  s.trace = trace;
  s.y = y;
  s.lde = lde;
  s.twist = plan.d_twist;
  s.scale = plan.d_scale;
  s.ztw = plan.d_ztw;
  s.L = (int)plan.log_rows;
  s.b = (int)plan.log_blowup;
  s.L1 = (int)plan.L1;
  s.L2 = (int)plan.L2;
  s.logT1 = (int)plan.logT1;
  s.logT2 = (int)plan.logT2;
  s.logT3 = (int)plan.logT3;
  s.logT2i = (int)plan.logT2i;
  s.bitrev = layout == V3DB_LAYOUT_BITREV;
  const size_t N = size_t(1) << (s.L + s.b);
  s.z = s.bitrev ? z : lde;
  s.zstride = N;
  return s;
}

v3db_status enqueue_lde(v3db_ctx *ctx, const uint64_t *trace, uint32_t n_cols, uint32_t log_rows,
                        uint32_t log_blowup, uint64_t shift, v3db_layout layout, uint64_t *lde,
                        uint64_t *scratch, hipStream_t stream) {
  const LdePlan *plan = nullptr;
  v3db_status st = get_plan(ctx, log_rows, log_blowup, shift, &plan);
  if (st != V3DB_OK) return st;
  uint64_t *y = scratch;
  uint64_t *z = scratch + (size_t(n_cols) << log_rows);
  const LdeTask s = lde_task(*plan, trace, y, z, lde, layout);
  const Twiddles tw = ctx->tw;
  const size_t sh1 = lde_lds_words(1, s.L1, s.L2, s.b, s.logT1) * 8;
  const size_t sh2 = lde_lds_words(2, s.L1, s.L2, s.b, s.logT2) * 8;
  const size_t sh3 = lde_lds_words(3, s.L1, s.L2, s.b, s.logT3) * 8;
  const size_t sh2i = lde_lds_words(4, s.L1, s.L2, s.b, s.logT2i) * 8;
  const unsigned t1 = (1u << s.L2) >> s.logT1, t2 = (1u << s.L1) >> s.logT2, t3 = (1u << (s.L2 + s.b)) >> s.logT3;
  const unsigned t2i = (1u << s.L1) >> s.logT2i;
  hipLaunchKernelGGL(k_lde_pass1, dim3(t1, n_cols), dim3(LDE_THREADS), sh1, stream, s, tw);
  hipLaunchKernelGGL(k_lde_pass2i, dim3(t2i, n_cols), dim3(LDE_THREADS), sh2i, stream, s, tw);
  // a chunk of columns at a time through passes 2 and 3, so a chunk's Z is still
  // in the Infinity Cache when pass 3 reads it
  const uint32_t chunk = n_cols < plan->chunk ? n_cols : plan->chunk;
  for (uint32_t c0 = 0; c0 < n_cols; c0 += chunk) {
    const uint32_t nc = (n_cols - c0) < chunk ? (n_cols - c0) : chunk;
    hipLaunchKernelGGL(k_lde_pass2, dim3(t2, nc), dim3(LDE_THREADS), sh2, stream, s, tw, (int)c0);
    hipLaunchKernelGGL(k_lde_pass3, dim3(t3, nc), dim3(LDE_THREADS), sh3, stream, s, tw, (int)c0);
  }
  return hip_check(hipGetLastError(), "LDE launch");
}

// Time one schedule on the given buffers: the best of three runs after a warm-up.
static v3db_status time_schedule(v3db_ctx *ctx, const LdeSchedule &sc, uint32_t L, uint32_t b, uint32_t n_cols,
                                 v3db_layout layout, uint64_t *trace, uint64_t *lde, uint64_t *scratch,
                                 hipStream_t stream, hipEvent_t e0, hipEvent_t e1, double *us) {
  // a private plan with this schedule (shift 7; the shift does not change the work)
  LdePlan p;
  v3db_status st = build_plan(ctx, L, b, 7, sc, p);
  if (st != V3DB_OK) return st;
  auto key = std::make_tuple(L, b, uint64_t(7));
  auto old = ctx->plans.find(key);
  LdePlan saved{};
  const bool had = old != ctx->plans.end();
  if (had) saved = old->second;
  ctx->plans[key] = p;
  double best = 1e30;
  for (int rep = 0; rep < 4 && st == V3DB_OK; rep++) {
    hipError_t e = hipEventRecord(e0, stream);
    if (e == hipSuccess) st = enqueue_lde(ctx, trace, n_cols, L, b, 7, layout, lde, scratch, stream);
    if (st == V3DB_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
    if (st == V3DB_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (st == V3DB_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) st = hip_check(e, "autotune timing");
    if (rep > 0 && st == V3DB_OK) best = std::min(best, double(ms) * 1e3);
  }
  if (had) ctx->plans[key] = saved;
  else ctx->plans.erase(key);
  free_plan(ctx, p);
  *us = best;
  return st;
}

v3db_status autotune_lde(v3db_ctx *ctx, uint32_t L, uint32_t b, uint32_t n_cols, v3db_layout layout,
                         LdeSchedule *out) {
  const size_t n = size_t(1) << L, N = n << b;
  uint64_t *trace = nullptr, *lde = nullptr, *scratch = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  v3db_status st = ctx_alloc(ctx, (void **)&trace, n_cols * n * 8, "autotune trace");
  if (st == V3DB_OK) st = ctx_alloc(ctx, (void **)&lde, n_cols * N * 8, "autotune LDE");
  const size_t sb = lde_scratch_bytes(n_cols, L, b, layout);
  if (st == V3DB_OK) st = ctx_alloc(ctx, (void **)&scratch, sb, "autotune scratch");
  hipError_t e = hipSuccess;
  if (st == V3DB_OK) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  if (st == V3DB_OK && e == hipSuccess) e = hipEventCreate(&e0);
  if (st == V3DB_OK && e == hipSuccess) e = hipEventCreate(&e1);
  if (st == V3DB_OK && e != hipSuccess) st = hip_check(e, "autotune setup");
  if (st == V3DB_OK) {
    hipLaunchKernelGGL(k_fill_pattern, dim3(1024), dim3(256), 0, stream, trace, n_cols * n);
    st = hip_check(hipGetLastError(), "autotune fill");
  }
  LdeSchedule best = default_schedule(L, b);
  double best_us = 0;
  if (st == V3DB_OK) st = time_schedule(ctx, best, L, b, n_cols, layout, trace, lde, scratch, stream, e0, e1, &best_us);
  auto consider = [&](LdeSchedule c) {
    if (st != V3DB_OK || !schedule_valid(c, L, b)) return;
    double us = 0;
    st = time_schedule(ctx, c, L, b, n_cols, layout, trace, lde, scratch, stream, e0, e1, &us);
    if (st == V3DB_OK && us < best_us * 0.98) {
      best = c;
      best_us = us;
    }
  };
  // coordinate search: the split, then each pass's tile cap, then the column chunk
  const LdeSchedule d = best;
  for (int delta : {-3, -2, -1, 1, 2, 3}) {
    LdeSchedule c = d;
    if ((int)c.L2 + delta < 0) continue;
    c.L2 = (uint32_t)((int)c.L2 + delta);
    consider(c);
  }
  for (int pass = 1; pass <= 3; pass++)
    for (uint32_t cap : {0u, 1u, 2u, 3u}) {
      LdeSchedule c = best;
      (pass == 1 ? c.cap1 : pass == 2 ? c.cap2 : c.cap3) = cap;
      consider(c);
    }
  if (n_cols > 1)
    for (uint32_t ch : {2u, 4u, 16u}) {
      LdeSchedule c = best;
      c.chunk = ch;
      consider(c);
    }
  if (stream) (void)hipStreamDestroy(stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  ctx_free(ctx, scratch, sb);
  ctx_free(ctx, lde, n_cols * N * 8);
  ctx_free(ctx, trace, n_cols * n * 8);
  if (st != V3DB_OK) return st;
  best.us = best_us;
  *out = best;
  return V3DB_OK;
}

}  // namespace v3db
