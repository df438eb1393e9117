// C-ABI entry points: context, errors, argument checks, scratch, and the
// single-trace calls. The batched path lives in batch.hip.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "internal.h"

namespace v3db {

static thread_local std::string g_last_error;

v3db_status set_error(v3db_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

v3db_status hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return V3DB_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return set_error(V3DB_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
  return set_error(V3DB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

v3db_status ctx_alloc(v3db_ctx *ctx, void **ptr, size_t bytes, const char *what) {
  if (ctx->budget && ctx->allocated + bytes > ctx->budget)
    return set_error(V3DB_ERR_OUT_OF_MEMORY, std::string(what) + ": context HBM budget exceeded (" +
                                                 std::to_string(ctx->allocated + bytes) + " > " +
                                                 std::to_string(ctx->budget) + " bytes)");
  hipError_t e = hipMalloc(ptr, bytes ? bytes : 1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(V3DB_ERR_OUT_OF_MEMORY, std::string(what) + ": hipMalloc of " + std::to_string(bytes) +
                                                 " bytes failed: " + hipGetErrorString(e));
  }
  ctx->allocated += bytes;
  return V3DB_OK;
}

void ctx_free(v3db_ctx *ctx, void *ptr, size_t bytes) {
  if (!ptr) return;
  (void)hipFree(ptr);
  ctx->allocated -= bytes;
}

v3db_status ctx_scratch(v3db_ctx *ctx, hipStream_t stream, size_t bytes, void **out) {
  ScratchBuf &sb = ctx->scratch[(void *)stream];
  if (sb.bytes < bytes) {
    if (sb.ptr) {
      // the old buffer may still be read by queued work on this stream
      hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return hip_check(e, "scratch resize sync");
      ctx_free(ctx, sb.ptr, sb.bytes);
      sb.ptr = nullptr;
      sb.bytes = 0;
    }
    v3db_status st = ctx_alloc(ctx, &sb.ptr, bytes, "scratch");
    if (st != V3DB_OK) return st;
    sb.bytes = bytes;
  }
  *out = sb.ptr;
  return V3DB_OK;
}

hipEvent_t prof_mark(v3db_ctx *ctx, hipStream_t stream) {
  if (!ctx->profiling) return nullptr;
  hipEvent_t e = nullptr;
  if (!ctx->event_pool.empty()) {
    e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(e, stream) != hipSuccess) {
    ctx->event_pool.push_back(e);
    return nullptr;
  }
  return e;
}

void prof_interval(v3db_ctx *ctx, int phase, hipEvent_t a, hipEvent_t b) {
  if (a && b) ctx->prof_pending.push_back({phase, {a, b}});
}

static void prof_drop(v3db_ctx *ctx) {
  for (auto &r : ctx->prof_pending) {
    ctx->event_pool.push_back(r.second.first);
    ctx->event_pool.push_back(r.second.second);
  }
  ctx->prof_pending.clear();
}

static bool validate_inputs_enabled() {
  const char *v = getenv("V3DB_VALIDATE");
  return v && v[0] == '1';
}

// Returns V3DB_OK or sets the error for an invalid LDE shape.
static v3db_status check_lde_args(const void *trace, uint32_t n_cols, uint32_t log_rows, uint32_t log_blowup,
                                  uint64_t shift, int layout, const void *lde) {
  if (!trace || !lde) return set_error(V3DB_ERR_INVALID_ARG, "lde: NULL trace or output pointer");
  if (n_cols == 0) return set_error(V3DB_ERR_INVALID_ARG, "lde: n_cols must be > 0");
  if (shift == 0 || shift >= gl::P) return set_error(V3DB_ERR_INVALID_ARG, "lde: shift must be in [1, p)");
  if (layout != V3DB_LAYOUT_NATURAL && layout != V3DB_LAYOUT_BITREV)
    return set_error(V3DB_ERR_INVALID_ARG, "lde: unknown layout");
  if (n_cols > V3DB_MAX_COLS) return set_error(V3DB_ERR_UNSUPPORTED, "lde: more than 65535 columns");
  if (log_rows > V3DB_MAX_LOG_ROWS || log_blowup > V3DB_MAX_LOG_BLOWUP || log_rows + log_blowup > V3DB_MAX_LOG_LDE)
    return set_error(V3DB_ERR_UNSUPPORTED, "lde: log_rows <= 24, log_blowup <= 4 and their sum <= 26 required");
  return V3DB_OK;
}

static v3db_status check_merkle_args(const void *mat, uint32_t n_cols, uint32_t log_leaves, uint32_t cap_height,
                                     const void *cap) {
  if (!mat || !cap) return set_error(V3DB_ERR_INVALID_ARG, "merkle: NULL matrix or cap pointer");
  if (n_cols == 0) return set_error(V3DB_ERR_INVALID_ARG, "merkle: n_cols must be > 0");
  if (cap_height > log_leaves) return set_error(V3DB_ERR_INVALID_ARG, "merkle: cap_height > log_leaves");
  if (log_leaves > V3DB_MAX_LOG_LDE) return set_error(V3DB_ERR_UNSUPPORTED, "merkle: log_leaves > 26");
  if (n_cols > V3DB_MAX_COLS) return set_error(V3DB_ERR_UNSUPPORTED, "merkle: more than 65535 columns");
  return V3DB_OK;
}

// Optional input check (V3DB_VALIDATE=1): counts elements >= p.
__global__ void k_count_noncanonical(const uint64_t *__restrict__ x, size_t n, unsigned int *bad) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  unsigned int local = 0;
  for (; i < n; i += stride) local += x[i] >= gl::P;
  if (local) atomicAdd(bad, local);
}

static v3db_status check_canonical(v3db_ctx *ctx, const uint64_t *x, size_t n, hipStream_t stream) {
  if (!validate_inputs_enabled() || n == 0) return V3DB_OK;
  unsigned int *d_bad = nullptr;
  v3db_status st = ctx_alloc(ctx, (void **)&d_bad, sizeof(unsigned int), "validation flag");
  if (st != V3DB_OK) return st;
  unsigned int bad = 0;
  hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(unsigned int), stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_count_noncanonical, dim3(1024), dim3(256), 0, stream, x, n, d_bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  ctx_free(ctx, d_bad, sizeof(unsigned int));
  if (e != hipSuccess) return hip_check(e, "validation");
  if (bad) return set_error(V3DB_ERR_NONCANONICAL, std::to_string(bad) + " input elements are >= p");
  return V3DB_OK;
}

// Optional index check (V3DB_VALIDATE=1): counts indices >= limit.
__global__ void k_count_out_of_range(const uint64_t *__restrict__ x, size_t n, uint64_t limit, unsigned int *bad) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  unsigned int local = 0;
  for (; i < n; i += stride) local += x[i] >= limit;
  if (local) atomicAdd(bad, local);
}

static v3db_status check_indices(v3db_ctx *ctx, const uint64_t *idx, size_t n, uint64_t limit, hipStream_t stream) {
  if (!validate_inputs_enabled() || n == 0) return V3DB_OK;
  unsigned int *d_bad = nullptr;
  v3db_status st = ctx_alloc(ctx, (void **)&d_bad, sizeof(unsigned int), "validation flag");
  if (st != V3DB_OK) return st;
  unsigned int bad = 0;
  hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(unsigned int), stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_count_out_of_range, dim3(64), dim3(256), 0, stream, idx, n, limit, d_bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  ctx_free(ctx, d_bad, sizeof(unsigned int));
  if (e != hipSuccess) return hip_check(e, "validation");
  if (bad) return set_error(V3DB_ERR_INVALID_ARG, std::to_string(bad) + " query indices are >= 2^log_leaves");
  return V3DB_OK;
}

static v3db_status check_open_args(const char *who, const void *a, const void *b, const void *c, uint32_t n_cols,
                                   uint32_t log_leaves, uint32_t cap_height, size_t n_q, const void *paths) {
  if (n_q && (!a || !b || !c)) return set_error(V3DB_ERR_INVALID_ARG, std::string(who) + ": NULL pointer");
  if (n_q && log_leaves > cap_height && !paths)
    return set_error(V3DB_ERR_INVALID_ARG, std::string(who) + ": NULL paths");
  if (n_cols == 0) return set_error(V3DB_ERR_INVALID_ARG, std::string(who) + ": n_cols must be > 0");
  if (cap_height > log_leaves) return set_error(V3DB_ERR_INVALID_ARG, std::string(who) + ": cap_height > log_leaves");
  if (log_leaves > V3DB_MAX_LOG_LDE) return set_error(V3DB_ERR_UNSUPPORTED, std::string(who) + ": log_leaves > 26");
  if (n_cols > V3DB_MAX_COLS) return set_error(V3DB_ERR_UNSUPPORTED, std::string(who) + ": more than 65535 columns");
  return V3DB_OK;
}

}  // namespace v3db

using namespace v3db;

extern "C" {

const char *v3db_last_error(void) { return g_last_error.c_str(); }

v3db_status v3db_ctx_create(int device, uint64_t poseidon_seed, size_t hbm_budget_bytes, v3db_ctx **out) {
  clear_error();
  if (!out) return set_error(V3DB_ERR_INVALID_ARG, "ctx_create: NULL out");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return set_error(V3DB_ERR_DEVICE, "ctx_create: no HIP device");
  if (device < 0 || device >= ndev) return set_error(V3DB_ERR_INVALID_ARG, "ctx_create: device out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_check(e, "ctx_create: hipSetDevice");
  v3db_ctx *ctx = new v3db_ctx();
  ctx->device = device;
  ctx->seed = poseidon_seed;
  ctx->budget = hbm_budget_bytes;
  if (!derive_poseidon(poseidon_seed, ctx->pos, ctx->mds_attempts)) {
    delete ctx;
    return set_error(V3DB_ERR_UNSUPPORTED, "ctx_create: no MDS circulant found in 1000 draws");
  }
  // the round constants followed by one row of zeros (the kernels add "next round's
  // constants" inside every round's linear layer, the last one included)
  uint64_t table[POS_TABLE_WORDS] = {};
  memcpy(table, ctx->pos.rc, sizeof(ctx->pos.rc));
  // then the rows of M[i][j] = a[(j - i) mod 12], for kernels that give each lane one row
  uint32_t *rows = reinterpret_cast<uint32_t *>(table + (ROUNDS + 1) * WIDTH);
  for (int i = 0; i < WIDTH; i++)
    for (int j = 0; j < WIDTH; j++) rows[i * WIDTH + j] = (uint32_t)ctx->pos.circ[(j - i + WIDTH) % WIDTH];
  v3db_status st = ctx_alloc(ctx, (void **)&ctx->d_pos, sizeof(table), "Poseidon constants");
  if (st == V3DB_OK)
    st = hip_check(hipMemcpy(ctx->d_pos, table, sizeof(table), hipMemcpyHostToDevice), "upload Poseidon constants");
  if (st == V3DB_OK) ctx->d_circ_rows = reinterpret_cast<const uint32_t *>(ctx->d_pos + (ROUNDS + 1) * WIDTH);
  // the matrix-core linear layer, when the circulant's entries allow it (V3DB_POSEIDON_VALU=1
  // keeps the VALU form regardless)
  if (st == V3DB_OK) {
    std::vector<uint64_t> mf(MF_TABLE_WORDS);
    const char *env = getenv("V3DB_POSEIDON_VALU");
    const bool force_valu = env && env[0] && strcmp(env, "0") != 0;
    if (build_mf_table(ctx->pos, mf.data()) && !force_valu) {
      st = ctx_alloc(ctx, (void **)&ctx->d_mf, MF_TABLE_WORDS * 8, "Poseidon matrix-core table");
      if (st == V3DB_OK)
        st = hip_check(hipMemcpy(ctx->d_mf, mf.data(), MF_TABLE_WORDS * 8, hipMemcpyHostToDevice),
                       "upload Poseidon matrix-core table");
      ctx->mf = st == V3DB_OK;
    }
  }
  if (st == V3DB_OK) st = build_twiddles(ctx);
  if (st == V3DB_OK) st = set_lde_kernel_attributes();
  if (st == V3DB_OK) st = set_batch_kernel_attributes();
  if (st == V3DB_OK) st = noalloc_setup(device);
  if (st != V3DB_OK) {
    v3db_ctx_destroy(ctx);
    return st;
  }
  *out = ctx;
  return V3DB_OK;
}

void v3db_ctx_destroy(v3db_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_batch_graphs(ctx);
  if (ctx->side_stream) (void)hipStreamDestroy(ctx->side_stream);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  free_tree_batch(ctx);
  prof_drop(ctx);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  ctx->event_pool.clear();
  for (auto &kv : ctx->scratch) ctx_free(ctx, kv.second.ptr, kv.second.bytes);
  ctx->scratch.clear();
  free_twiddles(ctx);
  ctx_free(ctx, ctx->d_pos, POS_TABLE_WORDS * 8);
  if (ctx->d_mf) ctx_free(ctx, ctx->d_mf, MF_TABLE_WORDS * 8);
  delete ctx;
}

v3db_status v3db_poseidon_constants(const v3db_ctx *ctx, uint64_t *rc_out, uint64_t *circ_out,
                                    uint32_t *attempts_out) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "poseidon_constants: NULL ctx");
  if (rc_out) memcpy(rc_out, ctx->pos.rc, sizeof(ctx->pos.rc));
  if (circ_out)
    for (int i = 0; i < WIDTH; i++) circ_out[i] = ctx->pos.circ[i];
  if (attempts_out) *attempts_out = ctx->mds_attempts;
  return V3DB_OK;
}

v3db_status v3db_profile_enable(v3db_ctx *ctx, int on) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "profile_enable: NULL ctx");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  prof_drop(ctx);
  ctx->profiling = on != 0;
  return V3DB_OK;
}

v3db_status v3db_profile_read(v3db_ctx *ctx, double *ms_out, uint64_t *count_out) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "profile_read: NULL ctx");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  v3db_status st = V3DB_OK;
  for (auto &r : ctx->prof_pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.second.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.second.first, r.second.second);
    if (e != hipSuccess) {
      st = hip_check(e, "profile_read");
      break;
    }
    if (ms_out) ms_out[r.first] += ms;
    if (count_out) count_out[r.first] += 1;
  }
  prof_drop(ctx);
  return st;
}

v3db_status v3db_set_option(v3db_ctx *ctx, v3db_option opt, uint64_t value) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "set_option: NULL ctx");
  std::lock_guard<std::mutex> g(ctx->mu);
  switch (opt) {
    case V3DB_OPT_BATCHING:
      ctx->batching = value != 0;
      return V3DB_OK;
    case V3DB_OPT_BATCH_GROUP_BYTES:
      if (value == 0) return set_error(V3DB_ERR_INVALID_ARG, "set_option: group size must be > 0");
      ctx->batch_group_bytes = (size_t)value;
      return V3DB_OK;
  }
  return set_error(V3DB_ERR_INVALID_ARG, "set_option: unknown option");
}

int v3db_ctx_hash_path(const v3db_ctx *ctx) { return ctx ? (ctx->mf ? 1 : 0) : -1; }

v3db_status v3db_derive_poseidon_constants(uint64_t poseidon_seed, uint64_t *rc_out, uint64_t *circ_out,
                                           uint32_t *attempts_out) {
  clear_error();
  PoseidonTables t;
  uint32_t attempts = 0;
  if (!derive_poseidon(poseidon_seed, t, attempts))
    return set_error(V3DB_ERR_UNSUPPORTED, "derive_poseidon_constants: no MDS circulant found in 1000 draws");
  if (rc_out) memcpy(rc_out, t.rc, sizeof(t.rc));
  if (circ_out)
    for (int i = 0; i < WIDTH; i++) circ_out[i] = t.circ[i];
  if (attempts_out) *attempts_out = attempts;
  return V3DB_OK;
}

v3db_status v3db_lde(v3db_ctx *ctx, const uint64_t *d_trace, uint32_t n_cols, uint32_t log_rows,
                     uint32_t log_blowup, uint64_t shift, v3db_layout layout, uint64_t *d_lde,
                     v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "lde: NULL ctx");
  v3db_status st = check_lde_args(d_trace, n_cols, log_rows, log_blowup, shift, layout, d_lde);
  if (st != V3DB_OK) return st;
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  st = check_canonical(ctx, d_trace, size_t(n_cols) << log_rows, s);
  if (st != V3DB_OK) return st;
  void *z = nullptr;
  st = ctx_scratch(ctx, s, lde_scratch_bytes(n_cols, log_rows, log_blowup, layout), &z);
  if (st != V3DB_OK) return st;
  return enqueue_lde(ctx, d_trace, n_cols, log_rows, log_blowup, shift, layout, d_lde, (uint64_t *)z, s);
}

v3db_status v3db_poseidon_permute(v3db_ctx *ctx, uint64_t *d_states, size_t count, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "permute: NULL ctx");
  if (count == 0) return V3DB_OK;
  if (!d_states) return set_error(V3DB_ERR_INVALID_ARG, "permute: NULL states");
  if (count > (size_t(1) << 40)) return set_error(V3DB_ERR_UNSUPPORTED, "permute: count too large");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  v3db_status st = check_canonical(ctx, d_states, count * WIDTH, s);
  if (st != V3DB_OK) return st;
  return enqueue_permute(ctx, d_states, count, s);
}

v3db_status v3db_merkle_commit(v3db_ctx *ctx, const uint64_t *d_mat, uint32_t n_cols, uint32_t log_leaves,
                               uint32_t cap_height, uint64_t *d_tree, uint64_t *d_cap, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "merkle_commit: NULL ctx");
  v3db_status st = check_merkle_args(d_mat, n_cols, log_leaves, cap_height, d_cap);
  if (st != V3DB_OK) return st;
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  st = check_canonical(ctx, d_mat, size_t(n_cols) << log_leaves, s);
  if (st != V3DB_OK) return st;
  uint64_t *tree = d_tree;
  if (!tree) {
    const size_t digests = (size_t(2) << log_leaves) - (size_t(1) << cap_height);
    void *p = nullptr;
    st = ctx_scratch(ctx, s, digests * DIGEST * 8, &p);
    if (st != V3DB_OK) return st;
    tree = (uint64_t *)p;
  }
  st = enqueue_leaf_hash(ctx, d_mat, n_cols, log_leaves, tree, s);
  if (st != V3DB_OK) return st;
  return enqueue_merkle_levels(ctx, tree, log_leaves, cap_height, d_cap, s);
}


static v3db::LdeSchedule to_internal(const v3db_schedule &s) {
  v3db::LdeSchedule r{};
  r.L2 = s.split_log;
  r.cap1 = s.tile_cap[0], r.cap2 = s.tile_cap[1], r.cap3 = s.tile_cap[2];
  r.chunk = s.chunk_cols;
  r.us = s.time_us;
  return r;
}

static v3db_schedule to_public(uint32_t L, uint32_t b, const v3db::LdeSchedule &s) {
  v3db_schedule r{};
  r.log_rows = L, r.log_blowup = b;
  r.split_log = s.L2;
  r.tile_cap[0] = s.cap1, r.tile_cap[1] = s.cap2, r.tile_cap[2] = s.cap3;
  r.chunk_cols = s.chunk;
  r.time_us = s.us;
  return r;
}

static v3db_status check_shape(const char *who, uint32_t L, uint32_t b) {
  if (L > V3DB_MAX_LOG_ROWS || b > V3DB_MAX_LOG_BLOWUP || L + b > V3DB_MAX_LOG_LDE)
    return set_error(V3DB_ERR_UNSUPPORTED, std::string(who) + ": shape beyond the build limits");
  return V3DB_OK;
}

// Install a schedule; the caller holds ctx->mu. Cached plans of the shape and every
// batched graph (which hold the plans' tables and launch shapes) are dropped.
static v3db_status install_schedule(v3db_ctx *ctx, uint32_t L, uint32_t b, const v3db::LdeSchedule &s) {
  (void)hipSetDevice(ctx->device);
  v3db_status st = hip_check(hipDeviceSynchronize(), "set_schedule: wait for device");
  if (st != V3DB_OK) return st;
  free_batch_graphs(ctx);
  drop_plans(ctx, L, b);
  ctx->tuned[{L, b}] = s;
  return V3DB_OK;
}

v3db_status v3db_autotune_lde(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, uint32_t n_cols,
                              v3db_layout layout, v3db_schedule *out) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "autotune_lde: NULL ctx");
  if (n_cols == 0 || n_cols > V3DB_MAX_COLS) return set_error(V3DB_ERR_INVALID_ARG, "autotune_lde: bad n_cols");
  if (layout != V3DB_LAYOUT_NATURAL && layout != V3DB_LAYOUT_BITREV)
    return set_error(V3DB_ERR_INVALID_ARG, "autotune_lde: unknown layout");
  v3db_status st = check_shape("autotune_lde", log_rows, log_blowup);
  if (st != V3DB_OK) return st;
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  v3db::LdeSchedule best;
  st = autotune_lde(ctx, log_rows, log_blowup, n_cols, layout, &best);
  if (st != V3DB_OK) return st;
  st = install_schedule(ctx, log_rows, log_blowup, best);
  if (st == V3DB_OK && out) *out = to_public(log_rows, log_blowup, best);
  return st;
}

v3db_status v3db_get_schedule(v3db_ctx *ctx, uint32_t log_rows, uint32_t log_blowup, v3db_schedule *out) {
  clear_error();
  if (!ctx || !out) return set_error(V3DB_ERR_INVALID_ARG, "get_schedule: NULL argument");
  v3db_status st = check_shape("get_schedule", log_rows, log_blowup);
  if (st != V3DB_OK) return st;
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->tuned.find({log_rows, log_blowup});
  *out = to_public(log_rows, log_blowup,
                   it != ctx->tuned.end() ? it->second : default_schedule(log_rows, log_blowup));
  return V3DB_OK;
}

v3db_status v3db_set_schedule(v3db_ctx *ctx, const v3db_schedule *s) {
  clear_error();
  if (!ctx || !s) return set_error(V3DB_ERR_INVALID_ARG, "set_schedule: NULL argument");
  v3db_status st = check_shape("set_schedule", s->log_rows, s->log_blowup);
  if (st != V3DB_OK) return st;
  const v3db::LdeSchedule in = to_internal(*s);
  if (!schedule_valid(in, s->log_rows, s->log_blowup))
    return set_error(V3DB_ERR_INVALID_ARG, "set_schedule: schedule out of bounds");
  std::lock_guard<std::mutex> g(ctx->mu);
  return install_schedule(ctx, s->log_rows, s->log_blowup, in);
}

v3db_status v3db_schedules_save(v3db_ctx *ctx, const char *path, size_t *count) {
  clear_error();
  if (!ctx || !path) return set_error(V3DB_ERR_INVALID_ARG, "schedules_save: NULL argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  FILE *f = fopen(path, "w");
  if (!f) return set_error(V3DB_ERR_INVALID_ARG, std::string("schedules_save: cannot open ") + path);
  size_t k = 0;
  for (const auto &kv : ctx->tuned) {
    const v3db::LdeSchedule &s = kv.second;
    fprintf(f, "v3db-schedule %u %u %u %u %u %u %u %.3f\n", kv.first.first, kv.first.second, s.L2, s.cap1,
            s.cap2, s.cap3, s.chunk, s.us);
    k++;
  }
  const bool ok = fclose(f) == 0;
  if (!ok) return set_error(V3DB_ERR_INVALID_ARG, std::string("schedules_save: write failed: ") + path);
  if (count) *count = k;
  return V3DB_OK;
}

v3db_status v3db_schedules_load(v3db_ctx *ctx, const char *path, size_t *count) {
  clear_error();
  if (!ctx || !path) return set_error(V3DB_ERR_INVALID_ARG, "schedules_load: NULL argument");
  FILE *f = fopen(path, "r");
  if (!f) return set_error(V3DB_ERR_INVALID_ARG, std::string("schedules_load: cannot open ") + path);
  std::lock_guard<std::mutex> g(ctx->mu);
  char line[256];
  size_t k = 0, lineno = 0;
  v3db_status st = V3DB_OK;
  while (st == V3DB_OK && fgets(line, sizeof line, f)) {
    lineno++;
    if (strncmp(line, "v3db-schedule ", 14) != 0) continue;
    unsigned L, b, l2, c1, c2, c3, ch;
    double us;
    v3db::LdeSchedule s{};
    if (sscanf(line + 14, "%u %u %u %u %u %u %u %lf", &L, &b, &l2, &c1, &c2, &c3, &ch, &us) != 8) {
      st = set_error(V3DB_ERR_INVALID_ARG, "schedules_load: malformed line " + std::to_string(lineno));
      break;
    }
    s.L2 = l2, s.cap1 = c1, s.cap2 = c2, s.cap3 = c3, s.chunk = ch, s.us = us;
    if (check_shape("schedules_load", L, b) != V3DB_OK || !schedule_valid(s, L, b)) {
      st = set_error(V3DB_ERR_INVALID_ARG, "schedules_load: schedule out of bounds on line " + std::to_string(lineno));
      break;
    }
    st = install_schedule(ctx, L, b, s);
    if (st == V3DB_OK) k++;
  }
  fclose(f);
  if (count) *count = k;
  return st;
}


v3db_status v3db_open_batch(v3db_ctx *ctx, const uint64_t *d_mat, uint32_t n_cols, uint32_t log_leaves,
                            const uint64_t *d_tree, uint32_t cap_height, const uint64_t *d_idx, size_t n_queries,
                            uint64_t *d_rows, uint64_t *d_paths, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "open_batch: NULL ctx");
  v3db_status st = check_open_args("open_batch", d_mat, d_tree, d_idx, n_cols, log_leaves, cap_height, n_queries,
                                   d_paths);
  if (st == V3DB_OK && n_queries && !d_rows) st = set_error(V3DB_ERR_INVALID_ARG, "open_batch: NULL rows");
  if (st != V3DB_OK || n_queries == 0) return st;
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  st = check_indices(ctx, d_idx, n_queries, uint64_t(1) << log_leaves, s);
  if (st != V3DB_OK) return st;
  return enqueue_open(ctx, d_mat, n_cols, log_leaves, d_tree, cap_height, d_idx, n_queries, d_rows, d_paths, s);
}

v3db_status v3db_verify_batch(v3db_ctx *ctx, const uint64_t *d_rows, uint32_t n_cols, uint32_t log_leaves,
                              uint32_t cap_height, const uint64_t *d_idx, size_t n_queries, const uint64_t *d_paths,
                              const uint64_t *d_cap, uint32_t *d_ok, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "verify_batch: NULL ctx");
  v3db_status st = check_open_args("verify_batch", d_rows, d_cap, d_idx, n_cols, log_leaves, cap_height, n_queries,
                                   d_paths);
  if (st == V3DB_OK && n_queries && !d_ok) st = set_error(V3DB_ERR_INVALID_ARG, "verify_batch: NULL ok");
  if (st != V3DB_OK || n_queries == 0) return st;
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  st = check_indices(ctx, d_idx, n_queries, uint64_t(1) << log_leaves, s);
  if (st != V3DB_OK) return st;
  return enqueue_verify(ctx, d_rows, n_cols, log_leaves, cap_height, d_idx, n_queries, d_paths, d_cap, d_ok, s);
}


v3db_status v3db_snapshot_commit(v3db_ctx *ctx, const v3db_snapshot *sn, uint64_t *d_list_roots,
                                 uint64_t *d_root_mk, uint64_t *d_root_cb, v3db_stream stream) {
  clear_error();
  if (!ctx || !sn) return set_error(V3DB_ERR_INVALID_ARG, "snapshot_commit: NULL ctx or snapshot");
  if (!sn->d_flag || !sn->d_item || !sn->d_codes || !sn->d_centroids || !sn->d_codebooks || !d_root_mk || !d_root_cb)
    return set_error(V3DB_ERR_INVALID_ARG, "snapshot_commit: NULL array");
  if (sn->m == 0 || sn->k == 0 || sn->dim == 0 || sn->dim % sn->m != 0)
    return set_error(V3DB_ERR_INVALID_ARG, "snapshot_commit: need m >= 1, k >= 1 and dim a positive multiple of m");
  if (sn->log_lists + sn->log_slots > V3DB_MAX_LOG_LDE || sn->m > 65535 || uint64_t(sn->k) * sn->dim >= (uint64_t(1) << 32))
    return set_error(V3DB_ERR_UNSUPPORTED, "snapshot_commit: shape beyond the build limits");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t n_list = size_t(1) << sn->log_lists, N = n_list << sn->log_slots;
  v3db_status st = check_canonical(ctx, sn->d_flag, N, s);
  if (st == V3DB_OK) st = check_canonical(ctx, sn->d_item, N, s);
  if (st == V3DB_OK) st = check_canonical(ctx, sn->d_codes, N * sn->m, s);
  if (st == V3DB_OK) st = check_canonical(ctx, sn->d_centroids, n_list * sn->dim, s);
  if (st == V3DB_OK) st = check_canonical(ctx, sn->d_codebooks, size_t(sn->k) * sn->dim, s);
  if (st != V3DB_OK) return st;
  void *z = nullptr;
  st = ctx_scratch(ctx, s, snapshot_scratch_words(sn->log_lists, sn->log_slots) * 8, &z);
  if (st != V3DB_OK) return st;
  return enqueue_snapshot(ctx, sn->log_lists, sn->log_slots, sn->m, sn->dim, sn->k, sn->d_flag, sn->d_item,
                          sn->d_codes, sn->d_centroids, sn->d_codebooks, d_list_roots, d_root_mk, d_root_cb,
                          (uint64_t *)z, s);
}


v3db_status v3db_grand_product(v3db_ctx *ctx, const uint64_t *d_cols, uint32_t width, uint64_t n, uint64_t alpha,
                               uint64_t beta, uint64_t *d_z, uint64_t *d_total, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "grand_product: NULL ctx");
  if (!d_total || (n && !d_cols)) return set_error(V3DB_ERR_INVALID_ARG, "grand_product: NULL pointer");
  if (width == 0) return set_error(V3DB_ERR_INVALID_ARG, "grand_product: width must be > 0");
  if (width > V3DB_MAX_COLS || n >= (uint64_t(1) << 40))
    return set_error(V3DB_ERR_UNSUPPORTED, "grand_product: width <= 65535 and n < 2^40 required");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  v3db_status st = check_canonical(ctx, d_cols, size_t(width) * n, s);
  if (st != V3DB_OK) return st;
  void *z = nullptr;
  st = ctx_scratch(ctx, s, grand_product_scratch_words(n) * 8, &z);
  if (st != V3DB_OK) return st;
  return enqueue_grand_product(ctx, d_cols, width, n, alpha, beta, d_z, d_total, (uint64_t *)z, s);
}


v3db_status v3db_fri_commit(v3db_ctx *ctx, const uint64_t *d_codeword, uint32_t log_n, uint64_t shift,
                            const uint64_t *betas, uint32_t rounds, uint32_t cap_height, uint64_t *d_folded,
                            uint64_t *d_trees, uint64_t *d_caps, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "fri_commit: NULL ctx");
  if (!d_codeword || !betas || !d_folded || !d_caps) return set_error(V3DB_ERR_INVALID_ARG, "fri_commit: NULL pointer");
  if (log_n > V3DB_MAX_LOG_LDE) return set_error(V3DB_ERR_UNSUPPORTED, "fri_commit: log_n > 26");
  if (rounds == 0 || rounds + cap_height > log_n)
    return set_error(V3DB_ERR_INVALID_ARG, "fri_commit: need 1 <= rounds and rounds + cap_height <= log_n");
  if (shift % gl::P == 0) return set_error(V3DB_ERR_INVALID_ARG, "fri_commit: shift is 0 mod p");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  v3db_status st = check_canonical(ctx, d_codeword, size_t(1) << log_n, s);
  if (st != V3DB_OK) return st;
  void *z = nullptr;
  if (!d_trees) {  // every round's tree at once: the rounds' trees are built in one batch
    st = ctx_scratch(ctx, s, fri_tree_digests(log_n, rounds, cap_height) * DIGEST * 8, &z);
    if (st != V3DB_OK) return st;
  }
  return enqueue_fri_commit(ctx, d_codeword, log_n, shift, betas, rounds, cap_height, d_folded, d_trees, d_caps,
                            (uint64_t *)z, s);
}

}  // extern "C"
