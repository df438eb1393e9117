// Commit of many traces: v3db_commit_batch.
#include <string>

#include "internal.h"

namespace v3db {

static size_t tree_digests(uint32_t log_leaves, uint32_t cap_height) {
  return (size_t(2) << log_leaves) - (size_t(1) << cap_height);
}

static v3db_status check_job(const v3db_commit_job &j, size_t idx) {
  const std::string pre = "commit job " + std::to_string(idx) + ": ";
  if (!j.d_trace || !j.d_cap) return set_error(V3DB_ERR_INVALID_ARG, pre + "NULL trace or cap pointer");
  if (j.n_cols == 0) return set_error(V3DB_ERR_INVALID_ARG, pre + "n_cols must be > 0");
  if (j.shift == 0 || j.shift >= gl::P) return set_error(V3DB_ERR_INVALID_ARG, pre + "shift must be in [1, p)");
  if (j.layout != V3DB_LAYOUT_NATURAL && j.layout != V3DB_LAYOUT_BITREV)
    return set_error(V3DB_ERR_INVALID_ARG, pre + "unknown layout");
  if (j.n_cols > V3DB_MAX_COLS || j.log_rows > V3DB_MAX_LOG_ROWS || j.log_blowup > V3DB_MAX_LOG_BLOWUP ||
      j.log_rows + j.log_blowup > V3DB_MAX_LOG_LDE)
    return set_error(V3DB_ERR_UNSUPPORTED, pre + "shape beyond the build limits");
  if (j.cap_height > j.log_rows + j.log_blowup)
    return set_error(V3DB_ERR_INVALID_ARG, pre + "cap_height > log2(LDE rows)");
  return V3DB_OK;
}

// Scratch one job needs when run alone: its LDE (if not given), then a region
// shared by the LDE's Z workspace and the tree (the tree is written only after
// the LDE has finished on the stream).
static size_t job_scratch(const v3db_commit_job &j) {
  const uint32_t logN = j.log_rows + j.log_blowup;
  size_t lde = j.d_lde ? 0 : (size_t(j.n_cols) << logN) * 8;
  size_t z = lde_scratch_bytes(j.n_cols, j.log_rows, j.log_blowup);
  size_t tree = j.d_tree ? 0 : tree_digests(logN, j.cap_height) * DIGEST * 8;
  return lde + (z > tree ? z : tree);
}

}  // namespace v3db

using namespace v3db;

extern "C" {

size_t v3db_commit_batch_scratch_bytes(const v3db_commit_job *jobs, size_t n_jobs) {
  size_t m = 0;
  for (size_t i = 0; jobs && i < n_jobs; i++) {
    const size_t b = job_scratch(jobs[i]);
    if (b > m) m = b;
  }
  return m;
}

v3db_status v3db_commit_batch(v3db_ctx *ctx, const v3db_commit_job *jobs, size_t n_jobs, v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "commit_batch: NULL ctx");
  if (n_jobs == 0) return V3DB_OK;
  if (!jobs) return set_error(V3DB_ERR_INVALID_ARG, "commit_batch: NULL jobs");
  for (size_t i = 0; i < n_jobs; i++) {
    v3db_status st = check_job(jobs[i], i);
    if (st != V3DB_OK) return st;
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  void *scratch = nullptr;
  v3db_status st = ctx_scratch(ctx, s, v3db_commit_batch_scratch_bytes(jobs, n_jobs), &scratch);
  if (st != V3DB_OK) return st;
  for (size_t i = 0; i < n_jobs; i++) {
    const v3db_commit_job &j = jobs[i];
    const uint32_t logN = j.log_rows + j.log_blowup;
    uint8_t *p = (uint8_t *)scratch;
    uint64_t *lde = j.d_lde;
    if (!lde) {
      lde = (uint64_t *)p;
      p += (size_t(j.n_cols) << logN) * 8;
    }
    uint64_t *z = (uint64_t *)p;
    uint64_t *tree = j.d_tree ? j.d_tree : (uint64_t *)p;
    hipEvent_t e0 = prof_mark(ctx, s);
    st = enqueue_lde(ctx, j.d_trace, j.n_cols, j.log_rows, j.log_blowup, j.shift, j.layout, lde, z, s);
    if (st != V3DB_OK) return st;
    hipEvent_t e1 = prof_mark(ctx, s);
    st = enqueue_leaf_hash(ctx, lde, j.n_cols, logN, tree, s);
    if (st != V3DB_OK) return st;
    hipEvent_t e2 = prof_mark(ctx, s);
    st = enqueue_merkle_levels(ctx, tree, logN, j.cap_height, j.d_cap, s);
    if (st != V3DB_OK) return st;
    hipEvent_t e3 = prof_mark(ctx, s);
    prof_interval(ctx, V3DB_PHASE_LDE, e0, e1);
    prof_interval(ctx, V3DB_PHASE_LEAF, e1, e2);
    prof_interval(ctx, V3DB_PHASE_MERKLE, e2, e3);
  }
  return V3DB_OK;
}

}  // extern "C"
