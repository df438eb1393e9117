// Merkle commitment that allocates nothing: the tree levels (scratch of
// v3db_merkle_commit when the caller passes no tree) live in a file-scope device
// array of fixed size, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops).
//
// The array's host-side name is not a device address: its address on each device is
// looked up once per device (at context creation, with that device current) and only
// that address is passed to kernels and copies. Every call on a device shares that
// device's array and leaves its last contents there; calls that overlap on one device
// (other streams, other host threads) race on it.
#include <mutex>

#include "internal.h"

namespace v3db {
namespace {

static __device__ __align__(256) uint8_t scratch[V3DB_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};  // the array's device address on each device, once looked up

}  // namespace

v3db_status noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES)
    return set_error(V3DB_ERR_UNSUPPORTED, "no-alloc scratch: device index beyond 63");
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[device]) return V3DB_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "no-alloc scratch address");
  g_scratch[device] = p;
  return V3DB_OK;
}

}  // namespace v3db

using namespace v3db;

extern "C" v3db_status v3db_merkle_commit_noalloc(v3db_ctx *ctx, const uint64_t *d_mat, uint32_t n_cols,
                                                  uint32_t log_leaves, uint32_t cap_height, uint64_t *d_cap,
                                                  v3db_stream stream) {
  clear_error();
  if (!ctx) return set_error(V3DB_ERR_INVALID_ARG, "merkle_commit_noalloc: NULL ctx");
  if (!d_mat || !d_cap) return set_error(V3DB_ERR_INVALID_ARG, "merkle_commit_noalloc: NULL d_mat or d_cap");
  if (n_cols == 0) return set_error(V3DB_ERR_INVALID_ARG, "merkle_commit_noalloc: n_cols must be > 0");
  if (cap_height > log_leaves) return set_error(V3DB_ERR_INVALID_ARG, "merkle_commit_noalloc: cap_height > log_leaves");
  if (n_cols > V3DB_MAX_COLS || log_leaves > V3DB_MAX_LOG_LDE)
    return set_error(V3DB_ERR_UNSUPPORTED, "merkle_commit_noalloc: shape beyond the build limits");
  const size_t digests = (size_t(2) << log_leaves) - (size_t(1) << cap_height);
  if (digests * DIGEST * 8 > size_t(V3DB_NOALLOC_SCRATCH_BYTES))
    return set_error(V3DB_ERR_UNSUPPORTED, "merkle_commit_noalloc: the tree needs " +
                                               std::to_string(digests * DIGEST * 8) + " bytes, more than the " +
                                               std::to_string(size_t(V3DB_NOALLOC_SCRATCH_BYTES)) +
                                               "-byte static scratch (at most 2^20 leaves)");
  void *tree = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    tree = ctx->device >= 0 && ctx->device < MAX_DEVICES ? g_scratch[ctx->device] : nullptr;
  }
  if (!tree) return set_error(V3DB_ERR_DEVICE, "merkle_commit_noalloc: no scratch address for this device");
  std::lock_guard<std::mutex> g(ctx->mu);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  v3db_status st = enqueue_leaf_hash(ctx, d_mat, n_cols, log_leaves, (uint64_t *)tree, s);
  if (st != V3DB_OK) return st;
  return enqueue_merkle_levels(ctx, (uint64_t *)tree, log_leaves, cap_height, d_cap, s);
}
