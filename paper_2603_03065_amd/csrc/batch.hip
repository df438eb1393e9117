// Commit of many traces: v3db_commit_batch.
//
// Traces in natural layout are committed together, phase by phase: one launch
// runs pass 1 of every column of every trace, then one launch each for pass 2,
// pass 3 and leaf hashing, then one launch per tree depth covering all traces
// that still have a level at that depth. Each launch's blocks look up their
// trace in a small table of item ranges, so traces of any mix of shapes fill
// the GPU together; small traces no longer leave most of it idle, and the long
// serial top of each tree overlaps with the other trees. The launch sequence
// for a given list of shapes is captured once as a HIP graph and replayed; each
// call only refreshes the device table of buffer pointers the graph's kernels
// read. Bit-reversed traces are committed one at a time with the single-trace
// kernels.
#include <string.h>

#include <algorithm>
#include <string>

#include "lde_dev.h"
#include "poseidon_mf.h"

namespace v3db {

namespace {

constexpr int POS_THREADS = 256;
constexpr int LEAF_ROWS = 256;     // rows per leaf-hashing block
constexpr int MERKLE_NODES = 256;  // nodes per Merkle block
constexpr int PASS_2I = 8;         // phase kind of pass 2's inverse part (k_batch_pass)

// Device descriptor of one trace of a batch.
struct BJob {
  lde::LdeTask t;        // natural layout: Z is built in the output (t.z = t.lde)
  uint64_t *tree;        // levels, leaves first
  uint64_t *cap;
  uint32_t n_cols, logN, cap_height, pad;
};

// Items of one launch: range r covers items [first, first + count) of job `job`.
struct BRange {
  uint32_t first, job, count, pad;
};

__device__ __forceinline__ int find_range(const BRange *__restrict__ r, int n, uint32_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(lde::LDE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_batch_pass(const BJob *__restrict__ jobs,
                                                                  const BRange *__restrict__ ranges, int n_ranges,
                                                                  int pass, Twiddles tw) {
  extern __shared__ uint64_t sh[];
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const lde::LdeTask t = jobs[r.job].t;
  const uint32_t local = blockIdx.x - r.first;
  if (pass == 1) {
    const int tiles = lde::lde_tiles1(t);
    lde::lde_pass1_tile(t, tw, sh, local / tiles, local % tiles);
  } else if (pass == PASS_2I) {
    const int tiles = lde::lde_tiles2i(t);
    lde::lde_pass2i_tile(t, tw, sh, local / tiles, local % tiles);
  } else if (pass == 2) {
    const int tiles = lde::lde_tiles2(t);
    const int col = local / tiles;
    lde::lde_pass2_tile(t, tw, sh, col, col, local % tiles);
  } else {
    const int tiles = lde::lde_tiles3(t);
    const int col = local / tiles;
    lde::lde_pass3_tile(t, tw, sh, col, col, local % tiles);
  }
}

__global__ void __launch_bounds__(POS_THREADS) k_batch_leaf(const BJob *__restrict__ jobs,
                                                             const BRange *__restrict__ ranges, int n_ranges,
                                                             const uint64_t *__restrict__ rc, pos::Circ c) {
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const BJob &j = jobs[r.job];
  const uint64_t n_rows = uint64_t(1) << j.logN;
  const uint64_t k = uint64_t(blockIdx.x - r.first) * LEAF_ROWS + threadIdx.x;
  if (k >= n_rows) return;
  uint32_t a[WIDTH];
  pos::circ_to_vgprs(c, a);
  uint64_t *d = j.tree + k * DIGEST;
  pos::leaf_digest(j.t.lde, j.n_cols, n_rows, k, d, rc, a);
  if (j.cap_height == j.logN) {
#pragma unroll
    for (int i = 0; i < DIGEST; i++) j.cap[k * DIGEST + i] = d[i];
  }
}

// The same with the matrix-core linear layer: each wave covers 64 consecutive rows
// (held to 128 VGPRs, four waves per SIMD, as the single-trace leaf kernel).
__global__ void __launch_bounds__(POS_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_batch_leaf_mf(const BJob *__restrict__ jobs,
                                                                const BRange *__restrict__ ranges, int n_ranges,
                                                                const uint64_t *__restrict__ rc,
                                                                const uint64_t *__restrict__ tab) {
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const BJob &j = jobs[r.job];
  const uint64_t n_rows = uint64_t(1) << j.logN;
  const uint64_t base = uint64_t(blockIdx.x - r.first) * LEAF_ROWS + (threadIdx.x & ~63u);
  if (base >= n_rows) return;  // whole waves only
  const pos::MfLane L = pos::mf_lane(tab);
  pos::leaf_digests_mf(j.t.lde, j.n_cols, n_rows, base, j.tree, L, rc, tab,
                       j.cap_height == j.logN ? j.cap : nullptr);
}

// Tree depth `depth` (1 = the level above the leaves) of every listed job.
__global__ void __launch_bounds__(POS_THREADS) k_batch_merkle(const BJob *__restrict__ jobs,
                                                               const BRange *__restrict__ ranges, int n_ranges,
                                                               int depth, const uint64_t *__restrict__ rc,
                                                               pos::Circ c) {
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const BJob &j = jobs[r.job];
  const uint32_t level = j.logN - depth;  // 2^level nodes at this level
  const uint64_t count = uint64_t(1) << level;
  const uint64_t k = uint64_t(blockIdx.x - r.first) * MERKLE_NODES + threadIdx.x;
  if (k >= count) return;
  uint32_t a[WIDTH];
  pos::circ_to_vgprs(c, a);
  // level L - d starts after 2^L + 2^(L-1) + ... + 2^(L-d+1) digests
  const uint64_t off_below = (uint64_t(2) << j.logN) - (uint64_t(2) << (level + 1));
  const uint64_t off_here = (uint64_t(2) << j.logN) - (uint64_t(2) << level);
  uint64_t *d = j.tree + (off_here + k) * DIGEST;
  pos::merkle_node(j.tree + off_below * DIGEST, k, d, rc, a);
  if (level == j.cap_height) {
#pragma unroll
    for (int i = 0; i < DIGEST; i++) j.cap[k * DIGEST + i] = d[i];
  }
}

__global__ void __launch_bounds__(POS_THREADS) k_batch_merkle_mf(const BJob *__restrict__ jobs,
                                                                  const BRange *__restrict__ ranges, int n_ranges,
                                                                  int depth, const uint64_t *__restrict__ rc,
                                                                  const uint64_t *__restrict__ tab) {
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const BJob &j = jobs[r.job];
  const uint32_t level = j.logN - depth;
  const uint64_t count = uint64_t(1) << level;
  const uint64_t base = uint64_t(blockIdx.x - r.first) * MERKLE_NODES + (threadIdx.x & ~63u);
  if (base >= count) return;
  const pos::MfLane L = pos::mf_lane(tab);
  const uint64_t off_below = (uint64_t(2) << j.logN) - (uint64_t(2) << (level + 1));
  const uint64_t off_here = (uint64_t(2) << j.logN) - (uint64_t(2) << level);
  pos::merkle_nodes_mf(j.tree + off_below * DIGEST, count, base, j.tree + off_here * DIGEST, L, rc, tab,
                       level == j.cap_height ? j.cap : nullptr);
}

// The same for depths with very few nodes in all: 32 lanes per node (pair_permute).
__global__ void __launch_bounds__(pos::PAIR_THREADS) k_batch_merkle_pair(const BJob *__restrict__ jobs,
                                                                         const BRange *__restrict__ ranges,
                                                                         int n_ranges, int depth,
                                                                         const uint64_t *__restrict__ rc,
                                                                         const uint32_t *__restrict__ circ_rows) {
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const BJob &j = jobs[r.job];
  const uint32_t level = j.logN - depth;
  const uint64_t count = uint64_t(1) << level;
  const int q = threadIdx.x % pos::PAIR_GROUP, grp = threadIdx.x / pos::PAIR_GROUP, g = q & 15;
  const uint64_t k = uint64_t(blockIdx.x - r.first) * pos::PAIR_PER_BLOCK + grp;
  const bool live = k < count;
  const uint64_t off_below = (uint64_t(2) << j.logN) - (uint64_t(2) << (level + 1));
  const uint64_t off_here = (uint64_t(2) << j.logN) - (uint64_t(2) << level);
  uint64_t s = 0;
  if (live && g < 2 * DIGEST) s = j.tree[(off_below + 2 * k) * DIGEST + g];
  s = pos::pair_permute(s, q, rc, circ_rows);
  if (live && q < DIGEST) {
    const uint64_t v = gl::canon(s);
    j.tree[(off_here + k) * DIGEST + q] = v;
    if (level == j.cap_height) j.cap[k * DIGEST + q] = v;
  }
}

// The same for depths with few nodes in all: 16 lanes per node (wide_permute).
__global__ void __launch_bounds__(pos::WIDE_THREADS) k_batch_merkle_wide(const BJob *__restrict__ jobs,
                                                                         const BRange *__restrict__ ranges,
                                                                         int n_ranges, int depth,
                                                                         const uint64_t *__restrict__ rc,
                                                                         const uint32_t *__restrict__ circ_rows) {
  const BRange r = ranges[find_range(ranges, n_ranges, blockIdx.x)];
  const BJob &j = jobs[r.job];
  const uint32_t level = j.logN - depth;
  const uint64_t count = uint64_t(1) << level;
  const int g = threadIdx.x % pos::WIDE_GROUP, grp = threadIdx.x / pos::WIDE_GROUP;
  const uint64_t k = uint64_t(blockIdx.x - r.first) * pos::WIDE_PER_BLOCK + grp;
  const bool live = k < count;
  const uint64_t off_below = (uint64_t(2) << j.logN) - (uint64_t(2) << (level + 1));
  const uint64_t off_here = (uint64_t(2) << j.logN) - (uint64_t(2) << level);
  uint64_t s = 0;
  if (live && g < 2 * DIGEST) s = j.tree[(off_below + 2 * k) * DIGEST + g];
  s = pos::wide_permute(s, g, rc, circ_rows);
  if (live && g < DIGEST) {
    const uint64_t v = gl::canon(s);
    j.tree[(off_here + k) * DIGEST + g] = v;
    if (level == j.cap_height) j.cap[k * DIGEST + g] = v;
  }
}

size_t tree_digests(uint32_t log_leaves, uint32_t cap_height) {
  return (size_t(2) << log_leaves) - (size_t(1) << cap_height);
}

v3db_status check_job(const v3db_commit_job &j, size_t idx) {
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

// Scratch one job needs when committed alone: its LDE (if not given), then a
// region shared by the LDE's scratch and the tree (the tree is written only
// after the LDE has finished on the stream).
size_t single_scratch(const v3db_commit_job &j) {
  const uint32_t logN = j.log_rows + j.log_blowup;
  const size_t lde = j.d_lde ? 0 : (size_t(j.n_cols) << logN) * 8;
  const size_t z = lde_scratch_bytes(j.n_cols, j.log_rows, j.log_blowup, j.layout);
  const size_t tree = j.d_tree ? 0 : tree_digests(logN, j.cap_height) * DIGEST * 8;
  return lde + std::max(z, tree);
}

// Scratch one job needs inside a batched group (everything coexists there):
// Y, plus its LDE and tree when the caller gives none.
size_t batched_scratch(const v3db_commit_job &j) {
  const uint32_t logN = j.log_rows + j.log_blowup;
  size_t b = (size_t(j.n_cols) << j.log_rows) * 8;
  if (!j.d_lde) b += (size_t(j.n_cols) << logN) * 8;
  if (!j.d_tree) b += tree_digests(logN, j.cap_height) * DIGEST * 8;
  return (b + 255) & ~size_t(255);
}

v3db_status commit_single(v3db_ctx *ctx, const v3db_commit_job &j, void *scratch, hipStream_t s) {
  const uint32_t logN = j.log_rows + j.log_blowup;
  uint8_t *p = (uint8_t *)scratch;
  uint64_t *lde = j.d_lde;
  if (!lde) {
    lde = (uint64_t *)p;
    p += (size_t(j.n_cols) << logN) * 8;
  }
  uint64_t *tree = j.d_tree ? j.d_tree : (uint64_t *)p;
  hipEvent_t e0 = prof_mark(ctx, s);
  v3db_status st = enqueue_lde(ctx, j.d_trace, j.n_cols, j.log_rows, j.log_blowup, j.shift, j.layout, lde,
                               (uint64_t *)p, s);
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
  return V3DB_OK;
}

struct Phase {
  int kind;   // 1..3 LDE pass (PASS_2I: pass 2's inverse part), 4 leaf hashing, 5 Merkle depth, 6 (7) Merkle
              // depth with 16 (32) lanes per node
  int depth;  // Merkle depth
  size_t ranges_off, n_ranges;
  uint32_t blocks;
  size_t lds;
};

struct GroupPlan {
  std::vector<BRange> ranges;
  std::vector<Phase> phases;
};

// Phase `kind` over the jobs: job i contributes items_of(i) blocks (a range of its own).
template <class F>
void add_phase(GroupPlan &g, size_t nj, int kind, int depth, size_t lds, F items_of) {
  Phase ph{kind, depth, g.ranges.size(), 0, 0, lds};
  uint32_t first = 0;
  for (size_t i = 0; i < nj; i++) {
    const uint32_t cnt = items_of(i);
    if (!cnt) continue;
    g.ranges.push_back(BRange{first, (uint32_t)i, cnt, 0});
    first += cnt;
  }
  ph.n_ranges = g.ranges.size() - ph.ranges_off;
  ph.blocks = first;
  if (ph.blocks) g.phases.push_back(ph);
}

// Leaf hashing and the Merkle depths of trees with 2^logN[i] leaves and cap heights
// cap[i]: one phase per depth over every tree that still has that depth, its layout
// (one node per lane, 16 or 32 lanes per node) chosen by the depth's total node count.
void add_tree_phases(GroupPlan &g, const std::vector<uint32_t> &logN, const std::vector<uint32_t> &cap) {
  const size_t nj = logN.size();
  add_phase(g, nj, 4, 0, 0, [&](size_t i) {
    const uint64_t rows = uint64_t(1) << logN[i];
    return (uint32_t)((rows + LEAF_ROWS - 1) / LEAF_ROWS);
  });
  uint32_t max_depth = 0;
  for (size_t i = 0; i < nj; i++) max_depth = std::max(max_depth, logN[i] - cap[i]);
  for (uint32_t d = 1; d <= max_depth; d++) {
    auto nodes_of = [&](size_t i) -> uint64_t {
      if (logN[i] < d || logN[i] - d < cap[i]) return 0;
      return uint64_t(1) << (logN[i] - d);
    };
    uint64_t total = 0;
    for (size_t i = 0; i < nj; i++) total += nodes_of(i);
    // few nodes at this depth in all: 16 or 32 lanes per node for a shorter chain
    const bool pair = total <= MERKLE_PAIR_MAX_NODES, wide = total <= MERKLE_WIDE_MAX_NODES;
    const uint64_t per_block = pair ? pos::PAIR_PER_BLOCK : wide ? pos::WIDE_PER_BLOCK : MERKLE_NODES;
    add_phase(g, nj, pair ? 7 : wide ? 6 : 5, (int)d, 0,
              [&](size_t i) -> uint32_t { return (uint32_t)((nodes_of(i) + per_block - 1) / per_block); });
  }
}

void plan_group(const std::vector<const LdePlan *> &plans, const std::vector<v3db_commit_job> &jobs,
                GroupPlan &g) {
  const size_t nj = jobs.size();
  size_t lds[4] = {0, 0, 0, 0};
  for (size_t i = 0; i < nj; i++) {
    const LdePlan &p = *plans[i];
    const int L1 = p.L1, L2 = p.L2, b = p.log_blowup;
    lds[1] = std::max(lds[1], lde::lde_lds_words(1, L1, L2, b, p.logT1) * 8);
    lds[2] = std::max(lds[2], lde::lde_lds_words(2, L1, L2, b, p.logT2) * 8);
    lds[3] = std::max(lds[3], lde::lde_lds_words(3, L1, L2, b, p.logT3) * 8);
    lds[0] = std::max(lds[0], lde::lde_lds_words(4, L1, L2, b, p.logT2i) * 8);
  }
  add_phase(g, nj, 1, 0, lds[1], [&](size_t i) { return jobs[i].n_cols * ((1u << plans[i]->L2) >> plans[i]->logT1); });
  add_phase(g, nj, PASS_2I, 0, lds[0],
            [&](size_t i) { return jobs[i].n_cols * ((1u << plans[i]->L1) >> plans[i]->logT2i); });
  add_phase(g, nj, 2, 0, lds[2], [&](size_t i) { return jobs[i].n_cols * ((1u << plans[i]->L1) >> plans[i]->logT2); });
  add_phase(g, nj, 3, 0, lds[3], [&](size_t i) {
    return jobs[i].n_cols * ((1u << (plans[i]->L2 + plans[i]->log_blowup)) >> plans[i]->logT3);
  });
  std::vector<uint32_t> logN(nj), cap(nj);
  for (size_t i = 0; i < nj; i++) {
    logN[i] = jobs[i].log_rows + jobs[i].log_blowup;
    cap[i] = jobs[i].cap_height;
  }
  add_tree_phases(g, logN, cap);
}

// Graphs are cached per stream too: a graph's table is rewritten only by calls
// on the stream that launches it, so the previous launch has finished reading it.
std::vector<uint64_t> shape_key(const std::vector<v3db_commit_job> &jobs, hipStream_t stream) {
  std::vector<uint64_t> k;
  k.reserve(jobs.size() * 3 + 1);
  k.push_back((uint64_t)(uintptr_t)stream);
  for (const auto &j : jobs) {
    k.push_back(uint64_t(j.n_cols) | uint64_t(j.log_rows) << 32 | uint64_t(j.log_blowup) << 40 |
                uint64_t(j.cap_height) << 48);
    k.push_back(j.shift);
    k.push_back(uint64_t(j.d_lde != nullptr) | uint64_t(j.d_tree != nullptr) << 1);
  }
  return k;
}

}  // namespace

// A captured launch sequence for one list of job shapes.
struct BatchGraph {
  std::vector<uint64_t> key;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void *d_table = nullptr;      // job descriptors, then item ranges, read by the graph's kernels
  size_t table_bytes = 0, jobs_bytes = 0;
  void *h_table = nullptr;      // pinned staging copy
  hipEvent_t staged = nullptr;  // the last upload from h_table has been read
  hipEvent_t done = nullptr;    // the last launch of the graph has finished
  uint64_t last_use = 0;
};

// The table of batches launched without a graph on one stream: kept and reused (grown
// only when a batch's table is larger), so such batches allocate nothing once it has
// reached its working size.
struct EagerTable {
  hipStream_t stream = nullptr;
  void *d = nullptr, *h = nullptr;
  size_t bytes = 0;
  hipEvent_t staged = nullptr;  // the last upload from h has been read
  hipEvent_t done = nullptr;    // the last batch's kernels have finished reading d
};

static void destroy_graph(v3db_ctx *ctx, BatchGraph *g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->staged) (void)hipEventDestroy(g->staged);
  if (g->done) (void)hipEventDestroy(g->done);
  if (g->h_table) (void)hipHostFree(g->h_table);
  if (g->d_table) ctx_free(ctx, g->d_table, g->table_bytes);
  delete g;
}

static void free_eager_table(v3db_ctx *ctx, EagerTable *t) {
  if (t->staged) (void)hipEventDestroy(t->staged);
  if (t->done) (void)hipEventDestroy(t->done);
  if (t->h) (void)hipHostFree(t->h);
  if (t->d) ctx_free(ctx, t->d, t->bytes);
  delete t;
}

// Callers have waited for the device (context teardown, schedule changes).
void free_batch_graphs(v3db_ctx *ctx) {
  for (BatchGraph *g : ctx->graphs) destroy_graph(ctx, g);
  ctx->graphs.clear();
  for (EagerTable *t : ctx->eager_tables) free_eager_table(ctx, t);
  ctx->eager_tables.clear();
  ctx->seen_keys.clear();
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  ctx->capture_stream = nullptr;
}

namespace {

// The kernels of every phase of g, in order, on stream cs; the job and range tables
// are on the device.
void launch_phases(v3db_ctx *ctx, const GroupPlan &g, const BJob *d_jobs, const BRange *d_ranges, hipStream_t cs) {
  const Twiddles tw = ctx->tw;
  const pos::Circ c = pos::circ_of(ctx);
  for (const Phase &ph : g.phases) {
    const BRange *rr = d_ranges + ph.ranges_off;
    const int nr = (int)ph.n_ranges;
    if (ph.kind <= 3 || ph.kind == PASS_2I)
      hipLaunchKernelGGL(k_batch_pass, dim3(ph.blocks), dim3(lde::LDE_THREADS), ph.lds, cs, d_jobs, rr, nr, ph.kind,
                         tw);
    else if (ph.kind == 4 && ctx->mf)
      hipLaunchKernelGGL(k_batch_leaf_mf, dim3(ph.blocks), dim3(POS_THREADS), 0, cs, d_jobs, rr, nr, ctx->d_pos,
                         ctx->d_mf);
    else if (ph.kind == 4)
      hipLaunchKernelGGL(k_batch_leaf, dim3(ph.blocks), dim3(POS_THREADS), 0, cs, d_jobs, rr, nr, ctx->d_pos, c);
    else if (ph.kind == 5 && ctx->mf)
      hipLaunchKernelGGL(k_batch_merkle_mf, dim3(ph.blocks), dim3(POS_THREADS), 0, cs, d_jobs, rr, nr, ph.depth,
                         ctx->d_pos, ctx->d_mf);
    else if (ph.kind == 5)
      hipLaunchKernelGGL(k_batch_merkle, dim3(ph.blocks), dim3(POS_THREADS), 0, cs, d_jobs, rr, nr, ph.depth,
                         ctx->d_pos, c);
    else if (ph.kind == 7)
      hipLaunchKernelGGL(k_batch_merkle_pair, dim3(ph.blocks), dim3(pos::PAIR_THREADS), 0, cs, d_jobs, rr, nr,
                         ph.depth, ctx->d_pos, ctx->d_circ_rows);
    else
      hipLaunchKernelGGL(k_batch_merkle_wide, dim3(ph.blocks), dim3(pos::WIDE_THREADS), 0, cs, d_jobs, rr, nr,
                         ph.depth, ctx->d_pos, ctx->d_circ_rows);
  }
}

v3db_status capture_group(v3db_ctx *ctx, const GroupPlan &g, BatchGraph *bg) {
  if (!ctx->capture_stream) {
    v3db_status st =
        hip_check(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking), "batch capture stream");
    if (st != V3DB_OK) return st;
  }
  const BJob *d_jobs = (const BJob *)bg->d_table;
  const BRange *d_ranges = (const BRange *)((uint8_t *)bg->d_table + bg->jobs_bytes);
  hipStream_t cs = ctx->capture_stream;
  v3db_status st = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st != V3DB_OK) return st;
  launch_phases(ctx, g, d_jobs, d_ranges, cs);
  const hipError_t le = hipGetLastError();
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &graph);
  bg->graph = graph;
  if (le != hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&bg->exec, graph, nullptr, nullptr, 0);
  return hip_check(e, "capture batch graph");
}

// Launch the phases of a group without a graph, with the job and range table staged
// through the stream's own reusable table.
v3db_status launch_eager(v3db_ctx *ctx, const GroupPlan &gp, const std::vector<BJob> &bj, hipStream_t s) {
  const size_t jobs_bytes = (bj.size() * sizeof(BJob) + 255) & ~size_t(255);
  const size_t bytes = jobs_bytes + gp.ranges.size() * sizeof(BRange);
  EagerTable *t = nullptr;
  for (EagerTable *x : ctx->eager_tables)
    if (x->stream == s) t = x;
  hipError_t e = hipSuccess;
  if (!t) {
    t = new EagerTable();
    t->stream = s;
    e = hipEventCreateWithFlags(&t->staged, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t->done, hipEventDisableTiming);
    if (e != hipSuccess) {
      free_eager_table(ctx, t);
      return hip_check(e, "batch table events");
    }
    ctx->eager_tables.push_back(t);
  }
  // the last upload from the staging copy must have been read before it is rewritten
  e = hipEventSynchronize(t->staged);
  if (e != hipSuccess) return hip_check(e, "batch staging wait");
  if (bytes > t->bytes) {
    // grow (rarely: the first size covers batches of dozens of jobs) once the kernels
    // still reading the old table are done
    e = hipEventSynchronize(t->done);
    if (e != hipSuccess) return hip_check(e, "batch table wait");
    if (t->h) (void)hipHostFree(t->h);
    if (t->d) ctx_free(ctx, t->d, t->bytes);
    t->h = t->d = nullptr;
    t->bytes = 0;
    const size_t want = std::max(bytes, size_t(256) << 10);
    v3db_status st = ctx_alloc(ctx, &t->d, want, "batch tables");
    if (st != V3DB_OK) return st;
    e = hipHostMalloc(&t->h, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      ctx_free(ctx, t->d, want);
      t->d = nullptr;
      return hip_check(e, "batch staging");
    }
    t->bytes = want;
  }
  memcpy(t->h, bj.data(), bj.size() * sizeof(BJob));
  memcpy((uint8_t *)t->h + jobs_bytes, gp.ranges.data(), gp.ranges.size() * sizeof(BRange));
  e = hipMemcpyAsync(t->d, t->h, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(t->staged, s);
  if (e != hipSuccess) return hip_check(e, "batch table upload");
  hipEvent_t e0 = prof_mark(ctx, s);
  launch_phases(ctx, gp, (const BJob *)t->d, (const BRange *)((uint8_t *)t->d + jobs_bytes), s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(t->done, s);
  if (e != hipSuccess) return hip_check(e, "batch launch");
  hipEvent_t e1 = prof_mark(ctx, s);
  prof_interval(ctx, V3DB_PHASE_BATCH, e0, e1);
  return V3DB_OK;
}

// The job descriptors of a group for this call's buffers.
std::vector<BJob> group_jobs(const std::vector<const LdePlan *> &plans, const std::vector<v3db_commit_job> &jobs,
                             uint8_t *scratch) {
  const size_t nj = jobs.size();
  std::vector<BJob> bj(nj);
  uint8_t *p = scratch;
  for (size_t i = 0; i < nj; i++) {
    const v3db_commit_job &j = jobs[i];
    const uint32_t logN = j.log_rows + j.log_blowup;
    uint64_t *y = (uint64_t *)p;
    uint8_t *q = p + (size_t(j.n_cols) << j.log_rows) * 8;
    uint64_t *lde = j.d_lde;
    if (!lde) {
      lde = (uint64_t *)q;
      q += (size_t(j.n_cols) << logN) * 8;
    }
    uint64_t *tree = j.d_tree ? j.d_tree : (uint64_t *)q;
    p += batched_scratch(j);
    BJob &b = bj[i];
    b.t = lde_task(*plans[i], j.d_trace, y, nullptr, lde, V3DB_LAYOUT_NATURAL);
    b.tree = tree;
    b.cap = j.d_cap;
    b.n_cols = j.n_cols;
    b.logN = logN;
    b.cap_height = j.cap_height;
    b.pad = 0;
  }
  return bj;
}

// Commit a group of natural-layout jobs together; scratch holds
// batched_scratch() of every job, in order. A list of shapes seen for the first time
// is launched directly (a server's batches rarely repeat); from its second call on it
// is captured as a graph and replayed.
v3db_status commit_group(v3db_ctx *ctx, const std::vector<v3db_commit_job> &jobs, uint8_t *scratch,
                         hipStream_t s) {
  const size_t nj = jobs.size();
  std::vector<const LdePlan *> plans(nj);
  for (size_t i = 0; i < nj; i++) {
    v3db_status st = get_plan(ctx, jobs[i].log_rows, jobs[i].log_blowup, jobs[i].shift, &plans[i]);
    if (st != V3DB_OK) return st;
  }
  const std::vector<uint64_t> key = shape_key(jobs, s);
  BatchGraph *bg = nullptr;
  for (BatchGraph *g : ctx->graphs)
    if (g->key == key) bg = g;
  GroupPlan gp;
  plan_group(plans, jobs, gp);
  const std::vector<BJob> bj = group_jobs(plans, jobs, scratch);
  if (!bg) {
    auto seen = std::find(ctx->seen_keys.begin(), ctx->seen_keys.end(), key);
    if (seen == ctx->seen_keys.end()) {
      if (ctx->seen_keys.size() >= 64) ctx->seen_keys.erase(ctx->seen_keys.begin());
      ctx->seen_keys.push_back(key);
      return launch_eager(ctx, gp, bj, s);
    }
    ctx->seen_keys.erase(seen);
    if (ctx->graphs.size() >= 8) {  // evict the least recently used, once its last launch is done
      auto it = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                 [](BatchGraph *a, BatchGraph *b) { return a->last_use < b->last_use; });
      hipError_t e = hipEventSynchronize((*it)->done);
      if (e != hipSuccess) return hip_check(e, "graph eviction wait");
      destroy_graph(ctx, *it);
      ctx->graphs.erase(it);
    }
    bg = new BatchGraph();
    bg->key = key;
    bg->jobs_bytes = (nj * sizeof(BJob) + 255) & ~size_t(255);
    bg->table_bytes = bg->jobs_bytes + gp.ranges.size() * sizeof(BRange);
    v3db_status st = ctx_alloc(ctx, &bg->d_table, bg->table_bytes, "batch tables");
    hipError_t e = hipSuccess;
    if (st == V3DB_OK) e = hipHostMalloc(&bg->h_table, bg->table_bytes, hipHostMallocDefault);
    if (st == V3DB_OK && e == hipSuccess) e = hipEventCreateWithFlags(&bg->staged, hipEventDisableTiming);
    if (st == V3DB_OK && e == hipSuccess) e = hipEventCreateWithFlags(&bg->done, hipEventDisableTiming);
    if (st == V3DB_OK && e != hipSuccess) st = hip_check(e, "batch staging");
    if (st == V3DB_OK) st = capture_group(ctx, gp, bg);
    if (st != V3DB_OK) {
      destroy_graph(ctx, bg);
      return st;
    }
    ctx->graphs.push_back(bg);
  }
  bg->last_use = ++ctx->graph_clock;
  // the previous upload from the staging buffer must have been read before it is rewritten
  hipError_t e = hipEventSynchronize(bg->staged);
  if (e != hipSuccess) return hip_check(e, "batch staging wait");
  memcpy(bg->h_table, bj.data(), nj * sizeof(BJob));
  memcpy((uint8_t *)bg->h_table + bg->jobs_bytes, gp.ranges.data(), gp.ranges.size() * sizeof(BRange));
  e = hipMemcpyAsync(bg->d_table, bg->h_table, bg->table_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(bg->staged, s);
  if (e != hipSuccess) return hip_check(e, "batch table upload");
  hipEvent_t e0 = prof_mark(ctx, s);
  e = hipGraphLaunch(bg->exec, s);
  if (e == hipSuccess) e = hipEventRecord(bg->done, s);
  if (e != hipSuccess) return hip_check(e, "batch graph launch");
  hipEvent_t e1 = prof_mark(ctx, s);
  prof_interval(ctx, V3DB_PHASE_BATCH, e0, e1);
  return V3DB_OK;
}

}  // namespace

static void free_tree_batch_tables(v3db_ctx *ctx) {
  if (ctx->tree_table_h) (void)hipHostFree(ctx->tree_table_h);
  if (ctx->tree_table_d) ctx_free(ctx, ctx->tree_table_d, ctx->tree_table_bytes);
  ctx->tree_table_h = ctx->tree_table_d = nullptr;
  ctx->tree_table_bytes = 0;
}

v3db_status enqueue_tree_batch(v3db_ctx *ctx, const TreeJob *jobs, size_t n, hipStream_t s) {
  if (n == 0) return V3DB_OK;
  std::vector<uint32_t> logN(n), cap(n);
  std::vector<BJob> bj(n);
  for (size_t i = 0; i < n; i++) {
    logN[i] = jobs[i].log_leaves;
    cap[i] = jobs[i].cap_height;
    BJob &b = bj[i];
    b = BJob{};
    b.t.lde = const_cast<uint64_t *>(jobs[i].mat);  // read only by the hashing kernels
    b.tree = jobs[i].tree;
    b.cap = jobs[i].cap;
    b.n_cols = jobs[i].n_cols;
    b.logN = jobs[i].log_leaves;
    b.cap_height = jobs[i].cap_height;
  }
  GroupPlan gp;
  add_tree_phases(gp, logN, cap);
  const size_t jobs_bytes = (n * sizeof(BJob) + 255) & ~size_t(255);
  const size_t bytes = jobs_bytes + gp.ranges.size() * sizeof(BRange);
  hipError_t e = hipSuccess;
  if (!ctx->tree_table_staged) e = hipEventCreateWithFlags(&ctx->tree_table_staged, hipEventDisableTiming);
  if (e == hipSuccess && !ctx->tree_table_done) e = hipEventCreateWithFlags(&ctx->tree_table_done, hipEventDisableTiming);
  if (e != hipSuccess) return hip_check(e, "tree batch events");
  // the last batch (possibly on another stream) may still read the device table and
  // the staging copy: wait for its upload before rewriting the staging copy, and
  // order this call's upload after its kernels
  e = hipEventSynchronize(ctx->tree_table_staged);
  if (e == hipSuccess && bytes > ctx->tree_table_bytes) {
    e = hipEventSynchronize(ctx->tree_table_done);
    if (e == hipSuccess) {
      free_tree_batch_tables(ctx);
      void *d = nullptr, *h = nullptr;
      v3db_status st = ctx_alloc(ctx, &d, bytes, "tree batch table");
      if (st != V3DB_OK) return st;
      e = hipHostMalloc(&h, bytes, hipHostMallocDefault);
      if (e != hipSuccess) {
        ctx_free(ctx, d, bytes);
        return hip_check(e, "tree batch staging");
      }
      ctx->tree_table_d = d;
      ctx->tree_table_h = h;
      ctx->tree_table_bytes = bytes;
    }
  }
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->tree_table_done, 0);
  if (e != hipSuccess) return hip_check(e, "tree batch table");
  memcpy(ctx->tree_table_h, bj.data(), n * sizeof(BJob));
  memcpy((uint8_t *)ctx->tree_table_h + jobs_bytes, gp.ranges.data(), gp.ranges.size() * sizeof(BRange));
  e = hipMemcpyAsync(ctx->tree_table_d, ctx->tree_table_h, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->tree_table_staged, s);
  if (e != hipSuccess) return hip_check(e, "tree batch upload");
  launch_phases(ctx, gp, (const BJob *)ctx->tree_table_d,
                (const BRange *)((uint8_t *)ctx->tree_table_d + jobs_bytes), s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(ctx->tree_table_done, s);
  return hip_check(e, "tree batch launch");
}

void free_tree_batch(v3db_ctx *ctx) {
  free_tree_batch_tables(ctx);
  if (ctx->tree_table_staged) (void)hipEventDestroy(ctx->tree_table_staged);
  if (ctx->tree_table_done) (void)hipEventDestroy(ctx->tree_table_done);
  ctx->tree_table_staged = ctx->tree_table_done = nullptr;
}

// The batched LDE passes use the same 8192-word tiles as the single-trace ones.
v3db_status set_batch_kernel_attributes() {
  return hip_check(hipFuncSetAttribute((const void *)k_batch_pass, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024),
                   "batch kernel LDS limit");
}

}  // namespace v3db

using namespace v3db;

extern "C" {

// A job is batched when it is in natural layout and at least one other such
// job comes with it (a lone trace gains nothing from the batched launches and
// keeps the single-trace LDE's cache-resident column chunks).
static size_t batchable_count(const v3db_commit_job *jobs, size_t n_jobs) {
  size_t k = 0;
  for (size_t i = 0; i < n_jobs; i++) k += jobs[i].layout == V3DB_LAYOUT_NATURAL;
  return k;
}

size_t v3db_commit_batch_scratch_bytes(const v3db_commit_job *jobs, size_t n_jobs) {
  if (!jobs) return 0;
  const bool batch = batchable_count(jobs, n_jobs) >= 2;
  size_t single = 0, batched = 0;
  for (size_t i = 0; i < n_jobs; i++) {
    if (batch && jobs[i].layout == V3DB_LAYOUT_NATURAL) batched += batched_scratch(jobs[i]);
    else single = std::max(single, single_scratch(jobs[i]));
  }
  return std::max(single, batched);
}

v3db_status v3db_commit_batch(v3db_ctx *ctx, const v3db_commit_job *jobs, size_t n_jobs, v3db_stream stream) {
  return v3db::commit_batch_impl(ctx, jobs, n_jobs, (hipStream_t)stream, nullptr, 0);
}

}  // extern "C"

v3db_status v3db::commit_batch_impl(v3db_ctx *ctx, const v3db_commit_job *jobs, size_t n_jobs, hipStream_t s,
                                    void *scratch_in, size_t scratch_bytes) {
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
  // Natural-layout jobs go through the batched graph, in groups whose scratch
  // stays within the group cap; the others (and every job when batching is
  // switched off) are committed one at a time.
  std::vector<v3db_commit_job> group, singles;
  std::vector<std::vector<v3db_commit_job>> groups;
  size_t gbytes = 0;
  const bool batch = ctx->batching && batchable_count(jobs, n_jobs) >= 2;
  for (size_t i = 0; i < n_jobs; i++) {
    const v3db_commit_job &j = jobs[i];
    if (j.layout != V3DB_LAYOUT_NATURAL || !batch) {
      singles.push_back(j);
      continue;
    }
    const size_t b = batched_scratch(j);
    if (!group.empty() && gbytes + b > ctx->batch_group_bytes) {
      groups.push_back(group);
      group.clear();
      gbytes = 0;
    }
    group.push_back(j);
    gbytes += b;
  }
  if (!group.empty()) groups.push_back(group);
  size_t need = 0;
  for (const auto &j : singles) need = std::max(need, single_scratch(j));
  for (const auto &gr : groups) {
    size_t b = 0;
    for (const auto &j : gr) b += batched_scratch(j);
    need = std::max(need, b);
  }
  void *scratch = scratch_in;
  v3db_status st = V3DB_OK;
  if (scratch) {
    if (scratch_bytes < need) return set_error(V3DB_ERR_INVALID_ARG, "commit_batch: scratch too small");
  } else {
    st = ctx_scratch(ctx, s, need, &scratch);
    if (st != V3DB_OK) return st;
  }
  for (const auto &gr : groups) {
    st = commit_group(ctx, gr, (uint8_t *)scratch, s);
    if (st != V3DB_OK) return st;
  }
  for (const auto &j : singles) {
    st = commit_single(ctx, j, scratch, s);
    if (st != V3DB_OK) return st;
  }
  return V3DB_OK;
}
