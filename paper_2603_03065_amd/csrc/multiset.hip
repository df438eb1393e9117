// Multiset-equality grand product over a table of tuples (tuple compression and
// SetEq of Sec. 4.5 "Gadgets and Cost Model"): c_i = sum_k x_{k,i} beta^k for the
// rows of a column-major table, and the running products
// z_i = prod_{j <= i} (alpha - c_j). Three launches: per tile of 4096 rows the
// compressed factors (written to z) and their product; one block scanning the tile
// products; per tile the inclusive scan of its factors times the tile's prefix.
#include "internal.h"

namespace v3db {

namespace {

constexpr int GP_THREADS = 256, GP_PER_THREAD = 16, GP_TILE = GP_THREADS * GP_PER_THREAD;
constexpr int SCAN_THREADS = 1024;

// Product of the 256 values in sh (one per thread); every thread returns it.
__device__ uint64_t block_product(uint64_t v, uint64_t *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int step = GP_THREADS / 2; step > 0; step >>= 1) {
    if ((int)threadIdx.x < step) sh[threadIdx.x] = gl::mul(sh[threadIdx.x], sh[threadIdx.x + step]);
    __syncthreads();
  }
  const uint64_t r = sh[0];
  __syncthreads();
  return r;
}

// Exclusive prefix products of one value per thread (Hillis-Steele over LDS,
// double-buffered); nthreads = blockDim.x.
__device__ uint64_t exclusive_scan(uint64_t v, uint64_t *sh) {
  const int t = threadIdx.x, nt = blockDim.x;
  uint64_t *a = sh, *b = sh + nt;
  a[t] = v;
  __syncthreads();
  for (int d = 1; d < nt; d <<= 1) {
    b[t] = t >= d ? gl::mul(a[t], a[t - d]) : a[t];
    __syncthreads();
    uint64_t *x = a;
    a = b, b = x;
  }
  const uint64_t r = t ? a[t - 1] : 1;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(GP_THREADS)
    k_gp_factors(const uint64_t *__restrict__ cols, uint32_t width, uint64_t n, uint64_t alpha, uint64_t beta,
                 uint64_t *__restrict__ z, uint64_t *__restrict__ partials) {
  __shared__ uint64_t sh[GP_THREADS];
  const uint64_t base = uint64_t(blockIdx.x) * GP_TILE;
  // Horner over the columns, highest first, for 8 of the thread's 16 rows at a time:
  // each column's 8 words are requested together (rows past the end read row n - 1 and
  // are dropped below), so the loads of a column overlap instead of following one another
  constexpr int G = 8;
  uint64_t prod = 1;
  for (int g = 0; g < GP_PER_THREAD; g += G) {
    uint64_t c[G];
#pragma unroll
    for (int k = 0; k < G; k++) {
      const uint64_t i = base + uint64_t(g + k) * GP_THREADS + threadIdx.x;
      c[k] = cols[uint64_t(width - 1) * n + (i < n ? i : n - 1)];
    }
    for (int w = (int)width - 2; w >= 0; w--) {
      uint64_t x[G];
#pragma unroll
      for (int k = 0; k < G; k++) {
        const uint64_t i = base + uint64_t(g + k) * GP_THREADS + threadIdx.x;
        x[k] = cols[uint64_t(w) * n + (i < n ? i : n - 1)];
      }
#pragma unroll
      for (int k = 0; k < G; k++) c[k] = gl::add(gl::mul(c[k], beta), x[k]);
    }
#pragma unroll
    for (int k = 0; k < G; k++) {
      const uint64_t i = base + uint64_t(g + k) * GP_THREADS + threadIdx.x;
      if (i < n) {
        const uint64_t d = gl::sub(alpha, c[k]);
        if (z) z[i] = d;
        prod = gl::mul(prod, d);
      }
    }
  }
  const uint64_t p = block_product(prod, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = p;
}

// offsets[b] = product of partials[0..b-1]; *total = product of all.
__global__ void __launch_bounds__(SCAN_THREADS)
    k_gp_scan_partials(const uint64_t *__restrict__ partials, uint64_t nb, uint64_t *__restrict__ offsets,
                       uint64_t *__restrict__ total) {
  __shared__ uint64_t sh[2 * SCAN_THREADS];
  const uint64_t per = (nb + SCAN_THREADS - 1) / SCAN_THREADS;  // consecutive partials per thread
  const uint64_t lo = uint64_t(threadIdx.x) * per;
  uint64_t p = 1;
  for (uint64_t b = lo; b < lo + per && b < nb; b++) p = gl::mul(p, partials[b]);
  uint64_t run = exclusive_scan(p, sh);
  if (threadIdx.x == SCAN_THREADS - 1) total[0] = gl::mul(run, p);
  if (offsets)
    for (uint64_t b = lo; b < lo + per && b < nb; b++) {
      offsets[b] = run;
      run = gl::mul(run, partials[b]);
    }
}

// Tile of 4096 factors in z: thread t takes 16 consecutive ones (LDS rows padded
// by one word per 16 so the 16-word runs of a half-wave fall in distinct banks).
__global__ void __launch_bounds__(GP_THREADS)
    k_gp_apply(uint64_t *__restrict__ z, uint64_t n, const uint64_t *__restrict__ offsets) {
  __shared__ uint64_t tile[GP_TILE + GP_TILE / GP_PER_THREAD];
  __shared__ uint64_t sh[2 * GP_THREADS];
  const uint64_t base = uint64_t(blockIdx.x) * GP_TILE;
  auto pos = [](int w) { return w + (w >> 4); };
  {
    // all 16 words requested before any is stored (rows past the end read row n - 1
    // and store 1)
    uint64_t x[GP_PER_THREAD];
#pragma unroll
    for (int k = 0; k < GP_PER_THREAD; k++) {
      const uint64_t i = base + k * GP_THREADS + threadIdx.x;
      x[k] = z[i < n ? i : n - 1];
    }
#pragma unroll
    for (int k = 0; k < GP_PER_THREAD; k++) {
      const int w = k * GP_THREADS + threadIdx.x;
      tile[pos(w)] = base + w < n ? x[k] : 1;
    }
  }
  __syncthreads();
  const int w0 = threadIdx.x * GP_PER_THREAD;
  uint64_t v[GP_PER_THREAD];
  uint64_t run = 1;
#pragma unroll
  for (int k = 0; k < GP_PER_THREAD; k++) {
    run = gl::mul(run, tile[pos(w0 + k)]);
    v[k] = run;
  }
  const uint64_t pre = gl::mul(exclusive_scan(run, sh), offsets[blockIdx.x]);
#pragma unroll
  for (int k = 0; k < GP_PER_THREAD; k++) tile[pos(w0 + k)] = gl::mul(pre, v[k]);
  __syncthreads();
  for (int k = 0; k < GP_PER_THREAD; k++) {
    const int w = k * GP_THREADS + threadIdx.x;
    const uint64_t i = base + w;
    if (i < n) z[i] = tile[pos(w)];
  }
}

}  // namespace

size_t grand_product_scratch_words(uint64_t n) {
  const uint64_t nb = (n + GP_TILE - 1) / GP_TILE;
  return 2 * (nb ? nb : 1);
}

v3db_status enqueue_grand_product(v3db_ctx *, const uint64_t *cols, uint32_t width, uint64_t n, uint64_t alpha,
                                  uint64_t beta, uint64_t *z, uint64_t *total, uint64_t *scratch,
                                  hipStream_t stream) {
  const uint64_t nb = (n + GP_TILE - 1) / GP_TILE;
  uint64_t *partials = scratch, *offsets = scratch + (nb ? nb : 1);
  if (nb) {
    hipLaunchKernelGGL(k_gp_factors, dim3((unsigned)nb), dim3(GP_THREADS), 0, stream, cols, width, n, alpha % gl::P,
                       beta % gl::P, z, partials);
  }
  hipLaunchKernelGGL(k_gp_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, stream, partials, nb, z ? offsets : nullptr,
                     total);
  if (nb && z) hipLaunchKernelGGL(k_gp_apply, dim3((unsigned)nb), dim3(GP_THREADS), 0, stream, z, n, offsets);
  return hip_check(hipGetLastError(), "grand product launch");
}

}  // namespace v3db
