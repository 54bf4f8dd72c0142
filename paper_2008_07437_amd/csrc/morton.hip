// Morton (Z-order) ordering of the locations (Section 5.3 orders locations
// this way so that nearby points share tiles, which lowers TLR ranks).
// Keys: floor(v * 2^16) clamped to [0, 65535], x bits at even and y bits at
// odd positions; the input index is appended below the key so equal keys keep
// their input order, and a bitonic network sorts the 64-bit composites.
#include "mvgeo_internal.h"

namespace mvg {

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ __forceinline__ uint32_t quant16(double v) {
  double q = floor(v * 65536.0);
  q = fmin(fmax(q, 0.0), 65535.0);
  return (uint32_t)q;
}

__global__ void k_morton_keys(const double *__restrict__ xs, const double *__restrict__ ys,
                              int64_t n, int64_t P, uint64_t *__restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  if (i < n) {
    const uint32_t m = spread16(quant16(xs[i])) | (spread16(quant16(ys[i])) << 1);
    key[i] = ((uint64_t)m << 32) | (uint64_t)i;
  } else {
    key[i] = ~(uint64_t)0;
  }
}

__global__ void k_bitonic_step(uint64_t *__restrict__ key, int64_t P, int64_t k, int64_t j) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int64_t ixj = i ^ j;
  if (ixj <= i) return;
  const bool up = (i & k) == 0;
  const uint64_t a = key[i], b = key[ixj];
  if ((a > b) == up) {
    key[i] = b;
    key[ixj] = a;
  }
}

__global__ void k_perm_out(const uint64_t *__restrict__ key, int64_t n, int64_t *__restrict__ perm,
                           const double *__restrict__ xs, const double *__restrict__ ys,
                           double *__restrict__ xo, double *__restrict__ yo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t src = (int64_t)(key[i] & 0xFFFFFFFFull);
  perm[i] = src;
  if (xo) xo[i] = xs[src];
  if (yo) yo[i] = ys[src];
}

int morton_sort(const double *d_x, const double *d_y, int64_t n, int64_t *d_perm, double *d_xs,
                double *d_ys, hipStream_t st) {
  int64_t P = 1;
  while (P < n) P <<= 1;
  uint64_t *key = nullptr;
  if (malloc_async((void **)&key, sizeof(uint64_t) * P, st) != hipSuccess) {
    hipGetLastError();
    set_error("morton_order: workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  const unsigned grid = (unsigned)((P + 255) / 256);
  hipLaunchKernelGGL(k_morton_keys, dim3(grid), dim3(256), 0, st, d_x, d_y, n, P, key);
  int rc = check_launch("morton_keys");
  for (int64_t k = 2; k <= P && !rc; k <<= 1)
    for (int64_t j = k >> 1; j > 0 && !rc; j >>= 1) {
      hipLaunchKernelGGL(k_bitonic_step, dim3(grid), dim3(256), 0, st, key, P, k, j);
      rc = check_launch("bitonic_step");
    }
  if (!rc) {
    hipLaunchKernelGGL(k_perm_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const uint64_t *)key, n, d_perm, d_x, d_y, d_xs, d_ys);
    rc = check_launch("perm_out");
  }
  hipFreeAsync(key, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = MVG_ERR_LAUNCH;
  return rc;
}

}  // namespace mvg
