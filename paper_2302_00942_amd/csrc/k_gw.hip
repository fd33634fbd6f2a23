// Element-wise and transpose kernels of the Gromov-Wasserstein loss matrix
// (App. "Fast Computation of Tensor Products", Alg. 2). The operator actions
// themselves are resident RFD integrations; these kernels form the marginals
// p = T 1 and q = T^T 1, the diagonal field diag(p), the transposes between
// the actions, the diagonal of C (C diag(p))^T, and the final
//   L[i][j] = v1[i] + v2[j] - 2 V[j][i].
// All matrices are row-major FP32 with explicit row pitches.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "rfd_internal.h"

namespace rfd {
namespace {

constexpr int kTile = 32;

// p[i] = sum_j T[i][j]: one workgroup per row, FP64 lane sums over a fixed
// stride, then a fixed tree over the workgroup.
__global__ __launch_bounds__(256) void k_gw_row_sums(const float* __restrict__ T, int64_t ldT, int m,
                                                     float* __restrict__ p) {
  __shared__ double red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int j = t; j < m; j += 256) s += (double)T[(int64_t)i * ldT + j];
  red[t] = s;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) p[i] = (float)red[0];
}

// q[j] = sum_i T[i][j]: one thread per column, rows in order (coalesced).
__global__ __launch_bounds__(256) void k_gw_col_sums(const float* __restrict__ T, int64_t ldT, int n, int m,
                                                     float* __restrict__ q) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (double)T[(int64_t)i * ldT + j];
  q[j] = (float)s;
}

// out (n x n) = diag(v).
__global__ __launch_bounds__(256) void k_gw_diag_field(const float* __restrict__ v, int n, float* __restrict__ out,
                                                       int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
  out[(int64_t)i * ld + j] = i == j ? v[i] : 0.f;
}

// out (cols x rows) = in^T (rows x cols), through a padded 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_gw_transpose(const float* __restrict__ in, int64_t ldi, int rows, int cols,
                                                      float* __restrict__ out, int64_t ldo) {
  __shared__ float tile[kTile][kTile + 1];
  const int r0 = blockIdx.y * kTile, c0 = blockIdx.x * kTile;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int k = ty; k < kTile; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = in[(int64_t)r * ldi + c];
  }
  __syncthreads();
  for (int k = ty; k < kTile; k += 8) {
    const int c = c0 + k, r = r0 + tx;  // out row c, column r
    if (c < cols && r < rows) out[(int64_t)c * ldo + r] = tile[tx][k];
  }
}

// v[i] = Z[i][i].
__global__ __launch_bounds__(256) void k_gw_take_diag(const float* __restrict__ Z, int64_t ld, int n,
                                                      float* __restrict__ v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = Z[(int64_t)i * ld + i];
}

// L[i][j] = v1[i] + v2[j] - 2 V[j][i] for V (m x n), through a padded tile;
// rounded as fma(-2, V[j][i], v1[i] + v2[j]).
__global__ __launch_bounds__(256) void k_gw_combine(const float* __restrict__ v1, const float* __restrict__ v2,
                                                    const float* __restrict__ V, int64_t ldV, int n, int m,
                                                    float* __restrict__ L, int64_t ldL) {
  __shared__ float tile[kTile][kTile + 1];
  const int j0 = blockIdx.y * kTile, i0 = blockIdx.x * kTile;  // V rows j, columns i
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < kTile; k += 8) {
    const int j = j0 + k, i = i0 + tx;
    if (j < m && i < n) tile[k][tx] = V[(int64_t)j * ldV + i];
  }
  __syncthreads();
  for (int k = ty; k < kTile; k += 8) {
    const int i = i0 + k, j = j0 + tx;
    if (i < n && j < m) L[(int64_t)i * ldL + j] = __builtin_fmaf(-2.f, tile[tx][k], v1[i] + v2[j]);
  }
}

}  // namespace

hipError_t launch_gw_margins(const float* T, int64_t ldT, int n, int m, float* p, float* q, hipStream_t st) {
  hipLaunchKernelGGL(k_gw_row_sums, dim3(n), dim3(256), 0, st, T, ldT, m, p);
  hipLaunchKernelGGL(k_gw_col_sums, dim3((m + 255) / 256), dim3(256), 0, st, T, ldT, n, m, q);
  return hipGetLastError();
}

hipError_t launch_gw_diag_field(const float* v, int n, float* out, int64_t ld, hipStream_t st) {
  const int64_t e = (int64_t)n * n;
  hipLaunchKernelGGL(k_gw_diag_field, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, v, n, out, ld);
  return hipGetLastError();
}

hipError_t launch_gw_transpose(const float* in, int64_t ldi, int rows, int cols, float* out, int64_t ldo,
                               hipStream_t st) {
  const dim3 grid((cols + kTile - 1) / kTile, (rows + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gw_transpose, grid, dim3(256), 0, st, in, ldi, rows, cols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_gw_take_diag(const float* Z, int64_t ld, int n, float* v, hipStream_t st) {
  hipLaunchKernelGGL(k_gw_take_diag, dim3((n + 255) / 256), dim3(256), 0, st, Z, ld, n, v);
  return hipGetLastError();
}

hipError_t launch_gw_combine(const float* v1, const float* v2, const float* V, int64_t ldV, int n, int m, float* L,
                             int64_t ldL, hipStream_t st) {
  const dim3 grid((n + kTile - 1) / kTile, (m + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gw_combine, grid, dim3(256), 0, st, v1, v2, V, ldV, n, m, L, ldL);
  return hipGetLastError();
}

}  // namespace rfd
