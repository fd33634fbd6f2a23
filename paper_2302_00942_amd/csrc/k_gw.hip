// Element-wise and transpose kernels of the Gromov-Wasserstein loss matrix
// (App. "Fast Computation of Tensor Products", Alg. 2). The operator actions
// themselves are wide-field RFD integrations; these kernels form the
// marginals p = T 1 and q = T^T 1 and the final
//   L[i][j] = v1[i] + v2[j] - 2 V[j][i],
// and transpose the cross term for the entry point that returns it.
// All matrices are row-major FP32 with explicit row pitches. A last small
// kernel re-points the slice descriptors of a wide-field integration.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "rfd_internal.h"

namespace rfd {
namespace {

constexpr int kTile = 32;
constexpr int kXcds = 8;  // workgroups are dealt to the 8 XCDs round-robin by linear id

// Tile of a 2-D grid for this workgroup such that each XCD takes a contiguous
// run of tiles in row-major order: row-adjacent tiles share the cache lines
// that straddle their boundary (rows are not line-aligned in general), and
// on one XCD they share its L2 instead of fetching those lines twice.
__device__ __forceinline__ void xcd_tile(int& tx, int& ty) {
  const int gx = gridDim.x, total = gx * gridDim.y;
  const int b = blockIdx.y * gx + blockIdx.x;
  const int q = total / kXcds, r = total % kXcds, x = b % kXcds, k = b / kXcds;
  const int t = x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
  tx = t % gx;
  ty = t / gx;
}

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

// Column sums in two passes with a fixed order: block b of kColRows rows
// gives part[b][j] (rows in order, coalesced over j) ...
constexpr int kColRows = 64;
__global__ __launch_bounds__(256) void k_gw_col_parts(const float* __restrict__ T, int64_t ldT, int n, int m,
                                                      double* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x, b = blockIdx.y;
  if (j >= m) return;
  const int r0 = b * kColRows, r1 = min(n, r0 + kColRows);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += (double)T[(int64_t)r * ldT + j];
  part[(size_t)b * m + j] = s;
}

// ... then q[j] = sum_b part[b][j]: 64 columns per workgroup, four row-block
// groups per column summed in order, the four group sums added in order.
__global__ __launch_bounds__(256) void k_gw_col_finish(const double* __restrict__ part, int nb, int m,
                                                       float* __restrict__ q) {
  __shared__ double red[4][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6, j = blockIdx.x * 64 + c;
  const int b0 = (int)(((int64_t)g * nb) / 4), b1 = (int)(((int64_t)(g + 1) * nb) / 4);
  double s = 0.0;
  if (j < m)
    for (int b = b0; b < b1; ++b) s += part[(size_t)b * m + j];
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && j < m) q[j] = (float)(((red[0][c] + red[1][c]) + red[2][c]) + red[3][c]);
}

// out (cols x rows) = in^T (rows x cols), through a padded 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_gw_transpose(const float* __restrict__ in, int64_t ldi, int rows, int cols,
                                                      float* __restrict__ out, int64_t ldo) {
  __shared__ float tile[kTile][kTile + 1];
  int bx, by;
  xcd_tile(bx, by);
  const int r0 = by * kTile, c0 = bx * kTile;
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

// L[i][j] = v1[i] + v2[j] - 2 V[j][i] for V (m x n), through a padded tile;
// rounded as fma(-2, V[j][i], v1[i] + v2[j]).
__global__ __launch_bounds__(256) void k_gw_combine(const float* __restrict__ v1, const float* __restrict__ v2,
                                                    const float* __restrict__ V, int64_t ldV, int n, int m,
                                                    float* __restrict__ L, int64_t ldL) {
  __shared__ float tile[kTile][kTile + 1];
  int bx, by;
  xcd_tile(bx, by);
  const int j0 = by * kTile, i0 = bx * kTile;  // V rows j, columns i
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

// Re-points the slices of a wide field: descriptor i reads F + i W.
__global__ __launch_bounds__(64) void k_wide_patch(CloudDesc* __restrict__ dcl, int nsl, const float* F, int64_t ldF,
                                                   int W) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= nsl) return;
  dcl[i].F = F + (size_t)i * W;
  dcl[i].ldF = ldF;
}

}  // namespace

hipError_t launch_wide_patch(CloudDesc* dcl, int nsl, const float* F, int64_t ldF, int W, hipStream_t st) {
  hipLaunchKernelGGL(k_wide_patch, dim3((nsl + 63) / 64), dim3(64), 0, st, dcl, nsl, F, ldF, W);
  return hipGetLastError();
}

size_t gw_margin_scratch_doubles(int n, int m) { return (size_t)((n + kColRows - 1) / kColRows) * m; }

hipError_t launch_gw_margins(const float* T, int64_t ldT, int n, int m, float* p, float* q, double* scratch,
                             hipStream_t st) {
  const int nb = (n + kColRows - 1) / kColRows;
  hipLaunchKernelGGL(k_gw_row_sums, dim3(n), dim3(256), 0, st, T, ldT, m, p);
  hipLaunchKernelGGL(k_gw_col_parts, dim3((m + 255) / 256, nb), dim3(256), 0, st, T, ldT, n, m, scratch);
  hipLaunchKernelGGL(k_gw_col_finish, dim3((m + 63) / 64), dim3(256), 0, st, scratch, nb, m, q);
  return hipGetLastError();
}

hipError_t launch_gw_transpose(const float* in, int64_t ldi, int rows, int cols, float* out, int64_t ldo,
                               hipStream_t st) {
  const dim3 grid((cols + kTile - 1) / kTile, (rows + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gw_transpose, grid, dim3(256), 0, st, in, ldi, rows, cols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_gw_combine(const float* v1, const float* v2, const float* V, int64_t ldV, int n, int m, float* L,
                             int64_t ldL, hipStream_t st) {
  const dim3 grid((n + kTile - 1) / kTile, (m + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gw_combine, grid, dim3(256), 0, st, v1, v2, V, ldV, n, m, L, ldL);
  return hipGetLastError();
}

}  // namespace rfd
