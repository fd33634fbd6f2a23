// Element-wise and transpose kernels of the Gromov-Wasserstein loss matrix
// (App. "Fast Computation of Tensor Products", Alg. 2). The operator actions
// themselves are wide-field RFD integrations (the final combination
// L[i][j] = v1[i] + v2[j] - 2 W3[i][j] is the epilogue of the last one's
// store); these kernels form the marginals p = T 1 and q = T^T 1 and
// transpose the cross term for the entry point that returns it.
// All matrices are row-major FP32 with explicit row pitches. Two small
// kernels re-point the slice descriptors of a wide-field integration.
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

// Marginals in one pass over T with a fixed summation order. A workgroup
// takes a tile of kMargRows rows x 256 columns, one column per thread:
// colpart[b][j] sums the tile's rows of column j in order; the tile is also
// staged in LDS, where eight threads per row sum 32 columns each (every
// eighth column, in order) and a three-step butterfly (read from the first
// of the eight) gives
// rowpart[c][i], the sum of row i over the tile's columns; all in FP64 ...
constexpr int kMargRows = 32;
__global__ __launch_bounds__(256) void k_gw_margin_parts(const float* __restrict__ T, int64_t ldT, int n, int m,
                                                         double* __restrict__ colpart, double* __restrict__ rowpart) {
  __shared__ float tile[kMargRows][256 + 1];
  const int t = threadIdx.x;
  const int j = blockIdx.x * 256 + t, r0 = blockIdx.y * kMargRows;
  float v[kMargRows];
#pragma unroll
  for (int r = 0; r < kMargRows; ++r) v[r] = (j < m && r0 + r < n) ? T[(int64_t)(r0 + r) * ldT + j] : 0.f;
  double cs = 0.0;
#pragma unroll
  for (int r = 0; r < kMargRows; ++r) {
    cs += (double)v[r];
    tile[r][t] = v[r];
  }
  if (j < m) colpart[(size_t)blockIdx.y * m + j] = cs;
  __syncthreads();
  const int r = t >> 3, seg = t & 7;
  double rs = 0.0;
#pragma unroll 8
  for (int k = 0; k < 32; ++k) rs += (double)tile[r][seg + 8 * k];
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) rs += __shfl_xor(rs, o);
  if (seg == 0 && r0 + r < n) rowpart[(size_t)blockIdx.x * n + r0 + r] = rs;
}

// ... then p[i] = sum_c rowpart[c][i] in order, one thread per row, and
// q[j] = sum_b colpart[b][j]: 64 columns per workgroup, four row-block groups
// per column summed in order, the four group sums added in order.
__global__ __launch_bounds__(256) void k_gw_row_finish(const double* __restrict__ rowpart, int nc, int n,
                                                       float* __restrict__ p) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < nc; ++c) s += rowpart[(size_t)c * n + i];
  p[i] = (float)s;
}

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

// Re-points the slices of a wide field: descriptor i reads F + i W.
__global__ __launch_bounds__(64) void k_wide_patch(CloudDesc* __restrict__ dcl, int nsl, const float* F, int64_t ldF,
                                                   int W) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= nsl) return;
  dcl[i].F = F + (size_t)i * W;
  dcl[i].ldF = ldF;
}

// Re-points the transposed outputs of a wide field and sets its epilogue:
// descriptor i writes rows [i W, i W + W) of out and reads a + i W, b.
__global__ __launch_bounds__(64) void k_wide_patch_out(CloudDesc* __restrict__ dcl, int nsl, float* out, int64_t ldO,
                                                       const float* a, const float* b, int W) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= nsl) return;
  dcl[i].out = out + (size_t)i * W * ldO;
  dcl[i].ldO = ldO;
  dcl[i].epi_a = a + (size_t)i * W;
  dcl[i].epi_b = b;
}

}  // namespace

hipError_t launch_wide_patch_out(CloudDesc* dcl, int nsl, float* out, int64_t ldO, const float* a, const float* b,
                                 int W, hipStream_t st) {
  hipLaunchKernelGGL(k_wide_patch_out, dim3((nsl + 63) / 64), dim3(64), 0, st, dcl, nsl, out, ldO, a, b, W);
  return hipGetLastError();
}

hipError_t launch_wide_patch(CloudDesc* dcl, int nsl, const float* F, int64_t ldF, int W, hipStream_t st) {
  hipLaunchKernelGGL(k_wide_patch, dim3((nsl + 63) / 64), dim3(64), 0, st, dcl, nsl, F, ldF, W);
  return hipGetLastError();
}

size_t gw_margin_scratch_doubles(int n, int m) {
  return (size_t)((n + kMargRows - 1) / kMargRows) * m + (size_t)((m + 255) / 256) * n;
}

hipError_t launch_gw_margins(const float* T, int64_t ldT, int n, int m, float* p, float* q, double* scratch,
                             hipStream_t st) {
  const int nb = (n + kMargRows - 1) / kMargRows, nc = (m + 255) / 256;
  double* colpart = scratch;
  double* rowpart = scratch + (size_t)nb * m;
  hipLaunchKernelGGL(k_gw_margin_parts, dim3(nc, nb), dim3(256), 0, st, T, ldT, n, m, colpart, rowpart);
  hipLaunchKernelGGL(k_gw_row_finish, dim3((n + 255) / 256), dim3(256), 0, st, rowpart, nc, n, p);
  hipLaunchKernelGGL(k_gw_col_finish, dim3((m + 63) / 64), dim3(256), 0, st, colpart, nb, m, q);
  return hipGetLastError();
}

hipError_t launch_gw_transpose(const float* in, int64_t ldi, int rows, int cols, float* out, int64_t ldo,
                               hipStream_t st) {
  const dim3 grid((cols + kTile - 1) / kTile, (rows + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gw_transpose, grid, dim3(256), 0, st, in, ldi, rows, cols, out, ldo);
  return hipGetLastError();
}

}  // namespace rfd
