// Spectrum of the RFD kernel matrix exp(lambda A B^T) from the low-rank
// factors (the route of the point-cloud and graph classification
// experiments): A B^T (N x N) and B^T A (m x m) share their non-zero
// eigenvalues, and A B^T has N - m more zeros when N >= m (for N < m,
// B^T A has m - N zeros that A B^T lacks). With non-negative weights
// B^T A = diag(c) Phi_u^T Phi_u diag(c) is symmetric; its eigenvalues mu are
// found by cyclic Jacobi in FP64, and the kernel's are exp(lambda mu) plus the
// eigenvalue 1 of the null space.
//
// One workgroup does everything: the m x m matrix (from the plan's Mraw and
// scales) lives in a global workspace; each Jacobi round applies m/2
// disjoint rotations (a round-robin schedule of pairs, so one sweep of m - 1
// rounds meets every pair once) as a column update A <- A J and a row update
// A <- J^T A. Sweeps stop when the off-diagonal sum of squares falls below
// 1e-30 of the matrix's, or after kMaxSweeps.
#include "rfd_internal.h"

namespace rfd {
namespace {

constexpr int kMaxSweeps = 40;

typedef __attribute__((address_space(1))) double gdouble_t;
__device__ __forceinline__ double ldg(const double* p) { return *(const gdouble_t*)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(gdouble_t*)p = v; }

// Pair t of round r over n (even) indices: n - 1 stays, the others rotate.
__device__ __forceinline__ void round_pair(int r, int t, int n, int& a, int& b) {
  if (t == 0) {
    a = r;
    b = n - 1;
  } else {
    a = (r + t) % (n - 1);
    b = (r - t + n - 1) % (n - 1);
  }
}

// Sum over the workgroup (fixed tree); every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(256) void k_spectrum(const double* __restrict__ Mraw, const double* __restrict__ cvec,
                                                  int Mp, int m, int f, double lambda, int64_t N, int which,
                                                  int64_t k, double* __restrict__ A, double* __restrict__ out,
                                                  int* __restrict__ flag) {
  __shared__ double red[256];
  __shared__ double rc[kMaxM / 2], rs[kMaxM / 2];
  __shared__ int ra[kMaxM / 2], rb[kMaxM / 2];
  __shared__ double mu[kMaxM];
  __shared__ double val[kMaxM];
  __shared__ int keep[kMaxM];
  const int t = threadIdx.x;
  const int n = m + (m & 1);  // even index count; index m is a dummy when m is odd
  const int fp = Mp / 2;
  // A = diag(c) Mraw diag(c) over the real features (canonical order)
  double fro = 0.0;
  for (int e = t; e < m * m; e += 256) {
    const int i = e / m, j = e - i * m;
    const int pi = i < f ? i : fp + (i - f), pj = j < f ? j : fp + (j - f);
    const double v = ldg(cvec + pi) * ldg(Mraw + (size_t)pi * Mp + pj) * ldg(cvec + pj);
    stg(A + e, v);
    fro += v * v;
  }
  fro = block_sum(fro, red);
  if (!isfinite(fro)) {
    if (t == 0) __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fro = 0.0;  // rotate nothing; the flag reports the input
  }
  for (int sweep = 0; sweep < kMaxSweeps && fro > 0.0; ++sweep) {
    double off = 0.0;
    for (int e = t; e < m * m; e += 256) {
      const int i = e / m, j = e - i * m;
      if (i != j) {
        const double v = ldg(A + e);
        off += v * v;
      }
    }
    off = block_sum(off, red);
    if (off <= 1e-30 * fro) break;  // uniform: every thread holds the same sums
    for (int r = 0; r < n - 1; ++r) {
      if (t < n / 2) {
        int a, b;
        round_pair(r, t, n, a, b);
        double c = 1.0, s = 0.0;
        if (a < m && b < m) {
          const double apq = ldg(A + (size_t)a * m + b);
          if (apq != 0.0) {
            const double app = ldg(A + (size_t)a * m + a), aqq = ldg(A + (size_t)b * m + b);
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        ra[t] = a;
        rb[t] = b;
        rc[t] = c;
        rs[t] = s;
      }
      __syncthreads();
      // A <- A J: columns a and b of every row
      for (int e = t; e < (n / 2) * m; e += 256) {
        const int q = e / m, i = e - q * m;
        const int a = ra[q], b = rb[q];
        if (a < m && b < m && rs[q] != 0.0) {
          const double c = rc[q], s = rs[q];
          const double x = ldg(A + (size_t)i * m + a), y = ldg(A + (size_t)i * m + b);
          stg(A + (size_t)i * m + a, c * x - s * y);
          stg(A + (size_t)i * m + b, s * x + c * y);
        }
      }
      __syncthreads();
      // A <- J^T A: rows a and b of every column
      for (int e = t; e < (n / 2) * m; e += 256) {
        const int q = e / m, j = e - q * m;
        const int a = ra[q], b = rb[q];
        if (a < m && b < m && rs[q] != 0.0) {
          const double c = rc[q], s = rs[q];
          const double x = ldg(A + (size_t)a * m + j), y = ldg(A + (size_t)b * m + j);
          stg(A + (size_t)a * m + j, c * x - s * y);
          stg(A + (size_t)b * m + j, s * x + c * y);
        }
      }
      __syncthreads();
    }
  }
  for (int i = t; i < m; i += 256) mu[i] = ldg(A + (size_t)i * m + i);
  __syncthreads();
  // for N < m, drop the m - N eigenvalues of smallest |mu| (ties by index)
  const int64_t drop = N < m ? (int64_t)m - N : 0;
  for (int i = t; i < m; i += 256) {
    int rank = 0;
    const double ai = fabs(mu[i]);
    for (int j = 0; j < m; ++j) {
      const double aj = fabs(mu[j]);
      rank += (aj < ai || (aj == ai && j < i)) ? 1 : 0;
    }
    keep[i] = rank >= drop ? 1 : 0;
    val[i] = exp(lambda * mu[i]);
  }
  __syncthreads();
  // ascending position of each kept value among all N: kept values below 1
  // first, then the N - m ones of the null space, then the rest
  const int64_t ones = N > m ? N - m : 0;
  int below = 0;
  for (int j = 0; j < m; ++j) below += (keep[j] && val[j] < 1.0) ? 1 : 0;
  for (int i = t; i < m; i += 256) {
    if (!keep[i]) continue;
    int64_t pos = 0;
    for (int j = 0; j < m; ++j)
      pos += (keep[j] && (val[j] < val[i] || (val[j] == val[i] && j < i))) ? 1 : 0;
    if (val[i] >= 1.0) pos += ones;
    const int64_t slot = which == 0 ? pos : N - 1 - pos;
    if (slot < k) stg(out + slot, val[i]);
  }
  // the ones occupy ascending positions [below, below + ones)
  const int64_t lo = which == 0 ? below : N - below - ones;
  for (int64_t p = lo + t; p < lo + ones && p < k; p += 256) stg(out + p, 1.0);
}

}  // namespace

hipError_t launch_spectrum(rfd_plan_s* p, int which, int64_t k, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_spectrum, dim3(1), dim3(256), 0, st, p->dev.Mraw, p->dev.cvec, p->dev_m, p->m, p->f,
                     p->params.lambda, p->N, which, k, p->dev.phi_ws, out, p->dev.flag);
  return hipGetLastError();
}

}  // namespace rfd
