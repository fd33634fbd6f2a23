// Spectrum of the RFD kernel matrix exp(lambda A B^T) from the low-rank
// factors (the route of the point-cloud and graph classification
// experiments): A B^T (N x N) and B^T A (m x m) share their non-zero
// eigenvalues, and A B^T has N - m more zeros when N >= m (for N < m,
// B^T A has m - N zeros that A B^T lacks). With non-negative weights
// B^T A = diag(c) Phi_u^T Phi_u diag(c) is symmetric; its eigenvalues mu are
// found in FP64 (Householder tridiagonalisation, then bisection), and the
// kernel's are exp(lambda mu) plus the eigenvalue 1 of the null space.
//
// One workgroup does everything: the m x m matrix (from the plan's Mraw and
// scales) lives in LDS when it fits (m <= 128), else in a global workspace; m - 2 Householder reflections reduce
// it to a symmetric tridiagonal T (each a product p = 2 A22 v over the
// trailing block and the rank-2 update A22 - v q^T - q v^T, with
// q = p - (v^T p) v), and every thread then finds one eigenvalue of T by
// bisection on its Sturm count (eigenvalues below x = negative pivots of
// T - x I), from the Gershgorin interval, until the interval cannot shrink.
#include "grid_barrier.h"
#include "rfd_internal.h"

namespace rfd {
namespace {

constexpr int kMaxBisect = 200;  // bisection steps per eigenvalue (about 60-70 reach the limit of FP64)

typedef __attribute__((address_space(1))) double gdouble_t;
__device__ __forceinline__ double ldg(const double* p) { return *(const gdouble_t*)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(gdouble_t*)p = v; }

// Sum over the workgroup in a fixed order (a butterfly in each wave, read
// from lane 0, then the four wave sums in order); every thread gets the
// result. Two barriers: the second lets red be reused at once.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  const double s = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return s;
}

// Eigenvalues of the tridiagonal T (diagonal dg, od[i] = T[i][i-1], od[0] = 0)
// and the selection of the k requested kernel eigenvalues; mu, val and keep
// are workgroup scratch of m entries. Every thread of the workgroup calls it.
__device__ __forceinline__ void spectrum_finish(const SpecArgs& sa, const double* dg, const double* od, double* mu,
                                                double* val, int* keep) {
  double* __restrict__ out = sa.out;
  const double lambda = sa.lambda;
  const int64_t N = sa.N, k = sa.k;
  const int m = sa.m, which = sa.which;
  const int t = threadIdx.x;
  // bisection on the Sturm count, one eigenvalue (the j-th smallest) per thread
  double emax2 = 1.0, lo = 0.0, hi = 0.0;
  for (int i = 0; i < m; ++i) {
    const double ei = fabs(od[i]), en = i + 1 < m ? fabs(od[i + 1]) : 0.0;
    emax2 = fmax(emax2, ei * ei);
    lo = i == 0 ? dg[i] - ei - en : fmin(lo, dg[i] - ei - en);
    hi = i == 0 ? dg[i] + ei + en : fmax(hi, dg[i] + ei + en);
  }
  const double pivmin = 2.2250738585072014e-308 * emax2;
  const double tol = 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi));  // absolute accuracy, 2 eps |T|
  for (int j = t; j < m; j += 256) {
    double a = lo, b = hi;
    for (int it = 0; it < kMaxBisect; ++it) {
      const double mid = 0.5 * (a + b);
      if (!(mid > a && mid < b) || b - a <= tol) break;
      int cnt = 0;
      double q = dg[0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0 ? 1 : 0;
      for (int i = 1; i < m; ++i) {
        q = dg[i] - mid - od[i] * od[i] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0 ? 1 : 0;
      }
      if (cnt > j)
        b = mid;
      else
        a = mid;
    }
    mu[j] = 0.5 * (a + b);
  }
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
  const int64_t first_one = which == 0 ? below : N - below - ones;
  for (int64_t p = first_one + t; p < first_one + ones && p < k; p += 256) stg(out + p, 1.0);
}

// The matrix lives in LDS (dynamic, m^2 doubles) when it fits, else in the
// global workspace Ag. One workgroup per cloud.
template <bool LDS>
__device__ __forceinline__ void spectrum_body(const SpecArgs& sa) {
  const double* __restrict__ Mraw = sa.Mraw;
  const double* __restrict__ cvec = sa.cvec;
  double* __restrict__ Ag = sa.Ag;
  int* __restrict__ flag = sa.flag;
  const int Mp = sa.Mp, m = sa.m, f = sa.f;
  extern __shared__ double As[];
  const auto ld = [&](size_t e) -> double {
    if constexpr (LDS) return As[e];
    else return ldg(Ag + e);
  };
  const auto st = [&](size_t e, double v) {
    if constexpr (LDS) As[e] = v;
    else stg(Ag + e, v);
  };
  // loads in flight per thread in the two passes over A22
  constexpr int GL = 16;
  __shared__ double red[4];
  __shared__ double vv[kMaxM], qq[kMaxM];
  __shared__ double dg[kMaxM], od[kMaxM];  // T: diagonal, and od[i] = T[i][i-1]
  __shared__ double mu[kMaxM];
  __shared__ double val[kMaxM];
  __shared__ int keep[kMaxM];
  const int t = threadIdx.x;
  const int fp = Mp / 2;
  // A = diag(c) Mraw diag(c) over the real features (canonical order)
  double fro = 0.0;
  for (int e = t; e < m * m; e += 256) {
    const int i = e / m, j = e - i * m;
    const int pi = i < f ? i : fp + (i - f), pj = j < f ? j : fp + (j - f);
    const double v = ldg(cvec + pi) * ldg(Mraw + (size_t)pi * Mp + pj) * ldg(cvec + pj);
    st(e, v);
    fro += v * v;
  }
  fro = block_sum(fro, red);
  if (!isfinite(fro) && t == 0) __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // Householder tridiagonalisation; every branch below is uniform over the
  // workgroup (it depends on block sums and LDS values only)
  for (int k = 0; k + 2 < m; ++k) {
    const int r = m - k - 1;  // order of the trailing block A22 = A[k+1.., k+1..]
    double tail = 0.0;
    for (int i = t; i < r; i += 256) {
      const double x = ld((size_t)(k + 1 + i) * m + k);
      vv[i] = x;
      if (i > 0) tail += x * x;
    }
    tail = block_sum(tail, red);  // also orders the vv stores before the reads below
    const double x0 = vv[0];
    if (t == 0) dg[k] = ld((size_t)k * m + k);
    if (!(tail > 0.0)) {  // the column is reduced already (or not finite: then nothing is rotated)
      if (t == 0) od[k + 1] = x0;
      __syncthreads();
      continue;
    }
    const double sq = x0 * x0 + tail;
    const double nrm = sqrt(sq);
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double vn = sqrt(2.0 * (sq - alpha * x0));  // |x - alpha e1|
    for (int i = t; i < r; i += 256) vv[i] = (i == 0 ? x0 - alpha : vv[i]) / vn;
    __syncthreads();
    // p = 2 A22 v (A22 is symmetric: thread i walks column i, coalesced over i)
    double vp = 0.0;
    for (int i = t; i < r; i += 256) {
      // eight partial sums (ps[u] adds the j = u mod 8 terms in increasing j),
      // GL loads in flight
      double ps[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int j = 0;
      for (; j + GL <= r; j += GL) {
        double x[GL];
#pragma unroll
        for (int u = 0; u < GL; ++u) x[u] = ld((size_t)(k + 1 + j + u) * m + (k + 1 + i));
#pragma unroll
        for (int g = 0; g < GL / 8; ++g)
#pragma unroll
          for (int u = 0; u < 8; ++u) ps[u] += x[8 * g + u] * vv[j + 8 * g + u];
      }
      for (; j + 8 <= r; j += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = ld((size_t)(k + 1 + j + u) * m + (k + 1 + i));
#pragma unroll
        for (int u = 0; u < 8; ++u) ps[u] += x[u] * vv[j + u];
      }
      for (; j < r; ++j) ps[j & 7] += ld((size_t)(k + 1 + j) * m + (k + 1 + i)) * vv[j];
      const double s = ((ps[0] + ps[1]) + (ps[2] + ps[3])) + ((ps[4] + ps[5]) + (ps[6] + ps[7]));
      qq[i] = 2.0 * s;
      vp += vv[i] * (2.0 * s);
    }
    const double beta = block_sum(vp, red);
    for (int i = t; i < r; i += 256) qq[i] -= beta * vv[i];
    __syncthreads();
    // rank-2 update: thread j walks column j of A22 (coalesced over j), GL
    // rows at a time: all loads, then all stores
    for (int j = t; j < r; j += 256) {
      const double vj = vv[j], qj = qq[j];
      int i = 0;
      for (; i + GL <= r; i += GL) {
        double x[GL];
#pragma unroll
        for (int u = 0; u < GL; ++u) x[u] = ld((size_t)(k + 1 + i + u) * m + (k + 1 + j));
#pragma unroll
        for (int u = 0; u < GL; ++u)
          st((size_t)(k + 1 + i + u) * m + (k + 1 + j), x[u] - (vv[i + u] * qj + qq[i + u] * vj));
      }
      for (; i < r; ++i)
        st((size_t)(k + 1 + i) * m + (k + 1 + j), ld((size_t)(k + 1 + i) * m + (k + 1 + j)) - (vv[i] * qj + qq[i] * vj));
    }
    if (t == 0) od[k + 1] = alpha;
    __syncthreads();
  }
  if (t == 0) {
    if (m >= 2) {
      dg[m - 2] = ld((size_t)(m - 2) * m + (m - 2));
      dg[m - 1] = ld((size_t)(m - 1) * m + (m - 1));
      od[m - 1] = ld((size_t)(m - 1) * m + (m - 2));
    } else {
      dg[0] = ld(0);
    }
    od[0] = 0.0;
  }
  __syncthreads();
  spectrum_finish(sa, dg, od, mu, val, keep);
}

template <bool LDS>
__global__ __launch_bounds__(256) void k_spectrum(SpecArgs sa) {
  spectrum_body<LDS>(sa);
}

template <bool LDS>
__global__ __launch_bounds__(256) void k_spectrum_batch(const SpecArgs* __restrict__ arr) {
  const SpecArgs sa = arr[blockIdx.x];
  spectrum_body<LDS>(sa);
}

// ------------------------------------------------------------------ cooperative
// A single call with m > 128 runs on W = ceil(m / 32) workgroups of a
// cooperative grid: column j of the matrix lives in the LDS of workgroup
// j % W (local column j / W), so the passes over the trailing block read LDS
// on W CUs instead of streaming the block through one CU's L2 port at every
// step. Step k: the owner of column k forms v from its column and publishes
// it (barrier); each workgroup forms p over its columns and publishes it
// (barrier); each workgroup then takes beta and q from the whole of v and p
// and updates its columns. Every value is formed as in spectrum_body — p as
// eight strided partial sums in increasing row order, combined in the same
// tree; beta by the same workgroup sum over the same lanes; the same update —
// so the eigenvalues are its bits, and WG 0 finishes as it does. v and the
// step's skip flag alternate between two slots, so the owner of step k + 1
// never overwrites what a workgroup may still read of step k. Published
// values are agent-scope stores (coherent once acknowledged, see GridBarrier).
constexpr int kCoopCols = 32;  // columns per workgroup
// column pitch m + 8 doubles: the eight columns a wave reads in the product
// fall on different banks
constexpr int kCoopPad = 8;
constexpr int kMaxCoopSpectrumGroups = (kMaxM + kCoopCols - 1) / kCoopCols;
static_assert(kMaxCoopSpectrumGroups <= 256, "more workgroups than the grid barrier counts");

__global__ __launch_bounds__(256) void k_spectrum_coop(SpecArgs sa, unsigned* bar_ctr, double* gws) {
  GridBarrier bar{bar_ctr, gridDim.x, 0u, sa.flag};
  extern __shared__ double cols[];  // [local column][row], column pitch CP
  const double* __restrict__ Mraw = sa.Mraw;
  const double* __restrict__ cvec = sa.cvec;
  const int W = (int)gridDim.x, w = (int)blockIdx.x, t = threadIdx.x;
  const int Mp = sa.Mp, m = sa.m, f = sa.f, fp = Mp / 2;
  double* const gv = gws;             // v, two slots of m
  double* const gflag = gv + 2 * m;   // step kept (1) or skipped (0), two slots
  double* const gp = gflag + 2;       // p, m
  double* const gdg = gp + m;         // T: diagonal
  double* const god = gdg + m;        // T: od[i] = T[i][i-1]
  double* const gfro = god + m;       // per workgroup: sum of squares of its entries
  __shared__ double red[4];
  __shared__ double vv[kMaxM], qq[kMaxM];
  __shared__ double dg[kMaxM], od[kMaxM];
  __shared__ double mu[kMaxM];
  __shared__ double val[kMaxM];
  __shared__ int keep[kMaxM];
  const int ncol = (m - w + W - 1) / W;  // columns w, w + W, ...
  const int CP = m + kCoopPad;
  // A = diag(c) Mraw diag(c) over the real features (canonical order), own columns
  double fro = 0.0;
  for (int e = t; e < ncol * m; e += 256) {
    const int lc = e / m, i = e - lc * m, j = lc * W + w;
    const int pi = i < f ? i : fp + (i - f), pj = j < f ? j : fp + (j - f);
    const double v = ldg(cvec + pi) * ldg(Mraw + (size_t)pi * Mp + pj) * ldg(cvec + pj);
    cols[lc * CP + i] = v;
    fro += v * v;
  }
  fro = block_sum(fro, red);
  if (t == 0) gst_agent(gfro + w, fro);
  for (int k = 0; k + 2 < m; ++k) {
    const int r = m - k - 1, slot = k & 1;
    if (w == k % W) {  // the owner of column k
      const double* col = cols + (k / W) * CP;
      double tail = 0.0;
      for (int i = t; i < r; i += 256) {
        const double x = col[k + 1 + i];
        vv[i] = x;
        if (i > 0) tail += x * x;
      }
      tail = block_sum(tail, red);
      const double x0 = vv[0];
      if (t == 0) gst_agent(gdg + k, col[k]);
      if (!(tail > 0.0)) {
        if (t == 0) {
          gst_agent(god + k + 1, x0);
          gst_agent(gflag + slot, 0.0);
        }
      } else {
        const double sq = x0 * x0 + tail;
        const double nrm = sqrt(sq);
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double vn = sqrt(2.0 * (sq - alpha * x0));
        for (int i = t; i < r; i += 256) gst_agent(gv + slot * m + i, (i == 0 ? x0 - alpha : vv[i]) / vn);
        if (t == 0) {
          gst_agent(god + k + 1, alpha);
          gst_agent(gflag + slot, 1.0);
        }
      }
    }
    bar.sync();
    if (!(ldg(gflag + slot) != 0.0)) continue;  // the column was reduced already: no rotation
    for (int i = t; i < r; i += 256) vv[i] = ldg(gv + slot * m + i);
    __syncthreads();
    // p over this workgroup's columns c > k: eight threads per column, lane u
    // adding the rows j = u (mod 8) of the trailing block in increasing order
    {
      const int lc0 = k + 1 > w ? (k + 1 - w + W - 1) / W : 0;
      const int u = t & 7;
      for (int lc = lc0 + (t >> 3); lc < ncol; lc += 256 / 8) {
        const double* col = cols + lc * CP + (k + 1);
        double ps = 0.0;
        for (int j = u; j < r; j += 8) ps += col[j] * vv[j];
        const double a = ps + __shfl_xor(ps, 1);  // ps0 + ps1, ps2 + ps3, ...
        const double b = a + __shfl_xor(a, 2);    // (ps0 + ps1) + (ps2 + ps3), ...
        const double sum = b + __shfl_xor(b, 4);
        if (u == 0) gst_agent(gp + (lc * W + w - (k + 1)), 2.0 * sum);
      }
    }
    bar.sync();
    double vp = 0.0;
    for (int i = t; i < r; i += 256) {
      const double pi = ldg(gp + i);
      qq[i] = pi;
      vp += vv[i] * pi;
    }
    const double beta = block_sum(vp, red);
    for (int i = t; i < r; i += 256) qq[i] -= beta * vv[i];
    __syncthreads();
    // rank-2 update of this workgroup's columns c > k: a wave per column, a
    // lane per row
    {
      const int lc0 = k + 1 > w ? (k + 1 - w + W - 1) / W : 0;
      for (int lc = lc0 + (t >> 6); lc < ncol; lc += 4) {
        const int jc = lc * W + w - (k + 1);
        const double vj = vv[jc], qj = qq[jc];
        double* col = cols + lc * CP + (k + 1);
        for (int i = t & 63; i < r; i += 64) col[i] = col[i] - (vv[i] * qj + qq[i] * vj);
      }
    }
    __syncthreads();
  }
  // the last 2 x 2 block of T
  if (t == 0) {
    if (m >= 2) {
      if (w == (m - 2) % W) {
        const double* col = cols + ((m - 2) / W) * CP;
        gst_agent(gdg + m - 2, col[m - 2]);
        gst_agent(god + m - 1, col[m - 1]);
      }
      if (w == (m - 1) % W) gst_agent(gdg + m - 1, cols[((m - 1) / W) * CP + m - 1]);
    } else if (w == 0) {
      gst_agent(gdg, cols[0]);
    }
  }
  bar.sync();
  bar.finish();
  if (w != 0) return;
  for (int i = t; i < m; i += 256) {
    dg[i] = ldg(gdg + i);
    od[i] = i == 0 ? 0.0 : ldg(god + i);
  }
  if (t == 0) {
    double tot = 0.0;
    for (int v = 0; v < W; ++v) tot += ldg(gfro + v);
    if (!isfinite(tot)) __hip_atomic_fetch_or(sa.flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  spectrum_finish(sa, dg, od, mu, val, keep);
}

}  // namespace

// The m x m core goes to LDS when it fits beside the kernel's own 15 KB.
static size_t spectrum_lds_max() {
  constexpr size_t kLdsLimit = 160 * 1024 - 16 * 1024;
  // whether the large-LDS attribute was accepted: decided once per process
  // (a function-local static is initialised by exactly one thread)
  static const bool lds_ok = [] {
    const bool a = hipFuncSetAttribute((const void*)k_spectrum<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kLdsLimit) == hipSuccess;
    const bool b = hipFuncSetAttribute((const void*)k_spectrum_batch<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit) == hipSuccess;
    return a && b;
  }();
  return lds_ok ? kLdsLimit : 48 * 1024;
}

SpecArgs spectrum_args(rfd_plan_s* p, int which, int64_t k, double* out) {
  SpecArgs a;
  a.Mraw = p->dev.Mraw;
  a.cvec = p->dev.cvec;
  a.Ag = p->dev.phi_ws;
  a.out = out;
  a.flag = p->dev.flag;
  a.lambda = p->params.lambda;
  a.N = p->N;
  a.k = k;
  a.Mp = p->dev_m;
  a.m = p->m;
  a.f = p->f;
  a.which = which;
  return a;
}

hipError_t launch_spectrum(rfd_plan_s* p, int which, int64_t k, double* out, hipStream_t st) {
  SpecArgs a = spectrum_args(p, which, k, out);
  const size_t bytes = sizeof(double) * (size_t)p->m * p->m;
  if (bytes <= spectrum_lds_max()) {
    hipLaunchKernelGGL(k_spectrum<true>, dim3(1), dim3(256), bytes, st, a);
    return hipGetLastError();
  }
  // the matrix does not fit one CU's LDS: its columns spread over W workgroups
  const int W = (p->m + kCoopCols - 1) / kCoopCols;
  const size_t lds = sizeof(double) * (size_t)kCoopCols * (p->m + kCoopPad);
  static const bool attr_ok = hipFuncSetAttribute((const void*)k_spectrum_coop,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)(sizeof(double) * kCoopCols * (kMaxM + kCoopPad))) == hipSuccess;
  if (!attr_ok || W > kMaxCoopSpectrumGroups) return hipErrorInvalidValue;
  unsigned* ctr = p->dev.barrier + kSpecBarrierOffset;
  double* gws = p->dev.phi_ws;  // v (2 m), flags (2), p, dg, od (m each), W sums: within the phi_1 workspace
  void* kargs[] = {&a, &ctr, &gws};
  return hipLaunchCooperativeKernel((const void*)k_spectrum_coop, dim3(W), dim3(256), kargs, (unsigned)lds, st);
}

hipError_t launch_spectrum_batch(const SpecArgs* dev_args, int n, int max_m, hipStream_t st) {
  const size_t bytes = sizeof(double) * (size_t)max_m * max_m;
  if (bytes <= spectrum_lds_max())
    hipLaunchKernelGGL(k_spectrum_batch<true>, dim3(n), dim3(256), bytes, st, dev_args);
  else
    hipLaunchKernelGGL(k_spectrum_batch<false>, dim3(n), dim3(256), 0, st, dev_args);
  return hipGetLastError();
}

}  // namespace rfd
