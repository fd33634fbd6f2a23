// FP64 phi_1 of the m x m RFD core on gfx950.
//
// S = lambda phi_1(lambda M), M = B^T A = diag(c) Mraw diag(c) diag(s), by
// scaling and squaring with truncated Taylor series evaluated by the
// Paterson-Stockmeyer scheme (no linear solve):
//
//   X = lambda M, s = max(0, ceil(log2(||X||_1 / theta_23))), Y = X / 2^s
//   P = sum_{k<=23} Y^k / (k+1)!  (phi_1(Y)),   E = sum_{k<=23} Y^k / k!  (e^Y)
//
// Both series are written as sum_j Y4^j B_j with B_j = sum_{i<4} c_{4j+i} Y^i
// and evaluated by Horner's rule in Y4 = Y^4 (five products each, the two
// chains side by side in the same phases). theta_23 = 2.014710780944616 is the
// largest 1-norm for which the backward error of the degree-23 Taylor
// approximant of exp stays below 2^-53: with T(Y) = e^{Y + h(Y)},
// ||h(Y)|| / ||Y|| <= sum_n |h_n| theta^{n-1} for the power series
// h(x) = log(e^{-x} T(x)) (the backward-error bound of Al-Mohy & Higham,
// SIAM J. Matrix Anal. Appl. 31(3), 2009, applied to Taylor polynomials).
// The scaling is undone with phi_1(2Y) = phi_1(Y) (e^Y + I) / 2 and
// e^{2Y} = e^Y e^Y, s times. Powers are formed from the unscaled X with the
// exact power-of-two factors 2^{-ks} applied in the products.
//
// One body serves two schedules: k_phi1_wg (one workgroup per cloud, for
// batches) and k_phi1_grid (one cloud over a cooperative grid, with a
// counter barrier between phases).
#include "rfd_internal.h"

namespace rfd {

struct Phi1Args {
  int m;               // padded size, a multiple of 64, <= 256
  int reserved;
  double lambda;
  const double* Mraw;  // m x m, canonical order (symmetric)
  const double* cvec;  // m, canonical order
  const double* svec;  // m, canonical order
  double* ws;          // phi1_ws_doubles(m)
  int* sdev;           // s
  double* S64;         // m x m canonical: lambda phi_1(lambda M)
  double* T64;         // m x m device order: diag(c s) S diag(c)
  int* flag;           // bit 0: non-finite input; bit 1: overflow in phi_1; bit 2: barrier timeout
  unsigned* barrier;   // grid barrier counter (zeroed before launch)
};

struct WgBarrier {
  __device__ __forceinline__ void sync() { __syncthreads(); }
};

// Two-level counter barrier over a cooperative grid. Workgroups arrive on the
// counter of their group of kBarGroup (128-byte apart lines); the last arrival
// of a group (seen from the returned count) bumps the top counter, which every
// workgroup polls. Counters only grow: round r waits for r * groups top
// arrivals. Arrivals are acquire-release, the poll is relaxed and followed by
// one acquire fence. The wait is bounded: on timeout the flag gets bit 2 and
// the workgroup proceeds, so every wave always exits.
constexpr int kBarGroup = 16;
constexpr int kBarStride = 32;        // unsigned words between counters (128 bytes)
constexpr int kBarWords = kBarStride * (1 + 256 / kBarGroup);
static_assert(kBarWords <= kBarrierWords, "barrier counters exceed the plan's buffer");

struct GridBarrier {
  unsigned* ctr;
  unsigned nblocks;
  unsigned round;
  int* flag;
  __device__ __forceinline__ void sync() {
    __syncthreads();
    if (threadIdx.x == 0) {
      ++round;
      const unsigned g = blockIdx.x / kBarGroup;
      const unsigned groups = (nblocks + kBarGroup - 1) / kBarGroup;
      const unsigned gsz = (g + 1 < groups) ? kBarGroup : nblocks - g * kBarGroup;
      __threadfence();
      const unsigned old =
          __hip_atomic_fetch_add(ctr + kBarStride * (1 + g), 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1 == round * gsz) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = round * groups;
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 24)) {
          __hip_atomic_fetch_or(flag, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __threadfence();
    }
    __syncthreads();
  }
};

// ------------------------------------------------------------------ GEMM tile
// 32 x 32 tile (ti, tj) of alpha A B for row-major m x m A and B. Each wave
// computes one 16 x 16 quadrant with four independent MFMA chains (k-steps
// taken round-robin, summed in a fixed order); the caller's epilogue gets
// (i, j, value) for the four values each lane holds.
template <int m, class EPI>
__device__ __forceinline__ void gemm_tile(int ti, int tj, const double* __restrict__ A,
                                          const double* __restrict__ B, double alpha, double* lds, EPI epi) {
  double* As = lds;                 // 32 x (m + 1)
  double* Bs = lds + 32 * (m + 1);  // m x 33
  const int tid = threadIdx.x;
  constexpr int NL = 16 * m / 256;  // double2 loads per thread and operand
  __syncthreads();
  // each operand's loads are all issued before its first LDS store
  {
    const double2* A2 = (const double2*)(A + (size_t)ti * 32 * m);
    double2 va[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 256 * q;  // 32 rows x m/2 double2
      va[q] = A2[(size_t)(e / (m / 2)) * (m / 2) + (e % (m / 2))];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 256 * q;
      const int i = e / (m / 2), k2 = e % (m / 2);
      As[i * (m + 1) + 2 * k2] = va[q].x;
      As[i * (m + 1) + 2 * k2 + 1] = va[q].y;
    }
  }
  {
    double2 vb[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 256 * q;  // m rows x 16 double2
      vb[q] = *(const double2*)(B + (size_t)(e >> 4) * m + tj * 32 + 2 * (e & 15));
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 256 * q;
      const int k = e >> 4, j2 = e & 15;
      Bs[k * 33 + 2 * j2] = vb[q].x;
      Bs[k * 33 + 2 * j2 + 1] = vb[q].y;
    }
  }
  __syncthreads();
  const int w = tid >> 6, l = tid & 63, qi = w >> 1, qj = w & 1;
  f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
  const double* ap = As + (qi * 16 + (l & 15)) * (m + 1) + (l >> 4);
  const double* bp = Bs + (l >> 4) * 33 + qj * 16 + (l & 15);
#pragma unroll 4
  for (int s = 0; s < m / 4; s += 4) {
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[4 * s], bp[4 * s * 33], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[4 * s + 4], bp[(4 * s + 4) * 33], acc1, 0, 0, 0);
    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[4 * s + 8], bp[(4 * s + 8) * 33], acc2, 0, 0, 0);
    acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[4 * s + 12], bp[(4 * s + 12) * 33], acc3, 0, 0, 0);
  }
  // f64 16x16x4 output layout: register r holds row 4 r + l/16, column l%16
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * 32 + qi * 16 + 4 * r + (l >> 4);
    const int j = tj * 32 + qj * 16 + (l & 15);
    epi(i, j, alpha * ((acc0[r] + acc1[r]) + (acc2[r] + acc3[r])));
  }
}

// ------------------------------------------------------------------ body
constexpr double kTheta23 = 2.014710780944616;

// 1/k! as a compile-time constant.
constexpr double inv_factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return 1.0 / f;
}

// Coefficient block j of the two series: B_j = sum_{i<4} c_{4j+i} Y^i, with
// c_k = 1/(k+1)! for phi_1 (chain 0) and 1/k! for exp (chain 1).
template <int J, int CHAIN>
__device__ __forceinline__ double coef_block(double id, double y, double y2, double y3) {
  constexpr int o = CHAIN == 0 ? 1 : 0;
  constexpr double c0 = inv_factorial(4 * J + o), c1 = inv_factorial(4 * J + 1 + o);
  constexpr double c2 = inv_factorial(4 * J + 2 + o), c3 = inv_factorial(4 * J + 3 + o);
  return ((c0 * id + c1 * y) + c2 * y2) + c3 * y3;
}

struct TaylorWs {
  const double* X0;  // lambda M (unscaled)
  double* Y2;
  double* Y3;
  double* Y4;
  double* R[2][2];   // [chain][ping-pong]
  double sc1;        // 2^-s
};

// Horner step J (J = 4 ... 0): R_chain <- Y4 R_chain + B_J, both chains.
template <int m, int J, class BAR>
__device__ __forceinline__ void horner_phase(const TaylorWs& w, int worker, int nw, double* lds, BAR& bar) {
  constexpr int nb = m / 32, nt = nb * nb;
  constexpr int src = (J + 1) & 1, dst = J & 1;
  for (int tile = worker; tile < 2 * nt; tile += nw) {
    const int tt = tile % nt;
    const auto form = [&](int i, int j, double& id, double& y, double& y2, double& y3) {
      const size_t e = (size_t)i * m + j;
      id = i == j ? 1.0 : 0.0;
      y = w.X0[e] * w.sc1;
      y2 = w.Y2[e];
      y3 = w.Y3[e];
    };
    if (tile < nt) {
      gemm_tile<m>(tt / nb, tt % nb, w.Y4, w.R[0][src], 1.0, lds, [&](int i, int j, double v) {
        double id, y, y2, y3;
        form(i, j, id, y, y2, y3);
        w.R[0][dst][(size_t)i * m + j] = v + coef_block<J, 0>(id, y, y2, y3);
      });
    } else {
      gemm_tile<m>(tt / nb, tt % nb, w.Y4, w.R[1][src], 1.0, lds, [&](int i, int j, double v) {
        double id, y, y2, y3;
        form(i, j, id, y, y2, y3);
        w.R[1][dst][(size_t)i * m + j] = v + coef_block<J, 1>(id, y, y2, y3);
      });
    }
  }
  bar.sync();
}

template <int m, class BAR>
__device__ __forceinline__ void phi1_body(const Phi1Args& a, int worker, int nw, double* lds, BAR& bar) {
  constexpr int nb = m / 32, nt = nb * nb;
  const size_t mm = (size_t)m * m;
  double* X0 = a.ws;        // lambda M
  double* Y2 = X0 + mm;
  double* Y3 = Y2 + mm;
  double* Y4 = Y3 + mm;
  double* R00 = Y4 + mm;    // phi_1 chain, two buffers
  double* R01 = R00 + mm;
  double* R10 = R01 + mm;   // exp chain, two buffers
  double* R11 = R10 + mm;
  double* colsum = R11 + mm;
  const int t = threadIdx.x;

  // ---- P0: X0 = lambda M, and column sums of |X0| (M is symmetric, so the
  // column sum of |X0| over rows is a row sum of |Mraw| scaled by c)
  for (size_t e = (size_t)worker * 256 + t; e < mm; e += (size_t)nw * 256) {
    const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
    X0[e] = a.lambda * a.cvec[i] * a.Mraw[e] * a.cvec[j] * a.svec[j];
  }
  for (int j = worker; j < m; j += nw) {
    __syncthreads();
    lds[t] = t < m ? a.cvec[t] * fabs(a.Mraw[(size_t)j * m + t]) : 0.0;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
      if (t < o) lds[t] = lds[t] + lds[t + o];
      __syncthreads();
    }
    if (t == 0) colsum[j] = fabs(a.lambda) * a.cvec[j] * lds[0];
  }
  bar.sync();

  // ---- s from the 1-norm (every worker, same arithmetic)
  double nrm = 0.0;
  for (int j = 0; j < m; ++j) nrm = fmax(nrm, colsum[j]);
  int s = 0;
  if (!(nrm <= 1e300)) s = 0;  // non-finite input: flagged by the reduction already
  else if (nrm > kTheta23) s = (int)ceil(log2(nrm / kTheta23));
  if (s > 1000) s = 1000;
  if (worker == 0 && t == 0) *a.sdev = s;
  const double sc1 = ldexp(1.0, -s), sc2 = ldexp(1.0, -2 * s);

  // ---- P1: Y2 = X0 X0 / 4^s
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile<m>(tile / nb, tile % nb, X0, X0, sc2, lds, [&](int i, int j, double v) { Y2[(size_t)i * m + j] = v; });
  bar.sync();
  // ---- P2: Y3 = Y2 X0 / 2^s (its epilogue also forms B_5 of both chains) and Y4 = Y2 Y2
  for (int tile = worker; tile < 2 * nt; tile += nw) {
    const int tt = tile % nt;
    if (tile < nt)
      gemm_tile<m>(tt / nb, tt % nb, Y2, X0, sc1, lds, [&](int i, int j, double y3) {
        const size_t e = (size_t)i * m + j;
        const double id = i == j ? 1.0 : 0.0, y = X0[e] * sc1, y2 = Y2[e];
        Y3[e] = y3;
        R01[e] = coef_block<5, 0>(id, y, y2, y3);
        R11[e] = coef_block<5, 1>(id, y, y2, y3);
      });
    else
      gemm_tile<m>(tt / nb, tt % nb, Y2, Y2, 1.0, lds, [&](int i, int j, double v) { Y4[(size_t)i * m + j] = v; });
  }
  bar.sync();
  // ---- P3..P7: Horner steps J = 4 ... 0 (J odd reads buffer 0, writes 1 ... ends in buffer 0)
  const TaylorWs w{X0, Y2, Y3, Y4, {{R00, R01}, {R10, R11}}, sc1};
  horner_phase<m, 4>(w, worker, nw, lds, bar);
  horner_phase<m, 3>(w, worker, nw, lds, bar);
  horner_phase<m, 2>(w, worker, nw, lds, bar);
  horner_phase<m, 1>(w, worker, nw, lds, bar);
  horner_phase<m, 0>(w, worker, nw, lds, bar);
  // ---- undo the scaling: P <- P (E + I) / 2, E <- E E
  double* Pc = R00;
  double* Ec = R10;
  double* Pn = R01;
  double* En = R11;
  for (int it = 0; it < s; ++it) {
    for (int tile = worker; tile < 2 * nt; tile += nw) {
      const int tt = tile % nt;
      if (tile < nt)
        gemm_tile<m>(tt / nb, tt % nb, Ec, Ec, 1.0, lds, [&](int i, int j, double v) { En[(size_t)i * m + j] = v; });
      else
        gemm_tile<m>(tt / nb, tt % nb, Pc, Ec, 0.5, lds, [&](int i, int j, double v) {
          const size_t e = (size_t)i * m + j;
          Pn[e] = v + 0.5 * Pc[e];
        });
    }
    bar.sync();
    double* x = Ec; Ec = En; En = x;
    x = Pc; Pc = Pn; Pn = x;
  }
  // ---- S = lambda P (canonical), T = diag(c s) S diag(c) in device order
  const int fq = m / 2;
  for (size_t e = (size_t)worker * 256 + t; e < mm; e += (size_t)nw * 256) {
    const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
    const double sv = a.lambda * Pc[e];
    if (!isfinite(sv)) __hip_atomic_fetch_or(a.flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.S64[e] = sv;
    const int di = i < fq ? 2 * i : 2 * (i - fq) + 1;
    const int dj = j < fq ? 2 * j : 2 * (j - fq) + 1;
    a.T64[(size_t)di * m + dj] = a.cvec[i] * a.svec[i] * sv * a.cvec[j];
  }
}

template <int M>
__global__ __launch_bounds__(256) void k_phi1_wg(const Phi1Args* __restrict__ args) {
  extern __shared__ double lds[];
  const Phi1Args a = args[blockIdx.x];
  WgBarrier bar;
  phi1_body<M>(a, 0, 1, lds, bar);
}

template <int M>
__global__ __launch_bounds__(256) void k_phi1_grid(Phi1Args a) {
  extern __shared__ double lds[];
  GridBarrier bar{a.barrier, gridDim.x, 0u, a.flag};
  phi1_body<M>(a, (int)blockIdx.x, (int)gridDim.x, lds, bar);
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// LDS bytes of the phi_1 kernels for padded size m.
static size_t phi1_lds_bytes(int m) { return (size_t)(32 * (m + 1) + m * 33) * 8; }

size_t phi1_ws_doubles(int m) { return 8 * (size_t)m * m + m; }

static void fill_args(rfd_plan_s* p, Phi1Args& a) {
  a.m = p->dev_m;
  a.reserved = 0;
  a.lambda = p->params.lambda;
  a.Mraw = p->dev.Mraw;
  a.cvec = p->dev.cvec;
  a.svec = p->dev.svec;
  a.ws = p->dev.phi_ws;
  a.sdev = p->dev.sdev;
  a.S64 = p->dev.S64;
  a.T64 = p->dev.T64;
  a.flag = p->dev.flag;
  a.barrier = p->dev.barrier;
}

template <int M>
static hipError_t launch_phi1_m(Phi1Args& a, hipStream_t st) {
  const size_t lds = phi1_lds_bytes(M);
  hipError_t e = hipFuncSetAttribute((const void*)k_phi1_grid<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  constexpr int nb = M / 32;
  // workgroups: the widest phases (Horner steps, squarings) have 2 nb^2 tiles;
  // fewer workgroups make the barrier cheaper and give each more tiles (the
  // count never changes results: each tile is computed the same way)
  int nw = tuned(kTunePhi1Workgroups, M, 0, 1, 0, 2 * nb * nb > 128 ? 128 : 2 * nb * nb);
  if (nw < 1) nw = 1;
  if (nw > 2 * nb * nb) nw = 2 * nb * nb;
  hipLaunchKernelGGL(k_zero_u32, dim3((kBarWords + 255) / 256), dim3(256), 0, st, a.barrier, kBarWords);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* kargs[] = {&a};
  ProfileScope prof(kKPhi1, st);
  return hipLaunchCooperativeKernel((const void*)k_phi1_grid<M>, dim3(nw), dim3(256), kargs, (unsigned)lds, st);
}

hipError_t launch_phi1(rfd_plan_s* p, hipStream_t st) {
  Phi1Args a;
  fill_args(p, a);
  switch (a.m) {
    case 64: return launch_phi1_m<64>(a, st);
    case 128: return launch_phi1_m<128>(a, st);
    case 256: return launch_phi1_m<256>(a, st);
    default: return hipErrorInvalidValue;
  }
}

void phi1_fill_args(rfd_plan_s* p, void* args_out) { fill_args(p, *(Phi1Args*)args_out); }

template <int M>
static hipError_t launch_phi1_batch_m(int n, const void* dev_args, hipStream_t st) {
  const size_t lds = phi1_lds_bytes(M);
  hipError_t e = hipFuncSetAttribute((const void*)k_phi1_wg<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  ProfileScope prof(kKPhi1Batch, st);
  hipLaunchKernelGGL(k_phi1_wg<M>, dim3(n), dim3(256), lds, st, (const Phi1Args*)dev_args);
  return hipGetLastError();
}

// Sets the LDS attribute of the per-cloud kernel (outside any graph capture)
// and launches it over n argument records already in device memory.
hipError_t launch_phi1_batch_dev(int M, int n, const void* dev_args, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (M) {
    case 64: return launch_phi1_batch_m<64>(n, dev_args, st);
    case 128: return launch_phi1_batch_m<128>(n, dev_args, st);
    case 256: return launch_phi1_batch_m<256>(n, dev_args, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_phi1_batch(rfd_plan_s** plans, int n, void* dev_args, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  std::vector<Phi1Args> h(n);
  for (int i = 0; i < n; ++i) fill_args(plans[i], h[i]);
  const int m = h[0].m;
  for (int i = 1; i < n; ++i)
    if (h[i].m != m) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyAsync(dev_args, h.data(), sizeof(Phi1Args) * n, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  switch (m) {
    case 64: return launch_phi1_batch_m<64>(n, dev_args, st);
    case 128: return launch_phi1_batch_m<128>(n, dev_args, st);
    case 256: return launch_phi1_batch_m<256>(n, dev_args, st);
    default: return hipErrorInvalidValue;
  }
}

size_t phi1_args_bytes() { return sizeof(Phi1Args); }

}  // namespace rfd
