// FP64 phi_1 of the m x m RFD core on gfx950.
//
// S = lambda phi_1(lambda M), M = B^T A = diag(c) Mraw diag(c) diag(s), by
// scaling and squaring with the [13/13] Pade approximant of exp (Higham 2005,
// "The scaling and squaring method for the matrix exponential revisited"):
//
//   Y = lambda M / 2^s,  s = max(0, ceil(log2(||lambda M||_1 / theta_13)))
//   U0 = b13 Y^12 + b11 Y^10 + ... + b3 Y^2 + b1 I,   U = Y U0   (odd part)
//   V  = b12 Y^12 + ... + b2 Y^2 + b0 I                         (even part)
//   (V - U) [E | P] = [V + U | 2 U0]
//
// E approximates e^Y. P approximates phi_1(Y): the same Pade approximant
// applied to the augmented matrix [[Y, I], [0, 0]] has top-right block
// q(Y)^{-1} (p~(Y) - q~(Y)) with p~, q~ the polynomials shifted down one
// power, and p~ - q~ = 2 U0 because q(x) = p(-x) (Al-Mohy & Higham 2011 use
// this augmentation for phi functions). The scaling is undone with
// phi_1(2Y) = phi_1(Y) (e^Y + I) / 2 and e^{2Y} = e^Y e^Y, s times.
//
// The linear solve is a right-looking blocked LU with partial pivoting
// (32-column panels); the 2m right-hand-side columns ride along as trailing
// columns, so forward elimination needs no separate pass, and back
// substitution runs per 32-column strip without any cross-workgroup sync.
//
// One body serves two schedules: k_phi1_wg (one workgroup per cloud, for
// batches) and k_phi1_grid (one cloud over a cooperative grid, with a
// counter barrier between phases).
#include "rfd_internal.h"

namespace rfd {

struct Lin {  // value(i, j) = sum_q c[q] a[q][i*m + j] + (i == j ? cI : 0)
  const double* a[3];
  double c[3];
  double cI;
};

struct Phi1Args {
  int m;               // padded size, a multiple of 32, <= 256
  int reserved;
  double lambda;
  double b[14];        // Pade [13/13] numerator coefficients
  const double* Mraw;  // m x m, canonical order
  const double* cvec;  // m, canonical order
  const double* svec;  // m, canonical order
  double* ws;          // 9 m^2 doubles
  int* piv;            // m
  int* sdev;           // s
  double* S64;         // m x m canonical: lambda phi_1(lambda M)
  double* T64;         // m x m device order: diag(c s) S diag(c)
  int* flag;           // bit 0: non-finite input; bit 1: overflow in phi_1; bit 2: barrier timeout
  unsigned* barrier;   // grid barrier counter (zeroed before launch)
};

__device__ __forceinline__ double lin_at(const Lin& L, int m, int i, int j) {
  double v = (i == j) ? L.cI : 0.0;
  if (L.a[0]) v += L.c[0] * L.a[0][(size_t)i * m + j];
  if (L.a[1]) v += L.c[1] * L.a[1][(size_t)i * m + j];
  if (L.a[2]) v += L.c[2] * L.a[2][(size_t)i * m + j];
  return v;
}

__device__ __forceinline__ Lin lin0() { return Lin{{nullptr, nullptr, nullptr}, {0, 0, 0}, 0.0}; }
__device__ __forceinline__ Lin lin1(const double* a, double c = 1.0) { return Lin{{a, nullptr, nullptr}, {c, 0, 0}, 0.0}; }

struct WgBarrier {
  __device__ void sync() { __syncthreads(); }
};

// Counter barrier over a cooperative grid. The counter only grows; round r
// waits for r * nblocks arrivals. The wait is bounded: on timeout the flag
// gets bit 2 and the workgroup proceeds, so every wave always exits.
struct GridBarrier {
  unsigned* ctr;
  unsigned nblocks;
  unsigned round;
  int* flag;
  __device__ void sync() {
    __syncthreads();
    if (threadIdx.x == 0) {
      ++round;
      __threadfence();
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = round * nblocks;
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
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
// out tile (32 x 32 at ti, tj) = alpha * A * B + C, A, B, C linear combinations.
// mode 1: the QR epilogue of U = Y U0: writes [V - U | V + U | 2 U0].
__device__ void gemm_tile(int m, int ti, int tj, const Lin& A, const Lin& B, double alpha, const Lin& C, double* out,
                          int mode, const double* V, const double* U0, double* lds) {
  double* As = lds;                     // 32 x (m + 1)
  double* Bs = lds + 32 * (m + 1);      // m x 33
  const int tid = threadIdx.x;
  __syncthreads();
  for (int e = tid; e < 32 * m; e += 256) {
    const int i = e / m, k = e - i * m;
    As[i * (m + 1) + k] = lin_at(A, m, ti * 32 + i, k);
  }
  for (int e = tid; e < m * 32; e += 256) {
    const int k = e >> 5, j = e & 31;
    Bs[k * 33 + j] = lin_at(B, m, k, tj * 32 + j);
  }
  __syncthreads();
  const int w = tid >> 6, l = tid & 63, qi = w >> 1, qj = w & 1;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  const double* ap = As + (qi * 16 + (l & 15)) * (m + 1) + (l >> 4);
  const double* bp = Bs + (l >> 4) * 33 + qj * 16 + (l & 15);
  for (int s = 0; s < m / 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[4 * s], bp[4 * s * 33], acc, 0, 0, 0);
  // f64 16x16x4 output layout: register r holds row 4 r + l/16, column l%16
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * 32 + qi * 16 + 4 * r + (l >> 4);
    const int j = tj * 32 + qj * 16 + (l & 15);
    if (mode == 0) {
      out[(size_t)i * m + j] = alpha * acc[r] + lin_at(C, m, i, j);
    } else {
      const size_t ld = 3 * (size_t)m;
      const double u = acc[r], v = V[(size_t)i * m + j], u0 = U0[(size_t)i * m + j];
      out[i * ld + j] = v - u;
      out[i * ld + m + j] = v + u;
      out[i * ld + 2 * m + j] = 2.0 * u0;
    }
  }
}

// ------------------------------------------------------------------ LU pieces
// Panel k: rows r0..m-1, columns r0..r0+31 of QR (row pitch 3m). Thread t
// holds row r0 + t in registers.
__device__ void lu_panel(int m, int k, double* QR, int* piv, int* flag, double* lds) {
  const int r0 = 32 * k, nr = m - r0;
  const size_t ld = 3 * (size_t)m;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  double* prow = lds;             // 32: pivot row
  double* srow = lds + 32;        // 32: row displaced by the swap
  double* redv = lds + 64;        // 4
  int* redi = (int*)(lds + 68);   // 4
  double r[32];
  const bool act = t < nr;
#pragma unroll
  for (int c = 0; c < 32; ++c) r[c] = act ? QR[(r0 + t) * ld + r0 + c] : 0.0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    double v = (act && t >= j) ? fabs(r[j]) : -1.0;
    int idx = t;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ov = __shfl_xor(v, o);
      const int oi = __shfl_xor(idx, o);
      if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    if (l == 0) { redv[w] = v; redi[w] = idx; }
    __syncthreads();
    double bv = redv[0];
    int p = redi[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (redv[q] > bv || (redv[q] == bv && redi[q] < p)) { bv = redv[q]; p = redi[q]; }
    }
    if (t == p) {
#pragma unroll
      for (int c = 0; c < 32; ++c) prow[c] = r[c];
    }
    if (t == j) {
#pragma unroll
      for (int c = 0; c < 32; ++c) srow[c] = r[c];
    }
    if (t == 0) piv[r0 + j] = r0 + p;
    __syncthreads();
    if (t == j) {
#pragma unroll
      for (int c = 0; c < 32; ++c) r[c] = prow[c];
    } else if (t == p) {
#pragma unroll
      for (int c = 0; c < 32; ++c) r[c] = srow[c];
    }
    double dv = prow[j];
    if (dv == 0.0) {
      if (t == 0) __hip_atomic_fetch_or(flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      dv = 1.0;
    }
    if (act && t > j) {
      const double lf = r[j] / dv;
      r[j] = lf;
#pragma unroll
      for (int c = j + 1; c < 32; ++c) r[c] -= lf * prow[c];
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < 32; ++c) QR[(r0 + t) * ld + r0 + c] = r[c];
  }
}

// Trailing update of one 32-column strip (columns cs..cs+31, cs >= r0 + 32)
// after panel k: apply the panel's row swaps, U12 = L11^{-1} A12, A22 -= L21 U12.
__device__ void lu_strip(int m, int k, int cs, double* QR, const int* piv, double* lds) {
  const int r0 = 32 * k, nr = m - r0;
  const size_t ld = 3 * (size_t)m;
  const int t = threadIdx.x;
  double* Sx = lds;             // nr x 33
  double* Lp = lds + nr * 33;   // nr x 33 (L11 over L21)
  __syncthreads();
  for (int e = t; e < nr * 32; e += 256) {
    const int i = e >> 5, c = e & 31;
    Sx[i * 33 + c] = QR[(r0 + i) * ld + cs + c];
    Lp[i * 33 + c] = QR[(r0 + i) * ld + r0 + c];
  }
  __syncthreads();
  if (t < 32) {
    // row swaps, in order, on column t
    for (int j = 0; j < 32; ++j) {
      const int p = piv[r0 + j] - r0;
      if (p != j) {
        const double a = Sx[j * 33 + t];
        Sx[j * 33 + t] = Sx[p * 33 + t];
        Sx[p * 33 + t] = a;
      }
    }
    // unit lower triangular solve on column t, in registers
    double x[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) x[i] = Sx[i * 33 + t];
#pragma unroll
    for (int i = 1; i < 32; ++i) {
      double v = x[i];
#pragma unroll
      for (int j = 0; j < i; ++j) v -= Lp[i * 33 + j] * x[j];
      x[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) Sx[i * 33 + t] = x[i];
  }
  __syncthreads();
  // A22 -= L21 U12 on the matrix cores: tiles of 16 rows x 16 columns
  const int w = t >> 6, l = t & 63;
  const int ntile = ((nr - 32) / 16) * 2;
  for (int tile = w; tile < ntile; tile += 4) {
    const int i0 = 32 + (tile >> 1) * 16, c0 = (tile & 1) * 16;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Lp[(i0 + (l & 15)) * 33 + 4 * s + (l >> 4)],
                                                 Sx[(4 * s + (l >> 4)) * 33 + c0 + (l & 15)], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * r + (l >> 4), c = c0 + (l & 15);
      Sx[i * 33 + c] -= acc[r];
    }
  }
  __syncthreads();
  for (int e = t; e < nr * 32; e += 256) {
    const int i = e >> 5, c = e & 31;
    QR[(r0 + i) * ld + cs + c] = Sx[i * 33 + c];
  }
}

// Back substitution U X = R for one 32-column strip of the right-hand side
// (columns m + cs .. of QR); X goes to dst (m x m, columns cs % m ..).
__device__ void back_strip(int m, int cs, const double* QR, double* dst, double* lds) {
  const size_t ld = 3 * (size_t)m;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  double* Rx = lds;               // m x 33
  double* Ub = lds + m * 33;      // m x 33: U[0..r0+31][r0..r0+31]
  __syncthreads();
  for (int e = t; e < m * 32; e += 256) {
    const int i = e >> 5, c = e & 31;
    Rx[i * 33 + c] = QR[i * ld + m + cs + c];
  }
  for (int k = m / 32 - 1; k >= 0; --k) {
    const int r0 = 32 * k;
    __syncthreads();
    for (int e = t; e < (r0 + 32) * 32; e += 256) {
      const int i = e >> 5, c = e & 31;
      Ub[i * 33 + c] = QR[i * ld + r0 + c];
    }
    __syncthreads();
    if (t < 32) {
      double x[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) x[i] = Rx[(r0 + i) * 33 + t];
#pragma unroll
      for (int i = 31; i >= 0; --i) {
        double v = x[i];
#pragma unroll
        for (int j = i + 1; j < 32; ++j) v -= Ub[(r0 + i) * 33 + j] * x[j];
        x[i] = v / Ub[(r0 + i) * 33 + i];
      }
#pragma unroll
      for (int i = 0; i < 32; ++i) Rx[(r0 + i) * 33 + t] = x[i];
    }
    __syncthreads();
    const int ntile = (r0 / 16) * 2;
    for (int tile = w; tile < ntile; tile += 4) {
      const int i0 = (tile >> 1) * 16, c0 = (tile & 1) * 16;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 8; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ub[(i0 + (l & 15)) * 33 + 4 * s + (l >> 4)],
                                                   Rx[(r0 + 4 * s + (l >> 4)) * 33 + c0 + (l & 15)], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 4 * r + (l >> 4), c = c0 + (l & 15);
        Rx[i * 33 + c] -= acc[r];
      }
    }
  }
  __syncthreads();
  const int col0 = cs % m;
  for (int e = t; e < m * 32; e += 256) {
    const int i = e >> 5, c = e & 31;
    dst[(size_t)i * m + col0 + c] = Rx[i * 33 + c];
  }
}

// ------------------------------------------------------------------ body
template <class BAR>
__device__ void phi1_body(const Phi1Args& a, int worker, int nw, double* lds, BAR& bar) {
  const int m = a.m, nb = m / 32, nt = nb * nb;
  const size_t mm = (size_t)m * m;
  double* Y = a.ws;
  double* Y2 = Y + mm;
  double* Y4 = Y2 + mm;
  double* Y6 = Y4 + mm;
  double* U0 = Y6 + mm;
  double* V = U0 + mm;
  double* QR = V + mm;  // m x 3m
  const int t = threadIdx.x;

  // ---- P0: 1-norm of lambda M (every worker, same arithmetic), s, Y
  double* red = lds;
  __syncthreads();
  double colsum = 0.0;
  if (t < m) {
    for (int i = 0; i < m; ++i) colsum += a.cvec[i] * fabs(a.Mraw[(size_t)i * m + t]);
    colsum *= a.cvec[t];
  }
  red[t] = colsum;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) red[t] = fmax(red[t], red[t + o]);
    __syncthreads();
  }
  const double nrm = fabs(a.lambda) * red[0];
  int s = 0;
  if (!(nrm <= 1e300)) s = 0;  // non-finite input: flagged by the reduction already
  else if (nrm > 5.371920351148152) s = (int)ceil(log2(nrm / 5.371920351148152));
  if (s > 1000) s = 1000;
  if (worker == 0 && t == 0) *a.sdev = s;
  const double scale = a.lambda * ldexp(1.0, -s);
  for (size_t e = (size_t)worker * 256 + t; e < mm; e += (size_t)nw * 256) {
    const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
    Y[e] = scale * a.cvec[i] * a.Mraw[e] * a.cvec[j] * a.svec[j];
  }
  bar.sync();

  const double* b = a.b;
  // ---- P1..P3: even powers
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile(m, tile / nb, tile % nb, lin1(Y), lin1(Y), 1.0, lin0(), Y2, 0, nullptr, nullptr, lds);
  bar.sync();
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile(m, tile / nb, tile % nb, lin1(Y2), lin1(Y2), 1.0, lin0(), Y4, 0, nullptr, nullptr, lds);
  bar.sync();
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile(m, tile / nb, tile % nb, lin1(Y4), lin1(Y2), 1.0, lin0(), Y6, 0, nullptr, nullptr, lds);
  bar.sync();
  // ---- P4: U0 and V
  for (int tile = worker; tile < 2 * nt; tile += nw) {
    const int tt = tile % nt;
    if (tile < nt) {
      Lin Bm{{Y6, Y4, Y2}, {b[13], b[11], b[9]}, 0.0};
      Lin Cm{{Y6, Y4, Y2}, {b[7], b[5], b[3]}, b[1]};
      gemm_tile(m, tt / nb, tt % nb, lin1(Y6), Bm, 1.0, Cm, U0, 0, nullptr, nullptr, lds);
    } else {
      Lin Bm{{Y6, Y4, Y2}, {b[12], b[10], b[8]}, 0.0};
      Lin Cm{{Y6, Y4, Y2}, {b[6], b[4], b[2]}, b[0]};
      gemm_tile(m, tt / nb, tt % nb, lin1(Y6), Bm, 1.0, Cm, V, 0, nullptr, nullptr, lds);
    }
  }
  bar.sync();
  // ---- P5: U = Y U0 and the system [V - U | V + U | 2 U0]
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile(m, tile / nb, tile % nb, lin1(Y), lin1(U0), 1.0, lin0(), QR, 1, V, U0, lds);
  bar.sync();
  // ---- P6: blocked LU with partial pivoting; right-hand sides ride along
  for (int k = 0; k < nb; ++k) {
    if (worker == 0) lu_panel(m, k, QR, a.piv, a.flag, lds);
    bar.sync();
    const int first = k + 1, nstrip = 3 * nb - first;
    for (int st = worker; st < nstrip; st += nw) lu_strip(m, k, 32 * (first + st), QR, a.piv, lds);
    bar.sync();
  }
  // ---- P7: back substitution per right-hand-side strip: E -> Y2, P -> Y4
  for (int st = worker; st < 2 * nb; st += nw) back_strip(m, 32 * st, QR, st < nb ? Y2 : Y4, lds);
  bar.sync();
  // ---- P8: undo the scaling: P <- P (E + I) / 2, E <- E E
  double* Ec = Y2;
  double* Pc = Y4;
  double* En = Y6;
  double* Pn = U0;
  for (int it = 0; it < s; ++it) {
    for (int tile = worker; tile < 2 * nt; tile += nw) {
      const int tt = tile % nt;
      if (tile < nt) gemm_tile(m, tt / nb, tt % nb, lin1(Ec), lin1(Ec), 1.0, lin0(), En, 0, nullptr, nullptr, lds);
      else gemm_tile(m, tt / nb, tt % nb, lin1(Pc), lin1(Ec), 0.5, lin1(Pc, 0.5), Pn, 0, nullptr, nullptr, lds);
    }
    bar.sync();
    double* x = Ec; Ec = En; En = x;
    x = Pc; Pc = Pn; Pn = x;
  }
  // ---- P9: S = lambda P (canonical), T = diag(c s) S diag(c) in device order
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

__global__ __launch_bounds__(256) void k_phi1_wg(const Phi1Args* __restrict__ args) {
  extern __shared__ double lds[];
  const Phi1Args a = args[blockIdx.x];
  WgBarrier bar;
  phi1_body(a, 0, 1, lds, bar);
}

__global__ __launch_bounds__(256) void k_phi1_grid(Phi1Args a) {
  extern __shared__ double lds[];
  GridBarrier bar{a.barrier, gridDim.x, 0u, a.flag};
  phi1_body(a, (int)blockIdx.x, (int)gridDim.x, lds, bar);
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// LDS bytes of the phi_1 kernels for padded size m.
static size_t phi1_lds_bytes(int m) {
  size_t gemm = (size_t)(32 * (m + 1) + m * 33) * 8;
  size_t two = (size_t)(2 * m * 33) * 8;
  size_t red = 256 * 8;
  size_t x = gemm > two ? gemm : two;
  return x > red ? x : red;
}

static void fill_args(rfd_plan_s* p, Phi1Args& a) {
  a.m = p->dev_m;
  a.reserved = 0;
  a.lambda = p->params.lambda;
  for (int k = 0; k < 14; ++k) a.b[k] = p->pade_b[k];
  a.Mraw = p->dev.Mraw;
  a.cvec = p->dev.cvec;
  a.svec = p->dev.svec;
  a.ws = p->dev.phi_ws;
  a.piv = p->dev.pivots;
  a.sdev = p->dev.sdev;
  a.S64 = p->dev.S64;
  a.T64 = p->dev.T64;
  a.flag = p->dev.flag;
  a.barrier = p->dev.barrier;
}

hipError_t launch_phi1(rfd_plan_s* p, hipStream_t st) {
  Phi1Args a;
  fill_args(p, a);
  const int m = a.m;
  const size_t lds = phi1_lds_bytes(m);
  hipError_t e = hipFuncSetAttribute((const void*)k_phi1_grid, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int nb = m / 32;
  int nw = 2 * nb * nb;  // the widest phase (U0 and V, and the squarings) has 2 nb^2 tiles
  if (nw > 128) nw = 128;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, a.barrier, 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* kargs[] = {&a};
  ProfileScope prof(kKPhi1, st);
  return hipLaunchCooperativeKernel((const void*)k_phi1_grid, dim3(nw), dim3(256), kargs, (unsigned)lds, st);
}

hipError_t launch_phi1_batch(rfd_plan_s** plans, int n, void* dev_args, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  std::vector<Phi1Args> h(n);
  for (int i = 0; i < n; ++i) fill_args(plans[i], h[i]);
  const int m = h[0].m;
  hipError_t e = hipMemcpyAsync(dev_args, h.data(), sizeof(Phi1Args) * n, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  const size_t lds = phi1_lds_bytes(m);
  e = hipFuncSetAttribute((const void*)k_phi1_wg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  ProfileScope prof(kKPhi1Batch, st);
  hipLaunchKernelGGL(k_phi1_wg, dim3(n), dim3(256), lds, st, (const Phi1Args*)dev_args);
  return hipGetLastError();
}

size_t phi1_args_bytes() { return sizeof(Phi1Args); }

}  // namespace rfd
