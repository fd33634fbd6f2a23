// FP64 phi_1 of the m x m RFD core on gfx950.
//
// S = lambda phi_1(lambda M), M = B^T A = diag(c) Mraw diag(c) diag(s), by
// scaling and squaring with the [13/13] Pade approximant of exp (Higham 2005,
// "The scaling and squaring method for the matrix exponential revisited"):
//
//   X = lambda M, s = max(0, ceil(log2(||X||_1 / theta_13))), Y = X / 2^s
//   U0 = b13 Y^12 + b11 Y^10 + ... + b3 Y^2 + b1 I,   U = Y U0   (odd part)
//   V  = b12 Y^12 + ... + b2 Y^2 + b0 I                         (even part)
//   Q = V - U,   P = Q^{-1} (2 U0),   E = I + Y P
//
// P is phi_1(Y) to Pade accuracy: the [13/13] approximant applied to the
// augmented matrix [[Y, I], [0, 0]] has top-right block Q^{-1} (p~(Y) - q~(Y))
// with p~, q~ the Pade polynomials shifted down one power, and p~ - q~ = 2 U0
// because q(x) = p(-x) (Al-Mohy & Higham 2011 use this augmentation for phi
// functions). E = Q^{-1}(V + U) = I + Y P because Q^{-1} commutes with Y. The
// scaling is undone with phi_1(2Y) = phi_1(Y) (e^Y + I) / 2 and
// e^{2Y} = e^Y e^Y, s times. Powers are formed from the unscaled X with the
// exact power-of-two factors 2^{-ks} applied in the products.
//
// The solve is a right-looking blocked LU with partial pivoting (32-column
// panels, the next panel factored in the same phase as the trailing update);
// the m right-hand-side columns ride along as trailing columns, so forward
// elimination needs no separate pass, and back substitution runs per
// 32-column strip without cross-workgroup sync.
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
  double b[14];        // Pade [13/13] numerator coefficients
  const double* Mraw;  // m x m, canonical order (symmetric)
  const double* cvec;  // m, canonical order
  const double* svec;  // m, canonical order
  double* ws;          // phi1_ws_doubles(m)
  int* piv;            // m
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

// Largest 32-bit key over the 64 lanes of a wave (DPP: swaps within quads,
// half-row and row mirrors, then the two row broadcasts; lane 63 ends with the
// maximum, which is read back into a uniform value).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

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

// ------------------------------------------------------------------ LU pieces
// Matrix QR: m rows, row pitch ld = 2m; columns [0, m) hold Q, [m, 2m) the
// right-hand sides. Panel k: rows r0..m-1, columns r0..r0+31, factored with
// partial pivoting; thread t holds panel row t in registers, the column steps
// are unrolled at compile time so every register index is static.
//
// Pivot choice: the 32-bit key of row t is the FP32 bit pattern of |a_tj|
// with its 8 low mantissa bits replaced by 255 - t; the largest key wins. The
// chosen pivot is within a factor 1 + 2^-15 of the column maximum (ties go to
// the smallest row), a deterministic partial-pivoting rule.
struct PanelCtx {
  double* rows;  // LDS: 2 x 2 x 32 doubles: [buffer][pivot row, displaced row]
  unsigned* red; // LDS: 2 x 4 per-wave maximum keys
  int* piv;      // global pivot vector
  int* flag;
  int r0, nr, t;
};

template <int J>
__device__ __forceinline__ void panel_step(double (&r)[32], const PanelCtx& c) {
  if constexpr (J < 32) {
    const int t = c.t, w = t >> 6;
    double* prow = c.rows + (J & 1) * 64;
    double* srow = prow + 32;
    unsigned* red = c.red + (J & 1) * 4;
    const bool cand = t < c.nr && t >= J;
    const unsigned key = cand ? ((__float_as_uint(fabsf((float)r[J])) & ~0xFFu) | (unsigned)(255 - t)) : 0u;
    const unsigned wm = wave_max_u32(key);
    if ((t & 63) == 0) red[w] = wm;
    __syncthreads();
    const unsigned best = max(max(red[0], red[1]), max(red[2], red[3]));
    const int p = best == 0u ? J : 255 - (int)(best & 0xFFu);
    if (t == p) {
#pragma unroll
      for (int k = J; k < 32; ++k) prow[k] = r[k];
    }
    if (t == J && p != J) {
#pragma unroll
      for (int k = J; k < 32; ++k) srow[k] = r[k];
    }
    if (t == 0) c.piv[c.r0 + J] = c.r0 + p;
    __syncthreads();
    if (p != J) {
      if (t == J) {
#pragma unroll
        for (int k = J; k < 32; ++k) r[k] = prow[k];
      } else if (t == p) {
#pragma unroll
        for (int k = J; k < 32; ++k) r[k] = srow[k];
      }
    }
    double dv = prow[J];
    if (dv == 0.0) {
      if (t == 0) __hip_atomic_fetch_or(c.flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      dv = 1.0;
    }
    if (t < c.nr && t > J) {
      const double lf = r[J] / dv;
      r[J] = lf;
#pragma unroll
      for (int k = J + 1; k < 32; ++k) r[k] -= lf * prow[k];
    }
    // no barrier here: the next step writes the other LDS buffer, and this
    // one is written again only after the next step's two barriers
    panel_step<J + 1>(r, c);
  }
}

template <int m>
__device__ __forceinline__ void lu_panel(int k, double* QR, int* piv, int* flag, double* lds) {
  const int r0 = 32 * k, nr = m - r0;
  const size_t ld = 2 * (size_t)m;
  const int t = threadIdx.x;
  double* Pn = lds;  // nr x 33 staging for coalesced loads and stores
  PanelCtx c{lds + 256 * 33, (unsigned*)(lds + 256 * 33 + 128), piv, flag, r0, nr, t};
  __syncthreads();
  {
    constexpr int NL = m / 8;
    double vp[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5;
      if (i < nr) vp[q] = QR[(r0 + i) * ld + r0 + (e & 31)];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5;
      if (i < nr) Pn[i * 33 + (e & 31)] = vp[q];
    }
  }
  __syncthreads();
  double r[32];
  const bool act = t < nr;
#pragma unroll
  for (int q = 0; q < 32; ++q) r[q] = act ? Pn[t * 33 + q] : 0.0;
  panel_step<0>(r, c);
  __syncthreads();
  if (act) {
#pragma unroll
    for (int q = 0; q < 32; ++q) Pn[t * 33 + q] = r[q];
  }
  __syncthreads();
  {
    constexpr int NL = m / 8;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5;
      if (i < nr) QR[(r0 + i) * ld + r0 + (e & 31)] = Pn[i * 33 + (e & 31)];
    }
  }
}

// Inverse of the upper triangular diagonal block U_kk (rows and columns
// 32k..32k+31 of QR, final once panel k is factored) into Ui (32 x 32,
// row-major): thread c < 32 solves U x = e_c in registers.
template <int m>
__device__ __forceinline__ void upper_inverse(int k, const double* QR, double* Ui, double* lds) {
  const int r0 = 32 * k;
  const size_t ld = 2 * (size_t)m;
  const int t = threadIdx.x;
  double* Ub = lds;  // 32 x 33
  __syncthreads();
  for (int e = t; e < 32 * 32; e += 256) Ub[(e >> 5) * 33 + (e & 31)] = QR[(r0 + (e >> 5)) * ld + r0 + (e & 31)];
  __syncthreads();
  if (t < 32) {
    double x[32];
#pragma unroll
    for (int i = 31; i >= 0; --i) {
      double v = (i == t) ? 1.0 : 0.0;
#pragma unroll
      for (int j = i + 1; j < 32; ++j) v -= Ub[i * 33 + j] * x[j];
      x[i] = v / Ub[i * 33 + i];
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) Ui[i * 32 + t] = x[i];
  }
}

// Trailing update of one 32-column strip (columns cs..cs+31, cs >= r0 + 32)
// after panel k: apply the panel's row swaps, U12 = L11^{-1} A12, A22 -= L21 U12.
template <int m>
__device__ __forceinline__ void lu_strip(int k, int cs, double* QR, const int* piv, double* lds) {
  const int r0 = 32 * k, nr = m - r0;
  const size_t ld = 2 * (size_t)m;
  const int t = threadIdx.x;
  double* Sx = lds;             // nr x 33
  double* Lp = lds + nr * 33;   // nr x 33 (L11 over L21)
  __syncthreads();
  {
    constexpr int NL = m / 8;  // upper bound of nr * 32 / 256
    double v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5, c = e & 31;
      if (i < nr) v[q] = QR[(r0 + i) * ld + cs + c];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5, c = e & 31;
      if (i < nr) Sx[i * 33 + c] = v[q];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5, c = e & 31;
      if (i < nr) v[q] = QR[(r0 + i) * ld + r0 + c];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q, i = e >> 5, c = e & 31;
      if (i < nr) Lp[i * 33 + c] = v[q];
    }
  }
  __syncthreads();
  if (t < 32) {
    // row swaps, in order, then the unit lower triangular solve, on column t
    for (int j = 0; j < 32; ++j) {
      const int p = piv[r0 + j] - r0;
      if (p != j) {
        const double a = Sx[j * 33 + t];
        Sx[j * 33 + t] = Sx[p * 33 + t];
        Sx[p * 33 + t] = a;
      }
    }
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
// (columns m + cs .. of QR) with the inverted diagonal blocks Uinv (nb blocks
// of 32 x 32): per block, X_k = Uinv_k R_k and R_{<k} -= U_{<k,k} X_k, both on
// the matrix cores. X goes to dst (m x m, columns cs ..).
template <int m>
__device__ __forceinline__ void back_strip(int cs, const double* QR, const double* Uinv, double* dst, double* lds) {
  const size_t ld = 2 * (size_t)m;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  double* Rx = lds;               // m x 33
  double* Ub = lds + m * 33;      // m x 33: U[0..r0-1][r0..r0+31], then Uinv_k in rows r0..r0+31
  __syncthreads();
  {
    constexpr int NL = m / 8;
    double vr[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q;
      vr[q] = QR[(e >> 5) * ld + m + cs + (e & 31)];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = t + 256 * q;
      Rx[(e >> 5) * 33 + (e & 31)] = vr[q];
    }
  }
  for (int k = m / 32 - 1; k >= 0; --k) {
    const int r0 = 32 * k;
    __syncthreads();
    {
      constexpr int NL = m / 8;
      double vu[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = t + 256 * q, i = e >> 5;
        if (i < r0) vu[q] = QR[i * ld + r0 + (e & 31)];
        else if (i < r0 + 32) vu[q] = Uinv[(size_t)k * 1024 + (i - r0) * 32 + (e & 31)];
      }
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = t + 256 * q, i = e >> 5;
        if (i < r0 + 32) Ub[i * 33 + (e & 31)] = vu[q];
      }
    }
    __syncthreads();
    // X_k = Uinv_k R_k: waves 0..3 take the four 16 x 16 quadrants
    {
      const int i0 = (w >> 1) * 16, c0 = (w & 1) * 16;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 8; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ub[(r0 + i0 + (l & 15)) * 33 + 4 * s + (l >> 4)],
                                                   Rx[(r0 + 4 * s + (l >> 4)) * 33 + c0 + (l & 15)], acc, 0, 0, 0);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) Rx[(r0 + i0 + 4 * r + (l >> 4)) * 33 + c0 + (l & 15)] = acc[r];
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
  for (int e = t; e < m * 32; e += 256) {
    const int i = e >> 5, c = e & 31;
    dst[(size_t)i * m + cs + c] = Rx[i * 33 + c];
  }
}

// ------------------------------------------------------------------ body
template <int m, class BAR>
__device__ __forceinline__ void phi1_body(const Phi1Args& a, int worker, int nw, double* lds, BAR& bar) {
  constexpr int nb = m / 32, nt = nb * nb;
  const size_t mm = (size_t)m * m;
  double* X0 = a.ws;        // lambda M
  double* Y2 = X0 + mm;
  double* Y4 = Y2 + mm;
  double* Y6 = Y4 + mm;
  double* W1 = Y6 + mm;
  double* Z1 = W1 + mm;
  double* C1 = Z1 + mm;
  double* C2 = C1 + mm;
  double* U0 = C2 + mm;
  double* V = U0 + mm;
  double* QR = V + mm;      // m x 2m
  double* colsum = QR + 2 * mm;
  double* Uinv = colsum + m;  // nb blocks of 32 x 32
  const int t = threadIdx.x;
  const double* b = a.b;

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
  else if (nrm > 5.371920351148152) s = (int)ceil(log2(nrm / 5.371920351148152));
  if (s > 1000) s = 1000;
  if (worker == 0 && t == 0) *a.sdev = s;
  const double sc1 = ldexp(1.0, -s), sc2 = ldexp(1.0, -2 * s);

  // ---- P1..P3: even powers of Y = X0 / 2^s; the last epilogue forms the
  // Pade combinations W1, Z1 (B operands) and C1, C2 (additive terms)
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile<m>(tile / nb, tile % nb, X0, X0, sc2, lds, [&](int i, int j, double v) { Y2[(size_t)i * m + j] = v; });
  bar.sync();
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile<m>(tile / nb, tile % nb, Y2, Y2, 1.0, lds, [&](int i, int j, double v) { Y4[(size_t)i * m + j] = v; });
  bar.sync();
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile<m>(tile / nb, tile % nb, Y4, Y2, 1.0, lds, [&](int i, int j, double y6) {
      const size_t e = (size_t)i * m + j;
      const double y4 = Y4[e], y2 = Y2[e], id = i == j ? 1.0 : 0.0;
      Y6[e] = y6;
      W1[e] = b[13] * y6 + b[11] * y4 + b[9] * y2;
      Z1[e] = b[12] * y6 + b[10] * y4 + b[8] * y2;
      C1[e] = b[7] * y6 + b[5] * y4 + b[3] * y2 + b[1] * id;
      C2[e] = b[6] * y6 + b[4] * y4 + b[2] * y2 + b[0] * id;
    });
  bar.sync();
  // ---- P4: U0 = Y6 W1 + C1,  V = Y6 Z1 + C2
  for (int tile = worker; tile < 2 * nt; tile += nw) {
    const int tt = tile % nt;
    if (tile < nt)
      gemm_tile<m>(tt / nb, tt % nb, Y6, W1, 1.0, lds,
                [&](int i, int j, double v) { const size_t e = (size_t)i * m + j; U0[e] = v + C1[e]; });
    else
      gemm_tile<m>(tt / nb, tt % nb, Y6, Z1, 1.0, lds,
                [&](int i, int j, double v) { const size_t e = (size_t)i * m + j; V[e] = v + C2[e]; });
  }
  bar.sync();
  // ---- P5: U = Y U0; system Q = V - U with right-hand side 2 U0
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile<m>(tile / nb, tile % nb, X0, U0, sc1, lds, [&](int i, int j, double u) {
      const size_t e = (size_t)i * m + j;
      QR[(size_t)i * 2 * m + j] = V[e] - u;
      QR[(size_t)i * 2 * m + m + j] = 2.0 * U0[e];
    });
  bar.sync();
  // ---- P6: blocked LU with partial pivoting, next panel factored in the
  // same phase as the trailing update (by the worker owning its strip)
  // The inverse of each diagonal U block is taken, off the critical path, by
  // the worker after the last strip owner in the phase following its panel.
  if (worker == 0) lu_panel<m>(0, QR, a.piv, a.flag, lds);
  bar.sync();
  for (int k = 0; k < nb; ++k) {
    const int nstrip = 2 * nb - k - 1;
    for (int st = worker; st < nstrip; st += nw) {
      lu_strip<m>(k, 32 * (k + 1 + st), QR, a.piv, lds);
      if (st == 0 && k + 1 < nb) lu_panel<m>(k + 1, QR, a.piv, a.flag, lds);
    }
    if (worker == nstrip % nw) upper_inverse<m>(k, QR, Uinv + (size_t)k * 1024, lds);
    bar.sync();
  }
  // ---- P7: back substitution per right-hand-side strip: P -> Y2
  double* Pc = Y2;
  for (int st = worker; st < nb; st += nw) back_strip<m>(32 * st, QR, Uinv, Pc, lds);
  bar.sync();
  // ---- P8: E = I + Y P -> Y4
  double* Ec = Y4;
  for (int tile = worker; tile < nt; tile += nw)
    gemm_tile<m>(tile / nb, tile % nb, X0, Pc, sc1, lds,
              [&](int i, int j, double v) { Ec[(size_t)i * m + j] = v + (i == j ? 1.0 : 0.0); });
  bar.sync();
  // ---- P9: undo the scaling: P <- P (E + I) / 2, E <- E E
  double* En = Y6;
  double* Pn = W1;
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
  // ---- P10: S = lambda P (canonical), T = diag(c s) S diag(c) in device order
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
static size_t phi1_lds_bytes(int m) {
  const size_t gemm = (size_t)(32 * (m + 1) + m * 33) * 8;
  const size_t strip = (size_t)(2 * m * 33) * 8;
  const size_t panel = (size_t)(256 * 33 + 128 + 8) * 8;
  size_t x = gemm > strip ? gemm : strip;
  return x > panel ? x : panel;
}

size_t phi1_ws_doubles(int m) { return 12 * (size_t)m * m + m + (size_t)(m / 32) * 1024; }

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

template <int M>
static hipError_t launch_phi1_m(Phi1Args& a, hipStream_t st) {
  const size_t lds = phi1_lds_bytes(M);
  hipError_t e = hipFuncSetAttribute((const void*)k_phi1_grid<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  constexpr int nb = M / 32;
  int nw = 2 * nb * nb;  // the widest phases (U0 and V, the squarings) have 2 nb^2 tiles
  if (nw > 128) nw = 128;
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
