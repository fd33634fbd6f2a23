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
#include "grid_barrier.h"
#include "rfd_internal.h"

namespace rfd {

struct Phi1Args {
  int m;               // padded size, a multiple of 64, <= 256
  int sym;             // 1: every weight is >= 0, so lambda M and every matrix of both chains is symmetric
  double lambda;
  const double* Mraw;  // m x m, canonical order (symmetric)
  const double* cvec;  // m, canonical order
  const double* svec;  // m, canonical order
  double* ws;          // phi1_ws_doubles(m)
  int* sdev;           // s
  double* S64;         // m x m canonical: lambda phi_1(lambda M)
  double* T64;         // m x m device order: diag(c s) S diag(c)
  int* flag;           // bit 0: non-finite input; bit 1: overflow in phi_1; bit 2: barrier timeout
  unsigned* barrier;   // grid barrier counters (zero at launch; each launch leaves them zero)
};

// The action form: G' = diag(c s) S diag(c) H0 for one channel block, without S.
struct ApplyArgs {
  const double* H0;  // m x d, device order: B^T F of the block
  int d;             // channels, <= kThinWidth
  int reserved;
  float* G32;        // m x d, device order
  __bf16* Gt16;      // BF16 hi (d x m), then lo at offset 64 m
  double* G64;       // m x kThinWidth, canonical: G = lambda phi_1(lambda M) H in FP64
};
constexpr int kThinWidth = 32;

// Global-typed accesses. The per-cloud kernels read their pointers from
// argument records in device memory, which the compiler cannot place in an
// address space, so plain accesses become flat ones; flat accesses also
// count against the LDS wait counter, so every LDS wait before a barrier
// would drain the loads in flight as well. All these buffers are global.
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) f64x2_t gf64x2;
__device__ __forceinline__ double gld(const double* p) { return *(const gdouble*)p; }
__device__ __forceinline__ double2 gld2(const double* p) {
  const f64x2_t v = *(const gf64x2*)p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gst(double* p, double v) { *(gdouble*)p = v; }

// One workgroup per cloud: the phases' global stores are waited for before
// the workgroup barrier, so every wave's next loads see them (the barrier
// alone does not wait for outstanding stores).
struct WgBarrier {
  __device__ __forceinline__ void sync() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  // a phase output (read by the same workgroup after sync)
  __device__ __forceinline__ void st(double* p, double v) const { gst(p, v); }
  __device__ __forceinline__ void finish() {}
};

// ------------------------------------------------------------------ GEMM tiles
// One workgroup computes the 32 x 32 tile (ti, tj) of C1 = alpha1 A1 B1 and,
// with NP = 2, of C2 = alpha2 A2 B2, for row-major m x m operands. The two
// products of a phase share a panel: SHARE == kShareA (A2 is A1: the row
// panel of A is loaded once) or kShareB (B2 is B1). K runs in blocks of KB
// through LDS. With ALL, every block's panels are loaded into registers up
// front (one memory round trip per tile) and staged through one LDS buffer;
// otherwise two LDS buffers alternate and the next block's panels are loaded
// while the current block is multiplied. Each wave computes one 16 x 16
// quadrant of each tile as one MFMA chain over the k steps in increasing
// order (k = 4 t .. 4 t + 3 in step t, lane (r, q) holding k = 4 t + q), then
// scales it by alpha: every kernel that forms these products uses this chain,
// so they give the same bits (dependent FP64 MFMAs issue back to back on
// gfx950: splitting the chain bought no speed). The NS side matrices the
// epilogue reads elementwise are loaded with the panels (ALL) or after the
// products; the epilogue gets (i, j, c1, c2, side values at (i, j)) for the
// four values each lane holds.
constexpr int kShareA = 0, kShareB = 1;
// doubles per LDS panel: A panels are 32 x KB (row pitch KB + 1), B panels
// KB x 32 (row pitch 33)
constexpr int panel_doubles(int KB) { return 32 * (KB + 1) > KB * 33 ? 32 * (KB + 1) : KB * 33; }
constexpr int gemm_lds_doubles(int KB, bool all) { return (all ? 1 : 2) * 3 * panel_doubles(KB); }

template <int NS>
struct Side {
  double v[NS > 0 ? NS : 1];
};

// LDB and LDC are the row pitches of the B operands and of the output/side
// matrices (m for m x m operands; the width of a thin operand block).
//
// gemm_range runs the tiles of virtual indices first, first + step, ... <
// end, map(idx, ti, tj) giving each tile. With ALL and a single K block
// (KB == m) the tiles are streamed: as soon as one tile's panels sit in LDS,
// the next tile's panel and side loads are issued, so they arrive while the
// current tile is multiplied. Every tile's arithmetic is that of a lone tile
// (the same products, summed in the same order), so results do not depend on
// how tiles are grouped into runs.
template <int m, int KB, bool ALL, int NP, int SHARE, int NS = 0, int LDB = m, int LDC = m, class MAP, class EPI>
__device__ __forceinline__ void gemm_range(int first, int end, int step, MAP map, const double* __restrict__ A1,
                                           const double* __restrict__ B1, const double* __restrict__ A2,
                                           const double* __restrict__ B2, double alpha1, double alpha2,
                                           double* lds, EPI epi, const double* S0 = nullptr,
                                           const double* S1 = nullptr, const double* S2 = nullptr,
                                           const double* S3 = nullptr) {
  constexpr int NA = (NP == 2 && SHARE == kShareB) ? 2 : 1;  // A row panels per block
  constexpr int NBP = (NP == 2 && SHARE == kShareA) ? 2 : 1; // B column panels per block
  constexpr int NB_K = m / KB;
  constexpr int PD = panel_doubles(KB);
  constexpr int AP = KB + 1;         // A panel row pitch
  constexpr int LQ = 32 * KB / 512;  // double2 per thread per panel
  constexpr int AH = KB / 2;         // double2 per A panel row
  constexpr int NR = ALL ? NB_K : 1; // blocks held in registers
  const int tid = threadIdx.x;
  const double* Ag[2] = {A1, A2};
  const double* Bg[2] = {B1, B2};
  double2 ra[NR][NA][LQ], rb[NR][NBP][LQ];
  int ti = 0, tj = 0;  // the tile whose panels are being loaded
  // A panel element e = tid + 256 q: row e / AH, double2 column e % AH;
  // B panel element e: row e / 16, double2 column e % 16
  const auto load = [&](int kb, int slot) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int q = 0; q < LQ; ++q) {
        const int e = tid + 256 * q, r = e / AH, c2 = e % AH;
        ra[slot][a][q] = gld2(Ag[a] + (size_t)(ti * 32 + r) * m + kb * KB + 2 * c2);
      }
#pragma unroll
    for (int b = 0; b < NBP; ++b)
#pragma unroll
      for (int q = 0; q < LQ; ++q) {
        const int e = tid + 256 * q, r = e >> 4, c2 = e & 15;
        rb[slot][b][q] = gld2(Bg[b] + (size_t)(kb * KB + r) * LDB + tj * 32 + 2 * c2);
      }
  };
  const auto store = [&](int slot, double* buf) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int q = 0; q < LQ; ++q) {
        const int e = tid + 256 * q, r = e / AH, c2 = e % AH;
        buf[a * PD + r * AP + 2 * c2] = ra[slot][a][q].x;
        buf[a * PD + r * AP + 2 * c2 + 1] = ra[slot][a][q].y;
      }
#pragma unroll
    for (int b = 0; b < NBP; ++b)
#pragma unroll
      for (int q = 0; q < LQ; ++q) {
        const int e = tid + 256 * q, r = e >> 4, c2 = e & 15;
        buf[(NA + b) * PD + r * 33 + 2 * c2] = rb[slot][b][q].x;
        buf[(NA + b) * PD + r * 33 + 2 * c2 + 1] = rb[slot][b][q].y;
      }
  };
  const int w = tid >> 6, l = tid & 63, qi = w >> 1, qj = w & 1;
  // output element r of this lane in tile (i0, j0): row i0*32 + qi*16 + 4r + l/16,
  // column j0*32 + qj*16 + l%16
  const auto out_index = [&](int i0, int j0, int r) {
    return (size_t)(i0 * 32 + qi * 16 + 4 * r + (l >> 4)) * LDC + j0 * 32 + qj * 16 + (l & 15);
  };
  const auto load_side = [&](Side<NS> (&side)[4]) {
    const double* sp[4] = {S0, S1, S2, S3};
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < NS; ++q) side[r].v[q] = gld(sp[q] + out_index(ti, tj, r));
  };
  const auto multiply = [&](const double* buf, f64x4 (&acc)[NP]) {
    const int ao = (qi * 16 + (l & 15)) * AP + (l >> 4);
    const int bo = (l >> 4) * 33 + qj * 16 + (l & 15);
#pragma unroll
    for (int t = 0; t < KB / 4; ++t) {
      const int k = 4 * t;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int pa = (NA == 2) ? p : 0, pb = (NBP == 2) ? p : 0;
        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(buf[pa * PD + ao + k], buf[(NA + pb) * PD + bo + k * 33], acc[p],
                                                      0, 0, 0);
      }
    }
  };
  const auto zero = [&](f64x4 (&acc)[NP]) {
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = f64x4{0.0, 0.0, 0.0, 0.0};
  };
  // f64 16x16x4 output layout: register r holds row 4 r + l/16, column l%16
  // an off-diagonal tile of a symmetric product is stored at (i, j) and (j, i):
  // the side matrices the epilogue reads are then symmetric too
  const auto epilogue = [&](int i0, int j0, const f64x4 (&acc)[NP], const Side<NS> (&side)[4]) {
    const bool mir = map.mirror(i0, j0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 * 32 + qi * 16 + 4 * r + (l >> 4);
      const int j = j0 * 32 + qj * 16 + (l & 15);
      const double v1 = alpha1 * acc[0][r];
      const double v2 = NP == 2 ? alpha2 * acc[NP - 1][r] : 0.0;
      epi(i, j, v1, v2, side[r]);
      if (mir) epi(j, i, v1, v2, side[r]);
    }
  };
  if constexpr (ALL && NB_K == 1) {
    if (first >= end) return;
    Side<NS> side[4], cur[4];
    map(first, ti, tj);
    load(0, 0);
    load_side(side);
    for (int idx = first; idx < end; idx += step) {
      const int ci = ti, cj = tj;
#pragma unroll
      for (int r = 0; r < 4; ++r) cur[r] = side[r];
      __syncthreads();  // the buffer's previous readers are done
      store(0, lds);
      if (idx + step < end) {  // the next tile's loads fly during this tile's products
        map(idx + step, ti, tj);
        load(0, 0);
        load_side(side);
      }
      __syncthreads();
      f64x4 acc[NP];
      zero(acc);
      multiply(lds, acc);
      epilogue(ci, cj, acc, cur);
    }
  } else {
    for (int idx = first; idx < end; idx += step) {
      map(idx, ti, tj);
      Side<NS> side[4];
      f64x4 acc[NP];
      zero(acc);
      if constexpr (ALL) {
#pragma unroll
        for (int kb = 0; kb < NB_K; ++kb) load(kb, kb);  // every load in flight at once
        load_side(side);
#pragma unroll
        for (int kb = 0; kb < NB_K; ++kb) {
          __syncthreads();  // the buffer's previous readers are done
          store(kb, lds);
          __syncthreads();
          multiply(lds, acc);
        }
      } else {
        __syncthreads();  // the buffers' previous readers are done
        load(0, 0);
        store(0, lds);
        __syncthreads();
#pragma unroll 1
        for (int kb = 0; kb < NB_K; ++kb) {
          if (kb + 1 < NB_K) load(kb + 1, 0);  // in flight during this block's products
          multiply(lds + (kb & 1) * 3 * PD, acc);
          if (kb + 1 < NB_K) store(0, lds + ((kb + 1) & 1) * 3 * PD);
          __syncthreads();
        }
        load_side(side);  // after the loop: no registers held across it
      }
      epilogue(ti, tj, acc, side);
    }
  }
}

// The tiles of one phase owned by worker `worker` of nw: full tiles t < nt
// (tile (t / nb, t % nb) of an m x m product) come first, then the thin row
// blocks t = nt .. nt + nthin - 1 (tile (t - nt, 0)), as in the loop
// for (t = worker; t < nt + nthin; t += nw).
// A symmetric product (sym) is formed from its upper block triangle only:
// tile t runs over the nb (nb + 1) / 2 tiles (i, j), i <= j, row by row, and
// an off-diagonal tile is also stored at its mirror position (j, i); a
// diagonal tile computes each of its elements itself.
struct FullTileMap {
  int nb;
  bool sym;
  __device__ void operator()(int t, int& ti, int& tj) const {
    if (!sym) {
      ti = t / nb;
      tj = t - ti * nb;
      return;
    }
    int i = 0;
    while (t >= nb - i) {
      t -= nb - i;
      ++i;
    }
    ti = i;
    tj = i + t;
  }
  __device__ bool mirror(int ti, int tj) const { return sym && ti != tj; }
  __device__ bool symmetric() const { return sym; }
  static constexpr bool kThin = false;
};
struct ThinTileMap {
  int nt;
  __device__ void operator()(int t, int& ti, int& tj) const {
    ti = t - nt;
    tj = 0;
  }
  __device__ bool mirror(int, int) const { return false; }
  __device__ bool symmetric() const { return false; }
  static constexpr bool kThin = true;
};
__host__ __device__ constexpr int full_tiles(int nb, bool sym) { return sym ? nb * (nb + 1) / 2 : nb * nb; }
// XCD-aware unit order for the symmetric m = 256 action form (36 full and 8
// thin units on 44 workgroups, the hardware dealing workgroup w to XCD w % 8):
// the units of one XCD share row and column panels (40 distinct panels per
// phase over the eight XCDs' L2s, against 83 in the plain order). Any order
// gives the same results: every unit is computed the same way.
__constant__ int kUnitOrder44[44] = {41, 5,  31, 40, 17, 0,  1,  16, 37, 11, 18, 33, 38, 6,  3,  15, 35, 4,  19, 42, 36, 13,
                                     8,  25, 14, 12, 30, 29, 39, 2,  10, 20, 32, 27, 24, 28, 22, 9,  7,  21, 43, 26, 23, 34};
__device__ __forceinline__ int phase_unit(int worker, int nw, int nb, bool sym) {
  return (nw == 44 && nb == 8 && sym) ? kUnitOrder44[worker] : worker;
}
struct PhaseTiles {
  int first_full, end_full, first_thin, end_thin, step;
  FullTileMap full;
  ThinTileMap thin;
  __device__ PhaseTiles(int worker, int nw, int nb, int nthin, bool sym)
      : end_full(full_tiles(nb, sym)), step(nw), full{nb, sym}, thin{full_tiles(nb, sym)} {
    const int u = phase_unit(worker, nw, nb, sym);
    const int nt = end_full;
    first_full = u;
    first_thin = u >= nt ? u : u + ((nt - u + nw - 1) / nw) * nw;
    end_thin = nt + nthin;
  }
};

// One product group of a phase for the streaming gemm and gemm_pair: the
// tiles first .. end - 1 (by step) of `map`, the B operands (B2 for the
// second product when NP = 2), the scales, the epilogue and its side matrices.
template <int NP_, int NS_, int LDB_, int LDC_, class MAP, class EPI>
struct Part {
  static constexpr int NP = NP_, NS = NS_, LDB = LDB_, LDC = LDC_;
  int first, end, step;
  MAP map;
  const double* B1;
  const double* B2;
  double alpha1, alpha2;
  EPI epi;
  const double* S[4];
};
template <int NP, int NS, int LDB, int LDC, class MAP, class EPI>
__device__ __forceinline__ Part<NP, NS, LDB, LDC, MAP, EPI> part(int first, int end, int step, MAP map,
                                                                 const double* B1, const double* B2, double alpha1,
                                                                 double alpha2, EPI epi, const double* S0 = nullptr,
                                                                 const double* S1 = nullptr,
                                                                 const double* S2 = nullptr,
                                                                 const double* S3 = nullptr) {
  return Part<NP, NS, LDB, LDC, MAP, EPI>{first, end, step, map, B1, B2, alpha1, alpha2, epi, {S0, S1, S2, S3}};
}
// No thin part.
struct NoThinEpi {
  __device__ void operator()(int, int, double, double, const Side<0>&) const {}
};
using NoPart = Part<1, 0, kThinWidth, kThinWidth, ThinTileMap, NoThinEpi>;

// Register-resident output for the one-workgroup-per-cloud kernels (m <=
// 128). A phase's full product group (the tiles of a FullTileMap: nb x nb
// tiles of 32 x 32, the upper block triangle when symmetric) and, optionally,
// its thin group (nb x 1 tiles of a ThinTileMap, B of width kThinWidth, the
// same A and the same number of products) are formed in one sweep over K.
// Wave w computes quadrant (w / 2, w % 2) of every tile, as in gemm_range, and
// keeps them all in registers (one 16 x 16 MFMA accumulator per tile and
// product) while K streams through LDS in slabs of 16 (four k steps),
// double-buffered, the next slab's loads in flight during the current slab's
// products; per k step a wave reads one A fragment per tile row and one B
// fragment per tile column. Each quadrant is one MFMA chain over the k steps
// in increasing order, scaled by alpha at the end: the arithmetic of
// gemm_range, so the results are its bits. A is read once per product and
// the B operands once per pass (two passes of half the tile rows for two
// products), against a 32-row and a 32-column panel per tile. With SHARE ==
// kShareB (no thin group) the two products have their own A (A1, A2) and
// one B.
constexpr int kStreamPA = 18;  // A slab row pitch (rows x 16 slab): conflict-free fragment reads
constexpr int stream_pb(int ldb) { return ldb + 16; }  // B slab row pitch (16 x ldb slab)
constexpr int stream_rows(int m, int np) { return np == 1 ? m : m / 2; }  // A rows per pass
constexpr int stream_buf_doubles(int m, int na, int nbp, int ldb, int np, int nthin) {
  return na * stream_rows(m, np) * kStreamPA + nbp * 16 * stream_pb(ldb) + nthin * 16 * stream_pb(kThinWidth);
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// LDS doubles of the streaming gemm over every phase shape (two buffers)
constexpr int stream_lds_doubles(int m) {
  return 2 * cmax(cmax(stream_buf_doubles(m, 1, 1, m, 1, 1), stream_buf_doubles(m, 1, 2, m, 2, 2)),
                  stream_buf_doubles(m, 2, 1, m, 2, 0));
}

template <int m, int SHARE, class FP, class TP>
__device__ __attribute__((noinline)) void gemm_stream(const double* __restrict__ A1, const double* __restrict__ A2,
                                                     FP f, TP t, bool do_full, double* lds) {
  constexpr bool TH = !std::is_same<TP, NoPart>::value;
  constexpr int NP = FP::NP;
  static_assert(!TH || (TP::NP == NP && SHARE == kShareA), "a thin group shares A and the product count");
  constexpr int NA = (NP == 2 && SHARE == kShareB) ? 2 : 1;
  constexpr int NBP = (NP == 2 && SHARE == kShareA) ? 2 : 1;
  constexpr int NT = TH ? NBP : 0;            // thin B slabs
  constexpr int NB = m / 32;                  // tile rows (and full tile columns)
  constexpr int R = stream_rows(m, NP) / 32;  // tile rows per pass
  constexpr int LDB = FP::LDB, TW = kThinWidth;
  constexpr int PA = kStreamPA, PB = stream_pb(LDB), PT = stream_pb(TW);
  constexpr int ASL = 32 * R * PA, BSL = 16 * PB, TSL = 16 * PT;  // slab sizes (doubles)
  constexpr int BUF = NA * ASL + NBP * BSL + NT * TSL;
  constexpr int NKB = m / 16;              // slabs
  constexpr int AQ = 32 * R * 8 / 256;     // double2 per thread per A slab
  constexpr int BH = LDB / 2, TH2 = TW / 2;  // double2 per B slab row
  constexpr int BQ = 16 * BH / 256;        // double2 per thread per B slab
  constexpr int TQ = 16 * TH2 / 256;       // double2 per thread per thin B slab
  static_assert(AQ >= 1 && BQ >= 1 && TQ >= 1 && 2 * BUF <= stream_lds_doubles(m), "slab shape");
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, qi = w >> 1, qj = w & 1;
  const bool sym = f.map.symmetric();
  const double* Ag[2] = {A1, A2};
  const double* Bg[2] = {f.B1, f.B2};
  const double* Tg[2] = {t.B1, t.B2};
  for (int r0 = 0; r0 < NB; r0 += R) {
    double2 ra[NA][AQ], rb[NBP][BQ], rt[NT > 0 ? NT : 1][TQ];
    // A slab element e = tid + 256 q: row e / 8 of the pass, double2 column
    // e % 8; B slab element e: row e / BH, double2 column e % BH
    const auto load = [&](int kb) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
          const int e = tid + 256 * q, r = e >> 3, c2 = e & 7;
          ra[a][q] = gld2(Ag[a] + (size_t)(r0 * 32 + r) * m + kb * 16 + 2 * c2);
        }
      if (do_full) {
#pragma unroll
        for (int b = 0; b < NBP; ++b)
#pragma unroll
          for (int q = 0; q < BQ; ++q) {
            const int e = tid + 256 * q, r = e / BH, c2 = e % BH;
            rb[b][q] = gld2(Bg[b] + (size_t)(kb * 16 + r) * LDB + 2 * c2);
          }
      }
#pragma unroll
      for (int b = 0; b < NT; ++b)
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
          const int e = tid + 256 * q, r = e / TH2, c2 = e % TH2;
          rt[b][q] = gld2(Tg[b] + (size_t)(kb * 16 + r) * TW + 2 * c2);
        }
    };
    const auto store = [&](double* buf) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
          const int e = tid + 256 * q, r = e >> 3, c2 = e & 7;
          *(double2*)(buf + a * ASL + r * PA + 2 * c2) = ra[a][q];
        }
      if (do_full) {
#pragma unroll
        for (int b = 0; b < NBP; ++b)
#pragma unroll
          for (int q = 0; q < BQ; ++q) {
            const int e = tid + 256 * q, r = e / BH, c2 = e % BH;
            *(double2*)(buf + NA * ASL + b * BSL + r * PB + 2 * c2) = rb[b][q];
          }
      }
#pragma unroll
      for (int b = 0; b < NT; ++b)
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
          const int e = tid + 256 * q, r = e / TH2, c2 = e % TH2;
          *(double2*)(buf + NA * ASL + NBP * BSL + b * TSL + r * PT + 2 * c2) = rt[b][q];
        }
    };
    f64x4 acc[R][NB][NP], act[R][NP];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j][p] = f64x4{0.0, 0.0, 0.0, 0.0};
        act[i][p] = f64x4{0.0, 0.0, 0.0, 0.0};
      }
    __syncthreads();  // the buffers' previous readers are done
    load(0);
    store(lds);
    __syncthreads();
    const int ao = (qi * 16 + (l & 15)) * PA + (l >> 4);
    const int bo = (l >> 4) * PB + qj * 16 + (l & 15);
    const int to = (l >> 4) * PT + qj * 16 + (l & 15);
#pragma unroll 1
    for (int kb = 0; kb < NKB; ++kb) {
      if (kb + 1 < NKB) load(kb + 1);  // in flight during this slab's products
      const double* buf = lds + (kb & 1) * BUF;
#pragma unroll
      for (int c = 0; c < 4; ++c) {  // the slab's four k steps, in order
        double af[NA][R];
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int i = 0; i < R; ++i) af[a][i] = buf[a * ASL + ao + i * 32 * PA + 4 * c];
        if (do_full) {
          double bf[NBP][NB];
#pragma unroll
          for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int j = 0; j < NB; ++j) bf[b][j] = buf[NA * ASL + b * BSL + bo + 4 * c * PB + j * 32];
#pragma unroll
          for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
              if (!sym || r0 + i <= j) {
#pragma unroll
                for (int p = 0; p < NP; ++p)
                  acc[i][j][p] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[NA == 2 ? p : 0][i],
                                                                      bf[NBP == 2 ? p : 0][j], acc[i][j][p], 0, 0, 0);
              }
        }
        if constexpr (TH) {
          double bt[NT];
#pragma unroll
          for (int b = 0; b < NT; ++b) bt[b] = buf[NA * ASL + NBP * BSL + b * TSL + to + 4 * c * PT];
#pragma unroll
          for (int i = 0; i < R; ++i)
#pragma unroll
            for (int p = 0; p < NP; ++p)
              act[i][p] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[0][i], bt[NT == 2 ? p : 0], act[i][p], 0, 0, 0);
        }
      }
      if (kb + 1 < NKB) store(lds + ((kb + 1) & 1) * BUF);
      __syncthreads();
    }
    // Epilogues, one tile row at a time: the side values of a whole row are
    // loaded together (with one product, the next row's while this row is
    // stored), since the epilogue's stores keep later loads from moving above
    // them. f64 16x16x4 output layout: register r holds row 4 r + l/16,
    // column l%16.
    if (do_full) {
      constexpr int NS = FP::NS, LDC = FP::LDC;
      constexpr int SB = NP == 1 ? 2 : 1;  // side buffers
      Side<NS> sd[SB][NB][4];
      const auto load_row = [&](int i, Side<NS> (&dst)[NB][4]) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (!(sym && r0 + i > j)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ii = (r0 + i) * 32 + qi * 16 + 4 * r + (l >> 4);
              const int jj = j * 32 + qj * 16 + (l & 15);
#pragma unroll
              for (int u = 0; u < NS; ++u) dst[j][r].v[u] = gld(f.S[u] + (size_t)ii * LDC + jj);
            }
          }
      };
      if constexpr (NS > 0 && SB == 2) load_row(0, sd[0]);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if constexpr (NS > 0 && SB == 2) {
          if (i + 1 < R) load_row(i + 1, sd[(i + 1) & 1]);
        } else if constexpr (NS > 0) {
          load_row(i, sd[0]);
        }
        const int ti = r0 + i;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if (sym && ti > j) continue;
          const bool mir = sym && ti != j;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ii = ti * 32 + qi * 16 + 4 * r + (l >> 4);
            const int jj = j * 32 + qj * 16 + (l & 15);
            const double v1 = f.alpha1 * acc[i][j][0][r];
            const double v2 = NP == 2 ? f.alpha2 * acc[i][j][NP - 1][r] : 0.0;
            f.epi(ii, jj, v1, v2, sd[i % SB][j][r]);
            if (mir) f.epi(jj, ii, v1, v2, sd[i % SB][j][r]);
          }
        }
      }
    }
    if constexpr (TH) {
      constexpr int NS = TP::NS;
      Side<NS> sd[R][4];
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = (r0 + i) * 32 + qi * 16 + 4 * r + (l >> 4);
          const int jj = qj * 16 + (l & 15);
#pragma unroll
          for (int u = 0; u < NS; ++u) sd[i][r].v[u] = gld(t.S[u] + (size_t)ii * TW + jj);
        }
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = (r0 + i) * 32 + qi * 16 + 4 * r + (l >> 4);
          const int jj = qj * 16 + (l & 15);
          const double v1 = t.alpha1 * act[i][0][r];
          const double v2 = NP == 2 ? t.alpha2 * act[i][NP - 1][r] : 0.0;
          t.epi(ii, jj, v1, v2, sd[i][r]);
        }
    }
  }
}

// A phase's full product group and thin group with one A (A1, and A2 for the
// second full product with SHARE == kShareB): one streaming sweep for the
// per-cloud kernels (KB = 0), two gemm_range calls otherwise. The full group
// is skipped when do_full is false.
template <int m, int KB, bool ALL, int SHARE, class FP, class TP>
__device__ __forceinline__ void gemm_pair(const double* A1, const double* A2, const FP& f, const TP& t, bool do_full,
                                          double* lds) {
  constexpr bool TH = !std::is_same<TP, NoPart>::value;
  if constexpr (KB == 0) {
    gemm_stream<m, SHARE>(A1, A2, f, t, do_full, lds);
  } else {
    if (do_full)
      gemm_range<m, KB, ALL, FP::NP, SHARE, FP::NS, FP::LDB, FP::LDC>(f.first, f.end, f.step, f.map, A1, f.B1,
                                                                      A2, f.B2, f.alpha1, f.alpha2, lds, f.epi,
                                                                      f.S[0], f.S[1], f.S[2], f.S[3]);
    if constexpr (TH)
      gemm_range<m, KB, ALL, TP::NP, kShareA, TP::NS, TP::LDB, TP::LDC>(t.first, t.end, t.step, t.map, A1, t.B1,
                                                                        A1, t.B2, t.alpha1, t.alpha2, lds, t.epi,
                                                                        t.S[0], t.S[1], t.S[2], t.S[3]);
  }
}

// ------------------------------------------------------------------ body
constexpr double kTheta23 = 2.014710780944616;

// Column sums of |lambda diag(c) M diag(c s)| (the matrix whose 1-norm sets
// the scaling): column j has entries lambda c_i M_ij c_j s_j, so its absolute
// sum is |lambda| c_j sum_i c_i |M_ij|, read along row j of the symmetric M.
// One wave per column: lane l adds rows l, l + 64, ... in order, then a fixed
// butterfly combines the lanes and lane 0 keeps the total.
// Columns go in groups of kEwGroup per wave, every load of a group issued
// before its stores (a store in between would keep the next column's loads
// from being issued early).
constexpr int kEwGroup = 8;
template <int m, class BAR>
__device__ __forceinline__ void column_abs_sums(const Phi1Args& a, int worker, int nw, double* colsum, BAR& bar) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int j0 = worker * 4 + w; j0 < m; j0 += kEwGroup * nw * 4) {
    double v[kEwGroup];
#pragma unroll
    for (int u = 0; u < kEwGroup; ++u) {
      const int j = j0 + u * nw * 4;
      double acc = 0.0;
      if (j < m) {
#pragma unroll
        for (int i = l; i < m; i += 64) acc += a.cvec[i] * fabs(a.Mraw[(size_t)j * m + i]);
      }
      v[u] = acc;
    }
#pragma unroll
    for (int u = 0; u < kEwGroup; ++u) {
      for (int o = 32; o >= 1; o >>= 1) v[u] += __shfl_xor(v[u], o);
      const int j = j0 + u * nw * 4;
      if (l == 0 && j < m) bar.st(colsum + j, fabs(a.lambda) * a.cvec[j] * v[u]);
    }
  }
}

// An elementwise pass over e = first, first + step, ... < n in groups of
// kEwGroup per thread: ld(e) reads and computes element e's value, st(e, v)
// stores it; every load of a group is issued before its stores (the compiler
// cannot move a load above a store that may alias it).
template <class LD, class ST>
__device__ __forceinline__ void ew_pass(size_t first, size_t step, size_t n, LD ld, ST st) {
  using V = decltype(ld(first));
  for (size_t e0 = first; e0 < n; e0 += kEwGroup * step) {
    V v[kEwGroup];
#pragma unroll
    for (int u = 0; u < kEwGroup; ++u) {
      const size_t e = e0 + u * step;
      if (e < n) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < kEwGroup; ++u) {
      const size_t e = e0 + u * step;
      if (e < n) st(e, v[u]);
    }
  }
}

// s = max(0, ceil(log2(||lambda M||_1 / theta_23))) from the column sums: a
// max over the threads' values, then over the four waves through LDS (a max
// is exact, so every workgroup gets the same s). Non-finite sums give s = 0;
// the non-finite input is flagged where M is formed.
template <int m>
__device__ __forceinline__ int scaling_power(const double* colsum, double* lds) {
  const int t = threadIdx.x;
  double v = t < m ? colsum[t] : 0.0;
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();  // earlier readers of lds are done
  if ((t & 63) == 0) lds[t >> 6] = v;
  __syncthreads();
  const double nrm = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
  __syncthreads();  // lds is free again
  int s = 0;
  if (!(nrm <= 1e300)) s = 0;
  else if (nrm > kTheta23) s = (int)ceil(log2(nrm / kTheta23));
  return s > 1000 ? 1000 : s;
}

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
  bool sym;          // symmetric chain (see FullTileMap)
};

// Horner step J (J = 4 ... 0): R_chain <- Y4 R_chain + B_J, both chains (one
// workgroup per tile, the Y4 row panel shared by the two products).
template <int m, int KB, bool ALL, int J, class BAR>
__device__ __forceinline__ void horner_phase(const TaylorWs& w, int worker, int nw, double* lds, BAR& bar) {
  constexpr int nb = m / 32;
  constexpr int src = (J + 1) & 1, dst = J & 1;
  {
    const PhaseTiles pt(worker, nw, nb, 0, w.sym);
    gemm_pair<m, KB, ALL, kShareA>(
        w.Y4, w.Y4,
        part<2, 3, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, w.R[0][src], w.R[1][src], 1.0, 1.0,
                         [&](int i, int j, double v0, double v1, const Side<3>& sd) {
                           const size_t e = (size_t)i * m + j;
                           const double id = i == j ? 1.0 : 0.0, y = sd.v[0] * w.sc1, y2 = sd.v[1], y3 = sd.v[2];
                           bar.st(w.R[0][dst] + e, v0 + coef_block<J, 0>(id, y, y2, y3));
                           bar.st(w.R[1][dst] + e, v1 + coef_block<J, 1>(id, y, y2, y3));
                         },
                         w.X0, w.Y2, w.Y3),
        NoPart{}, true, lds);
  }
  bar.sync();
}

template <int m, int KB, bool ALL, class BAR>
__device__ __forceinline__ void phi1_body(const Phi1Args& a, int worker, int nw, double* lds, BAR& bar) {
  constexpr int nb = m / 32;
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
  ew_pass((size_t)worker * 256 + t, (size_t)nw * 256, mm,
          [&](size_t e) {
            const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
            return a.lambda * a.cvec[i] * a.Mraw[e] * a.cvec[j] * a.svec[j];
          },
          [&](size_t e, double v) { bar.st(X0 + e, v); });
  column_abs_sums<m>(a, worker, nw, colsum, bar);
  bar.sync();

  // ---- s from the 1-norm (every worker, same value)
  const int s = scaling_power<m>(colsum, lds);
  if (worker == 0 && t == 0) *a.sdev = s;
  const double sc1 = ldexp(1.0, -s), sc2 = ldexp(1.0, -2 * s);

  // ---- P1: Y2 = X0 X0 / 4^s
  {
    const PhaseTiles pt(worker, nw, nb, 0, a.sym != 0);
    gemm_pair<m, KB, ALL, kShareA>(X0, X0,
                                   part<1, 0, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, X0, X0, sc2, 0.0,
                                                    [&](int i, int j, double v, double, const Side<0>&) {
                                                      bar.st(Y2 + (size_t)i * m + j, v);
                                                    }),
                                   NoPart{}, true, lds);
  }
  bar.sync();
  // ---- P2: Y3 = Y2 X0 / 2^s (its epilogue also forms B_5 of both chains) and Y4 = Y2 Y2
  {
    const PhaseTiles pt(worker, nw, nb, 0, a.sym != 0);
    gemm_pair<m, KB, ALL, kShareA>(
        Y2, Y2,
        part<2, 2, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, X0, Y2, sc1, 1.0,
                         [&](int i, int j, double y3, double y4, const Side<2>& sd) {
                           const size_t e = (size_t)i * m + j;
                           const double id = i == j ? 1.0 : 0.0, y = sd.v[0] * sc1, y2 = sd.v[1];
                           bar.st(Y3 + e, y3);
                           bar.st(Y4 + e, y4);
                           bar.st(R01 + e, coef_block<5, 0>(id, y, y2, y3));
                           bar.st(R11 + e, coef_block<5, 1>(id, y, y2, y3));
                         },
                         X0, Y2),
        NoPart{}, true, lds);
  }
  bar.sync();
  // ---- P3..P7: Horner steps J = 4 ... 0 (J odd reads buffer 0, writes 1 ... ends in buffer 0)
  const TaylorWs w{X0, Y2, Y3, Y4, {{R00, R01}, {R10, R11}}, sc1, a.sym != 0};
  horner_phase<m, KB, ALL, 4>(w, worker, nw, lds, bar);
  horner_phase<m, KB, ALL, 3>(w, worker, nw, lds, bar);
  horner_phase<m, KB, ALL, 2>(w, worker, nw, lds, bar);
  horner_phase<m, KB, ALL, 1>(w, worker, nw, lds, bar);
  horner_phase<m, KB, ALL, 0>(w, worker, nw, lds, bar);
  // ---- undo the scaling: P <- P (E + I) / 2, E <- E E
  double* Pc = R00;
  double* Ec = R10;
  double* Pn = R01;
  double* En = R11;
  for (int it = 0; it < s; ++it) {
    {
      const PhaseTiles pt(worker, nw, nb, 0, a.sym != 0);
      gemm_pair<m, KB, ALL, kShareB>(Ec, Pc,
                                     part<2, 1, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, Ec, Ec, 1.0, 0.5,
                                                      [&](int i, int j, double e2, double pe, const Side<1>& sd) {
                                                        const size_t e = (size_t)i * m + j;
                                                        bar.st(En + e, e2);
                                                        bar.st(Pn + e, pe + 0.5 * sd.v[0]);
                                                      },
                                                      Pc),
                                     NoPart{}, true, lds);
    }
    bar.sync();
    double* x = Ec; Ec = En; En = x;
    x = Pc; Pc = Pn; Pn = x;
  }
  // ---- S = lambda P (canonical), T = diag(c s) S diag(c) in device order
  const int fq = m / 2;
  ew_pass((size_t)worker * 256 + t, (size_t)nw * 256, mm,
          [&](size_t e) {
            const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
            const double sv = a.lambda * Pc[e];
            return make_double2(sv, a.cvec[i] * a.svec[i] * sv * a.cvec[j]);
          },
          [&](size_t e, double2 v) {
            const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
            if (!isfinite(v.x)) __hip_atomic_fetch_or(a.flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a.S64[e] = v.x;
            const int di = i < fq ? 2 * i : 2 * (i - fq) + 1;
            const int dj = j < fq ? 2 * j : 2 * (j - fq) + 1;
            a.T64[(size_t)di * m + dj] = v.y;
          });
}

// ------------------------------------------------------------------ action form
// phi_1 applied to a thin block v = diag(c) H0 (m x 32, canonical order) with
// the same Taylor degree and scaling: since every factor is a polynomial in Y
// they commute, so
//   phi_1(2^s Y) v = prod_{k<s} (E_k + I)/2 . phi_1(Y) v,   E_k = e^{2^k Y},
// and only the exp chain needs m x m products (Horner steps, then squarings);
// phi_1(Y) v takes thin Horner steps on Y v, Y^2 v, Y^3 v, and each squaring
// phase applies (E_k + I)/2 to the thin block. The result leaves as G' in
// device order (FP32 and a BF16 hi + lo pair), as the core product writes it.

// Horner step J of both chains: E <- Y4 E + B_J (full tiles) and
// W <- Y4 W + B_J v (thin tiles, B_J v from v, Y v, Y^2 v, Y^3 v).
template <int m, int KB, bool ALL, int J, class BAR>
__device__ __forceinline__ void apply_horner(const TaylorWs& w, double* const (&E)[2], const double* V,
                                             const double* U1, const double* U2, const double* U3,
                                             double* const (&W)[2], int worker, int nw, double* lds, BAR& bar) {
  constexpr int nb = m / 32, TW = kThinWidth;
  constexpr int src = (J + 1) & 1, dst = J & 1;
  {
    const PhaseTiles pt(worker, nw, nb, nb, w.sym);
    gemm_pair<m, KB, ALL, kShareA>(
        w.Y4, w.Y4,
        part<1, 3, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, E[src], E[src], 1.0, 0.0,
                         [&](int i, int j, double v, double, const Side<3>& sd) {
                           const double id = i == j ? 1.0 : 0.0;
                           bar.st(E[dst] + (size_t)i * m + j,
                               v + coef_block<J, 1>(id, sd.v[0] * w.sc1, sd.v[1], sd.v[2]));
                         },
                         w.X0, w.Y2, w.Y3),
        part<1, 4, TW, TW>(pt.first_thin, pt.end_thin, pt.step, pt.thin, W[src], W[src], 1.0, 0.0,
                           [&](int i, int j, double v, double, const Side<4>& sd) {
                             bar.st(W[dst] + (size_t)i * TW + j,
                                 v + coef_block<J, 0>(sd.v[0], sd.v[1], sd.v[2], sd.v[3]));
                           },
                           V, U1, U2, U3),
        true, lds);
  }
  bar.sync();
}

template <int m, int KB, bool ALL, class BAR>
__device__ __forceinline__ void apply_body(const Phi1Args& a, const ApplyArgs& ap, int worker, int nw, double* lds,
                                           BAR& bar) {
  constexpr int nb = m / 32, TW = kThinWidth;
  const size_t mm = (size_t)m * m, mt = (size_t)m * TW;
  double* X0 = a.ws;
  double* Y2 = X0 + mm;
  double* Y3 = Y2 + mm;
  double* Y4 = Y3 + mm;
  double* E0 = Y4 + mm;  // exp chain, two buffers
  double* E1 = E0 + mm;
  double* colsum = a.ws + 8 * mm;
  double* V = colsum + m;  // thin blocks, m x TW each
  double* U1 = V + mt;
  double* U2 = U1 + mt;
  double* U3 = U2 + mt;
  double* W0 = U3 + mt;
  double* W1 = W0 + mt;
  const int t = threadIdx.x, f = m / 2, d = ap.d;

  // ---- P0: X0 = lambda M, column sums of |X0|, and v = diag(c) H0 (canonical, zero past d)
  ew_pass((size_t)worker * 256 + t, (size_t)nw * 256, mm,
          [&](size_t e) {
            const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
            return a.lambda * a.cvec[i] * a.Mraw[e] * a.cvec[j] * a.svec[j];
          },
          [&](size_t e, double v) { bar.st(X0 + e, v); });
  ew_pass((size_t)worker * 256 + t, (size_t)nw * 256, mt,
          [&](size_t e) {
            const int i = (int)(e / TW), c = (int)(e - (size_t)i * TW);
            const int di = i < f ? 2 * i : 2 * (i - f) + 1;
            return c < d ? a.cvec[i] * ap.H0[(size_t)di * d + c] : 0.0;
          },
          [&](size_t e, double v) { bar.st(V + e, v); });
  column_abs_sums<m>(a, worker, nw, colsum, bar);
  bar.sync();
  const int s = scaling_power<m>(colsum, lds);
  if (worker == 0 && t == 0) *a.sdev = s;
  const double sc1 = ldexp(1.0, -s), sc2 = ldexp(1.0, -2 * s);

  // ---- P1: Y2 = X0 X0 / 4^s; U1 = Y v
  {
    const PhaseTiles pt(worker, nw, nb, nb, a.sym != 0);
    gemm_pair<m, KB, ALL, kShareA>(X0, X0,
                                   part<1, 0, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, X0, X0, sc2, 0.0,
                                                    [&](int i, int j, double v, double, const Side<0>&) {
                                                      bar.st(Y2 + (size_t)i * m + j, v);
                                                    }),
                                   part<1, 0, TW, TW>(pt.first_thin, pt.end_thin, pt.step, pt.thin, V, V, sc1, 0.0,
                                                      [&](int i, int j, double v, double, const Side<0>&) {
                                                        bar.st(U1 + (size_t)i * TW + j, v);
                                                      }),
                                   true, lds);
  }
  bar.sync();
  // ---- P2: Y3 = Y2 Y, Y4 = Y2 Y2 (with B_5 of the exp chain); U2 = Y2 v, U3 = Y2 U1 (with B_5 v)
  {
    const PhaseTiles pt(worker, nw, nb, nb, a.sym != 0);
    gemm_pair<m, KB, ALL, kShareA>(
        Y2, Y2,
        part<2, 2, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, X0, Y2, sc1, 1.0,
                         [&](int i, int j, double y3, double y4, const Side<2>& sd) {
                           const size_t e = (size_t)i * m + j;
                           const double id = i == j ? 1.0 : 0.0;
                           bar.st(Y3 + e, y3);
                           bar.st(Y4 + e, y4);
                           bar.st(E1 + e, coef_block<5, 1>(id, sd.v[0] * sc1, sd.v[1], y3));
                         },
                         X0, Y2),
        part<2, 2, TW, TW>(pt.first_thin, pt.end_thin, pt.step, pt.thin, V, U1, 1.0, 1.0,
                           [&](int i, int j, double u2, double u3, const Side<2>& sd) {
                             const size_t e = (size_t)i * TW + j;
                             bar.st(U2 + e, u2);
                             bar.st(U3 + e, u3);
                             bar.st(W1 + e, coef_block<5, 0>(sd.v[0], sd.v[1], u2, u3));
                           },
                           V, U1),
        true, lds);
  }
  bar.sync();
  // ---- Horner steps J = 4 ... 0 (results in E0 and W0)
  const TaylorWs w{X0, Y2, Y3, Y4, {{nullptr, nullptr}, {nullptr, nullptr}}, sc1, a.sym != 0};
  double* const E[2] = {E0, E1};
  double* const W[2] = {W0, W1};
  apply_horner<m, KB, ALL, 4>(w, E, V, U1, U2, U3, W, worker, nw, lds, bar);
  apply_horner<m, KB, ALL, 3>(w, E, V, U1, U2, U3, W, worker, nw, lds, bar);
  apply_horner<m, KB, ALL, 2>(w, E, V, U1, U2, U3, W, worker, nw, lds, bar);
  apply_horner<m, KB, ALL, 1>(w, E, V, U1, U2, U3, W, worker, nw, lds, bar);
  apply_horner<m, KB, ALL, 0>(w, E, V, U1, U2, U3, W, worker, nw, lds, bar);
  // ---- squaring: W <- (E W + W) / 2, E <- E E (the last E is not needed)
  double* Ec = E0;
  double* En = E1;
  double* Wc = W0;
  double* Wn = W1;
  for (int it = 0; it < s; ++it) {
    {
      const PhaseTiles pt(worker, nw, nb, nb, a.sym != 0);
      gemm_pair<m, KB, ALL, kShareA>(
          Ec, Ec,
          part<1, 0, m, m>(pt.first_full, pt.end_full, pt.step, pt.full, Ec, Ec, 1.0, 0.0,
                           [&](int i, int j, double v, double, const Side<0>&) { bar.st(En + (size_t)i * m + j, v); }),
          part<1, 1, TW, TW>(pt.first_thin, pt.end_thin, pt.step, pt.thin, Wc, Wc, 0.5, 0.0,
                             [&](int i, int j, double v, double, const Side<1>& sd) {
                               bar.st(Wn + (size_t)i * TW + j, v + 0.5 * sd.v[0]);
                             },
                             Wc),
          it + 1 < s, lds);
    }
    bar.sync();
    double* x = Ec; Ec = En; En = x;
    x = Wc; Wc = Wn; Wn = x;
  }
  // ---- G' = diag(c s) lambda w in device order, as FP32 and a BF16 hi + lo pair
  ew_pass((size_t)worker * 256 + t, (size_t)nw * 256, (size_t)m * d,
          [&](size_t e) {
            const int i = (int)(e / d), c = (int)(e - (size_t)i * d);
            const double sv = a.lambda * Wc[(size_t)i * TW + c];
            return make_double2(sv, a.cvec[i] * a.svec[i] * sv);
          },
          [&](size_t e, double2 v) {
            const int i = (int)(e / d), c = (int)(e - (size_t)i * d);
            if (!isfinite(v.x)) __hip_atomic_fetch_or(a.flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gst(ap.G64 + (size_t)i * TW + c, v.x);
            const int di = i < f ? 2 * i : 2 * (i - f) + 1;
            const float g = (float)v.y;
            const __bf16 hi = (__bf16)g;
            ap.G32[(size_t)di * d + c] = g;
            ap.Gt16[(size_t)c * m + di] = hi;
            ap.Gt16[(size_t)kMaxDBlocks * kDBlock * m + (size_t)c * m + di] = (__bf16)(g - (float)hi);
          });
}

// K blocks: the cooperative kernel (one workgroup per CU) issues all of a
// tile's loads at once and stages 128-wide blocks, one memory round trip per
// tile. The one-workgroup-per-cloud kernels pipeline 32-wide blocks through
// two LDS buffers (50 KB) and are held to 256 registers per lane, so two
// clouds share a CU (two waves per SIMD hide each other's LDS and memory
// waits); a whole tile as one block would take 101 KB of LDS and 512
// registers, one cloud per CU. The k order of every MFMA chain is the same
// for any block width, so both kernels give the same bits.
constexpr int kWgKB = 32, kGridKB = 128;
template <int M>
constexpr int wg_kb() { return M <= 128 ? 0 : kWgKB; }
template <int M>
constexpr bool wg_all() { return false; }
// waves per SIMD the per-cloud kernels are compiled for: one with the
// register-resident output (m <= 128), two otherwise
template <int M>
constexpr int wg_waves() { return M <= 128 ? 1 : 2; }

template <int M>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(wg_waves<M>()))) void k_phi1_wg(const Phi1Args* __restrict__ args) {
  extern __shared__ double lds[];
  const Phi1Args a = args[blockIdx.x];
  WgBarrier bar;
  phi1_body<M, wg_kb<M>(), wg_all<M>()>(a, 0, 1, lds, bar);
}

constexpr int kMaxWorkers = 256;  // one workgroup per CU (a workgroup's LDS allows no second)

template <int M>
__global__ __launch_bounds__(256) void k_phi1_grid(Phi1Args a) {
  extern __shared__ double lds[];
  GridBarrier bar{a.barrier, gridDim.x, 0u, a.flag};
  phi1_body<M, (M < kGridKB ? M : kGridKB), true>(a, (int)blockIdx.x, (int)gridDim.x, lds, bar);
  bar.finish();
}

template <int M>
__global__ __launch_bounds__(256) void k_phi1_apply_grid(Phi1Args a, ApplyArgs ap) {
  extern __shared__ double lds[];
  GridBarrier bar{a.barrier, gridDim.x, 0u, a.flag};
  apply_body<M, (M < kGridKB ? M : kGridKB), true>(a, ap, (int)blockIdx.x, (int)gridDim.x, lds, bar);
  bar.finish();
}

template <int M>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(wg_waves<M>()))) void k_phi1_apply_wg(const Phi1Args* __restrict__ args,
                                                      const ApplyArgs* __restrict__ aargs) {
  extern __shared__ double lds[];
  const Phi1Args a = args[blockIdx.x];
  const ApplyArgs ap = aargs[blockIdx.x];
  WgBarrier bar;
  apply_body<M, wg_kb<M>(), wg_all<M>()>(a, ap, 0, 1, lds, bar);
}

// LDS bytes of the phi_1 kernels for padded size m.
static size_t phi1_lds_bytes(int KB, bool all) { return (size_t)gemm_lds_doubles(KB, all) * sizeof(double); }
// LDS bytes of the per-cloud kernels
template <int M>
static size_t wg_lds_bytes() {
  return wg_kb<M>() == 0 ? sizeof(double) * (size_t)stream_lds_doubles(M) : phi1_lds_bytes(wg_kb<M>(), wg_all<M>());
}

size_t phi1_ws_doubles(int m) { return 8 * (size_t)m * m + m + 6 * (size_t)m * kThinWidth; }

static void fill_args(rfd_plan_s* p, Phi1Args& a) {
  a.m = p->dev_m;
  a.sym = 1;
  for (double w : p->w)
    if (w < 0.0) a.sym = 0;
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
  const size_t lds = phi1_lds_bytes(M < kGridKB ? M : kGridKB, true);
  hipError_t e = hipFuncSetAttribute((const void*)k_phi1_grid<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  constexpr int nb = M / 32;
  // workgroups: every phase has full_tiles(nb, sym) tiles (pairs of products);
  // fewer workgroups make the barrier cheaper and give each more tiles (the
  // count never changes results: each tile is computed the same way)
  const int tiles = full_tiles(nb, a.sym != 0);
  int nw = tuned(kTunePhi1Workgroups, M, 0, 1, 0, tiles < kMaxWorkers ? tiles : kMaxWorkers);
  if (nw < 1) nw = 1;
  if (nw > tiles) nw = tiles;
  if (nw > kMaxWorkers) nw = kMaxWorkers;
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

template <int M>
static hipError_t launch_apply_m(Phi1Args& a, ApplyArgs& ap, hipStream_t st) {
  const size_t lds = phi1_lds_bytes(M < kGridKB ? M : kGridKB, true);
  hipError_t e =
      hipFuncSetAttribute((const void*)k_phi1_apply_grid<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  constexpr int nb = M / 32;
  const int units = full_tiles(nb, a.sym != 0) + nb;  // full tiles plus thin row tiles
  const int nw = units < kMaxWorkers ? units : kMaxWorkers;
  void* kargs[] = {&a, &ap};
  ProfileScope prof(kKPhi1Apply, st);
  return hipLaunchCooperativeKernel((const void*)k_phi1_apply_grid<M>, dim3(nw), dim3(256), kargs, (unsigned)lds,
                                    st);
}

hipError_t launch_phi1_apply(rfd_plan_s* p, int d, hipStream_t st) {
  if (d < 1 || d > kThinWidth) return hipErrorInvalidValue;
  Phi1Args a;
  fill_args(p, a);
  ApplyArgs ap{p->dev.H0, d, 0, p->dev.G32, p->dev.Gt16, p->dev.G64};
  p->action_d = d;
  switch (a.m) {
    case 64: return launch_apply_m<64>(a, ap, st);
    case 128: return launch_apply_m<128>(a, ap, st);
    case 256: return launch_apply_m<256>(a, ap, st);
    default: return hipErrorInvalidValue;
  }
}

int phi1_apply_max_width() { return kThinWidth; }

int phi1_grid_workers_max(rfd_plan_s* p) {
  Phi1Args a;
  fill_args(p, a);
  const int tiles = full_tiles(a.m / 32, a.sym != 0);
  return tiles < kMaxWorkers ? tiles : kMaxWorkers;
}

void phi1_fill_apply_args(rfd_plan_s* p, int d, void* out) {
  *(ApplyArgs*)out = ApplyArgs{p->dev.H0, d, 0, p->dev.G32, p->dev.Gt16, p->dev.G64};
  p->action_d = d;
}

size_t phi1_apply_args_bytes() { return sizeof(ApplyArgs); }

template <int M>
static hipError_t launch_apply_batch_m(int n, const void* dev_args, const void* dev_aargs, hipStream_t st) {
  const size_t lds = wg_lds_bytes<M>();
  hipError_t e =
      hipFuncSetAttribute((const void*)k_phi1_apply_wg<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  ProfileScope prof(kKPhi1Batch, st);
  hipLaunchKernelGGL(k_phi1_apply_wg<M>, dim3(n), dim3(256), lds, st, (const Phi1Args*)dev_args,
                     (const ApplyArgs*)dev_aargs);
  return hipGetLastError();
}

hipError_t launch_phi1_apply_batch_dev(int M, int n, const void* dev_args, const void* dev_aargs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (M) {
    case 64: return launch_apply_batch_m<64>(n, dev_args, dev_aargs, st);
    case 128: return launch_apply_batch_m<128>(n, dev_args, dev_aargs, st);
    case 256: return launch_apply_batch_m<256>(n, dev_args, dev_aargs, st);
    default: return hipErrorInvalidValue;
  }
}

void phi1_fill_args(rfd_plan_s* p, void* args_out) { fill_args(p, *(Phi1Args*)args_out); }

template <int M>
static hipError_t launch_phi1_batch_m(int n, const void* dev_args, hipStream_t st) {
  const size_t lds = wg_lds_bytes<M>();
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
