// Split-N streaming kernels of the RFD integrator on gfx950.
//
//   k_bta     one pass over a cloud: recompute the random features of a chunk
//             of points into LDS and accumulate, on the matrix cores, the
//             Gram B^T A (upper triangle) and/or B^T F; one FP32 partial per
//             workgroup (Sec. 2.4: B^T A and B^T x of the GFI formula).
//   k_reduce  two-level fixed-order FP64 sum of the partials -> M (canonical
//             order) and H0 (device order); flags non-finite sums.
//   k_gcore   G' = T H0 (FP64) with T = diag(c s) S diag(c), S = lambda phi_1(lambda M).
//   k_expand  out = F + Phi G' with the features of each point computed in
//             registers directly in the MFMA operand layout.
//
// Features are never stored in HBM: both passes evaluate cos/sin of the FP32
// phase omega_k . x (in revolutions, reduced by fract) with the hardware
// transcendental unit. Feature columns are kept unscaled on the device; the
// scale c_k and sign s_k live in the m x m core.
#include <type_traits>

#include "rfd_internal.h"

namespace rfd {

// ------------------------------------------------------------------ helpers
// sin and cos of 2 pi th for a phase th in revolutions
__device__ __forceinline__ void rev_sincos(float th, float& s, float& c) {
  float t = __builtin_amdgcn_fractf(th);  // exact: th - floor(th) in [0, 1)
  s = __builtin_amdgcn_sinf(t);           // sin(2 pi t)
  c = __builtin_amdgcn_cosf(t);           // cos(2 pi t)
}
__device__ __forceinline__ void phase_sincos(float4 w, float x, float y, float z, float& s, float& c) {
  rev_sincos(fmaf(w.z, z, fmaf(w.y, y, w.x * x)), s, c);
}

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Two floats rounded to BF16 (nearest even) in one word, a in the low half:
// a single v_cvt_pk_bf16_f32.
__device__ __forceinline__ unsigned pack_bf16x2(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

// Global-typed accesses. The batched kernels read their pointers from cloud
// records in device memory, which the compiler cannot place in an address
// space, so plain accesses become flat ones; flat accesses also count
// against the LDS wait counter, so the LDS wait before every barrier would
// drain the next chunk's or tile's loads in flight as well. Every buffer
// these kernels touch is global memory.
typedef float f32x4v_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4v_t __attribute__((ext_vector_type(4)));
#define RFD_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ float gldf(const float* p) { return *(const RFD_GLOBAL float*)p; }
__device__ __forceinline__ double gldd(const double* p) { return *(const RFD_GLOBAL double*)p; }
__device__ __forceinline__ float4 gld4(const float* p) {
  const f32x4v_t v = *(const RFD_GLOBAL f32x4v_t*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 gldu4(const void* p) {
  const u32x4v_t v = *(const RFD_GLOBAL u32x4v_t*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstf(float* p, float v) { *(RFD_GLOBAL float*)p = v; }
__device__ __forceinline__ void gstd(double* p, double v) { *(RFD_GLOBAL double*)p = v; }
__device__ __forceinline__ void gsth(__bf16* p, __bf16 v) { *(RFD_GLOBAL __bf16*)p = v; }
__device__ __forceinline__ void gst4(float* p, float4 v) {
  *(RFD_GLOBAL f32x4v_t*)p = f32x4v_t{v.x, v.y, v.z, v.w};
}

// Gram tile schedule. The NB x NB grid of 32 x 32 blocks of the symmetric
// Gram has NB (NB + 1) / 2 distinct tiles: one per vertex (diagonal) and one
// per edge of the complete graph on the NB feature blocks. Orienting every
// edge towards one endpoint K groups the tiles into stars that share the MFMA
// operand F_K; with a near-regular orientation every wave gets the same static
// shape: segments of SEG[g] slots, slot 0 of a segment being the diagonal tile
// (K, K) (except for NB = 2) and the other slots tiles (K, J). A tile computed as (K, J) with
// K > J is the transpose of the upper-triangle tile; the reduction writes both
// mirror images, so orientation does not matter there.
//   NB = 8: circulant tournament on blocks 0..6 (i -> i+1, i+2, i+3 mod 7),
//           7 -> 0..3, 4..6 -> 7; waves pair an out-degree-4 block with an
//           out-degree-3 block: 9 tiles each.
//   NB = 4: 0 -> 1, 2; 1 -> 2, 3; 2 -> 3; 3 -> 0; the shorter stars repeat
//           their diagonal tile in the spare slot (computed, not stored).
//   NB = 2: waves 0, 1 the diagonal tiles, wave 2 the tile (0, 1).
template <int NB>
struct GramSched;
template <>
struct GramSched<8> {
  static constexpr int NSEG = 2, SLOTS = 9;
  static constexpr int SEG[2] = {5, 4};
};
template <>
struct GramSched<4> {
  static constexpr int NSEG = 1, SLOTS = 3;
  static constexpr int SEG[1] = {3};
};
template <>
struct GramSched<2> {
  static constexpr int NSEG = 1, SLOTS = 1;
  static constexpr int SEG[1] = {1};
};

// (K, J) of slot s of wave w; returns false for a spare slot (not stored).
__host__ __device__ inline bool gram_slot(int NB, int w, int s, int& K, int& J) {
  if (NB == 8) {
    if (s < 5) {
      const int k0[4] = {7, 4, 5, 6};
      const int j0[4][4] = {{0, 1, 2, 3}, {5, 6, 0, 7}, {6, 0, 1, 7}, {0, 1, 2, 7}};
      K = k0[w];
      J = s == 0 ? K : j0[w][s - 1];
    } else {
      K = w;
      J = s == 5 ? w : w + (s - 5);
    }
    return true;
  }
  if (NB == 4) {
    const int j4[4][3] = {{0, 1, 2}, {1, 2, 3}, {2, 3, -1}, {3, 0, -1}};
    K = w;
    J = j4[w][s];
    if (J < 0) {
      J = K;
      return false;
    }
    return true;
  }
  // NB == 2
  const int k2[4] = {0, 1, 0, 0}, jj[4] = {0, 1, 1, 0};
  K = k2[w];
  J = jj[w];
  return w < 3;
}

__host__ __device__ constexpr int gram_slots(int NB) { return NB == 8 ? 9 : (NB == 4 ? 3 : 1); }

template <int M, int PREC>
struct BtaShape {
  static constexpr int NB = M / 32;                 // 32-wide feature blocks
  static constexpr int SLOTS = gram_slots(NB);      // Gram tiles per wave
  static constexpr int RB = M / 16;                 // 16-row blocks for B^T F
  static constexpr int RPW = RB / 4;                // row blocks per wave
  // LDS row pitch (elements) of the feature and field tiles: conflict-free reads
  static constexpr int PITCH = PREC ? (kChunk + 8) : (kChunk + 1);
  using elem = typename std::conditional<PREC != 0, __bf16, float>::type;
};

// Channel blocks of a pass over d channels: 1, 2 or 4 blocks of 16. A Gram
// pass without a field still carries one (all-zero) block: that variant
// keeps the register allocation of the fused kernel.
int dblocks(int d) {
  if (d <= 16) return 1;
  if (d <= 32) return 2;
  return 4;
}

size_t bta_partial_floats(int m, int d, bool gram) {
  const int NB = m / 32;
  const size_t g = gram ? (size_t)4 * gram_slots(NB) * 1024 : 0;
  return g + (size_t)(m / 16) * dblocks(d) * 256;
}

// Number of partials (= workgroups) of a split-N pass over N points: at
// least 16 chunks per partial when the pass carries the Gram (its partials
// are m(m+1)/2 floats, so fewer of them), 2 otherwise; at most 512 partials
// (two workgroups per CU), or 768 for a field pass of one channel block over
// at least 8 chunks per partial, whose registers and LDS leave room for three
// workgroups per CU (all but the FP32 pass at m = 256, whose feature tile
// alone takes 66 KB of LDS); with fewer chunks the extra partials cost more
// in the reduction than they gain. A function of N, m, the precision, the
// pass kind and the channel blocks only, so a cloud gets the same partition
// alone and in a batch.
constexpr int kMinChunksPerPartGram = 16;
constexpr int kMinChunksPerPart = 2;
int bta_partials(int64_t N, int m, int d, bool gram, int prec) {
  const int64_t chunks = (N + kChunk - 1) / kChunk;
  const int per = gram ? kMinChunksPerPartGram : kMinChunksPerPart;
  int64_t parts = (chunks + per - 1) / per;
  const bool three_per_cu = !gram && dblocks(d) == 1 && !(prec == 0 && m > 128) && chunks >= 768 * 8;
  const int cap = three_per_cu ? 768 : 512;
  if (parts > cap) parts = cap;
  if (parts < 1) parts = 1;
  return (int)parts;
}

// ------------------------------------------------------------------ k_bta
// Accumulators: Gram slots acc[s] (32x32 f32: 16 regs), B^T F tiles hacc[r][cb]
// (16x16: 4 regs). The wave index w only selects LDS rows and partial slots.
template <int M, int PREC, bool GRAM, int DB>
__device__ __forceinline__ void bta_mma(const typename BtaShape<M, PREC>::elem* __restrict__ phi,
                                        const typename BtaShape<M, PREC>::elem* __restrict__ fs,
                                        const typename BtaShape<M, PREC>::elem* __restrict__ fsl,
                                        f32x16 (&acc)[BtaShape<M, PREC>::SLOTS],
                                        f32x4 (&hacc)[BtaShape<M, PREC>::RPW][DB], int lane, int w) {
  using S = BtaShape<M, PREC>;
  using G = GramSched<S::NB>;
  constexpr int P = S::PITCH;
  if constexpr (PREC) {
    // BF16: Gram with 32x32x16, B^T F with 16x16x32.
    if constexpr (GRAM) {
      // the four K steps unrolled: a step's LDS operand reads can be issued
      // during the previous step's MFMAs
#pragma unroll
      for (int ks = 0; ks < kChunk / 16; ++ks) {
        const __bf16* base = phi + (lane & 31) * P + ks * 16 + 8 * (lane >> 5);
        int s0 = 0;
#pragma unroll
        for (int g = 0; g < G::NSEG; ++g) {
          int K, J;
          gram_slot(S::NB, w, s0, K, J);
          const bf16x8 a = *(const bf16x8*)(base + K * 32 * P);
          if constexpr (S::NB == 2) {  // slot 0 of wave 2 is the off-diagonal tile
            const bf16x8 b0 = *(const bf16x8*)(base + J * 32 * P);
            acc[s0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc[s0], 0, 0, 0);
          } else {
            acc[s0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, acc[s0], 0, 0, 0);
          }
#pragma unroll
          for (int q = 1; q < G::SEG[g]; ++q) {
            gram_slot(S::NB, w, s0 + q, K, J);
            const bf16x8 bj = *(const bf16x8*)(base + J * 32 * P);
            acc[s0 + q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bj, acc[s0 + q], 0, 0, 0);
          }
          s0 += G::SEG[g];
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < kChunk / 32; ++ks) {
      // F enters as a hi + lo pair of BF16 values (F = hi + lo to ~16 bits)
      bf16x8 fb[DB], fbl[DB];
#pragma unroll
      for (int cb = 0; cb < DB; ++cb) {
        fb[cb] = *(const bf16x8*)(fs + (cb * 16 + (lane & 15)) * P + ks * 32 + 8 * (lane >> 4));
        fbl[cb] = *(const bf16x8*)(fsl + (cb * 16 + (lane & 15)) * P + ks * 32 + 8 * (lane >> 4));
      }
#pragma unroll
      for (int r = 0; r < S::RPW; ++r) {
        const int R = w + 4 * r;
        const bf16x8 fa = *(const bf16x8*)(phi + (R * 16 + (lane & 15)) * P + ks * 32 + 8 * (lane >> 4));
#pragma unroll
        for (int cb = 0; cb < DB; ++cb) {
          hacc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[cb], hacc[r][cb], 0, 0, 0);
          hacc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fbl[cb], hacc[r][cb], 0, 0, 0);
        }
      }
    }
  } else {
    // FP32: Gram with 32x32x2, B^T F with 16x16x4.
    if constexpr (GRAM) {
#pragma unroll 2
      for (int ks = 0; ks < kChunk / 2; ++ks) {
        const float* base = phi + (lane & 31) * P + ks * 2 + (lane >> 5);
        int s0 = 0;
#pragma unroll
        for (int g = 0; g < G::NSEG; ++g) {
          int K, J;
          gram_slot(S::NB, w, s0, K, J);
          const float a = base[K * 32 * P];
          if constexpr (S::NB == 2) {  // slot 0 of wave 2 is the off-diagonal tile
            acc[s0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, base[J * 32 * P], acc[s0], 0, 0, 0);
          } else {
            acc[s0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, a, acc[s0], 0, 0, 0);
          }
#pragma unroll
          for (int q = 1; q < G::SEG[g]; ++q) {
            gram_slot(S::NB, w, s0 + q, K, J);
            acc[s0 + q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, base[J * 32 * P], acc[s0 + q], 0, 0, 0);
          }
          s0 += G::SEG[g];
        }
      }
    }
#pragma unroll 4
    for (int ks = 0; ks < kChunk / 4; ++ks) {
      float fb[DB];
#pragma unroll
      for (int cb = 0; cb < DB; ++cb) fb[cb] = fs[(cb * 16 + (lane & 15)) * P + ks * 4 + (lane >> 4)];
#pragma unroll
      for (int r = 0; r < S::RPW; ++r) {
        const int R = w + 4 * r;
        const float fa = phi[(R * 16 + (lane & 15)) * P + ks * 4 + (lane >> 4)];
#pragma unroll
        for (int cb = 0; cb < DB; ++cb)
          hacc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, fb[cb], hacc[r][cb], 0, 0, 0);
      }
    }
  }
}

template <int M, int PREC, bool GRAM, int DB>
__device__ __forceinline__ void bta_store(float* __restrict__ part, f32x16 (&acc)[BtaShape<M, PREC>::SLOTS],
                                          f32x4 (&hacc)[BtaShape<M, PREC>::RPW][DB], int lane, int w) {
  using S = BtaShape<M, PREC>;
  if constexpr (GRAM) {
#pragma unroll
    for (int sl = 0; sl < S::SLOTS; ++sl) {
      int K, J;
      if (gram_slot(S::NB, w, sl, K, J)) {
        float* tp = part + (size_t)(w * S::SLOTS + sl) * 1024;
#pragma unroll
        for (int r = 0; r < 16; ++r) gstf(tp + r * 64 + lane, acc[sl][r]);
      }
    }
  }
  float* hp = part + (GRAM ? (size_t)4 * S::SLOTS * 1024 : 0);
#pragma unroll
  for (int r = 0; r < S::RPW; ++r) {
    const int R = w + 4 * r;
#pragma unroll
    for (int cb = 0; cb < DB; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) gstf(hp + ((size_t)R * DB + cb) * 256 + q * 64 + lane, hacc[r][cb][q]);
  }
}

// One workgroup of a split-N pass: part b of nparts handles chunks
// [b*nchunks/nparts, (b+1)*nchunks/nparts) of its cloud and writes its
// partial at `part`. With Xcopy, the points it reads are also written there
// (the plan's resident copy of the cloud), so no separate copy pass is needed.
template <int M, int PREC, bool GRAM, int DB>
__device__ __forceinline__ void bta_body(const float* __restrict__ X, float* __restrict__ Xcopy, int64_t N,
                                         const float4* __restrict__ om,
                                         const float* __restrict__ F, int64_t ldF, int d, int b, int nparts,
                                         float* __restrict__ part) {
  using S = BtaShape<M, PREC>;
  using E = typename S::elem;
  constexpr int P = S::PITCH;
  constexpr int FQ = M / 2;
  __shared__ float4 oms[FQ];
  __shared__ __attribute__((aligned(16))) E phi[M * P];
  __shared__ __attribute__((aligned(16))) E fs[DB * 16 * P];
  __shared__ __attribute__((aligned(16))) E fsl[PREC ? DB * 16 * P : 1];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int k = tid; k < FQ; k += 256) oms[k] = gld4((const float*)(om + k));

  f32x16 acc[S::SLOTS];
  f32x4 hacc[S::RPW][DB];
#pragma unroll
  for (int i = 0; i < S::SLOTS; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
#pragma unroll
  for (int i = 0; i < S::RPW; ++i)
#pragma unroll
    for (int c = 0; c < DB; ++c) hacc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int64_t nchunks = (N + kChunk - 1) / kChunk;
  // even split of the chunks over the parts (depends only on N)
  const int64_t c0 = ((int64_t)b * nchunks) / nparts;
  const int64_t c1 = ((int64_t)(b + 1) * nchunks) / nparts;

  const int pp = tid & 31;   // point pair within the chunk
  const int kq = tid >> 5;   // frequency phase 0..7
  constexpr int DC = DB * 16;
  constexpr int FPT = kChunk * DC / 256;  // field values per thread per chunk
  // registers of one chunk: the coordinates of points pa, pa + 1 and FPT field
  // values; the next chunk's are loaded while the current one is multiplied
  float xa = 0.f, ya = 0.f, za = 0.f, xb = 0.f, yb = 0.f, zb = 0.f;
  float fv[FPT];
  // BF16 staging item q of this thread: channel c, point pair pp2. A wave
  // covers 16 channels x 4 point pairs, so its 32-bit LDS writes at word
  // c * P/2 + pp2 (P/2 = 36) hit 64 distinct banks.
  const auto field_pair = [&](int q, int& c, int& pp2) {
    const int b = (tid >> 6) + 4 * q;  // block: 8 point-pair blocks per 16-channel block
    c = (b >> 3) * 16 + (tid & 15);
    pp2 = (b & 7) * 4 + ((tid >> 4) & 3);
  };
  const auto load_chunk = [&](int64_t base) {
    const int64_t pa = base + 2 * pp, pb = pa + 1;
    if (base + kChunk <= N) {
      xa = gldf(X + pa * 3); ya = gldf(X + pa * 3 + 1); za = gldf(X + pa * 3 + 2);
      xb = gldf(X + pb * 3); yb = gldf(X + pb * 3 + 1); zb = gldf(X + pb * 3 + 2);
    } else {
      xa = ya = za = xb = yb = zb = 0.f;
      if (pa < N) { xa = gldf(X + pa * 3); ya = gldf(X + pa * 3 + 1); za = gldf(X + pa * 3 + 2); }
      if (pb < N) { xb = gldf(X + pb * 3); yb = gldf(X + pb * 3 + 1); zb = gldf(X + pb * 3 + 2); }
    }
    if constexpr (PREC) {
      // lane: channel tid % 16 of a 16-channel block, point pair (tid / 16) % 4
      // of a 4-pair block; the wave and q pick the blocks (see field_pair)
#pragma unroll
      for (int q = 0; q < FPT / 2; ++q) {
        int c, pp2;
        field_pair(q, c, pp2);
        const int64_t g0 = base + 2 * pp2;
        fv[2 * q] = (g0 < N && c < d) ? gldf(F + g0 * ldF + c) : 0.f;
        fv[2 * q + 1] = (g0 + 1 < N && c < d) ? gldf(F + (g0 + 1) * ldF + c) : 0.f;
      }
    } else {
#pragma unroll
      for (int q = 0; q < FPT; ++q) {
        const int idx = tid + 256 * q;
        const int p = idx / DC, c = idx - p * DC;
        const int64_t gp = base + p;
        fv[q] = (gp < N && c < d) ? gldf(F + gp * ldF + c) : 0.f;
      }
    }
  };
  // features of points pa, pa + 1 into LDS (device order rows); points past
  // N (only in a cloud's last chunk) get zero features
  const auto features = [&](int64_t pa, bool va, bool vb, auto masked) {
#pragma unroll 2
    for (int k = kq; k < FQ; k += 8) {
      const float4 w = oms[k];
      float sa, ca, sb, cb;
      phase_sincos(w, xa, ya, za, sa, ca);
      phase_sincos(w, xb, yb, zb, sb, cb);
      if constexpr (decltype(masked)::value) {
        if (!va) { sa = 0.f; ca = 0.f; }
        if (!vb) { sb = 0.f; cb = 0.f; }
      }
      if constexpr (PREC) {
        *(unsigned*)(phi + (2 * k) * P + 2 * pp) = pack_bf16x2(ca, cb);
        *(unsigned*)(phi + (2 * k + 1) * P + 2 * pp) = pack_bf16x2(sa, sb);
      } else {
        phi[(2 * k) * P + 2 * pp] = ca;
        phi[(2 * k) * P + 2 * pp + 1] = cb;
        phi[(2 * k + 1) * P + 2 * pp] = sa;
        phi[(2 * k + 1) * P + 2 * pp + 1] = sb;
      }
    }
  };
  if (c0 < c1) load_chunk(c0 * kChunk);
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int64_t base = ch * kChunk;
    __syncthreads();  // previous chunk's MFMA reads are done (and oms is visible)
    const int64_t pa = base + 2 * pp;
    if (base + kChunk <= N)  // full chunk (uniform branch): no masking
      features(pa, true, true, std::false_type{});
    else
      features(pa, pa < N, pa + 1 < N, std::true_type{});
    // ---- field chunk, transposed to [channel][point] (BF16: hi and lo parts)
    if constexpr (PREC) {
#pragma unroll
      for (int q = 0; q < FPT / 2; ++q) {
        int c, pp2;
        field_pair(q, c, pp2);
        const float v0 = fv[2 * q], v1 = fv[2 * q + 1];
        const unsigned hi = pack_bf16x2(v0, v1);
        const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
        *(unsigned*)(fs + c * P + 2 * pp2) = hi;
        *(unsigned*)(fsl + c * P + 2 * pp2) = pack_bf16x2(v0 - h0, v1 - h1);
      }
    } else {
#pragma unroll
      for (int q = 0; q < FPT; ++q) {
        const int idx = tid + 256 * q;
        const int p = idx / DC, c = idx - p * DC;
        fs[c * P + p] = fv[q];
      }
    }
    // The plan's copy of the chunk's points, written after their features
    // and the field staging: a store right after the prefetch would wait for
    // its loads, and one before the features would be waited for with them.
    if (Xcopy && kq == 0) {
      if (pa < N) { gstf(Xcopy + pa * 3, xa); gstf(Xcopy + pa * 3 + 1, ya); gstf(Xcopy + pa * 3 + 2, za); }
      if (pa + 1 < N) { gstf(Xcopy + pa * 3 + 3, xb); gstf(Xcopy + pa * 3 + 4, yb); gstf(Xcopy + pa * 3 + 5, zb); }
    }
    if (ch + 1 < c1) load_chunk(base + kChunk);  // in flight during the products below
    __syncthreads();
    bta_mma<M, PREC, GRAM, DB>(phi, fs, fsl, acc, hacc, lane, wave);
  }
  bta_store<M, PREC, GRAM, DB>(part, acc, hacc, lane, wave);
}

// grid: nparts workgroups of 256 threads, one per partial.
template <int M, int PREC, bool GRAM, int DB>
__global__ __launch_bounds__(256) void k_bta(const float* __restrict__ X, float* __restrict__ Xcopy, int64_t N,
                                             const float4* __restrict__ om, const float* __restrict__ F,
                                             int64_t ldF, int d, float* __restrict__ partials, size_t part_stride) {
  bta_body<M, PREC, GRAM, DB>(X, Xcopy, N, om, F, ldF, d, (int)blockIdx.x, (int)gridDim.x,
                              partials + (size_t)blockIdx.x * part_stride);
}

// Batched pass: one workgroup per (cloud, part) work item.
template <int M, int PREC, bool GRAM, int DB>
__global__ __launch_bounds__(256) void k_bta_batch(const CloudDesc* __restrict__ cl, const int2* __restrict__ work,
                                                   size_t part_stride) {
  const int2 wi = work[blockIdx.x];
  const CloudDesc& c = cl[wi.x];
  bta_body<M, PREC, GRAM, DB>(c.X, c.Xcopy, c.N, c.om, c.F, c.ldF, c.d, wi.y, c.nparts,
                              c.partials + (size_t)wi.y * part_stride);
}

// ------------------------------------------------------------------ k_gram_nd
// The Gram pass over points in D dimensions, D != 3 (node features as points
// of R^D, for the kernel's spectrum): one workgroup per partial with
// k_bta's chunk split, MFMA schedule and partial layout (its Gram pass
// without a field: one all-zero channel block). A chunk's points and the
// f x D frequencies sit in LDS; a feature's phase is the FP32 sum
// w_0 x_0 + ... + w_{D-1} x_{D-1} accumulated in coordinate order with fused
// multiply-adds (the 3-D pass's own order when D = 3).
constexpr int kGramNdPitch = kMaxDim + 1;  // LDS row pitch of a chunk's points (floats)
template <int M, int PREC>
__global__ __launch_bounds__(256) void k_gram_nd(const float* __restrict__ X, int64_t N, int D,
                                                 const float* __restrict__ omD, float* __restrict__ partials,
                                                 size_t part_stride) {
  using S = BtaShape<M, PREC>;
  using E = typename S::elem;
  constexpr int P = S::PITCH;
  constexpr int FQ = M / 2;
  __shared__ float oms[FQ * kMaxDim];
  __shared__ float xs[kChunk * kGramNdPitch];
  __shared__ __attribute__((aligned(16))) E phi[M * P];
  __shared__ __attribute__((aligned(16))) E fs[16 * P];
  __shared__ __attribute__((aligned(16))) E fsl[PREC ? 16 * P : 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < FQ * D; e += 256) oms[e] = gldf(omD + e);
  for (int e = tid; e < 16 * P; e += 256) fs[e] = (E)0.f;
  if constexpr (PREC)
    for (int e = tid; e < 16 * P; e += 256) fsl[e] = (E)0.f;
  f32x16 acc[S::SLOTS];
  f32x4 hacc[S::RPW][1];
#pragma unroll
  for (int i = 0; i < S::SLOTS; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
#pragma unroll
  for (int i = 0; i < S::RPW; ++i) hacc[i][0] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int b = blockIdx.x, nparts = gridDim.x;
  const int64_t nchunks = (N + kChunk - 1) / kChunk;
  const int64_t c0 = ((int64_t)b * nchunks) / nparts;
  const int64_t c1 = ((int64_t)(b + 1) * nchunks) / nparts;
  const int pp = tid & 31;  // point pair within the chunk
  const int kq = tid >> 5;  // frequency phase 0..7
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int64_t base = ch * kChunk;
    __syncthreads();  // the previous chunk's reads of xs and phi are done
    for (int e = tid; e < kChunk * D; e += 256) {
      const int q = e / D, c = e - q * D;
      xs[q * kGramNdPitch + c] = base + q < N ? gldf(X + (base + q) * D + c) : 0.f;
    }
    __syncthreads();
    const bool va = base + 2 * pp < N, vb = base + 2 * pp + 1 < N;
    const float* xa = xs + (2 * pp) * kGramNdPitch;
    const float* xb = xa + kGramNdPitch;
    for (int k = kq; k < FQ; k += 8) {
      const float* w = oms + k * D;
      float tha = w[0] * xa[0], thb = w[0] * xb[0];
      for (int c = 1; c < D; ++c) {
        tha = fmaf(w[c], xa[c], tha);
        thb = fmaf(w[c], xb[c], thb);
      }
      float sa, ca, sb, cb;
      rev_sincos(tha, sa, ca);
      rev_sincos(thb, sb, cb);
      if (!va) sa = ca = 0.f;  // points past N: zero features
      if (!vb) sb = cb = 0.f;
      if constexpr (PREC) {
        *(unsigned*)(phi + (2 * k) * P + 2 * pp) = pack_bf16x2(ca, cb);
        *(unsigned*)(phi + (2 * k + 1) * P + 2 * pp) = pack_bf16x2(sa, sb);
      } else {
        phi[(2 * k) * P + 2 * pp] = ca;
        phi[(2 * k) * P + 2 * pp + 1] = cb;
        phi[(2 * k + 1) * P + 2 * pp] = sa;
        phi[(2 * k + 1) * P + 2 * pp + 1] = sb;
      }
    }
    __syncthreads();
    bta_mma<M, PREC, true, 1>(phi, fs, fsl, acc, hacc, lane, wave);
  }
  bta_store<M, PREC, true, 1>(partials + (size_t)b * part_stride, acc, hacc, lane, wave);
}

// ------------------------------------------------------------------ k_reduce
// Two-level fixed-order FP64 sum of the partials. Level 1: thread (e, g) adds
// the partials of group g (contiguous, increasing order) for element e.
// Level 2: thread e adds the group sums in order and scatters the result. The
// grouping depends only on the number of partials, i.e. on N.
constexpr int kReduceGroups = 16;

__host__ __device__ inline size_t reduce_elems(int m, int DB, bool gram) {
  return (gram ? (size_t)4 * gram_slots(m / 32) * 1024 : 0) + (size_t)(m / 16) * DB * 256;
}

__device__ __forceinline__ void reduce1_body(const float* __restrict__ partials, size_t stride, int nparts, size_t E,
                                             double* __restrict__ lvl, size_t e, int g) {
  if (e >= E) return;
  const int b0 = (int)(((int64_t)g * nparts) / kReduceGroups);
  const int b1 = (int)(((int64_t)(g + 1) * nparts) / kReduceGroups);
  double s = 0.0;
  int b = b0;
  // 16 loads in flight per step, added in increasing b
  for (; b + 16 <= b1; b += 16) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = gldf(partials + (size_t)(b + u) * stride + e);
#pragma unroll
    for (int u = 0; u < 16; ++u) s += (double)v[u];
  }
  for (; b + 4 <= b1; b += 4) {
    const float v0 = gldf(partials + (size_t)b * stride + e);
    const float v1 = gldf(partials + (size_t)(b + 1) * stride + e);
    const float v2 = gldf(partials + (size_t)(b + 2) * stride + e);
    const float v3 = gldf(partials + (size_t)(b + 3) * stride + e);
    s += (double)v0;
    s += (double)v1;
    s += (double)v2;
    s += (double)v3;
  }
  for (; b < b1; ++b) s += (double)gldf(partials + (size_t)b * stride + e);
  gstd(lvl + (size_t)g * E + e, s);
}

// Gram slot (I, J) of element e of a Gram partial, false for a spare slot.
__device__ __forceinline__ bool reduce_slot(size_t e, size_t ng, int NB, int slots, int& I, int& J) {
  if (e >= ng) return true;
  const int t = (int)(e >> 10);
  return gram_slot(NB, t / slots, t % slots, I, J);
}

// Writes the reduced element e (Gram tile element or B^T F element) into
// Mraw (both triangles, canonical order) or H0, flagging non-finite sums.
__device__ __forceinline__ void reduce_scatter(double s, size_t e, size_t ng, int I, int J, int m, int d, int DB,
                                               double* __restrict__ Mraw, double* __restrict__ H0,
                                               int* __restrict__ flag) {
  if (!isfinite(s)) __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int f = m / 2;
  if (e < ng) {
    const int r = (int)((e >> 6) & 15), l = (int)(e & 63);
    const int row = I * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    const int col = J * 32 + (l & 31);
    const int ci = dev_to_canon(row, f), cj = dev_to_canon(col, f);
    gstd(Mraw + (size_t)ci * m + cj, s);
    gstd(Mraw + (size_t)cj * m + ci, s);
  } else {
    const size_t eh = e - ng;
    const int tile = (int)(eh >> 8), q = (int)((eh >> 6) & 3), l = (int)(eh & 63);
    const int R = tile / DB, cb = tile - R * DB;
    const int row = R * 16 + 4 * (l >> 4) + q;
    const int ch = cb * 16 + (l & 15);
    if (ch < d) gstd(H0 + (size_t)row * d + ch, s);
  }
}

__device__ __forceinline__ void reduce2_body(const double* __restrict__ lvl, size_t E, int m, int d, int DB, int gram,
                                             double* __restrict__ Mraw, double* __restrict__ H0, int* __restrict__ flag,
                                             size_t e) {
  const int NB = m / 32;
  const int slots = gram_slots(NB);
  const size_t ng = gram ? (size_t)4 * slots * 1024 : 0;
  if (e >= E) return;
  int I = 0, J = 0;
  if (!reduce_slot(e, ng, NB, slots, I, J)) return;  // spare slot: never written
  double s = 0.0;
#pragma unroll
  for (int g = 0; g < kReduceGroups; ++g) s += gldd(lvl + (size_t)g * E + e);
  reduce_scatter(s, e, ng, I, J, m, d, DB, Mraw, H0, flag);
}

// Both levels in one thread: the same group sums, added in the same order,
// so the result is bitwise that of reduce1 + reduce2 (for few partials).
constexpr int kFusedReduceMaxParts = 64;
constexpr int kFusedInFlight = 8;  // loads in flight per thread in the one-launch reduction
__device__ __forceinline__ void reduce_fused_body(const float* __restrict__ partials, size_t stride, int nparts,
                                                  size_t E, int m, int d, int DB, int gram, double* __restrict__ Mraw,
                                                  double* __restrict__ H0, int* __restrict__ flag, size_t e) {
  const int NB = m / 32;
  const int slots = gram_slots(NB);
  const size_t ng = gram ? (size_t)4 * slots * 1024 : 0;
  if (e >= E) return;
  int I = 0, J = 0;
  if (!reduce_slot(e, ng, NB, slots, I, J)) return;
  // The partials stream in blocks of kFusedInFlight loads (a load per round
  // trip would leave the thread waiting on each); the sums are the group loop
  // s = sum_g (sum_{b in g} P_b), every group's sum (zero for an empty group)
  // added to s in group order.
  double s = 0.0, sg = 0.0;
  int g = 0;
  int gend = (int)((int64_t)nparts / kReduceGroups);  // end of group 0
  const auto add = [&](int b, float v) {
    while (b >= gend) {  // close the groups that end before partial b
      s += sg;
      sg = 0.0;
      ++g;
      gend = (int)(((int64_t)(g + 1) * nparts) / kReduceGroups);
    }
    sg += (double)v;
  };
  int b0 = 0;
  for (; b0 + kFusedInFlight <= nparts; b0 += kFusedInFlight) {
    float v[kFusedInFlight];
#pragma unroll
    for (int u = 0; u < kFusedInFlight; ++u) v[u] = gldf(partials + (size_t)(b0 + u) * stride + e);
#pragma unroll
    for (int u = 0; u < kFusedInFlight; ++u) add(b0 + u, v[u]);
  }
  for (; b0 < nparts; ++b0) add(b0, gldf(partials + (size_t)b0 * stride + e));
  for (; g < kReduceGroups; ++g) {  // the last group with partials, then any empty ones
    s += sg;
    sg = 0.0;
  }
  reduce_scatter(s, e, ng, I, J, m, d, DB, Mraw, H0, flag);
}

__global__ __launch_bounds__(256) void k_reduce1(const float* __restrict__ partials, size_t stride, int nparts,
                                                 size_t E, double* __restrict__ lvl) {
  reduce1_body(partials, stride, nparts, E, lvl, (size_t)blockIdx.x * 256 + threadIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void k_reduce2(const double* __restrict__ lvl, size_t E, int m, int d, int DB,
                                                 int gram, double* __restrict__ Mraw, double* __restrict__ H0,
                                                 int* __restrict__ flag) {
  reduce2_body(lvl, E, m, d, DB, gram, Mraw, H0, flag, (size_t)blockIdx.x * 256 + threadIdx.x);
}

// Batched reduction: blockIdx.z is the cloud.
__global__ __launch_bounds__(256) void k_reduce1_batch(const CloudDesc* __restrict__ cl, size_t stride, size_t E) {
  const CloudDesc& c = cl[blockIdx.z];
  reduce1_body(c.partials, stride, c.nparts, E, c.lvl, (size_t)blockIdx.x * 256 + threadIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void k_reduce2_batch(const CloudDesc* __restrict__ cl, size_t E, int m, int DB,
                                                       int gram) {
  const CloudDesc& c = cl[blockIdx.z];
  reduce2_body(c.lvl, E, m, c.d, DB, gram, c.Mraw, c.H0, c.flag, (size_t)blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_reduce_fused(const float* __restrict__ partials, size_t stride, int nparts,
                                                      size_t E, int m, int d, int DB, int gram,
                                                      double* __restrict__ Mraw, double* __restrict__ H0,
                                                      int* __restrict__ flag) {
  reduce_fused_body(partials, stride, nparts, E, m, d, DB, gram, Mraw, H0, flag,
                    (size_t)blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_reduce_fused_batch(const CloudDesc* __restrict__ cl, size_t stride, size_t E,
                                                            int m, int DB, int gram) {
  const CloudDesc& c = cl[blockIdx.y];
  reduce_fused_body(c.partials, stride, c.nparts, E, m, c.d, DB, gram, c.Mraw, c.H0, c.flag,
                    (size_t)blockIdx.x * 256 + threadIdx.x);
}

// ------------------------------------------------------------------ k_gcore
// G'[j][c] = sum_i T[j][i] H0[i][c] (device order), FP64, one workgroup per
// kGcoreRows rows x 16 channels with both operands staged in LDS; each sum is
// split over four threads (terms i = 4s + q in part q, the parts added as
// (p0 + p1) + (p2 + p3)), so its dependent chain is m/4 long. Stored as FP32
// [j][c] and as a BF16 hi + lo pair, transposed [c][j] (lo at offset 64 m).
constexpr int kGcoreRows = 4;
__device__ __forceinline__ void gcore_body(const double* __restrict__ T, const double* __restrict__ H0, int m, int d,
                                           float* __restrict__ G32, __bf16* __restrict__ Gt16, int j0, int c0) {
  __shared__ double ts[kGcoreRows * kMaxM];
  __shared__ double hs[kMaxM * 16];
  const int t = threadIdx.x;
  // every load of the two operand tiles in flight at once (m <= 256: at most
  // 4 + 16 per thread), then staged into LDS
  constexpr int QT = kGcoreRows * kMaxM / 256;
  constexpr int QH = 16 * kMaxM / 256;
  double tv[QT], hv[QH];
#pragma unroll
  for (int q = 0; q < QT; ++q) {
    const int e = t + 256 * q;  // the rows j0 .. j0 + kGcoreRows - 1 are contiguous in T
    tv[q] = e < kGcoreRows * m ? gldd(T + (size_t)j0 * m + e) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const int e = t + 256 * q;
    const int ih = e >> 4, c = e & 15;
    hv[q] = (e < 16 * m && c0 + c < d) ? gldd(H0 + (size_t)ih * d + c0 + c) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < QT; ++q) {
    const int e = t + 256 * q;
    if (e < kGcoreRows * m) ts[(e / m) * kMaxM + e % m] = tv[q];
  }
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const int e = t + 256 * q;
    if (e < 16 * m) hs[e] = hv[q];
  }
  __syncthreads();
  const int part = t & 3, c = (t >> 2) & 15, r = t >> 6;
  double s = 0.0;
  for (int i = part; i < m; i += 4) s += ts[r * kMaxM + i] * hs[i * 16 + c];
  s += __shfl_xor(s, 1);  // p0 + p1 (and p2 + p3)
  s += __shfl_xor(s, 2);  // (p0 + p1) + (p2 + p3): addition commutes, so every part holds the same sum
  const int j = j0 + r, ch = c0 + c;
  if (part != 0 || ch >= d) return;
  const float g = (float)s;
  const __bf16 hi = (__bf16)g;
  gstf(G32 + (size_t)j * d + ch, g);
  gsth(Gt16 + (size_t)ch * m + j, hi);                                                         // hi part, d x m
  gsth(Gt16 + (size_t)kMaxDBlocks * kDBlock * m + (size_t)ch * m + j, (__bf16)(g - (float)hi));  // lo part
}

__global__ __launch_bounds__(256) void k_gcore(const double* __restrict__ T, const double* __restrict__ H0, int m,
                                               int d, float* __restrict__ G32, __bf16* __restrict__ Gt16) {
  gcore_body(T, H0, m, d, G32, Gt16, blockIdx.x * kGcoreRows, blockIdx.y * 16);
}

__global__ __launch_bounds__(256) void k_gcore_batch(const CloudDesc* __restrict__ cl, int m) {
  const CloudDesc& c = cl[blockIdx.z];
  if ((int)blockIdx.y * 16 >= c.d) return;
  gcore_body(c.T64, c.H0, m, c.d, c.G32, c.Gt16, blockIdx.x * kGcoreRows, blockIdx.y * 16);
}

// ------------------------------------------------------------------ k_expand
// Output layout of the products, chosen by the number of channel blocks.
// One block (d <= 16): the products are formed as (Phi G')^T = G'^T Phi^T
// (G'^T the MFMA A operand), so lane (g, pl) holds channels 4g .. 4g+3 of
// point tile*16 + pl, and the residual loads and output stores are one
// 16-byte access per lane covering whole 64-byte rows (VEC, when rows and
// bases allow it). Wider fields: the direct form, lane (g, pl) holding
// channel cb*16 + pl of points tile*16 + 4g + q (q = 0..3), four rows per
// access; a 16-byte piece per lane there would spread every access over 16
// rows 64 * DB bytes apart, which measured slower for DB >= 2.
template <int DB>
constexpr bool kRowPieces = DB == 1;

template <int DB>
__device__ __forceinline__ void load_residual(const float* F, int64_t ldF, int d, int64_t N, int64_t tile, int g,
                                              int pl, bool vec, float (&fres)[DB][4]) {
  if constexpr (kRowPieces<DB>) {
    const int64_t pr = tile * 16 + pl;
    const int c = 4 * g;
    if (vec) {
      float4 v = {0.f, 0.f, 0.f, 0.f};
      if (c < d && pr < N) v = gld4(F + pr * ldF + c);
      fres[0][0] = v.x; fres[0][1] = v.y; fres[0][2] = v.z; fres[0][3] = v.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) fres[0][q] = (c + q < d && pr < N) ? gldf(F + pr * ldF + c + q) : 0.f;
    }
  } else {
#pragma unroll
    for (int cb = 0; cb < DB; ++cb) {
      const int c = cb * 16 + pl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t pr = tile * 16 + 4 * g + q;
        fres[cb][q] = (c < d && pr < N) ? gldf(F + pr * ldF + c) : 0.f;
      }
    }
  }
}

// Residual of a diagonal field diag(w) (square, sliced): the slice's channel
// c is column col0 + c, so point p has w[c] (w already offset by col0) where
// p == col0 + c and zero elsewhere; same lane layout as load_residual.
template <int DB>
__device__ __forceinline__ void diag_residual(const float* w, int64_t col0, int d, int64_t N, int64_t tile, int g,
                                              int pl, float (&fres)[DB][4]) {
  if constexpr (kRowPieces<DB>) {
    const int64_t pr = tile * 16 + pl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * g + q;
      fres[0][q] = (c < d && pr < N && pr == col0 + c) ? gldf(w + c) : 0.f;
    }
  } else {
#pragma unroll
    for (int cb = 0; cb < DB; ++cb) {
      const int c = cb * 16 + pl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t pr = tile * 16 + 4 * g + q;
        fres[cb][q] = (c < d && pr < N && pr == col0 + c) ? gldf(w + c) : 0.f;
      }
    }
  }
}

// TOUT: the result is stored transposed, out[c * ldO + p] (channel-major),
// for fields whose transpose is the next operand; the direct layout then
// writes four consecutive points of one channel per lane.
// EPI (with TOUT): the stored value is fma(-2, result, ea[c] + eb[p]).
template <int DB, bool TOUT, bool EPI = false>
__device__ __forceinline__ void store_out(float* out, int64_t ldO, const float* __restrict__ rowscale, int d,
                                          int64_t N, int64_t tile, int g, int pl, bool vec,
                                          const float (&fres)[DB][4], const f32x4 (&acc)[DB],
                                          const float* __restrict__ ea = nullptr,
                                          const float* __restrict__ eb = nullptr) {
  if constexpr (TOUT) {
    if constexpr (kRowPieces<DB>) {
      const int64_t pr = tile * 16 + pl;
      if (pr >= N) return;
      const float sc = rowscale ? gldf(rowscale + pr) : 1.f;
      const float ebp = EPI ? gldf(eb + pr) : 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 4 * g + q;
        if (c >= d) continue;
        float v = fres[0][q] + acc[0][q];
        if (rowscale) v = sc * v;
        if constexpr (EPI) v = __builtin_fmaf(-2.f, v, gldf(ea + c) + ebp);
        gstf(out + (int64_t)c * ldO + pr, v);
      }
    } else {
      const int64_t p0 = tile * 16 + 4 * g;
      const bool vt = ((ldO & 3) == 0) && (((uintptr_t)out & 15) == 0) && p0 + 3 < N;
      float ebq[4] = {0.f, 0.f, 0.f, 0.f};  // the epilogue's point terms, loaded once per tile
      if constexpr (EPI) {
        if (p0 + 3 < N && ((uintptr_t)(eb + p0) & 15) == 0) {
          const float4 e4 = gld4(eb + p0);
          ebq[0] = e4.x; ebq[1] = e4.y; ebq[2] = e4.z; ebq[3] = e4.w;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) ebq[q] = p0 + q < N ? gldf(eb + p0 + q) : 0.f;
        }
      }
#pragma unroll
      for (int cb = 0; cb < DB; ++cb) {
        const int c = cb * 16 + pl;
        if (c >= d) continue;
        const float eac = EPI ? gldf(ea + c) : 0.f;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = fres[cb][q] + acc[cb][q];
          if (rowscale && p0 + q < N) v[q] *= gldf(rowscale + p0 + q);
          if constexpr (EPI) v[q] = __builtin_fmaf(-2.f, v[q], eac + ebq[q]);
        }
        if (vt) {
          gst4(out + (int64_t)c * ldO + p0, float4{v[0], v[1], v[2], v[3]});
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (p0 + q < N) gstf(out + (int64_t)c * ldO + p0 + q, v[q]);
        }
      }
    }
    return;
  }
  if constexpr (kRowPieces<DB>) {
    const int64_t pr = tile * 16 + pl;
    if (pr >= N) return;
    const int c = 4 * g;
    const float sc = rowscale ? gldf(rowscale + pr) : 1.f;
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = fres[0][q] + acc[0][q];
      if (rowscale) v[q] = sc * v[q];
    }
    if (vec) {
      if (c < d) gst4(out + pr * ldO + c, float4{v[0], v[1], v[2], v[3]});
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (c + q < d) gstf(out + pr * ldO + c + q, v[q]);
    }
  } else {
#pragma unroll
    for (int cb = 0; cb < DB; ++cb) {
      const int c = cb * 16 + pl;
      if (c < d) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t pr = tile * 16 + 4 * g + q;
          if (pr < N) {
            const float v = fres[cb][q] + acc[cb][q];
            gstf(out + pr * ldO + c, rowscale ? gldf(rowscale + pr) * v : v);
          }
        }
      }
    }
  }
}

// out = F + Phi G'. Each wave owns tiles of 16 points; lane l handles point
// l%16 and the feature group g = l/16 of every K step (the outputs it then
// holds follow the layout above). Point tiles are distributed round-robin
// over the waves of the grid.
// Point tiles [t_first + wave, t_end) with stride t_step are processed by the
// four waves of the workgroup.
// DIAG: the field is diag(w) of a square sliced field (see diag_residual):
// F is the slice's part of w and ldF its first column; nothing of the n x n
// field is read.
template <int M, int PREC, int DB, bool TOUT = false, bool DIAG = false, bool EPI = false>
__device__ __forceinline__ void expand_body(const float* __restrict__ X, int64_t N, const float4* __restrict__ om,
                                            const float* __restrict__ G32, const __bf16* __restrict__ Gt16, int d,
                                            const float* F, int64_t ldF, float* out, int64_t ldO,
                                            const float* __restrict__ rowscale, int64_t t_first, int64_t t_end,
                                            int64_t t_step, const float* __restrict__ ea = nullptr,
                                            const float* __restrict__ eb = nullptr) {
  constexpr int FQ = M / 2;
  constexpr int GP = M + 8;  // BF16 row pitch of G'^T in LDS: conflict-free 16-byte reads
  __shared__ float4 oms[FQ];
  __shared__ float gs[PREC ? 1 : M * DB * 16];
  __shared__ __attribute__((aligned(16))) __bf16 gth[PREC ? DB * 16 * GP : 8];
  __shared__ __attribute__((aligned(16))) __bf16 gtl[PREC ? DB * 16 * GP : 8];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int k = tid; k < FQ; k += 256) oms[k] = gld4((const float*)(om + k));
  if constexpr (PREC) {
    // 16-byte pieces of the G'^T rows (hi and lo); rows past d are zero
    const uint4* gh = (const uint4*)Gt16;
    const uint4* gl = (const uint4*)(Gt16 + (size_t)kMaxDBlocks * kDBlock * M);
    for (int idx = tid; idx < DB * 16 * (M / 8); idx += 256) {
      const int c = idx / (M / 8), j8 = idx - c * (M / 8);
      const bool ok = c < d;
      const uint4 z = {0u, 0u, 0u, 0u};
      *(uint4*)(gth + c * GP + 8 * j8) = ok ? gldu4(gh + (size_t)c * (M / 8) + j8) : z;
      *(uint4*)(gtl + c * GP + 8 * j8) = ok ? gldu4(gl + (size_t)c * (M / 8) + j8) : z;
    }
  }
  if constexpr (!PREC) {
    if (d == DB * 16) {  // G' rows fill the channel blocks: a straight copy
      for (int idx = tid; idx < M * DB * 4; idx += 256) ((float4*)gs)[idx] = gld4(G32 + 4 * (size_t)idx);
    } else {
      for (int idx = tid; idx < M * DB * 16; idx += 256) {
        const int j = idx / (DB * 16), c = idx - j * (DB * 16);
        gs[idx] = c < d ? gldf(G32 + (size_t)j * d + c) : 0.f;
      }
    }
  }
  __syncthreads();
  const int g = lane >> 4, pl = lane & 15;
  // 16-byte residual loads and output stores (one-block layout): every row
  // starts 16-byte aligned
  const bool vec = ((d | ldF | ldO) & 3) == 0 && (((uintptr_t)F | (uintptr_t)out) & 15) == 0;
  const int64_t ntiles = t_end;
  const int64_t wstride = t_step;

  // a wave's next tile (its point and residual F values) is loaded while the
  // current one is computed
  float xn = 0.f, yn = 0.f, zn = 0.f;
  float fn[DB][4];
  const auto load_tile = [&](int64_t tile) {
    const int64_t p = tile * 16 + pl;
    xn = yn = zn = 0.f;
    if (p < N) { xn = gldf(X + p * 3); yn = gldf(X + p * 3 + 1); zn = gldf(X + p * 3 + 2); }
    if constexpr (DIAG)
      diag_residual(F, ldF, d, N, tile, g, pl, fn);
    else
      load_residual(F, ldF, d, N, tile, g, pl, vec, fn);
  };
  if (t_first + (tid >> 6) < ntiles) load_tile(t_first + (tid >> 6));

  // the products of one tile: acc = (Phi G')^T (one channel block) or Phi G'
  const auto products = [&](float x, float y, float z, f32x4 (&acc)[DB]) {
    if constexpr (PREC) {
#pragma unroll
      for (int cb = 0; cb < DB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
      for (int s = 0; s < M / 32; ++s) {
        u32x4_t aw;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float sn, cs;
          phase_sincos(oms[16 * s + 4 * g + i], x, y, z, sn, cs);
          aw[i] = pack_bf16x2(cs, sn);
        }
        const bf16x8 a = __builtin_bit_cast(bf16x8, aw);
#pragma unroll
        for (int cb = 0; cb < DB; ++cb) {
          const int off = (cb * 16 + pl) * GP + s * 32 + 8 * g;
          const bf16x8 bh = *(const bf16x8*)(gth + off);
          const bf16x8 bl = *(const bf16x8*)(gtl + off);
          if constexpr (kRowPieces<DB>) {
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, a, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, a, acc[cb], 0, 0, 0);
          } else {
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[cb], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int cb = 0; cb < DB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
      // K steps in pairs: lane group g uses frequency k = 4t + g, cos then sin.
#pragma unroll 4
      for (int t = 0; t < FQ / 4; ++t) {
        const int k = 4 * t + g;
        float sn, cs;
        phase_sincos(oms[k], x, y, z, sn, cs);
#pragma unroll
        for (int cb = 0; cb < DB; ++cb) {
          const float b0 = gs[(2 * k) * (DB * 16) + cb * 16 + pl];
          const float b1 = gs[(2 * k + 1) * (DB * 16) + cb * 16 + pl];
          if constexpr (kRowPieces<DB>) {
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, cs, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, sn, acc[cb], 0, 0, 0);
          } else {
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(cs, b0, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(sn, b1, acc[cb], 0, 0, 0);
          }
        }
      }
    }
  };
  int64_t tile = t_first + (tid >> 6);
  if constexpr (!TOUT && !DIAG && !EPI) {
    // Interior tiles of a field of full 16-channel blocks without row
    // scaling: all 16 points below N and, like the tile each prefetches,
    // inside this call's range [t_first, t_end). Every load and store there
    // is unconditional, so no wait for the prefetch also waits for the
    // previous tile's stores.
    const int64_t nfull = N / 16 < ntiles ? N / 16 : ntiles;
    const bool full = kRowPieces<DB> ? (vec && d == 16) : d == DB * 16;
    if (full && rowscale == nullptr && tile + wstride < nfull) {
      // the first tile's loads arrive here, so no wait inside the loop
      // covers them (such a wait would also cover the previous tile's store)
      asm volatile("" ::"v"(xn), "v"(yn), "v"(zn));
#pragma unroll
      for (int cb = 0; cb < DB; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) asm volatile("" ::"v"(fn[cb][q]));
      for (; tile + wstride < nfull; tile += wstride) {
        const float x = xn, y = yn, z = zn;
        float fres[DB][4];
#pragma unroll
        for (int cb = 0; cb < DB; ++cb)
#pragma unroll
          for (int q = 0; q < 4; ++q) fres[cb][q] = fn[cb][q];
        const int64_t nt = tile + wstride;
        const int64_t p = nt * 16 + pl;
        xn = gldf(X + p * 3); yn = gldf(X + p * 3 + 1); zn = gldf(X + p * 3 + 2);
        if constexpr (kRowPieces<DB>) {
          const float4 v = gld4(F + p * ldF + 4 * g);
          fn[0][0] = v.x; fn[0][1] = v.y; fn[0][2] = v.z; fn[0][3] = v.w;
        } else {
#pragma unroll
          for (int cb = 0; cb < DB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) fn[cb][q] = gldf(F + (nt * 16 + 4 * g + q) * ldF + cb * 16 + pl);
        }
        f32x4 acc[DB];
        products(x, y, z, acc);
        if constexpr (kRowPieces<DB>) {
          gst4(out + (tile * 16 + pl) * ldO + 4 * g, float4{fres[0][0] + acc[0][0], fres[0][1] + acc[0][1],
                                                            fres[0][2] + acc[0][2], fres[0][3] + acc[0][3]});
        } else {
#pragma unroll
          for (int cb = 0; cb < DB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              gstf(out + (tile * 16 + 4 * g + q) * ldO + cb * 16 + pl, fres[cb][q] + acc[cb][q]);
        }
      }
    }
  }
  for (; tile < ntiles; tile += wstride) {
    const float x = xn, y = yn, z = zn;
    float fres[DB][4];
#pragma unroll
    for (int cb = 0; cb < DB; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) fres[cb][q] = fn[cb][q];
    if (tile + wstride < ntiles) load_tile(tile + wstride);
    f32x4 acc[DB];
    products(x, y, z, acc);
    store_out<DB, TOUT, EPI>(out, ldO, rowscale, d, N, tile, g, pl, vec, fres, acc, ea, eb);
  }
}

// The expansion without the matrix cores, for fields of DV <= 4 channels
// (the A (G) step with m d small): one thread per point evaluates its
// features in turn (rounded to BF16 in BF16 mode, as the matrix-core path
// feeds them) and accumulates the d channels of Phi_i G' with FP32 FMAs, G'
// in FP32 from LDS (every lane reads the same word: a broadcast).
template <int M, int PREC, int DV>
__device__ __forceinline__ void expand_valu_body(const float* __restrict__ X, int64_t N,
                                                 const float4* __restrict__ om, const float* __restrict__ G32, int d,
                                                 const float* __restrict__ F, int64_t ldF, float* __restrict__ out,
                                                 int64_t ldO, const float* __restrict__ rowscale, int64_t p_first,
                                                 int64_t p_end, int64_t p_step) {
  constexpr int FQ = M / 2;
  __shared__ float4 oms[FQ];
  __shared__ float gs[M * DV];
  const int tid = threadIdx.x;
  for (int k = tid; k < FQ; k += 256) oms[k] = gld4((const float*)(om + k));
  for (int idx = tid; idx < M * DV; idx += 256) {
    const int j = idx / DV, c = idx - j * DV;
    gs[idx] = c < d ? gldf(G32 + (size_t)j * d + c) : 0.f;
  }
  __syncthreads();
  for (int64_t p = p_first + tid; p < p_end; p += p_step) {
    const float x = gldf(X + p * 3), y = gldf(X + p * 3 + 1), z = gldf(X + p * 3 + 2);
    float acc[DV];
#pragma unroll
    for (int c = 0; c < DV; ++c) acc[c] = 0.f;
#pragma unroll 4
    for (int k = 0; k < FQ; ++k) {
      float sn, cs;
      phase_sincos(oms[k], x, y, z, sn, cs);
      if constexpr (PREC) {
        cs = (float)(__bf16)cs;
        sn = (float)(__bf16)sn;
      }
#pragma unroll
      for (int c = 0; c < DV; ++c) {
        acc[c] = fmaf(cs, gs[(2 * k) * DV + c], acc[c]);
        acc[c] = fmaf(sn, gs[(2 * k + 1) * DV + c], acc[c]);
      }
    }
    const float sc = rowscale ? gldf(rowscale + p) : 1.f;
#pragma unroll
    for (int c = 0; c < DV; ++c) {
      if (c < d) {
        const float v = gldf(F + p * ldF + c) + acc[c];
        gstf(out + p * ldO + c, rowscale ? sc * v : v);
      }
    }
  }
}

template <int M, int PREC, int DV>
__global__ __launch_bounds__(256) void k_expand_valu(const float* __restrict__ X, int64_t N,
                                                     const float4* __restrict__ om, const float* __restrict__ G32,
                                                     int d, const float* F, int64_t ldF, float* out, int64_t ldO,
                                                     const float* __restrict__ rowscale) {
  expand_valu_body<M, PREC, DV>(X, N, om, G32, d, F, ldF, out, ldO, rowscale, (int64_t)blockIdx.x * 256, N,
                                (int64_t)gridDim.x * 256);
}

// Batched: work item (cloud, first tile) covers the points of tpi tiles of 16.
// Every cloud takes the kValuMaxD-channel body with its own d; channels past
// d carry zero G' rows, and each kept channel sees the same FMAs in the same
// order as in the single-cloud kernel of its exact width, so the bits agree.
template <int M, int PREC>
__global__ __launch_bounds__(256) void k_expand_valu_batch(const CloudDesc* __restrict__ cl,
                                                           const int2* __restrict__ work, int tpi) {
  const int2 wi = work[blockIdx.x];
  const CloudDesc& c = cl[wi.x];
  const int64_t p0 = (int64_t)wi.y * 16;
  int64_t p1 = p0 + (int64_t)tpi * 16;
  if (p1 > c.N) p1 = c.N;
  expand_valu_body<M, PREC, kValuMaxD>(c.X, c.N, c.om, c.G32, c.d, c.F, c.ldF, c.out, c.ldO, nullptr, p0, p1, 256);
}

template <int M, int PREC, int DB>
__global__ __launch_bounds__(256) void k_expand(const float* __restrict__ X, int64_t N,
                                                const float4* __restrict__ om, const float* __restrict__ G32,
                                                const __bf16* __restrict__ Gt16, int d, const float* F,
                                                int64_t ldF, float* out, int64_t ldO,
                                                const float* __restrict__ rowscale) {
  expand_body<M, PREC, DB>(X, N, om, G32, Gt16, d, F, ldF, out, ldO, rowscale, (int64_t)blockIdx.x * 4,
                           (N + 15) / 16, (int64_t)gridDim.x * 4);
}

// Batched expansion: one workgroup per (cloud, first tile) work item, each
// covering `tpi` tiles of 16 points (a launch-geometry choice: any tpi gives
// the same result).
template <int M, int PREC, int DB, bool TOUT, bool DIAG, bool EPI>
__global__ __launch_bounds__(256) void k_expand_batch(const CloudDesc* __restrict__ cl, const int2* __restrict__ work,
                                                      int tpi) {
  const int2 wi = work[blockIdx.x];
  const CloudDesc& c = cl[wi.x];
  const int64_t ntiles = (c.N + 15) / 16;
  int64_t t_end = (int64_t)wi.y + tpi;
  if (t_end > ntiles) t_end = ntiles;
  expand_body<M, PREC, DB, TOUT, DIAG, EPI>(c.X, c.N, c.om, c.G32, c.Gt16, c.d, c.F, c.ldF, c.out, c.ldO, nullptr,
                                            wi.y, t_end, 4, c.epi_a, c.epi_b);
}

// ------------------------------------------------------------------ launchers
template <int M, int PREC, bool GRAM>
static hipError_t bta_dispatch_db(int DB, dim3 grid, const float* X, float* Xcopy, int64_t N, const float4* om,
                                  const float* F, int64_t ldF, int d, float* parts, size_t stride, hipStream_t st) {
  switch (DB) {
    case 1:
      hipLaunchKernelGGL((k_bta<M, PREC, GRAM, 1>), grid, dim3(256), 0, st, X, Xcopy, N, om, F, ldF, d, parts, stride);
      return hipGetLastError();
    case 2:
      hipLaunchKernelGGL((k_bta<M, PREC, GRAM, 2>), grid, dim3(256), 0, st, X, Xcopy, N, om, F, ldF, d, parts, stride);
      return hipGetLastError();
    case 4:
      if constexpr (!(GRAM && M == 256)) {
        hipLaunchKernelGGL((k_bta<M, PREC, GRAM, 4>), grid, dim3(256), 0, st, X, Xcopy, N, om, F, ldF, d, parts, stride);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_bta(rfd_plan_s* p, const float* X, int64_t N, const float* F, int64_t ldF, int d, bool gram,
                      hipStream_t st, float* xcopy) {
  const int M = p->dev_m, prec = p->params.precision;
  const int DB = dblocks(d);
  const int nparts = bta_partials(N, M, d, gram, prec);
  const size_t stride = bta_partial_floats(M, d, gram);
  dim3 grid(nparts);
  const float4* om = p->dev.om;
  float* parts = p->dev.partials;
  ProfileScope prof(gram ? kKGram : kKBta, st);
#define RFD_BTA(MM, PP)                                                                                     \
  if (M == MM && prec == PP) {                                                                              \
    return gram ? bta_dispatch_db<MM, PP, true>(DB, grid, X, xcopy, N, om, F, ldF, d, parts, stride, st)    \
                : bta_dispatch_db<MM, PP, false>(DB, grid, X, xcopy, N, om, F, ldF, d, parts, stride, st);  \
  }
  RFD_BTA(64, 0)
  RFD_BTA(64, 1)
  RFD_BTA(128, 0)
  RFD_BTA(128, 1)
  RFD_BTA(256, 0)
  RFD_BTA(256, 1)
#undef RFD_BTA
  return hipErrorInvalidValue;
}

hipError_t launch_gram_nd(rfd_plan_s* p, const float* X, int64_t N, hipStream_t st) {
  const int M = p->dev_m, prec = p->params.precision, D = plan_dim(p->params);
  if (D < 1 || D > kMaxDim || !p->dev.omD) return hipErrorInvalidValue;
  const int nparts = bta_partials(N, M, 0, true, prec);
  const size_t stride = bta_partial_floats(M, 0, true);
  ProfileScope prof(kKGram, st);
#define RFD_GND(MM, PP)                                                                                    \
  if (M == MM && prec == PP) {                                                                             \
    hipLaunchKernelGGL((k_gram_nd<MM, PP>), dim3(nparts), dim3(256), 0, st, X, N, D, p->dev.omD,          \
                       p->dev.partials, stride);                                                           \
    return hipGetLastError();                                                                              \
  }
  RFD_GND(64, 0)
  RFD_GND(64, 1)
  RFD_GND(128, 0)
  RFD_GND(128, 1)
  RFD_GND(256, 0)
  RFD_GND(256, 1)
#undef RFD_GND
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(rfd_plan_s* p, int64_t N, int d, bool gram, hipStream_t st) {
  const int M = p->dev_m, prec = p->params.precision;
  const int DB = dblocks(d);
  const int nparts = bta_partials(N, M, d, gram, prec);
  const size_t stride = bta_partial_floats(M, d, gram);
  const size_t E = reduce_elems(M, DB, gram);
  ProfileScope prof(kKReduce, st);
  if (nparts <= kFusedReduceMaxParts) {
    hipLaunchKernelGGL(k_reduce_fused, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, p->dev.partials, stride,
                       nparts, E, M, d, DB, gram ? 1 : 0, p->dev.Mraw, p->dev.H0, p->dev.flag);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_reduce1, dim3((unsigned)((E + 255) / 256), kReduceGroups), dim3(256), 0, st, p->dev.partials,
                     stride, nparts, E, p->dev.lvl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce2, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, p->dev.lvl, E, M, d, DB,
                     gram ? 1 : 0, p->dev.Mraw, p->dev.H0, p->dev.flag);
  return hipGetLastError();
}

size_t reduce_scratch_doubles(int m) { return (size_t)kReduceGroups * reduce_elems(m, kMaxDBlocks, true); }

hipError_t launch_gcore(rfd_plan_s* p, int d, hipStream_t st) {
  const int M = p->dev_m;
  dim3 grid((unsigned)(M / kGcoreRows), (unsigned)((d + 15) / 16));
  ProfileScope prof(kKGcore, st);
  hipLaunchKernelGGL(k_gcore, grid, dim3(256), 0, st, p->dev.T64, p->dev.H0, M, d, p->dev.G32, p->dev.Gt16);
  return hipGetLastError();
}

template <int M, int PREC>
static hipError_t expand_dispatch(int DB, dim3 grid, const float* X, int64_t N, const float4* om, const float* G32,
                                  const __bf16* Gt16, int d, const float* F, int64_t ldF, float* out, int64_t ldO,
                                  const float* rowscale, hipStream_t st) {
  switch (DB) {
    case 1:
      hipLaunchKernelGGL((k_expand<M, PREC, 1>), grid, dim3(256), 0, st, X, N, om, G32, Gt16, d, F, ldF, out, ldO, rowscale);
      break;
    case 2:
      hipLaunchKernelGGL((k_expand<M, PREC, 2>), grid, dim3(256), 0, st, X, N, om, G32, Gt16, d, F, ldF, out, ldO, rowscale);
      break;
    case 4:
      hipLaunchKernelGGL((k_expand<M, PREC, 4>), grid, dim3(256), 0, st, X, N, om, G32, Gt16, d, F, ldF, out, ldO, rowscale);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int M, int PREC>
static hipError_t expand_valu_dispatch(int64_t N, const float* X, const float4* om, const float* G32, int d,
                                       const float* F, int64_t ldF, float* out, int64_t ldO, const float* rowscale,
                                       hipStream_t st) {
  int64_t nwg = (N + 255) / 256;
  if (nwg > 4096) nwg = 4096;
  if (nwg < 1) nwg = 1;
  const dim3 grid((unsigned)nwg);
  switch (d) {
    case 1:
      hipLaunchKernelGGL((k_expand_valu<M, PREC, 1>), grid, dim3(256), 0, st, X, N, om, G32, d, F, ldF, out, ldO,
                         rowscale);
      break;
    case 2:
      hipLaunchKernelGGL((k_expand_valu<M, PREC, 2>), grid, dim3(256), 0, st, X, N, om, G32, d, F, ldF, out, ldO,
                         rowscale);
      break;
    case 3:
      hipLaunchKernelGGL((k_expand_valu<M, PREC, 3>), grid, dim3(256), 0, st, X, N, om, G32, d, F, ldF, out, ldO,
                         rowscale);
      break;
    case 4:
      hipLaunchKernelGGL((k_expand_valu<M, PREC, 4>), grid, dim3(256), 0, st, X, N, om, G32, d, F, ldF, out, ldO,
                         rowscale);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Default from measurements on MI355X (resident integrate, 1M and 100k
// points, m = 64 and 128): in FP32 the FMA path takes 0.43-0.58 of the
// FP32-matrix-core expansion's time for d <= 3; in BF16 it is 4-8% faster at
// d = 1 and up to 19% slower at d = 3.
int expand_path(int M, int prec, int d) {
  if (d < 1 || d > kValuMaxD) return kExpandMfma;
  const int rule = (prec == 0 || d == 1) ? kExpandValu : kExpandMfma;
  (void)M;
  return tuned(kTuneExpandPath, M, prec, 1, (int64_t)1 << d, rule);
}

hipError_t launch_expand(rfd_plan_s* p, const float* X, int64_t N, const float* F, int64_t ldF, int d, float* out,
                         int64_t ldO, const float* rowscale, hipStream_t st) {
  const int M = p->dev_m, prec = p->params.precision;
  if (expand_path(M, prec, d) == kExpandValu) {
    const float4* om = p->dev.om;
    ProfileScope prof(kKExpand, st);
#define RFD_EXPV(MM, PP) \
  if (M == MM && prec == PP) return expand_valu_dispatch<MM, PP>(N, X, om, p->dev.G32, d, F, ldF, out, ldO, rowscale, st);
    RFD_EXPV(64, 0)
    RFD_EXPV(64, 1)
    RFD_EXPV(128, 0)
    RFD_EXPV(128, 1)
    RFD_EXPV(256, 0)
    RFD_EXPV(256, 1)
#undef RFD_EXPV
    return hipErrorInvalidValue;
  }
  const int DB = dblocks(d);
  const int64_t ntiles = (N + 15) / 16;
  // tiles of 16 points per wave: launch geometry only (results do not depend on it)
  const int tpw = tuned(kTuneExpandTilesPerWave, M, prec, DB, N, default_expand_tiles_per_wave(N, prec));
  int64_t nwg = (ntiles + 4 * tpw - 1) / (4 * tpw);
  if (nwg > 2048) nwg = 2048;
  if (nwg < 1) nwg = 1;
  dim3 grid((unsigned)nwg);
  const float4* om = p->dev.om;
  ProfileScope prof(kKExpand, st);
#define RFD_EXP(MM, PP) \
  if (M == MM && prec == PP) return expand_dispatch<MM, PP>(DB, grid, X, N, om, p->dev.G32, p->dev.Gt16, d, F, ldF, out, ldO, rowscale, st);
  RFD_EXP(64, 0)
  RFD_EXP(64, 1)
  RFD_EXP(128, 0)
  RFD_EXP(128, 1)
  RFD_EXP(256, 0)
  RFD_EXP(256, 1)
#undef RFD_EXP
  return hipErrorInvalidValue;
}

// Diagonal of a square wide-field integration (d = N, slices of 64 channels):
// v[i] = F[i][i] + sum_j phi_j(x_i) G'_s[j][c] with s = i / 64, c = i % 64 and
// G'_s = T H0 of slice s, the features in FP32 as the expansion forms them
// and the sum in FP64. Only the diagonal is formed: no other element of the
// result is read or written. One thread per point.
template <int M>
__global__ __launch_bounds__(256) void k_wide_diag(const CloudDesc* __restrict__ cl, int64_t N,
                                                   float* __restrict__ v) {
  __shared__ float4 oms[M / 2];
  for (int k = threadIdx.x; k < M / 2; k += 256) oms[k] = gld4((const float*)(cl[0].om + k));
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const CloudDesc& c = cl[i / 64];
  const int ch = (int)(i % 64);
  const float x = gldf(c.X + 3 * i), y = gldf(c.X + 3 * i + 1), z = gldf(c.X + 3 * i + 2);
  double s = 0.0;
#pragma unroll 4
  for (int k = 0; k < M / 2; ++k) {
    float sn, cs;
    phase_sincos(oms[k], x, y, z, sn, cs);
    s += (double)cs * gldf(c.G32 + (size_t)(2 * k) * c.d + ch);
    s += (double)sn * gldf(c.G32 + (size_t)(2 * k + 1) * c.d + ch);
  }
  gstf(v + i, (float)((double)gldf(c.F + i * c.ldF + ch) + s));
}

// B^T diag(w) of a square sliced field, formed directly: slice s's H0 column
// c is phi(x_i) w_i for i = 64 s + c (unscaled device-order features, the
// product in FP64). One thread per point; no n x n field is read.
template <int M>
__global__ __launch_bounds__(256) void k_wide_diag_h0(const CloudDesc* __restrict__ cl, int64_t N,
                                                      const float* __restrict__ w) {
  __shared__ float4 oms[M / 2];
  for (int k = threadIdx.x; k < M / 2; k += 256) oms[k] = gld4((const float*)(cl[0].om + k));
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const CloudDesc& c = cl[i / 64];
  const int ch = (int)(i % 64);
  const float x = gldf(c.X + 3 * i), y = gldf(c.X + 3 * i + 1), z = gldf(c.X + 3 * i + 2);
  const double wi = (double)gldf(w + i);
#pragma unroll 4
  for (int k = 0; k < M / 2; ++k) {
    float sn, cs;
    phase_sincos(oms[k], x, y, z, sn, cs);
    gstd(c.H0 + (size_t)(2 * k) * c.d + ch, (double)cs * wi);
    gstd(c.H0 + (size_t)(2 * k + 1) * c.d + ch, (double)sn * wi);
  }
}

hipError_t launch_wide_diag_h0(int M, const CloudDesc* dcl, int64_t N, const float* w, hipStream_t st) {
  const dim3 grid((unsigned)((N + 255) / 256));
  if (M == 64) hipLaunchKernelGGL(k_wide_diag_h0<64>, grid, dim3(256), 0, st, dcl, N, w);
  else if (M == 128) hipLaunchKernelGGL(k_wide_diag_h0<128>, grid, dim3(256), 0, st, dcl, N, w);
  else if (M == 256) hipLaunchKernelGGL(k_wide_diag_h0<256>, grid, dim3(256), 0, st, dcl, N, w);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_wide_diag(int M, const CloudDesc* dcl, int64_t N, float* v, hipStream_t st) {
  const dim3 grid((unsigned)((N + 255) / 256));
  if (M == 64) hipLaunchKernelGGL(k_wide_diag<64>, grid, dim3(256), 0, st, dcl, N, v);
  else if (M == 128) hipLaunchKernelGGL(k_wide_diag<128>, grid, dim3(256), 0, st, dcl, N, v);
  else if (M == 256) hipLaunchKernelGGL(k_wide_diag<256>, grid, dim3(256), 0, st, dcl, N, v);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------ batched launchers
template <int M, int PREC, bool GRAM>
static hipError_t bta_batch_db(int DB, int nwork, const CloudDesc* dcl, const int2* dwork, size_t stride,
                               hipStream_t st) {
  switch (DB) {
    case 1:
      hipLaunchKernelGGL((k_bta_batch<M, PREC, GRAM, 1>), dim3(nwork), dim3(256), 0, st, dcl, dwork, stride);
      return hipGetLastError();
    case 2:
      hipLaunchKernelGGL((k_bta_batch<M, PREC, GRAM, 2>), dim3(nwork), dim3(256), 0, st, dcl, dwork, stride);
      return hipGetLastError();
    case 4:
      if constexpr (M != 256 || !GRAM) {  // the Gram at m = 256 takes at most 32 channels
        hipLaunchKernelGGL((k_bta_batch<M, PREC, GRAM, 4>), dim3(nwork), dim3(256), 0, st, dcl, dwork, stride);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
}

template <int M, int PREC>
static hipError_t bta_batch_gram(bool gram, int DB, int nwork, const CloudDesc* dcl, const int2* dwork, size_t stride,
                                 hipStream_t st) {
  return gram ? bta_batch_db<M, PREC, true>(DB, nwork, dcl, dwork, stride, st)
              : bta_batch_db<M, PREC, false>(DB, nwork, dcl, dwork, stride, st);
}

hipError_t launch_bta_batch(int M, int prec, int DB, bool gram, const CloudDesc* dcl, const int2* dwork, int nwork,
                            hipStream_t st) {
  const size_t stride = bta_partial_floats(M, 16 * DB, gram);
  ProfileScope prof(kKBtaBatch, st);
  if (M == 64) return prec ? bta_batch_gram<64, 1>(gram, DB, nwork, dcl, dwork, stride, st) : bta_batch_gram<64, 0>(gram, DB, nwork, dcl, dwork, stride, st);
  if (M == 128) return prec ? bta_batch_gram<128, 1>(gram, DB, nwork, dcl, dwork, stride, st) : bta_batch_gram<128, 0>(gram, DB, nwork, dcl, dwork, stride, st);
  if (M == 256) return prec ? bta_batch_gram<256, 1>(gram, DB, nwork, dcl, dwork, stride, st) : bta_batch_gram<256, 0>(gram, DB, nwork, dcl, dwork, stride, st);
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_batch(int M, int DB, bool gram, const CloudDesc* dcl, int ncl, int max_parts, hipStream_t st) {
  const size_t stride = bta_partial_floats(M, 16 * DB, gram);
  const size_t E = reduce_elems(M, DB, gram);
  ProfileScope prof(kKReduce, st);
  if (max_parts <= kFusedReduceMaxParts) {
    hipLaunchKernelGGL(k_reduce_fused_batch, dim3((unsigned)((E + 255) / 256), (unsigned)ncl), dim3(256), 0, st, dcl,
                       stride, E, M, DB, gram ? 1 : 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_reduce1_batch, dim3((unsigned)((E + 255) / 256), kReduceGroups, (unsigned)ncl), dim3(256), 0, st,
                     dcl, stride, E);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce2_batch, dim3((unsigned)((E + 255) / 256), 1, (unsigned)ncl), dim3(256), 0, st, dcl, E, M,
                     DB, gram ? 1 : 0);
  return hipGetLastError();
}

int fused_reduce_max_parts() { return kFusedReduceMaxParts; }

hipError_t launch_gcore_batch(int M, int dmax, const CloudDesc* dcl, int ncl, hipStream_t st) {
  ProfileScope prof(kKGcore, st);
  hipLaunchKernelGGL(k_gcore_batch, dim3((unsigned)(M / kGcoreRows), (unsigned)((dmax + 15) / 16), (unsigned)ncl), dim3(256),
                     0, st, dcl, M);
  return hipGetLastError();
}

template <int M, int PREC, bool TOUT, bool DIAG, bool EPI>
static hipError_t expand_batch_db(int DB, int nwork, const CloudDesc* dcl, const int2* dwork, int tpi,
                                  hipStream_t st) {
  switch (DB) {
    case 1:
      hipLaunchKernelGGL((k_expand_batch<M, PREC, 1, TOUT, DIAG, EPI>), dim3(nwork), dim3(256), 0, st, dcl, dwork, tpi);
      break;
    case 2:
      hipLaunchKernelGGL((k_expand_batch<M, PREC, 2, TOUT, DIAG, EPI>), dim3(nwork), dim3(256), 0, st, dcl, dwork, tpi);
      break;
    case 4:
      hipLaunchKernelGGL((k_expand_batch<M, PREC, 4, TOUT, DIAG, EPI>), dim3(nwork), dim3(256), 0, st, dcl, dwork, tpi);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The combinations in use: plain; transposed; transposed from a diagonal
// field; transposed with the epilogue.
template <int M, int PREC>
static hipError_t expand_batch_t(bool tout, bool diag, bool epi, int DB, int nwork, const CloudDesc* dcl,
                                 const int2* dwork, int tpi, hipStream_t st) {
  if ((diag || epi) && !tout) return hipErrorInvalidValue;
  if (diag && epi) return hipErrorInvalidValue;
  if (diag) return expand_batch_db<M, PREC, true, true, false>(DB, nwork, dcl, dwork, tpi, st);
  if (epi) return expand_batch_db<M, PREC, true, false, true>(DB, nwork, dcl, dwork, tpi, st);
  return tout ? expand_batch_db<M, PREC, true, false, false>(DB, nwork, dcl, dwork, tpi, st)
              : expand_batch_db<M, PREC, false, false, false>(DB, nwork, dcl, dwork, tpi, st);
}

hipError_t launch_expand_valu_batch(int M, int prec, const CloudDesc* dcl, const int2* dwork, int nwork, int tpi,
                                    hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  ProfileScope prof(kKExpandBatch, st);
#define RFD_EXPVB(MM, PP)                                                                                    \
  if (M == MM && prec == PP) {                                                                               \
    hipLaunchKernelGGL((k_expand_valu_batch<MM, PP>), dim3(nwork), dim3(256), 0, st, dcl, dwork, tpi);     \
    return hipGetLastError();                                                                                \
  }
  RFD_EXPVB(64, 0)
  RFD_EXPVB(64, 1)
  RFD_EXPVB(128, 0)
  RFD_EXPVB(128, 1)
  RFD_EXPVB(256, 0)
  RFD_EXPVB(256, 1)
#undef RFD_EXPVB
  return hipErrorInvalidValue;
}

hipError_t launch_expand_batch(int M, int prec, int DB, const CloudDesc* dcl, const int2* dwork, int nwork, int tpi,
                               hipStream_t st, bool tout, bool diag, bool epi) {
  ProfileScope prof(kKExpandBatch, st);
  if (M == 64) return prec ? expand_batch_t<64, 1>(tout, diag, epi, DB, nwork, dcl, dwork, tpi, st) : expand_batch_t<64, 0>(tout, diag, epi, DB, nwork, dcl, dwork, tpi, st);
  if (M == 128) return prec ? expand_batch_t<128, 1>(tout, diag, epi, DB, nwork, dcl, dwork, tpi, st) : expand_batch_t<128, 0>(tout, diag, epi, DB, nwork, dcl, dwork, tpi, st);
  if (M == 256) return prec ? expand_batch_t<256, 1>(tout, diag, epi, DB, nwork, dcl, dwork, tpi, st) : expand_batch_t<256, 0>(tout, diag, epi, DB, nwork, dcl, dwork, tpi, st);
  return hipErrorInvalidValue;
}

}  // namespace rfd
