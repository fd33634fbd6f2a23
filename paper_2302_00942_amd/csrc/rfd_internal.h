// Internal declarations of the RFD library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

#include "rfd.h"

namespace rfd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxM = 256;        // largest supported number of feature columns
constexpr int kMaxDim = 64;       // largest coordinate dimension of the points
constexpr int kMaxD = 1024;       // largest field width per call
constexpr int kChunk = 64;        // points per chunk of the split-N passes
constexpr int kDBlock = 16;       // channels per MFMA block of the field
constexpr int kMaxDBlocks = 4;    // channel blocks handled by one pass (64 channels)
constexpr int kBarrierWords = 2048; // words of the grid-barrier counters of a plan
constexpr int kSpecBarrierOffset = 1024;  // the cooperative spectrum's counters (phi_1 uses the words below)

// Device feature order: column 2k holds cos(2 pi omega_k . x), column 2k+1
// holds sin(2 pi omega_k . x), both unscaled. The paper's order
// [cos_0..cos_{f-1} | sin_0..sin_{f-1}] with the scale c_k is restored at the
// host boundary (rfd_plan_core) and folded into the m x m core T.
__host__ __device__ inline int dev_to_canon(int j, int f) { return (j & 1) ? f + (j >> 1) : (j >> 1); }

// One cloud of a batched launch (device-side descriptor).
struct CloudDesc {
  const float* X;     // points (the caller's)
  float* Xcopy;       // the plan's resident copy, written by the split-N pass
  int64_t N;
  const float4* om;   // frequencies
  const float* F;
  int64_t ldF;
  float* out;
  int64_t ldO;
  float* partials;    // the plan's split-N partials
  double* lvl;        // the plan's level-1 reduction buffer
  double* Mraw;
  double* H0;
  const double* T64;
  float* G32;
  __bf16* Gt16;
  int* flag;
  int d;
  int nparts;
  // optional epilogue of a transposed store: out = fma(-2, result,
  // epi_a[c] + epi_b[p]) for channel c, point p (null: plain store)
  const float* epi_a;
  const float* epi_b;
};

// Scratch and resident buffers of one plan.
struct PlanDev {
  float4* om = nullptr;       // f x float4
  float* omD = nullptr;       // f x D frequencies of a plan of dimension D != 3 (zero rows past f)
  double* cvec = nullptr;     // m: c_j in canonical order
  double* svec = nullptr;     // m: sign_j in canonical order
  float* X = nullptr;         // copy of the cloud
  int64_t Xcap = 0;
  double* Mraw = nullptr;     // m x m
  double* H0 = nullptr;       // m x 64, device order: unscaled Phi^T F of one channel slice
  double* S64 = nullptr;      // m x m, canonical order, lambda phi_1(lambda M)
  double* T64 = nullptr;      // m x m, device order
  float* G32 = nullptr;       // m x 64, device order: G' = T H0 of one channel slice
  __bf16* Gt16 = nullptr;     // 2 x 64 x m: G'^T as BF16 hi, then BF16 lo
  double* G64 = nullptr;      // m x 32, canonical: G = S H of the last phi_1 action (FP64)
  double* phi_ws = nullptr;   // phi_1 workspace (phi1_ws_doubles)
  int* sdev = nullptr;        // scaling power s
  unsigned* barrier = nullptr;// grid barrier counter
  int* flag = nullptr;        // non-finite flag
  double* lvl = nullptr;      // level-1 sums of the partial reduction
  float* partials = nullptr;  // split-N partial sums
  size_t partials_cap = 0;    // in floats
  bool external = false;      // every buffer is a piece of a caller's arena (never freed, never grown)
};

}  // namespace rfd

struct rfd_plan_s {
  rfd_params params{};
  int m = 0, f = 0;
  double sigma = 0, radius = 0;
  std::vector<float> omega;   // f x D
  std::vector<double> w;      // f
  double wsum_abs = 0;        // sum |w_k|
  bool any_growth = false;    // lambda * w_k > 0 for some k
  int64_t N = -1;             // cloud size after rfd_features (-1: none)
  bool core_ready = false;    // S and T hold phi_1 of the current cloud's core
  int action_d = 0;           // channels of the last phi_1 action in G64 (0: none)
  int dev_m = 0;              // padded feature count used on the device: 64, 128 or 256
  int device = 0;
  rfd::PlanDev dev;
};

namespace rfd {

// Coordinate dimension of a plan's points (params.dim, 0 meaning 3).
inline int plan_dim(const rfd_params& p) { return p.dim == 0 ? 3 : p.dim; }
// Entry points that apply the kernel to a field run on 3-D points only.
inline bool plan_is_3d(const rfd_plan_s* p) { return plan_dim(p->params) == 3; }

// Kernel ids of the optional per-launch timing (profile.cpp).
enum KernelId {
  kKGram = 0, kKBta, kKReduce, kKPhi1, kKGcore, kKExpand, kKPhi1Batch, kKBtaBatch, kKExpandBatch,
  kKPhi1Apply, kNumKernelIds
};

// Brackets one launch with hipEvents on its stream while profiling is on.
class ProfileScope {
 public:
  ProfileScope(int id, hipStream_t st);
  ~ProfileScope();
  ProfileScope(const ProfileScope&) = delete;
  ProfileScope& operator=(const ProfileScope&) = delete;

 private:
  int id_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  bool active_ = false;
};
const char* kernel_name(int id);

// Kernels and launchers (k_stream.hip, k_phi1.hip).
// xcopy (may be null): where the pass also writes the points it reads.
hipError_t launch_bta(rfd_plan_s* p, const float* X, int64_t N, const float* F, int64_t ldF,
                      int d, bool gram, hipStream_t st, float* xcopy = nullptr);
hipError_t launch_reduce(rfd_plan_s* p, int64_t N, int d, bool gram, hipStream_t st);
// The Gram pass of a plan of dimension D != 3 over N x D points (partials as
// launch_bta's Gram pass without a field, for launch_reduce(p, N, 0, true)).
hipError_t launch_gram_nd(rfd_plan_s* p, const float* X, int64_t N, hipStream_t st);
hipError_t launch_phi1(rfd_plan_s* p, hipStream_t st);
hipError_t launch_phi1_batch(rfd_plan_s** plans, int n, void* dev_args, hipStream_t st);
// G' of one block of d <= phi1_apply_max_width() channels straight from H0,
// without forming S (the plan's S and T are then stale: see ensure_core).
hipError_t launch_phi1_apply(rfd_plan_s* p, int d, hipStream_t st);
int phi1_apply_max_width();
// Most workers the cooperative phi_1 kernel of this plan uses (its tiles per phase, at most one XCD's CUs).
int phi1_grid_workers_max(rfd_plan_s* p);
// Batched action form: one workgroup per cloud over Phi1Args / apply records.
hipError_t launch_phi1_apply_batch_dev(int M, int n, const void* dev_args, const void* dev_aargs, hipStream_t st);
void phi1_fill_apply_args(rfd_plan_s* p, int d, void* out);  // writes one apply record
size_t phi1_apply_args_bytes();
// Forms S and T (phi_1 kernel) if the last core computation used the action form.
rfd_status ensure_core(rfd_plan_s* p, hipStream_t st);
size_t phi1_args_bytes();
size_t phi1_ws_doubles(int m);
hipError_t launch_gcore(rfd_plan_s* p, int d, hipStream_t st);
hipError_t launch_expand(rfd_plan_s* p, const float* X, int64_t N, const float* F, int64_t ldF,
                         int d, float* out, int64_t ldO, const float* rowscale, hipStream_t st);
// Batched stages over device descriptor arrays.
// gram: the pass also forms the feature Gram (one-shot batches); without it only
// B^T F of each descriptor's field (resident clouds, slices of a wide field).
hipError_t launch_bta_batch(int M, int prec, int DB, bool gram, const CloudDesc* dcl, const int2* dwork, int nwork,
                            hipStream_t st);
hipError_t launch_reduce_batch(int M, int DB, bool gram, const CloudDesc* dcl, int ncl, int max_parts, hipStream_t st);
int fused_reduce_max_parts();  // most partials the one-launch reduction takes
hipError_t launch_gcore_batch(int M, int dmax, const CloudDesc* dcl, int ncl, hipStream_t st);
// tout: each descriptor's result is stored transposed (out[c * ldO + p]).
// diag (with tout only): each descriptor's field is a slice of diag(w), F
// pointing at the slice's part of w and ldF holding its first column.
// epi (with tout only): the descriptors' epi_a / epi_b epilogue.
hipError_t launch_expand_batch(int M, int prec, int DB, const CloudDesc* dcl, const int2* dwork, int nwork, int tpi,
                               hipStream_t st, bool tout = false, bool diag = false, bool epi = false);
hipError_t launch_phi1_batch_dev(int M, int n, const void* dev_args, hipStream_t st);
void phi1_fill_args(rfd_plan_s* p, void* args_out);  // writes one Phi1Args
int dblocks(int d);
// Gromov-Wasserstein loss matrix (k_gw.hip): row-major FP32 matrices.
// p = T 1 and q = T^T 1 (n x m coupling), FP64 sums in a fixed order; scratch
// holds gw_margin_scratch_doubles(n, m) doubles.
hipError_t launch_gw_margins(const float* T, int64_t ldT, int n, int m, float* p, float* q, double* scratch,
                             hipStream_t st);
size_t gw_margin_scratch_doubles(int n, int m);
hipError_t launch_gw_transpose(const float* in, int64_t ldi, int rows, int cols, float* out, int64_t ldo,
                               hipStream_t st);
// Resident integration of a wide field on one plan, one launch per stage over
// its 64-channel slices (wide.cpp). Shapes and buffers are fixed at creation;
// wide_set_input re-points the field (same width) on the stream.
struct WideField {
  rfd_plan_s* p = nullptr;
  int64_t N = 0;
  int d = 0, nsl = 0, DB = 4, nparts = 1, tpi = 64;
  bool tout = false;         // result stored transposed (d x N)
  const float* diag = nullptr;  // the field is diag(diag) (square; F unused)
  bool epi = false;             // transposed store with the epi_a / epi_b epilogue
  // what the descriptors were last re-pointed to (a repeat call enqueues no patch)
  const void* cur_in = nullptr;
  const void* cur_out = nullptr;
  int64_t cur_ld = -1;
  CloudDesc* dcl = nullptr;  // one descriptor per slice (device)
  int2* dwork_bta = nullptr;
  int2* dwork_exp = nullptr;
  int nwork_bta = 0, nwork_exp = 0;
  void* arena = nullptr;     // per-slice partials, H0, G32, Gt16
};
// trans_out: the result is written transposed, out (d x N, leading dimension
// ldO >= N) = (F + A S B^T F)^T; out must not overlap F.
// diag_of (square fields, with trans_out): the field is diag(diag_of), never
// materialised; F and ldF are ignored.
rfd_status wide_create(rfd_plan_s* p, int d, const float* F, int64_t ldF, float* out, int64_t ldO, WideField* w,
                       bool trans_out = false, const float* diag_of = nullptr);
hipError_t wide_set_input(WideField* w, const float* F, int64_t ldF, hipStream_t st);
// Transposed-store fields: re-points the output (d x N, leading dimension ldO)
// and sets the epilogue out = fma(-2, result, a[c] + b[p]) (a, b non-null).
hipError_t wide_set_output_epilogue(WideField* w, float* out, int64_t ldO, const float* a, const float* b,
                                    hipStream_t st);
hipError_t wide_enqueue(const WideField* w, hipStream_t st);  // needs the plan's S and T (ensure_core)
// Square fields (d = N) only: v = the diagonal of the integrated field, with
// no other element formed.
hipError_t wide_diag_enqueue(const WideField* w, float* v, hipStream_t st);
hipError_t launch_wide_diag(int M, const CloudDesc* dcl, int64_t N, float* v, hipStream_t st);  // k_stream.hip
// Square fields diag(w) only (a wide field created with diag_of set): the
// integration of diag(w), stored transposed, from B^T diag(w) formed directly.
hipError_t wide_diag_field_enqueue(const WideField* w, hipStream_t st);
hipError_t launch_wide_diag_h0(int M, const CloudDesc* dcl, int64_t N, const float* w, hipStream_t st);
size_t wide_device_bytes(const WideField* w);
void wide_free(WideField* w);
hipError_t launch_wide_patch(CloudDesc* dcl, int nsl, const float* F, int64_t ldF, int W, hipStream_t st);  // k_gw.hip
hipError_t launch_wide_patch_out(CloudDesc* dcl, int nsl, float* out, int64_t ldO, const float* a, const float* b,
                                 int W, hipStream_t st);  // k_gw.hip
// Spectrum of the kernel matrix of one cloud (k_spectrum.hip): the plan's core,
// its phi_1 workspace (global path), the output and the selection.
struct SpecArgs {
  const double* Mraw;
  const double* cvec;
  double* Ag;
  double* out;
  int* flag;
  double lambda;
  int64_t N;
  int64_t k;
  int Mp, m, f, which;
};
SpecArgs spectrum_args(rfd_plan_s* p, int which, int64_t k, double* out);
hipError_t launch_spectrum(rfd_plan_s* p, int which, int64_t k, double* out, hipStream_t st);
hipError_t launch_spectrum_batch(const SpecArgs* dev_args, int n, int max_m, hipStream_t st);
void release_spectrum_records();  // frees the batched spectrum's record buffers (spectrum.cpp)
// Elementwise steps of the Wasserstein-barycenter iteration (k_bary.hip);
// fields N x k row-major, rho < 0: no floor.
constexpr int kMaxBaryInputs = 16;
hipError_t launch_bary_init(const float* a, int64_t N, int k, float* v, float* F, unsigned long long* ctr,
                            hipStream_t st);
hipError_t launch_bary_ratio(const float* a, const float* mus, int64_t ldmu, int64_t N, int k, float rho,
                             const float* K, float* F, unsigned long long* ctr, hipStream_t st);
hipError_t launch_bary_update(const float* a, int64_t N, int k, const float* alpha, float rho, const float* K,
                              float* v, float* F, float* mu, unsigned long long* ctr, hipStream_t st);
// Launch-geometry tuning (autotune.cpp): knobs that change speed, never results.
enum TuneKnob { kTuneExpandTilesPerWave = 0, kTuneBatchExpandTilesPerItem = 1, kTunePhi1Workgroups = 2,
                kTuneExpandPath = 3, kNumTuneKnobs };
// Arithmetic of the expansion out = F + A G' for fields of at most
// kValuMaxD channels: the matrix cores or FP32 FMAs (k_expand_valu). Unlike
// the geometry knobs this one selects different (equally valid) roundings;
// its table entry is keyed by (m, precision, d) and read by every expansion
// of such a field, single or batched.
constexpr int kValuMaxD = 4;
constexpr int kExpandMfma = 1, kExpandValu = 2;
int expand_path(int M, int prec, int d);
// Batched FMA-path expansion over (cloud, first tile) items of clouds whose
// expand_path is kExpandValu.
hipError_t launch_expand_valu_batch(int M, int prec, const CloudDesc* dcl, const int2* dwork, int nwork, int tpi,
                                    hipStream_t st);
int tuned(int knob, int M, int prec, int DB, int64_t N, int fallback);
void set_tuned(int knob, int M, int prec, int DB, int64_t N, int value);
int default_expand_tiles_per_wave(int64_t N, int prec);
int default_batch_tiles_per_item();
void set_capturing(bool on);  // suspends per-kernel timing during graph capture
int bta_partials(int64_t N, int m, int d, bool gram, int prec);  // number of workgroups / partials
size_t phi1_args_bytes();
// host helpers shared by the single-cloud and batched entry points (host_plan.cpp)
rfd_status ensure_partials(rfd_plan_s* p, size_t floats, hipStream_t st);
rfd_status ensure_x(rfd_plan_s* p, int64_t N, hipStream_t st);
int slice_width(int dev_m, bool gram);
// Host overflow guard of the core (exact bound |lambda| N sum|w| / f on the
// spectral norm of lambda M, checked when some lambda w_k > 0).
bool range_exceeded(const rfd_plan_s* p, int64_t N);
// A side stream on which phi_1 runs between two events (see enqueue_phi1).
struct PhiLane {
  hipStream_t st;
  hipEvent_t before, after;
};
rfd_status features_enqueue(rfd_plan_s* p, const float* X, int64_t N, hipStream_t st, const PhiLane* lane);
// Channels [first_channel_done, d) of out = rowscale . (F + A S B^T F) (rowscale may be null).
rfd_status integrate_enqueue(rfd_plan_s* p, const float* F, int64_t ldF, int d, float* out, int64_t ldO,
                             hipStream_t st, int first_channel_done, const float* rowscale);
rfd_status oneshot_enqueue(rfd_plan_s* p, const float* X, int64_t N, const float* F, int64_t ldF, int d,
                           float* out, int64_t ldO, hipStream_t st, const PhiLane* lane);
rfd_status check_field_args(int64_t N, const float* F, int64_t ldF, int d, const float* out, int64_t ldO);
// Partial-buffer floats a pass over N points with d channels needs.
size_t partial_floats_needed(const rfd_plan_s* p, int64_t N, int d, bool gram);
size_t partial_floats_for(int M, int prec, int64_t N, int d, bool gram);
// Largest partial buffer (floats) over the channel slices of one request.
size_t request_partial_floats(int M, int prec, int64_t N, int d, bool oneshot);
int padded_m(int m);                       // device feature count: 64, 128 or 256
size_t plan_fixed_bytes(int M);            // device bytes of a plan before any cloud
size_t plan_device_bytes(const rfd_plan_s* p);
rfd_status check_params(const rfd_params* p);
void free_plan_device(rfd_plan_s* p);      // frees the plan and its buffers without a device-wide wait
size_t bta_partial_floats(int m, int d, bool gram);              // floats per partial
size_t reduce_scratch_doubles(int m);                            // level-1 reduction buffer

}  // namespace rfd
