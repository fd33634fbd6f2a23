/*
 * rfd.h -- C ABI of the RFDiffusion (RFD) graph-field integrator on one
 * AMD Instinct MI355X (gfx950).
 *
 * What it computes (Choromanski et al., "Efficient Graph Field Integrators
 * Meet Point Clouds", ICML 2023, arXiv 2302.00942):
 *
 *   Graph-field integration (Sec. 1, Eq. 1): out(v) = sum_w K(w, v) F(w) for
 *   every point v of a cloud X = {x_i} in R^3, with the graph diffusion kernel
 *   K = exp(lambda W) (Sec. 2, Eq. 3) of the epsilon-NN graph
 *   W(i, j) = 1[||x_i - x_j|| <= eps] (Sec. 2.4, Eq. "w").
 *
 *   W is never built. Random Fourier features give W ~= A B^T with
 *   A, B in R^{N x m} (Sec. 2.4): f = m/2 frequencies omega_k drawn from a
 *   truncated Gaussian with pdf p, importance weights w_k = tau(omega_k) /
 *   p(omega_k) (tau = Fourier transform of the ball indicator), and real
 *   features Phi(x) = [c_k cos(2 pi omega_k.x) || c_k sin(2 pi omega_k.x)],
 *   c_k = sqrt(|w_k| / f); B = Phi, A = Phi diag(sgn w, sgn w). This is the
 *   real-part estimator of the Lemma 2.5 proof (App. A.4).
 *
 *   The low-rank exponential (Sec. 2.4, the identity displayed after the
 *   feature maps and the bracket order of the GFI formula that follows) is
 *   applied in phi_1 form, which needs no inverse of B^T A:
 *       out = F + A (lambda phi_1(lambda B^T A)) (B^T F),
 *       phi_1(Y) = sum_{k>=0} Y^k / (k+1)!,
 *   with phi_1 evaluated in FP64 by the degree-23 Taylor series
 *   (Paterson-Stockmeyer) with scaling and squaring.
 *
 * Memory: every X, F and out pointer is DEVICE memory owned by the caller.
 * F and out are row-major N x d float32 arrays with leading dimensions
 * ldF, ldO >= d (in elements). A plan owns its own device buffers (the
 * frequencies, a copy of X, the m x m core and scratch), allocated with
 * hipMalloc when created or when a cloud needs more room, and freed by
 * rfd_plan_destroy. Nothing throws across this ABI: every call returns an
 * rfd_status. Objects are thread-compatible (one thread at a time per plan),
 * not thread-safe; the server object is thread-safe.
 */
#ifndef RFD_H
#define RFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RFD_OK = 0,
  RFD_ERR_INVALID_ARG = 1,   /* bad size, null pointer, m odd or <= 0, eps <= 0, ld < d ... */
  RFD_ERR_RANGE = 2,         /* exp(lambda A B^T) could overflow FP64 (see rfd_features) */
  RFD_ERR_OUT_OF_BUDGET = 3, /* server: the request can never fit the HBM budget */
  RFD_ERR_NONFINITE = 4,     /* NaN or Inf in X or F, or produced in the core */
  RFD_ERR_DEVICE = 5,        /* a HIP runtime call failed */
  RFD_ERR_NOT_READY = 6,     /* rfd_integrate before rfd_features; rfd_wait timed out */
  RFD_ERR_SHUTDOWN = 7       /* server is shutting down */
} rfd_status;

/* Shape of the neighbourhood f(z) = 1[||z|| <= eps] (Sec. 2.4). */
typedef enum {
  RFD_BALL_L2 = 0,  /* Euclidean ball: tau = (sin u - u cos u)/(2 pi^2 r^3), u = 2 pi eps r */
  RFD_BOX_LINF = 1  /* max-norm box: tau = prod_i sin(2 pi eps w_i)/(pi w_i) */
} rfd_shape;

/* Arithmetic of the two thin products and the Gram (features always come
 * from FP32 phases; accumulation is FP32; phi_1 is FP64). */
typedef enum {
  RFD_FP32 = 0,  /* FP32 features, FP32 matrix cores (v_mfma_f32_*_f32) */
  RFD_BF16 = 1   /* features rounded to BF16 (RNE) as MFMA operands; the field F
                    (pass 1) and G (pass 2) enter as a BF16 hi + lo pair
                    (hi = bf16(x), lo = bf16(x - hi), two MFMAs), so the features
                    are the only BF16 rounding on the data path */
} rfd_precision;

typedef struct {
  int32_t m;          /* real feature columns, even, 2 <= m <= 256 (f = m/2 frequencies) */
  int32_t shape;      /* rfd_shape */
  int32_t precision;  /* rfd_precision */
  int32_t dim;        /* coordinate dimension D of the points, 1 <= D <= 64; 0 means 3. Points in D
                         dimensions (the graph-classification appendix: node features as vectors
                         in R^D) are taken by rfd_features, rfd_features_sync, rfd_plan_core and the
                         spectrum calls; every entry point that applies the kernel to a field needs
                         D = 3 and returns RFD_ERR_INVALID_ARG otherwise. For D != 3 the ball's
                         transform is tau = eps^(D/2) J_{D/2}(2 pi eps r) / r^(D/2), its preset
                         radius the first zero of J_{D/2} over 2 pi eps, the preset sigma
                         R / sqrt(D + 6) (R/3 at D = 3), and the frequency law N(0, sigma^2 I_D)
                         truncated to the D-ball or D-box (Sec. 2.4). */
  double eps;         /* neighbourhood radius, > 0 */
  double lambda;      /* diffusion strength in exp(lambda W); any sign */
  double sigma;       /* Gaussian scale of the frequency law; 0 with radius 0 = preset */
  double radius;      /* truncation radius R of the frequency law; 0 with sigma 0 = preset:
                         ball R = 0.7151483/eps (first zero of tau), box R = 1/(2 eps);
                         sigma = R/3. The preset keeps every weight >= 0. */
  uint64_t seed;      /* SplitMix64 seed of the frequency stream */
  const float* omega; /* optional HOST array of f x D frequencies (row-major); NULL = sample */
} rfd_params;

typedef struct rfd_plan_s* rfd_plan_t;
typedef struct rfd_server_s* rfd_server_t;
typedef void* rfd_stream_t; /* a hipStream_t; NULL = the default stream */

/* ---------------------------------------------------------------- plans */

/* Validates params, samples the f frequencies on the host (SplitMix64 ->
 * 53-bit uniforms -> Box-Muller, both outputs in order, D per candidate ->
 * times sigma -> rejected outside the ball/box of radius R, the squared norm
 * summed in coordinate order, in FP64 -> rounded to FP32) or
 * takes them from params->omega, computes the weights w = tau/p in FP64 and
 * uploads the frequencies. Errors: RFD_ERR_INVALID_ARG. */
rfd_status rfd_plan_create(const rfd_params* params, rfd_plan_t* out_plan);

/* Device bytes of a plan that lives in a caller's arena (rfd_plan_create_in)
 * sized for clouds of up to N_max points and fields of up to d_max channels:
 * the plan's fixed buffers (core, phi_1 workspace, reduction groups), the
 * point copy (12 B per point) and the split-N partials of the widest
 * one-shot or resident pass. Host only. Errors: those of rfd_plan_create's
 * parameter checks, RFD_ERR_INVALID_ARG for N_max < 0 or d_max outside
 * [0, 1024]. */
rfd_status rfd_plan_workspace_size(const rfd_params* params, int64_t N_max, int32_t d_max, size_t* bytes);

/* rfd_plan_create with every device buffer of the plan carved from the
 * caller's arena (device memory, 256-byte aligned, `bytes` >=
 * rfd_plan_workspace_size(params, N_max, d_max)), so the caller (a torch
 * tensor, a pool) owns all device memory the plan uses (Sec. 1, Eq. 1: the
 * integrator as a library call inside a larger program). The plan never
 * allocates or frees device memory: a call that would need more than the
 * sizing (a cloud of more than N_max points, a field wider than d_max) returns
 * RFD_ERR_OUT_OF_BUDGET before any launch. The arena must outlive the plan;
 * rfd_plan_destroy leaves it to the caller. Errors: RFD_ERR_INVALID_ARG (null
 * or unaligned arena, sizes), RFD_ERR_OUT_OF_BUDGET (bytes too small), those
 * of rfd_plan_create. */
rfd_status rfd_plan_create_in(const rfd_params* params, void* arena_dev, size_t bytes, int64_t N_max,
                              int32_t d_max, rfd_plan_t* out_plan);

/* Host only (no device memory, no GPU needed): the f frequencies and FP64
 * weights that rfd_plan_create would produce for these params, written to
 * caller-owned host arrays of f x D floats and f doubles. Errors:
 * RFD_ERR_INVALID_ARG as for rfd_plan_create. */
rfd_status rfd_params_frequencies(const rfd_params* params, float* omega_fx3, double* w_f);

/* Copies the plan's FP32 frequencies (f x D, row-major) and FP64 weights (f)
 * to host arrays; either pointer may be NULL. */
rfd_status rfd_plan_export(rfd_plan_t plan, float* omega_fx3, double* w_f);

/* Features of a cloud: copies X (N x 3 float32, device, row-major) into the
 * plan, computes M = B^T A (split over N, fixed-order reduction, FP64 result)
 * and S = lambda phi_1(lambda M) in FP64 (Taylor 23, scaling and squaring).
 * For a plan of dimension D != 3, X is N x D and is not kept (the plan then
 * serves rfd_plan_core and the spectrum calls only).
 * Enqueued on `stream`; returns once enqueued. Errors found on the host are
 * returned at once: RFD_ERR_INVALID_ARG (N < 0), RFD_ERR_RANGE when lambda
 * and the weights allow growth (lambda * w > 0 for some k) and the exact
 * bound |lambda| N sum|w|/f exceeds 700. Device-side findings (non-finite X
 * or core) are reported by rfd_plan_check. N = 0 is valid: out = F. */
rfd_status rfd_features(rfd_plan_t plan, const float* X_dev, int64_t N, rfd_stream_t stream);

/* rfd_features with its status reported synchronously: waits for `stream`
 * after the enqueue and returns what the device found for the plan (as
 * rfd_plan_check does: RFD_ERR_NONFINITE for a non-finite point or core,
 * RFD_ERR_RANGE for an overflowing phi_1), so plan errors surface at this
 * call. Errors otherwise those of rfd_features. */
rfd_status rfd_features_sync(rfd_plan_t plan, const float* X_dev, int64_t N, rfd_stream_t stream);

/* out = F + A (S (B^T F)) for the plan's cloud: K4 (split-N B^T F), K5
 * (reduce, G = S H) and K6 (out = F + A G), enqueued on `stream`. out may
 * alias F (each row of F is read before that row of out is written).
 * d = 0 is a no-op. Errors: RFD_ERR_NOT_READY if rfd_features has not run;
 * RFD_ERR_INVALID_ARG for ld < d, d < 0, d > 1024 or null pointers. */
rfd_status rfd_integrate(rfd_plan_t plan, const float* F_dev, int64_t ldF, int32_t d,
                         float* out_dev, int64_t ldO, rfd_stream_t stream);

/* out = diag(scale) (F + A (S (B^T F))): rfd_integrate with each output row i
 * multiplied by scale[i] (device, N float32; NULL = no scaling) in the
 * expansion's store. This is one step of a scaling loop such as the
 * Wasserstein-barycenter iteration (App. D, Alg. 1). Same errors and aliasing
 * rules as rfd_integrate. */
rfd_status rfd_integrate_scaled(rfd_plan_t plan, const float* F_dev, int64_t ldF, int32_t d,
                                float* out_dev, int64_t ldO, const float* scale_dev,
                                rfd_stream_t stream);

/* One-shot: rfd_features followed by rfd_integrate, with the Gram and B^T F
 * computed in ONE pass over X and F (B^T [A | F]); two passes in total.
 * Errors: those of rfd_features and rfd_integrate. */
rfd_status rfd_integrate_oneshot(rfd_plan_t plan, const float* X_dev, int64_t N,
                                 const float* F_dev, int64_t ldF, int32_t d,
                                 float* out_dev, int64_t ldO, rfd_stream_t stream);

/* rfd_integrate_oneshot for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it makes no hipMalloc, hipFree or other allocating call. The
 * buffers its kernels need besides X, F and out (split-N partials, the core
 * and field block, the phi_1 workspace, G', barrier counters, a status flag)
 * live in one fixed 20 MiB device array of the library, which every device it
 * runs on holds until the process ends. Limits: N <= 65536 points and
 * d <= 32 channels for m > 128 (d <= 64 for m <= 128), so the whole field
 * goes through the one fused pass; larger requests get RFD_ERR_OUT_OF_BUDGET
 * before any launch. The kernels and the split of the cloud are those of
 * rfd_integrate_oneshot, so out is bitwise the same. Points are read from
 * X_dev in both passes (X must stay valid until the stream completes) and the
 * plan's resident cloud, core and buffers are left as they were; device
 * findings (non-finite values) are added to the plan's flag for
 * rfd_plan_check. All calls on one GPU share the array: calls that overlap on
 * one GPU (two streams, two threads) race and give wrong results; serialise
 * them. The current device must be the plan's (else RFD_ERR_INVALID_ARG).
 * Other errors: those of rfd_integrate_oneshot. */
rfd_status rfd_integrate_oneshot_noalloc(rfd_plan_t plan, const float* X_dev, int64_t N,
                                         const float* F_dev, int64_t ldF, int32_t d,
                                         float* out_dev, int64_t ldO, rfd_stream_t stream);

/* Waits for `stream` and reports what the device found for this plan since
 * the last check: RFD_OK or RFD_ERR_NONFINITE (clears the flag). */
rfd_status rfd_plan_check(rfd_plan_t plan, rfd_stream_t stream);

/* Copies the plan's M (m x m, FP64, row-major) and S = lambda phi_1(lambda M)
 * (m x m, FP64, row-major) to host arrays after synchronising `stream`; also
 * the scaling power s used for phi_1. Any pointer may be NULL. M here is
 * B^T A in the feature scaling c_k (the same matrix the paper's core uses). */
rfd_status rfd_plan_core(rfd_plan_t plan, double* M_mxm, double* S_mxm, int32_t* s_out,
                         rfd_stream_t stream);

/* The plan's cloud size (the N of the last rfd_features / one-shot call, -1
 * before any), its feature count m and the padded count the device uses (64,
 * 128 or 256). Host only; any pointer may be NULL. Callers that pass F and
 * out to rfd_integrate check their row counts against N with it. */
rfd_status rfd_plan_info(rfd_plan_t plan, int64_t* N_out, int32_t* m_out, int32_t* padded_m_out);

/* The field block of the last one-shot call (or batch item) whose phi_1 ran
 * in action form (fields of <= 32 channels): H = B^T F (m x d, FP64,
 * row-major, the paper's feature order, Sec. 2.4) as the phi_1 kernel read
 * it, and G = lambda phi_1(lambda M) H (m x d, FP64) as it computed it, before
 * G is rounded for the expansion. Synchronises `stream` first. Any pointer
 * may be NULL; *d_out gets d. Errors: RFD_ERR_NOT_READY if no action-form
 * call has run on the plan. For checking the FP64 core arithmetic. */
rfd_status rfd_plan_action(rfd_plan_t plan, double* H_mxd, double* G_mxd, int32_t* d_out,
                           rfd_stream_t stream);

void rfd_plan_destroy(rfd_plan_t plan);

/* --------------------------------------------------------------- batches */

typedef struct rfd_batch_s* rfd_batch_t;

/* A batch of one-shot integrations over many clouds of uneven size: item i
 * integrates field Fs[i] (Ns[i] x ds[i], leading dimension ldFs[i]) on cloud
 * Xs[i] (Ns[i] x 3) into outs[i] with plans[i]. All plans share m and
 * precision; each item has its own plan; 1 <= ds[i] <= 64 (<= 32 when
 * m > 128); all pointers are device memory that must stay valid while the
 * batch exists. Each stage is ONE launch over the flattened work list:
 * (cloud, part) for the feature/Gram/B^T F pass, (cloud, element block) for
 * the reduction and G = S H, one workgroup per cloud for phi_1, (cloud,
 * 1024-point block) for the expansion. The split of a cloud into parts
 * depends only on its own N, so results equal the per-cloud entry points.
 * Creation sizes the plans' buffers (hipMalloc) and uploads the work lists.
 * Errors: RFD_ERR_INVALID_ARG (mixed m or precision, a plan used twice,
 * sizes), RFD_ERR_DEVICE. */
rfd_status rfd_batch_create(const rfd_plan_t* plans, const float* const* Xs, const int64_t* Ns,
                            const float* const* Fs, const int64_t* ldFs, const int32_t* ds,
                            float* const* outs, const int64_t* ldOs, int32_t n, rfd_batch_t* out);

/* Enqueues the batch on `stream`. Returns RFD_ERR_INVALID_ARG if a plan's
 * buffers were reallocated since creation (a standalone call on a larger
 * cloud); create the batch again then. The first launch runs eagerly; the second,
 * on a non-default stream, records the launch sequence into a hipGraph;
 * later launches replay that graph (one hipGraphLaunch). Per-cloud device
 * findings are reported by rfd_plan_check on each plan. */
rfd_status rfd_batch_launch(rfd_batch_t batch, rfd_stream_t stream);

/* Autotunes the batch's expansion geometry (tiles of 16 points per
 * workgroup: 8 ... 256): runs the batch once eagerly, then times `reps`
 * expansion launches per candidate with hipEvents on `stream`, keeps the
 * fastest for this batch and records it in the process-wide tuning table
 * (key: m, precision, channel blocks, log2 of the batch's total points) for
 * batches created later. The geometry never changes results. The outputs
 * hold the batch's result on return; the next launch records a new graph.
 * Errors: RFD_ERR_INVALID_ARG (reps < 1, an out aliasing its F, stale plan
 * buffers), RFD_ERR_DEVICE. */
rfd_status rfd_batch_tune(rfd_batch_t batch, int32_t reps, rfd_stream_t stream);

/* The batch's current expansion tiles per workgroup. */
int32_t rfd_batch_tiles_per_item(rfd_batch_t batch);

/* Waits for the device and frees the batch (not the plans). */
void rfd_batch_destroy(rfd_batch_t batch);

/* One-off batch: create, launch eagerly, synchronise `stream`, destroy. */
rfd_status rfd_integrate_batch(const rfd_plan_t* plans, const float* const* Xs, const int64_t* Ns,
                               const float* const* Fs, const int64_t* ldFs, const int32_t* ds,
                               float* const* outs, const int64_t* ldOs, int32_t n, rfd_stream_t stream);

/* --------------------------------------------------------------- autotuning */

/* Autotunes the expansion geometry (tiles of 16 points per wave: 1 ... 16) of
 * rfd_integrate for this plan's cloud and field width: computes G for the
 * first channel slice, times `reps` expansion launches per candidate with
 * hipEvents on `stream`, and records the fastest in the process-wide tuning
 * table (key: m, precision, channel blocks, log2 N), which every later
 * launch of that key uses (graphs already recorded keep their geometry).
 * The geometry never changes results. On return (enqueued) out holds
 * rfd_integrate(F). Errors: those of rfd_integrate; RFD_ERR_INVALID_ARG for
 * reps < 1 or out == F. */
rfd_status rfd_autotune(rfd_plan_t plan, const float* F_dev, int64_t ldF, int32_t d,
                        float* out_dev, int64_t ldO, int32_t reps, rfd_stream_t stream);

/* Autotunes the number of workgroups of the cooperative phi_1 kernel for the
 * plan's padded m (candidates: (m/32)^2, its half and its quarter): re-runs phi_1 on the plan's core `reps` times per
 * candidate, timed with hipEvents on `stream`, and records the fastest in the
 * tuning table (key: m). The count never changes results. Requires features
 * (rfd_features or a one-shot call). Errors: RFD_ERR_INVALID_ARG,
 * RFD_ERR_NOT_READY, RFD_ERR_DEVICE. */
rfd_status rfd_autotune_phi1(rfd_plan_t plan, int32_t reps, rfd_stream_t stream);

/* Writes the tuning table as text, one entry per line
 * "knob m precision channel_blocks log2N value", into buf (with a final NUL)
 * when cap is large enough; returns the bytes needed. */
int32_t rfd_tune_export(char* buf, int32_t cap);

/* Merges entries in the export format into the table; the whole text is
 * validated first (RFD_ERR_INVALID_ARG leaves the table unchanged). */
rfd_status rfd_tune_import(const char* text);

/* Clears the tuning table (defaults apply again). */
void rfd_tune_reset(void);

/* ------------------------------------------------------ repeated application */

typedef struct rfd_loop_s* rfd_loop_t;

/* A loop of `iterations` in-place steps on the vector block v (N x d,
 * leading dimension ldv, device): step t applies plan k = t mod nplans,
 *     v <- diag(scales[k]) exp(lambda_k A_k B_k^T) v,
 * with every plan's features already computed (rfd_features) on clouds of the
 * same N; scales may be NULL or hold NULL entries (no scaling). Creation sizes
 * the plans' buffers so that no launch allocates. Errors: RFD_ERR_INVALID_ARG
 * (sizes, unequal N, more than 16 plans), RFD_ERR_NOT_READY. */
rfd_status rfd_loop_create(const rfd_plan_t* plans, const float* const* scales, int32_t nplans,
                           float* v, int64_t ldv, int32_t d, int32_t iterations, rfd_loop_t* out);

/* Enqueues the whole loop on `stream`. The first launch runs eagerly; the
 * second, on a non-default stream, records the iterations into a hipGraph;
 * later launches replay it (one hipGraphLaunch). Returns RFD_ERR_INVALID_ARG
 * if a plan's buffers or cloud size changed since creation. */
rfd_status rfd_loop_launch(rfd_loop_t loop, rfd_stream_t stream);

/* Waits for the device and frees the loop (not the plans). */
void rfd_loop_destroy(rfd_loop_t loop);

/* ----------------------------------------------------- spectrum of the kernel */

/* The k smallest (which = 0, ascending) or k largest (which = 1, descending)
 * of the N eigenvalues of the kernel matrix exp(lambda A B^T) of the plan's
 * cloud, written as doubles to out_dev (device, k entries), computed from
 * the low-rank factors as the classification experiments do (Sec. 3,
 * point-cloud classification; the graph-classification appendix):
 * A B^T and the m x m core M = B^T A share their non-zero eigenvalues mu, so
 * the kernel's eigenvalues are exp(lambda mu) and, for N > m, the eigenvalue
 * 1 with multiplicity N - m (for N < m, the m - N eigenvalues of M of
 * smallest |mu| are its extra zeros and are left out). M is symmetric when
 * every weight is non-negative (the default main-lobe sampling); its
 * eigenvalues are found in FP64 (Householder tridiagonalisation, then
 * bisection on the Sturm count) by one workgroup on `stream`, using the
 * plan's M from rfd_features and its phi_1 workspace (do not overlap with
 * other work on the same plan). Errors: RFD_ERR_NOT_READY
 * (no features), RFD_ERR_INVALID_ARG (which not 0 or 1, k < 0, k > N, null
 * out with k > 0, a negative weight); a non-finite M is reported by
 * rfd_plan_check. k = 0 is a no-op. */
rfd_status rfd_plan_spectrum(rfd_plan_t plan, int32_t which, int64_t k, double* out_dev, rfd_stream_t stream);

/* rfd_plan_spectrum for n plans at once (one workgroup per cloud, one
 * launch): cloud i's k values go to outs[i] (device). Each plan appears once
 * and meets rfd_plan_spectrum's conditions, with k <= its N; the feature
 * counts may differ. The call copies n argument records into a device buffer
 * the library keeps per device and reuses (it is allocated only when n
 * exceeds every earlier n on the device; rfd_library_release frees it), and
 * synchronises `stream` before returning; concurrent calls are serialised. Errors: those of
 * rfd_plan_spectrum, RFD_ERR_INVALID_ARG for n < 0, null arrays or a plan
 * given twice; n = 0 or k = 0 is a no-op. */
rfd_status rfd_spectrum_batch(const rfd_plan_t* plans, int32_t n, int32_t which, int64_t k, double* const* outs,
                              rfd_stream_t stream);

/* ------------------------------------------------- Wasserstein barycenter */

typedef struct rfd_bary_s* rfd_bary_t;

/* The scaling iteration for the entropic Wasserstein barycenter of k
 * distributions on a resident plan's cloud (App. D, Alg. 1, "Fast Computation
 * of Wasserstein Barycenter"), with the kernel K = exp(lambda A B^T) applied
 * by the low-rank integrator. From v^i = 1, each iteration computes, for
 * every i, w^i = mu^i / K(a v^i), d^i = v^i K(a w^i), then
 * mu = prod_i (d^i)^alpha_i and v^i = v^i mu / d^i; the k distributions are
 * the channels of one N x k field, so an iteration is two integrations of
 * width k plus three elementwise kernels. mu restarts from the all-ones
 * vector every iteration (the listing initialises it once; without the
 * restart the update has no fixed point). floor >= 0 switches on a safeguard:
 * every kernel output below floor times its input is raised to that bound
 * (floor = 1 is the bound exp(lambda W) x >= x of the exact kernel for
 * lambda >= 0, which the random-feature estimate can violate); floor < 0
 * applies K as estimated. Arguments: a = area weights (device, N float32),
 * mus = inputs (device, N x k float32, leading dimension ldmu >= k),
 * alpha = k host weights, mu_out = result (device, N float32), all kept
 * alive by the caller while the object exists; 1 <= k <= 16,
 * iterations >= 1. The plan must have its features (rfd_features). Creation
 * allocates the N x k work fields; launches do not. Errors:
 * RFD_ERR_NOT_READY (no features), RFD_ERR_INVALID_ARG (sizes, null
 * pointers, a negative or non-finite alpha, N = 0), RFD_ERR_DEVICE. */
rfd_status rfd_bary_create(rfd_plan_t plan, const float* a_dev, const float* mus_dev, int64_t ldmu, int32_t k,
                           const double* alpha, int32_t iterations, double floor, float* mu_out_dev,
                           rfd_bary_t* out);

/* Runs all iterations on `stream` (async): the first launch eagerly, the
 * second records them into a hipGraph, later ones replay it; every launch
 * starts from v = 1, so each gives the same bits. RFD_ERR_INVALID_ARG if the
 * plan's buffers or cloud size changed since creation. */
rfd_status rfd_bary_launch(rfd_bary_t bary, rfd_stream_t stream);

/* Number of kernel outputs the floor raised during the last launch (waits
 * for `stream`). */
rfd_status rfd_bary_floored(rfd_bary_t bary, int64_t* count, rfd_stream_t stream);

void rfd_bary_destroy(rfd_bary_t bary);

/* ------------------------------------------- Gromov-Wasserstein loss matrix */

typedef struct rfd_gw_s* rfd_gw_t;

/* Workspace for the loss matrix of the Gromov-Wasserstein iterations with the
 * Euclidean loss (App. "Fast Computation of Tensor Products", Alg. 2), where
 * the cost matrices are the RFD operators of two clouds: C = exp(lambda A B^T)
 * of plan pc (source cloud, n points) and D likewise of plan pd (target
 * cloud, m points), both with rfd_features already run on their clouds.
 * C and D enter only through their actions (resident integrations). The
 * identity behind Alg. 2 assumes symmetric costs, which holds for RFD
 * operators whose weights are all positive (the default main-lobe sampling).
 * Allocates one max(n, m)^2 float buffer plus per-slice scratch, and forms
 * both plans' S, so that rfd_gw_loss allocates nothing. The plans must outlive
 * the workspace and keep their cloud sizes. Errors: RFD_ERR_INVALID_ARG (null
 * or identical plans, n or m < 1 or > 32768), RFD_ERR_NOT_READY (no
 * features), RFD_ERR_DEVICE. */
rfd_status rfd_gw_create(rfd_plan_t pc, rfd_plan_t pd, rfd_gw_t* out);

/* L = v1 1^T + 1 v2^T - 2 C T D^T for the coupling T (n x m float32,
 * row-major, leading dimension ldT >= m, device), written to L (n x m,
 * ldL >= m, device; overlapping T is an error), with p = T 1, q = T^T 1,
 * v1 = diag(C (C diag p)^T) = C^{o2} p and v2 = D^{o2} q, each Hadamard-square
 * action taken as two operator actions (the subsection "Estimating the Action
 * of Hadamard Square of Matrices on Vectors"), and C T D^T as
 * (D (C T)^T)^T (Alg. 2, step 3). The marginals are summed in FP64 in a fixed
 * order; the operator actions follow the plans' precision. Enqueued on
 * `stream`. Errors: RFD_ERR_INVALID_ARG (null pointers, ld < m, a plan's
 * cloud size changed since rfd_gw_create). A non-finite T is reported by
 * rfd_plan_check on the plans. */
rfd_status rfd_gw_loss(rfd_gw_t gw, const float* T_dev, int64_t ldT, float* L_dev, int64_t ldL,
                       rfd_stream_t stream);

/* The three terms of the same loss separately, as the line search of the
 * fused GW iterations uses them (App. "Gromov Wasserstein Distance", the
 * cost c_{C,D} and the tensor product): v1 = C^{o2} p (n floats),
 * v2 = D^{o2} q (m floats) and W3 = C T D^T (n x m, ldW >= m), all device,
 * computed exactly as in rfd_gw_loss (L = v1 1^T + 1 v2^T - 2 W3 with the
 * same roundings). Errors as for rfd_gw_loss. */
rfd_status rfd_gw_terms(rfd_gw_t gw, const float* T_dev, int64_t ldT, float* v1_dev, float* v2_dev,
                        float* W3_dev, int64_t ldW, rfd_stream_t stream);

/* Waits for the device and frees the workspace (not the plans). */
void rfd_gw_destroy(rfd_gw_t gw);

/* ---------------------------------------------------------------- server */

/* The server admits integration requests of mixed N, d and m and runs them
 * with continuous batching: a worker thread admits queued requests (FIFO)
 * whenever one of `max_inflight` slots is free and the device memory of the
 * request's plan fits the HBM budget, evicting idle cached plans (least
 * recently used first) to make room; admitted requests run on a pool of
 * streams, so requests that arrive while others run are admitted as slots and
 * memory free up, and their kernels overlap on the device. Plans stay
 * resident between requests, cached by their parameters: a request whose
 * cloud_key names a cloud whose features a cached plan holds runs the
 * integrate passes only; otherwise the one-shot path runs on an idle plan
 * with the same parameters (no allocation) or on a new plan. Each request's
 * result equals rfd_integrate_oneshot (or rfd_integrate on the resident
 * features) of the same inputs, bitwise, whatever else runs beside it. The
 * budget counts the plans' own device memory (frequencies, core, workspaces,
 * the copy of X, partial sums), not the callers' F and out. All functions
 * are thread-safe. */

typedef struct {
  const float* X;     /* device, N x 3; read before the request completes */
  int64_t N;
  const float* F;     /* device, N x d; must stay valid until the request completes */
  int64_t ldF;
  int32_t d;
  int32_t reserved;
  float* out;         /* device, N x d; written by the time the request completes */
  int64_t ldO;
  rfd_params params;  /* params.omega must be NULL (frequencies come from the seed) */
  uint64_t cloud_key; /* nonzero: the caller's name for this cloud (same key = same X and N),
                         so later requests on it reuse the resident features; 0 = no reuse */
} rfd_request;

typedef struct {
  rfd_status status;  /* the request's outcome */
  int32_t reserved;
  double t_submit, t_start, t_done; /* seconds on the host steady clock: submitted, admitted
                                       (work enqueued), completion seen by the worker */
} rfd_result;

/* Starts a server on the current device: hbm_budget_bytes > 0 bounds the
 * device memory of its resident plans; 1 <= max_inflight <= 64 requests run
 * at once. Errors: RFD_ERR_INVALID_ARG, RFD_ERR_DEVICE. */
rfd_status rfd_server_create(size_t hbm_budget_bytes, int32_t max_inflight, rfd_server_t* out);

/* Queues one request and returns at once with its ticket. The server runs
 * the request on its own non-blocking streams, which are not ordered after
 * the caller's streams: X, F and out must be ready (the work producing them
 * complete) when rfd_submit is called. Once rfd_wait has returned the
 * request's status, out is complete on the device. Errors (nothing is
 * queued): RFD_ERR_INVALID_ARG as for rfd_integrate_oneshot or a non-NULL
 * params.omega; RFD_ERR_OUT_OF_BUDGET when the request alone can never fit
 * the budget; RFD_ERR_SHUTDOWN. N = 0 or d = 0 completes at once. */
rfd_status rfd_submit(rfd_server_t server, const rfd_request* req, uint64_t* ticket);

/* Waits up to timeout_s seconds (< 0: without limit) for a ticket. Returns
 * RFD_ERR_NOT_READY on timeout (the ticket stays valid) and
 * RFD_ERR_INVALID_ARG for an unknown or already collected ticket; otherwise
 * fills *res (may be NULL), forgets the ticket and returns the request's
 * status: RFD_OK, RFD_ERR_RANGE, RFD_ERR_NONFINITE, RFD_ERR_DEVICE, or
 * RFD_ERR_SHUTDOWN for a request still queued when the server was destroyed. */
rfd_status rfd_wait(rfd_server_t server, uint64_t ticket, double timeout_s, rfd_result* res);

/* Current device bytes of the resident plans, number of plans, queued and
 * in-flight requests (any pointer may be NULL). */
rfd_status rfd_server_stats(rfd_server_t server, size_t* device_bytes, int32_t* plans,
                            int32_t* queued, int32_t* inflight);

/* Finishes the in-flight requests, completes the queued ones with
 * RFD_ERR_SHUTDOWN, frees every plan and the server. Call it only after every
 * thread's rfd_wait on this server has returned. */
void rfd_server_destroy(rfd_server_t server);

const char* rfd_status_string(rfd_status s);

/* --------------------------------------------------------------- profiling */

/* Turns per-kernel timing on (1) or off (0) for the whole process. While on,
 * every kernel launch of the library is bracketed by two hipEvents recorded
 * on the stream it is launched on (a few microseconds of overhead each). */
void rfd_profile_enable(int on);

/* Synchronises the device, then writes per-kernel total milliseconds and
 * launch counts for the first n kernel ids (either array may be NULL) and
 * returns the number of kernel ids; reset != 0 clears the totals. */
int32_t rfd_profile_read(double* total_ms, int64_t* counts, int32_t n, int32_t reset);

/* Name of kernel id i (a static string), "?" when out of range. */
const char* rfd_profile_kernel_name(int32_t id);

/* Destroys the HIP objects the library keeps process-wide (the timing event
 * pool, with profiling switched off, and the batched spectrum's argument
 * buffers) after a device-wide wait, so that nothing
 * of the library's is left for the runtime's exit-time teardown. Objects the
 * caller created (plans, batches, loops, servers, GW workspaces) are the
 * caller's to destroy first. Later calls recreate what they need. */
void rfd_library_release(void);

#ifdef __cplusplus
}
#endif
#endif /* RFD_H */
