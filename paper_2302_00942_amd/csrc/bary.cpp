// Wasserstein barycenter on a resident RFD plan (App. D, Alg. 1): k input
// distributions on the plan's cloud, the kernel K = exp(lambda A B^T)
// applied by the low-rank integrator. One iteration is two integrations of
// the N x k field (all k distributions as channels) with the elementwise
// steps around them (k_bary.hip):
//   F = a (x) v;  K1 = FM(F);  w = mu_in / K1;  F = a (x) w;  K2 = FM(F);
//   d = v (x) K2;  mu = prod_i d_i^alpha_i;  v = v (x) mu / d.
// mu restarts from the all-ones vector every iteration (the weighted
// geometric mean of the current marginals); the optional floor replaces each
// kernel output below rho times its input by that bound. All iterations are
// recorded once into a hipGraph and replayed.
#include <math.h>

#include <vector>

#include "rfd_internal.h"

struct rfd_bary_s {
  rfd_plan_s* p = nullptr;
  int64_t N = 0;
  int k = 0, iters = 0, launches = 0;
  float rho = -1.f;
  const float* a = nullptr;
  const float* mus = nullptr;
  int64_t ldmu = 0;
  float* mu = nullptr;
  float* v = nullptr;  // N x k scaling vectors
  float* F = nullptr;  // N x k integration input
  float* K = nullptr;  // N x k integration output
  float* alpha = nullptr;
  unsigned long long* floored = nullptr;
  const void* bound[3] = {};  // the plan's point copy, partial buffer and N at creation
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

#define HIPCK(x)                                  \
  do {                                            \
    if ((x) != hipSuccess) return RFD_ERR_DEVICE; \
  } while (0)

rfd_status enqueue(rfd_bary_s* b, hipStream_t st) {
  const int64_t N = b->N;
  const int k = b->k;
  HIPCK(rfd::launch_bary_init(b->a, N, k, b->v, b->F, b->floored, st));
  for (int t = 0; t < b->iters; ++t) {
    rfd_status s = rfd::integrate_enqueue(b->p, b->F, k, k, b->K, k, st, 0, nullptr);
    if (s != RFD_OK) return s;
    HIPCK(rfd::launch_bary_ratio(b->a, b->mus, b->ldmu, N, k, b->rho, b->K, b->F, b->floored, st));
    s = rfd::integrate_enqueue(b->p, b->F, k, k, b->K, k, st, 0, nullptr);
    if (s != RFD_OK) return s;
    HIPCK(rfd::launch_bary_update(b->a, N, k, b->alpha, b->rho, b->K, b->v, b->F, b->mu, b->floored, st));
  }
  return RFD_OK;
}

void free_bary(rfd_bary_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->v) (void)hipFree(b->v);
  delete b;
}

}  // namespace

extern "C" {

rfd_status rfd_bary_create(rfd_plan_t p, const float* a, const float* mus, int64_t ldmu, int32_t k,
                           const double* alpha, int32_t iterations, double floor, float* mu_out, rfd_bary_t* out) {
  if (!out) return RFD_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || !a || !mus || !alpha || !mu_out || k < 1 || k > rfd::kMaxBaryInputs || ldmu < k || iterations < 1 ||
      !rfd::plan_is_3d(p))
    return RFD_ERR_INVALID_ARG;
  for (int i = 0; i < k; ++i)
    if (!(alpha[i] >= 0.0) || !isfinite(alpha[i])) return RFD_ERR_INVALID_ARG;
  if (!isfinite(floor)) return RFD_ERR_INVALID_ARG;
  if (p->N < 0) return RFD_ERR_NOT_READY;
  if (p->N == 0) return RFD_ERR_INVALID_ARG;
  rfd_bary_s* b = new (std::nothrow) rfd_bary_s();
  if (!b) return RFD_ERR_DEVICE;
  b->p = p;
  b->N = p->N;
  b->k = k;
  b->iters = iterations;
  b->rho = floor < 0.0 ? -1.f : (float)floor;
  b->a = a;
  b->mus = mus;
  b->ldmu = ldmu;
  b->mu = mu_out;
  const size_t nk = (size_t)b->N * k;
  // v, F, K, then alpha (k floats) and the 64-bit counter, in one allocation
  const size_t bytes = sizeof(float) * (3 * nk + rfd::kMaxBaryInputs) + 2 * sizeof(unsigned long long);
  if (hipMalloc((void**)&b->v, bytes + 256) != hipSuccess) {
    b->v = nullptr;
    free_bary(b);
    return RFD_ERR_DEVICE;
  }
  b->F = b->v + nk;
  b->K = b->F + nk;
  b->alpha = b->K + nk;
  b->floored = (unsigned long long*)(((uintptr_t)(b->alpha + rfd::kMaxBaryInputs) + 15) & ~(uintptr_t)15);
  std::vector<float> al(rfd::kMaxBaryInputs, 0.f);
  for (int i = 0; i < k; ++i) al[i] = (float)alpha[i];
  rfd_status s = RFD_OK;
  if (hipMemcpy(b->alpha, al.data(), sizeof(float) * al.size(), hipMemcpyHostToDevice) != hipSuccess)
    s = RFD_ERR_DEVICE;
  // S and T, and partials for the widest slice, before anything is recorded;
  // this call has no stream, so the device is idle around them
  if (s == RFD_OK && !p->core_ready) {
    s = hipDeviceSynchronize() == hipSuccess ? rfd::ensure_core(p, nullptr) : RFD_ERR_DEVICE;
    if (s == RFD_OK && hipDeviceSynchronize() != hipSuccess) s = RFD_ERR_DEVICE;
  }
  if (s == RFD_OK) s = rfd::ensure_partials(p, rfd::partial_floats_needed(p, b->N, k, false), nullptr);
  if (s != RFD_OK) {
    free_bary(b);
    return s;
  }
  b->bound[0] = p->dev.X;
  b->bound[1] = p->dev.partials;
  b->bound[2] = (const void*)(intptr_t)p->N;
  *out = b;
  return RFD_OK;
}

rfd_status rfd_bary_launch(rfd_bary_t b, rfd_stream_t stream) {
  if (!b) return RFD_ERR_INVALID_ARG;
  rfd_plan_s* p = b->p;
  if (p->dev.X != b->bound[0] || p->dev.partials != b->bound[1] || (const void*)(intptr_t)p->N != b->bound[2])
    return RFD_ERR_INVALID_ARG;  // the plan's buffers or cloud size changed since creation
  hipStream_t st = (hipStream_t)stream;
  // a one-shot call on the plan since then may have left S and T stale
  const rfd_status cs = rfd::ensure_core(p, st);
  if (cs != RFD_OK) return cs;
  if (b->exec) {
    HIPCK(hipGraphLaunch(b->exec, st));
    return RFD_OK;
  }
  if (b->launches == 0 || st == nullptr) {
    ++b->launches;
    return enqueue(b, st);
  }
  rfd::set_capturing(true);
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
  rfd_status s = e == hipSuccess ? enqueue(b, st) : RFD_ERR_DEVICE;
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  rfd::set_capturing(false);
  if (s != RFD_OK || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return s != RFD_OK ? s : RFD_ERR_DEVICE;
  }
  b->graph = g;
  HIPCK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  ++b->launches;
  HIPCK(hipGraphLaunch(b->exec, st));
  return RFD_OK;
}

rfd_status rfd_bary_floored(rfd_bary_t b, int64_t* count, rfd_stream_t stream) {
  if (!b || !count) return RFD_ERR_INVALID_ARG;
  HIPCK(hipStreamSynchronize((hipStream_t)stream));
  unsigned long long c = 0;
  HIPCK(hipMemcpy(&c, b->floored, sizeof(c), hipMemcpyDeviceToHost));
  *count = (int64_t)c;
  return RFD_OK;
}

void rfd_bary_destroy(rfd_bary_t b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_bary(b);
}

}  // extern "C"
