// Repeated application of resident RFD operators to one block of vectors,
// v <- s_k . exp(lambda_k A_k B_k^T) v with k cycling over the plans: the
// alternating scaling loop of the Wasserstein-barycenter algorithm (App. D,
// Alg. 1) with fixed features. Every iteration is the resident-plan integrate
// (split-N B^T v, reduce, G = S H, expansion with the scale fused into its
// store); the whole loop is recorded once into a hipGraph and replayed.
#include <math.h>

#include <vector>

#include "rfd_internal.h"

struct rfd_loop_s {
  std::vector<rfd_plan_s*> plans;
  std::vector<const float*> scales;
  std::vector<const void*> bound;  // per plan: X copy, partial buffer, N at creation
  float* v = nullptr;
  int64_t ldv = 0;
  int d = 0, iters = 0, launches = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

#define HIPCK(x)                                  \
  do {                                            \
    if ((x) != hipSuccess) return RFD_ERR_DEVICE; \
  } while (0)

constexpr int kMaxLoopPlans = 16;

rfd_status enqueue(rfd_loop_s* L, hipStream_t st) {
  const int n = (int)L->plans.size();
  for (int t = 0; t < L->iters; ++t) {
    rfd_plan_s* p = L->plans[t % n];
    rfd_status s = rfd::integrate_enqueue(p, L->v, L->ldv, L->d, L->v, L->ldv, st, 0, L->scales[t % n]);
    if (s != RFD_OK) return s;
  }
  return RFD_OK;
}

bool stale(const rfd_loop_s* L) {
  for (size_t i = 0; i < L->plans.size(); ++i) {
    const rfd_plan_s* p = L->plans[i];
    if (p->dev.X != L->bound[3 * i] || p->dev.partials != L->bound[3 * i + 1] ||
        (const void*)(intptr_t)p->N != L->bound[3 * i + 2])
      return true;
  }
  return false;
}

void free_loop(rfd_loop_s* L) {
  if (L->exec) (void)hipGraphExecDestroy(L->exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  delete L;
}

}  // namespace

extern "C" {

rfd_status rfd_loop_create(const rfd_plan_t* plans, const float* const* scales, int32_t nplans, float* v,
                           int64_t ldv, int32_t d, int32_t iterations, rfd_loop_t* out) {
  if (!out) return RFD_ERR_INVALID_ARG;
  *out = nullptr;
  if (!plans || nplans < 1 || nplans > kMaxLoopPlans || iterations < 1 || d < 1 || d > rfd::kMaxD || !v ||
      ldv < d)
    return RFD_ERR_INVALID_ARG;
  const int64_t N = plans[0] ? plans[0]->N : -1;
  for (int i = 0; i < nplans; ++i) {
    if (!plans[i] || !rfd::plan_is_3d(plans[i])) return RFD_ERR_INVALID_ARG;
    if (plans[i]->N < 0) return RFD_ERR_NOT_READY;
    if (plans[i]->N != N) return RFD_ERR_INVALID_ARG;  // one vector block shared by every operator
  }
  if (N == 0) return RFD_ERR_INVALID_ARG;
  rfd_loop_s* L = new (std::nothrow) rfd_loop_s();
  if (!L) return RFD_ERR_DEVICE;
  L->v = v;
  L->ldv = ldv;
  L->d = d;
  L->iters = iterations;
  for (int i = 0; i < nplans; ++i) {
    rfd_plan_s* p = plans[i];
    // S and T must exist before any launch is recorded; this call has no
    // stream, so the device is idle around the phi_1 launch
    if (!p->core_ready) {
      rfd_status cs = hipDeviceSynchronize() == hipSuccess ? rfd::ensure_core(p, nullptr) : RFD_ERR_DEVICE;
      if (cs == RFD_OK && hipDeviceSynchronize() != hipSuccess) cs = RFD_ERR_DEVICE;
      if (cs != RFD_OK) {
        free_loop(L);
        return cs;
      }
    }
    // size the partial buffer for the widest channel slice now, so that no
    // launch of the loop allocates
    const int W = rfd::slice_width(p->dev_m, false);
    size_t need = 0;
    for (int c0 = 0; c0 < d; c0 += W) {
      const size_t f = rfd::partial_floats_needed(p, N, d - c0 < W ? d - c0 : W, false);
      need = f > need ? f : need;
    }
    rfd_status s = rfd::ensure_partials(p, need, nullptr);
    if (s != RFD_OK) {
      free_loop(L);
      return s;
    }
    L->plans.push_back(p);
    L->scales.push_back(scales ? scales[i] : nullptr);
  }
  for (rfd_plan_s* p : L->plans) {
    L->bound.push_back(p->dev.X);
    L->bound.push_back(p->dev.partials);
    L->bound.push_back((const void*)(intptr_t)p->N);
  }
  *out = L;
  return RFD_OK;
}

rfd_status rfd_loop_launch(rfd_loop_t L, rfd_stream_t stream) {
  if (!L) return RFD_ERR_INVALID_ARG;
  if (stale(L)) return RFD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  // The recorded launches read each plan's S and T. A one-shot call on a plan
  // since then (same cloud size, so the same buffers) may have applied phi_1
  // in action form to a new cloud and left S and T stale: form them first.
  for (rfd_plan_s* p : L->plans) {
    const rfd_status cs = rfd::ensure_core(p, st);
    if (cs != RFD_OK) return cs;
  }
  if (L->exec) {
    HIPCK(hipGraphLaunch(L->exec, st));
    return RFD_OK;
  }
  if (L->launches == 0 || st == nullptr) {
    ++L->launches;
    return enqueue(L, st);
  }
  rfd::set_capturing(true);
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
  rfd_status s = e == hipSuccess ? enqueue(L, st) : RFD_ERR_DEVICE;
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  rfd::set_capturing(false);
  if (s != RFD_OK || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return s != RFD_OK ? s : RFD_ERR_DEVICE;
  }
  L->graph = g;
  HIPCK(hipGraphInstantiate(&L->exec, g, nullptr, nullptr, 0));
  ++L->launches;
  HIPCK(hipGraphLaunch(L->exec, st));
  return RFD_OK;
}

void rfd_loop_destroy(rfd_loop_t L) {
  if (!L) return;
  (void)hipDeviceSynchronize();
  free_loop(L);
}

}  // extern "C"
