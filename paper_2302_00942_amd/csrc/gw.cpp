// Loss matrix of the Gromov-Wasserstein iterations with RFD operators in place
// of the two cost matrices (App. "Fast Computation of Tensor Products",
// Alg. 2, with the Hadamard-square action of the preceding subsection):
//
//   p = T 1, q = T^T 1
//   v1 = diag(FM_C(FM_C(diag p)^T))      (= C^{o2} p)
//   v2 = diag(FM_D(FM_D(diag q)^T))      (= D^{o2} q)
//   w3 = (FM_D(FM_C(T)^T))^T             (= C T D^T)
//   L  = v1 1^T + 1 v2^T - 2 w3
//
// FM_C is a resident integration on the plan of the source cloud (n points),
// FM_D one on the plan of the target cloud (m points). Each of the six
// matrix-valued fields is integrated as one wide field (all 64-channel slices
// in one launch per stage). An action whose result is transposed next stores
// it transposed (no transpose pass), and the second action of each
// Hadamard-square term forms only the diagonal that the term keeps. Every
// step runs on the caller's stream.
#include <new>

#include "rfd_internal.h"

struct rfd_gw_s {
  rfd_plan_s* pc = nullptr;
  rfd_plan_s* pd = nullptr;
  int n = 0, m = 0;
  const float* xc = nullptr;  // the plans' point copies the wide fields were bound to
  const float* xd = nullptr;
  float* B = nullptr;    // max(n, m)^2 floats
  float* vec = nullptr;  // p (n), q (m), v1 (n), v2 (m)
  double* colpart = nullptr;  // column-sum partials of the coupling
  // wide integrations: C on diag(p) with the result stored transposed in B,
  // then C on B forming only the diagonal (likewise D); C on T stored
  // transposed in B (m x n); D on B either in place (the terms) or stored
  // transposed into L with the final combination as its epilogue (the loss)
  rfd::WideField c_sq1, c_sq2, d_sq1, d_sq2, c_t, d_cross, d_loss;
};

namespace {

#define HIPCK(x)                                  \
  do {                                            \
    if ((x) != hipSuccess) return RFD_ERR_DEVICE; \
  } while (0)

#define RFDCK(x)                 \
  do {                           \
    const rfd_status s_ = (x);   \
    if (s_ != RFD_OK) return s_; \
  } while (0)

constexpr int kMaxGwPoints = 32768;  // largest n or m (one max(n, m)^2 float buffer: 4 GiB)

void free_gw(rfd_gw_s* g) {
  for (rfd::WideField* w : {&g->c_sq1, &g->c_sq2, &g->d_sq1, &g->d_sq2, &g->c_t, &g->d_cross, &g->d_loss})
    rfd::wide_free(w);
  void* ptrs[] = {g->B, g->vec, g->colpart};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete g;
}

// v = diag(FM(FM(diag w)^T)) on k x k fields: W1 integrates diag(w) (never
// materialised: B^T diag(w) is formed from the features directly and the
// residual is the diagonal) and stores the result transposed in B, W2
// integrates B forming only the diagonal of its result.
rfd_status hadamard_square(const rfd::WideField& W1, const rfd::WideField& W2, float* v, hipStream_t st) {
  HIPCK(rfd::wide_diag_field_enqueue(&W1, st));
  HIPCK(rfd::wide_diag_enqueue(&W2, v, st));
  return RFD_OK;
}

// p, q, v1, v2 into g->vec and FM_C(T)^T (m x n) into g->B.
rfd_status enqueue_terms(rfd_gw_s* g, const float* T, int64_t ldT, hipStream_t st) {
  if (!T || ldT < g->m) return RFD_ERR_INVALID_ARG;
  if (g->pc->N != g->n || g->pd->N != g->m) return RFD_ERR_INVALID_ARG;  // a cloud changed size
  // the wide fields read the plans' point copies bound at creation: a larger
  // call in between reallocates them
  if (g->pc->dev.X != g->xc || g->pd->dev.X != g->xd) return RFD_ERR_INVALID_ARG;
  const int n = g->n, m = g->m;
  float *p = g->vec, *q = p + n, *v1 = q + m, *v2 = v1 + n;
  RFDCK(rfd::ensure_core(g->pc, st));
  RFDCK(rfd::ensure_core(g->pd, st));
  HIPCK(rfd::launch_gw_margins(T, ldT, n, m, p, q, g->colpart, st));
  RFDCK(hadamard_square(g->c_sq1, g->c_sq2, v1, st));
  RFDCK(hadamard_square(g->d_sq1, g->d_sq2, v2, st));
  // B = FM_C(T)^T (m x n)
  HIPCK(rfd::wide_set_input(&g->c_t, T, ldT, st));
  HIPCK(rfd::wide_enqueue(&g->c_t, st));
  return RFD_OK;
}

}  // namespace

extern "C" {

rfd_status rfd_gw_create(rfd_plan_t pc, rfd_plan_t pd, rfd_gw_t* out) {
  if (!out) return RFD_ERR_INVALID_ARG;
  *out = nullptr;
  if (!pc || !pd || pc == pd || !rfd::plan_is_3d(pc) || !rfd::plan_is_3d(pd)) return RFD_ERR_INVALID_ARG;
  if (pc->N < 0 || pd->N < 0) return RFD_ERR_NOT_READY;
  if (pc->N < 1 || pd->N < 1 || pc->N > kMaxGwPoints || pd->N > kMaxGwPoints) return RFD_ERR_INVALID_ARG;
  rfd_gw_s* g = new (std::nothrow) rfd_gw_s();
  if (!g) return RFD_ERR_DEVICE;
  g->pc = pc;
  g->pd = pd;
  const int n = (int)pc->N, m = (int)pd->N;
  g->n = n;
  g->m = m;
  g->xc = pc->dev.X;
  g->xd = pd->dev.X;
  const size_t k = (size_t)(n > m ? n : m);
  bool ok = hipMalloc((void**)&g->B, sizeof(float) * k * k) == hipSuccess &&
            hipMalloc((void**)&g->vec, sizeof(float) * 2 * (size_t)(n + m)) == hipSuccess &&
            hipMalloc((void**)&g->colpart, sizeof(double) * rfd::gw_margin_scratch_doubles(n, m)) == hipSuccess;
  rfd_status s = ok ? RFD_OK : RFD_ERR_DEVICE;
  // S and T of both plans now, so that no call of the loss forms them
  for (rfd_plan_s* p : {pc, pd}) {
    if (s == RFD_OK && !p->core_ready) {
      s = hipDeviceSynchronize() == hipSuccess ? rfd::ensure_core(p, nullptr) : RFD_ERR_DEVICE;
      if (s == RFD_OK && hipDeviceSynchronize() != hipSuccess) s = RFD_ERR_DEVICE;
    }
  }
  float* p = g->vec;  // p (n), then q (m)
  if (s == RFD_OK) s = rfd::wide_create(pc, n, nullptr, n, g->B, n, &g->c_sq1, true, p);
  if (s == RFD_OK) s = rfd::wide_create(pc, n, g->B, n, nullptr, n, &g->c_sq2);
  if (s == RFD_OK) s = rfd::wide_create(pd, m, nullptr, m, g->B, m, &g->d_sq1, true, p + n);
  if (s == RFD_OK) s = rfd::wide_create(pd, m, g->B, m, nullptr, m, &g->d_sq2);
  if (s == RFD_OK) s = rfd::wide_create(pc, m, nullptr, m, g->B, n, &g->c_t, true);
  if (s == RFD_OK) s = rfd::wide_create(pd, n, g->B, n, g->B, n, &g->d_cross);
  if (s == RFD_OK) s = rfd::wide_create(pd, n, g->B, n, nullptr, m, &g->d_loss, true);
  if (s != RFD_OK) {
    free_gw(g);
    return s;
  }
  *out = g;
  return RFD_OK;
}

rfd_status rfd_gw_loss(rfd_gw_t g, const float* T, int64_t ldT, float* L, int64_t ldL, rfd_stream_t stream) {
  if (!g || !L || ldL < g->m) return RFD_ERR_INVALID_ARG;
  if (T) {  // L and T must not overlap (T is the caller's input and stays intact)
    const char *t0 = (const char*)T, *t1 = (const char*)(T + ((size_t)(g->n - 1) * ldT + g->m));
    const char *l0 = (const char*)L, *l1 = (const char*)(L + ((size_t)(g->n - 1) * ldL + g->m));
    if (t0 < l1 && l0 < t1) return RFD_ERR_INVALID_ARG;
  }
  const hipStream_t st = (hipStream_t)stream;
  RFDCK(enqueue_terms(g, T, ldT, st));
  // L = (FM_D(B))^T combined as fma(-2, ., v1[i] + v2[j]) in the store
  const float *v1 = g->vec + g->n + g->m, *v2 = v1 + g->n;
  HIPCK(rfd::wide_set_output_epilogue(&g->d_loss, L, ldL, v1, v2, st));
  HIPCK(rfd::wide_enqueue(&g->d_loss, st));
  return RFD_OK;
}

rfd_status rfd_gw_terms(rfd_gw_t g, const float* T, int64_t ldT, float* v1, float* v2, float* W3, int64_t ldW,
                        rfd_stream_t stream) {
  if (!g || !v1 || !v2 || !W3 || ldW < g->m) return RFD_ERR_INVALID_ARG;
  const hipStream_t st = (hipStream_t)stream;
  RFDCK(enqueue_terms(g, T, ldT, st));
  HIPCK(rfd::wide_enqueue(&g->d_cross, st));  // B <- FM_D(B) = W3^T
  const int n = g->n, m = g->m;
  const float* dv1 = g->vec + n + m;
  HIPCK(hipMemcpyAsync(v1, dv1, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
  HIPCK(hipMemcpyAsync(v2, dv1 + n, sizeof(float) * m, hipMemcpyDeviceToDevice, st));
  HIPCK(rfd::launch_gw_transpose(g->B, n, m, n, W3, ldW, st));
  return RFD_OK;
}

void rfd_gw_destroy(rfd_gw_t g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  free_gw(g);
}

}  // extern "C"
