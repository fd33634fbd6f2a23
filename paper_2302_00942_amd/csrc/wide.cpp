// Resident integration of a wide field (d = hundreds to thousands of
// channels) in one launch per stage: each 64-channel slice of the field is one
// descriptor of the batched stages (split-N B^T F without the Gram, the
// one-launch reduction, G' = T H0, the expansion), so the number of launches
// does not grow with d and the slices fill the chip together. Each slice has
// its own partial sums, H0 and G'; the plan's features, X copy and T are
// shared. The geometry (partials per slice, tiles per expansion item) is
// fixed at creation.
#include <algorithm>
#include <vector>

#include "rfd_internal.h"

namespace rfd {

namespace {

constexpr int kWideSlice = 64;          // channels per slice
constexpr int kWideTargetItems = 2048;  // work items per stage the geometry aims for

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

void wide_free(WideField* w) {
  void* ptrs[] = {w->dcl, w->dwork_bta, w->dwork_exp, w->arena};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  *w = WideField();
}

rfd_status wide_create(rfd_plan_s* p, int d, const float* F, int64_t ldF, float* out, int64_t ldO, WideField* w,
                       bool trans_out, const float* diag_of) {
  *w = WideField();
  if (p->N < 1 || d < 1) return RFD_ERR_INVALID_ARG;
  if (diag_of && (d != p->N || !trans_out)) return RFD_ERR_INVALID_ARG;
  const int M = p->dev_m, prec = p->params.precision;
  const int64_t N = p->N;
  const int nsl = (d + kWideSlice - 1) / kWideSlice;
  const int DB = dblocks(std::min(d, kWideSlice));
  const int per_slice_parts = bta_partials(N, M, kWideSlice, false, prec);
  const int nparts = std::max(1, std::min({per_slice_parts, fused_reduce_max_parts(),
                                           (kWideTargetItems + nsl - 1) / nsl}));
  const int64_t ntiles = (N + 15) / 16;
  int tpi = (int)std::min<int64_t>(64, std::max<int64_t>(4, (ntiles * nsl + kWideTargetItems - 1) / kWideTargetItems));
  tpi = (tpi + 3) & ~3;
  const size_t stride = bta_partial_floats(M, 16 * DB, false);
  const size_t b_part = align256(sizeof(float) * stride * nparts);
  const size_t b_h0 = align256(sizeof(double) * M * kWideSlice);
  const size_t b_g32 = align256(sizeof(float) * M * kWideSlice);
  const size_t b_gt = align256(sizeof(__bf16) * 2 * kWideSlice * M);
  const size_t per = b_part + b_h0 + b_g32 + b_gt;
  std::vector<CloudDesc> cl(nsl);
  std::vector<int2> wb, we;
  if (hipMalloc(&w->arena, per * nsl) != hipSuccess) return RFD_ERR_DEVICE;
  char* base = (char*)w->arena;
  for (int s = 0; s < nsl; ++s) {
    char* a = base + per * s;
    CloudDesc& c = cl[s];
    c.X = p->dev.X;
    c.Xcopy = nullptr;
    c.N = N;
    c.om = p->dev.om;
    if (diag_of) {  // the slice's part of the diagonal, and its first column
      c.F = diag_of + (size_t)s * kWideSlice;
      c.ldF = (int64_t)s * kWideSlice;
    } else {
      c.F = F ? F + (size_t)s * kWideSlice : nullptr;
      c.ldF = ldF;
    }
    c.out = out ? out + (size_t)s * kWideSlice * (trans_out ? (size_t)ldO : 1) : nullptr;
    c.ldO = ldO;
    c.partials = (float*)a;
    c.lvl = nullptr;  // nparts <= fused_reduce_max_parts(): one-launch reduction
    c.Mraw = nullptr;  // no Gram
    c.H0 = (double*)(a + b_part);
    c.T64 = p->dev.T64;
    c.G32 = (float*)(a + b_part + b_h0);
    c.Gt16 = (__bf16*)(a + b_part + b_h0 + b_g32);
    c.flag = p->dev.flag;
    c.d = std::min(kWideSlice, d - s * kWideSlice);
    c.nparts = nparts;
    for (int b = 0; b < nparts; ++b) wb.push_back(make_int2(s, b));
    for (int64_t t0 = 0; t0 < ntiles; t0 += tpi) we.push_back(make_int2(s, (int)t0));
  }
  w->p = p;
  w->N = N;
  w->d = d;
  w->nsl = nsl;
  w->DB = DB;
  w->nparts = nparts;
  w->tpi = tpi;
  w->tout = trans_out;
  w->diag = diag_of;
  w->nwork_bta = (int)wb.size();
  w->nwork_exp = (int)we.size();
  bool ok = hipMalloc((void**)&w->dcl, sizeof(CloudDesc) * nsl) == hipSuccess &&
            hipMalloc((void**)&w->dwork_bta, sizeof(int2) * wb.size()) == hipSuccess &&
            hipMalloc((void**)&w->dwork_exp, sizeof(int2) * we.size()) == hipSuccess &&
            hipMemcpy(w->dcl, cl.data(), sizeof(CloudDesc) * nsl, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(w->dwork_bta, wb.data(), sizeof(int2) * wb.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(w->dwork_exp, we.data(), sizeof(int2) * we.size(), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    wide_free(w);
    return RFD_ERR_DEVICE;
  }
  return RFD_OK;
}

size_t wide_device_bytes(const WideField* w) {
  if (!w->arena) return 0;
  const int M = w->p->dev_m;
  const size_t per = align256(sizeof(float) * bta_partial_floats(M, 16 * w->DB, false) * w->nparts) +
                     align256(sizeof(double) * M * kWideSlice) + align256(sizeof(float) * M * kWideSlice) +
                     align256(sizeof(__bf16) * 2 * kWideSlice * M);
  return per * w->nsl + sizeof(CloudDesc) * w->nsl + sizeof(int2) * (w->nwork_bta + w->nwork_exp);
}

hipError_t wide_set_input(WideField* w, const float* F, int64_t ldF, hipStream_t st) {
  if (F == w->cur_in && ldF == w->cur_ld) return hipSuccess;  // already points there (stream order)
  const hipError_t e = launch_wide_patch(w->dcl, w->nsl, F, ldF, kWideSlice, st);
  if (e == hipSuccess) {
    w->cur_in = F;
    w->cur_ld = ldF;
  }
  return e;
}

hipError_t wide_set_output_epilogue(WideField* w, float* out, int64_t ldO, const float* a, const float* b,
                                    hipStream_t st) {
  if (!w->tout || !a || !b) return hipErrorInvalidValue;
  w->epi = true;
  if (out == w->cur_out && ldO == w->cur_ld && a == w->cur_in) return hipSuccess;  // already set (stream order)
  const hipError_t e = launch_wide_patch_out(w->dcl, w->nsl, out, ldO, a, b, kWideSlice, st);
  if (e == hipSuccess) {
    w->cur_out = out;
    w->cur_ld = ldO;
    w->cur_in = a;
  }
  return e;
}

// Split-N B^T F of every slice, the reduction and G' = T H0.
static hipError_t wide_core(const WideField* w, hipStream_t st) {
  const int M = w->p->dev_m, prec = w->p->params.precision;
  hipError_t e = launch_bta_batch(M, prec, w->DB, false, w->dcl, w->dwork_bta, w->nwork_bta, st);
  if (e == hipSuccess) e = launch_reduce_batch(M, w->DB, false, w->dcl, w->nsl, w->nparts, st);
  if (e == hipSuccess) e = launch_gcore_batch(M, std::min(w->d, kWideSlice), w->dcl, w->nsl, st);
  return e;
}

hipError_t wide_enqueue(const WideField* w, hipStream_t st) {
  hipError_t e = wide_core(w, st);
  if (e == hipSuccess)
    e = launch_expand_batch(w->p->dev_m, w->p->params.precision, w->DB, w->dcl, w->dwork_exp, w->nwork_exp, w->tpi, st,
                            w->tout, false, w->epi);
  return e;
}

hipError_t wide_diag_field_enqueue(const WideField* w, hipStream_t st) {
  if (!w->diag) return hipErrorInvalidValue;
  const int M = w->p->dev_m, prec = w->p->params.precision;
  hipError_t e = launch_wide_diag_h0(M, w->dcl, w->N, w->diag, st);
  if (e == hipSuccess) e = launch_gcore_batch(M, std::min(w->d, kWideSlice), w->dcl, w->nsl, st);
  if (e == hipSuccess) e = launch_expand_batch(M, prec, w->DB, w->dcl, w->dwork_exp, w->nwork_exp, w->tpi, st, true, true);
  return e;
}

hipError_t wide_diag_enqueue(const WideField* w, float* v, hipStream_t st) {
  if ((int64_t)w->d != w->N) return hipErrorInvalidValue;
  hipError_t e = wide_core(w, st);
  if (e == hipSuccess) e = launch_wide_diag(w->p->dev_m, w->dcl, w->N, v, st);
  return e;
}

}  // namespace rfd
