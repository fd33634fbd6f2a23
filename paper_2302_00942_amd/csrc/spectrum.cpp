// Spectrum of the RFD kernel matrix from the plan's low-rank factors
// (k_spectrum.hip): the entry points check their arguments on the host and
// enqueue one kernel with one workgroup per cloud.
#include "rfd_internal.h"

#include <vector>

extern "C" {

rfd_status rfd_plan_spectrum(rfd_plan_t p, int32_t which, int64_t k, double* out, rfd_stream_t stream) {
  if (!p || (which != 0 && which != 1) || k < 0) return RFD_ERR_INVALID_ARG;
  if (p->N < 0) return RFD_ERR_NOT_READY;
  if (k > p->N) return RFD_ERR_INVALID_ARG;
  if (k == 0) return RFD_OK;
  if (!out) return RFD_ERR_INVALID_ARG;
  for (double w : p->w)
    if (w < 0.0) return RFD_ERR_INVALID_ARG;  // signed weights: B^T A is not symmetric
  return rfd::launch_spectrum(p, which, k, out, (hipStream_t)stream) == hipSuccess ? RFD_OK : RFD_ERR_DEVICE;
}

rfd_status rfd_spectrum_batch(const rfd_plan_t* plans, int32_t n, int32_t which, int64_t k, double* const* outs,
                              rfd_stream_t stream) {
  if (!plans || n < 0 || (which != 0 && which != 1) || k < 0 || (n > 0 && !outs)) return RFD_ERR_INVALID_ARG;
  if (n == 0 || k == 0) return RFD_OK;
  std::vector<rfd::SpecArgs> args;
  int max_m = 0;
  for (int i = 0; i < n; ++i) {
    rfd_plan_s* p = plans[i];
    if (!p || !outs[i]) return RFD_ERR_INVALID_ARG;
    if (p->N < 0) return RFD_ERR_NOT_READY;
    if (k > p->N) return RFD_ERR_INVALID_ARG;
    for (int j = 0; j < i; ++j)
      if (plans[j] == p) return RFD_ERR_INVALID_ARG;  // one workspace per plan
    for (double w : p->w)
      if (w < 0.0) return RFD_ERR_INVALID_ARG;
    args.push_back(rfd::spectrum_args(p, which, k, outs[i]));
    max_m = p->m > max_m ? p->m : max_m;
  }
  hipStream_t st = (hipStream_t)stream;
  rfd::SpecArgs* dargs = nullptr;
  if (hipMalloc((void**)&dargs, sizeof(rfd::SpecArgs) * n) != hipSuccess) return RFD_ERR_DEVICE;
  hipError_t e = hipMemcpyAsync(dargs, args.data(), sizeof(rfd::SpecArgs) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = rfd::launch_spectrum_batch(dargs, n, max_m, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the records (and the host copy) are released below
  (void)hipFree(dargs);
  return e == hipSuccess ? RFD_OK : RFD_ERR_DEVICE;
}

}  // extern "C"
