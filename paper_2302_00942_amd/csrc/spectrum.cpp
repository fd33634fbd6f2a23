// Spectrum of the RFD kernel matrix from the plan's low-rank factors
// (k_spectrum.hip): the entry point checks its arguments on the host and
// enqueues one single-workgroup kernel.
#include "rfd_internal.h"

namespace rfd {
hipError_t launch_spectrum(rfd_plan_s* p, int which, int64_t k, double* out, hipStream_t st);
}  // namespace rfd

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

}  // extern "C"
