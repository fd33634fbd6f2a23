// Spectrum of the RFD kernel matrix from the plan's low-rank factors
// (k_spectrum.hip): the entry points check their arguments on the host and
// enqueue one kernel with one workgroup per cloud.
#include "rfd_internal.h"

#include <mutex>
#include <vector>

namespace {

// Device copies of the batched argument records: one grow-only buffer per
// device, reused by every call (each call waits for its launch before it
// returns, and the mutex keeps concurrent calls from sharing it), so a call
// allocates only when it has more clouds than any earlier call on the device.
struct RecordCache {
  std::mutex mu;
  std::vector<void*> buf;
  std::vector<size_t> cap;
};

RecordCache& records() {
  static RecordCache c;
  return c;
}

}  // namespace

namespace rfd {

void release_spectrum_records() {
  RecordCache& c = records();
  std::lock_guard<std::mutex> g(c.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (size_t dev = 0; dev < c.buf.size(); ++dev) {
    if (!c.buf[dev]) continue;
    (void)hipSetDevice((int)dev);
    (void)hipFree(c.buf[dev]);
    c.buf[dev] = nullptr;
    c.cap[dev] = 0;
  }
  (void)hipSetDevice(cur);
}

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
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return RFD_ERR_DEVICE;
  RecordCache& c = records();
  std::lock_guard<std::mutex> g(c.mu);
  if (c.buf.size() <= (size_t)dev) {
    c.buf.resize(dev + 1, nullptr);
    c.cap.resize(dev + 1, 0);
  }
  const size_t bytes = sizeof(rfd::SpecArgs) * n;
  if (c.cap[dev] < bytes) {
    size_t want = c.cap[dev] ? 2 * c.cap[dev] : sizeof(rfd::SpecArgs) * 64;
    while (want < bytes) want *= 2;
    if (c.buf[dev]) (void)hipFree(c.buf[dev]);  // the previous call waited for its launch
    c.buf[dev] = nullptr;
    c.cap[dev] = 0;
    if (hipMalloc(&c.buf[dev], want) != hipSuccess) return RFD_ERR_DEVICE;
    c.cap[dev] = want;
  }
  rfd::SpecArgs* dargs = (rfd::SpecArgs*)c.buf[dev];
  hipError_t e = hipMemcpyAsync(dargs, args.data(), bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = rfd::launch_spectrum_batch(dargs, n, max_m, st);
  // the records are reused by the next call, and the host copy is released on return
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? RFD_OK : RFD_ERR_DEVICE;
}

}  // extern "C"
