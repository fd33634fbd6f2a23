// One-shot integration that allocates no device memory: every buffer the
// one-shot kernels use besides the caller's inputs and outputs (split-N
// partials, the reduced core and field block, the phi_1 workspace, G', the
// grid-barrier counters and the status flag) is carved out of one fixed
// device array of this file, `scratch`, so the call makes no hipMalloc, no
// hipFree and no allocating library call. For callers that cannot allocate
// (graph capture, tight serving loops). The kernels and the split of the
// cloud are those of rfd_integrate_oneshot, so the results are the same bits.
#include <mutex>

#include "rfd_internal.h"

// The one scratch array. In host code its name only stands in for the symbol:
// the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[(size_t)20 << 20];

namespace {

// Largest cloud and field: the fused first pass then covers the whole field
// (one channel slice), the cloud has at most 64 split-N partials (the
// one-launch reduction) and the points are read from the caller's X (the plan
// keeps no copy).
constexpr int64_t kMaxPoints = 65536;
constexpr size_t kScratchBytes = sizeof(scratch);
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

__global__ void k_zero_words(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// The plan's status flag takes the bits the call's kernels set.
__global__ void k_fold_flag(const int* from, int* into) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int f = *from;
    if (f) __hip_atomic_fetch_or(into, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Carves the buffers of a plan with padded feature count M out of `base`;
// returns the bytes used (256-byte aligned pieces).
size_t carve(unsigned char* base, int M, int prec, int d, rfd::PlanDev& o) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    unsigned char* q = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  const size_t mm = (size_t)M * M;
  o.Mraw = (double*)take(sizeof(double) * mm);
  o.H0 = (double*)take(sizeof(double) * M * 64);
  o.S64 = (double*)take(sizeof(double) * mm);
  o.T64 = (double*)take(sizeof(double) * mm);
  o.G32 = (float*)take(sizeof(float) * M * 64);
  o.Gt16 = (__bf16*)take(sizeof(__bf16) * 2 * M * 64);
  o.G64 = (double*)take(sizeof(double) * M * 32);
  o.phi_ws = (double*)take(sizeof(double) * rfd::phi1_ws_doubles(M));
  o.sdev = (int*)take(sizeof(int));
  o.flag = (int*)take(sizeof(int));
  o.barrier = (unsigned*)take(sizeof(unsigned) * rfd::kBarrierWords);
  const size_t floats = rfd::partial_floats_for(M, prec, kMaxPoints, d, true);
  o.partials = (float*)take(sizeof(float) * floats);
  o.partials_cap = floats;
  o.lvl = nullptr;  // at most 64 partials: the one-launch reduction
  o.X = nullptr;
  o.Xcap = 0;
  o.external = true;  // nothing may grow these buffers
  return off;
}

}  // namespace

extern "C" {

rfd_status rfd_integrate_oneshot_noalloc(rfd_plan_t p, const float* X, int64_t N, const float* F, int64_t ldF,
                                         int32_t d, float* out, int64_t ldO, rfd_stream_t stream) {
  if (!p || !rfd::plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  if (N < 0 || (N > 0 && !X)) return RFD_ERR_INVALID_ARG;
  rfd_status s = rfd::check_field_args(N, F, ldF, d, out, ldO);
  if (s != RFD_OK) return s;
  if (N == 0 || d == 0) return RFD_OK;
  const int M = p->dev_m;
  if (N > kMaxPoints || d > rfd::slice_width(M, true)) return RFD_ERR_OUT_OF_BUDGET;
  if (rfd::range_exceeded(p, N)) return RFD_ERR_RANGE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) return RFD_ERR_INVALID_ARG;
  unsigned char* base = (unsigned char*)scratch_address(dev);
  if (!base) return RFD_ERR_DEVICE;
  rfd::PlanDev sd;
  if (carve(base, M, p->params.precision, d, sd) > kScratchBytes) return RFD_ERR_OUT_OF_BUDGET;
  sd.om = p->dev.om;
  sd.cvec = p->dev.cvec;
  sd.svec = p->dev.svec;
  hipStream_t st = (hipStream_t)stream;
  // the call's kernels see the scratch buffers through the plan; the plan's
  // own buffers and state are restored before returning (nothing of its
  // resident cloud changes)
  const rfd::PlanDev own = p->dev;
  const int64_t own_N = p->N;
  const bool own_ready = p->core_ready;
  const int own_action = p->action_d;
  p->dev = sd;
  p->N = N;
  hipError_t e = hipSuccess;
  // counters and flag start at zero (a fill kernel: the call may be captured)
  const int nz = rfd::kBarrierWords;
  hipLaunchKernelGGL(k_zero_words, dim3((nz + 255) / 256), dim3(256), 0, st, sd.barrier, nz);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)sd.flag, 1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = rfd::launch_bta(p, X, N, F, ldF, d, true, st, nullptr);
  if (e == hipSuccess) e = rfd::launch_reduce(p, N, d, true, st);
  if (e == hipSuccess) {
    if (d <= rfd::phi1_apply_max_width()) {
      e = rfd::launch_phi1_apply(p, d, st);
    } else {
      e = rfd::launch_phi1(p, st);
      if (e == hipSuccess) e = rfd::launch_gcore(p, d, st);
    }
  }
  if (e == hipSuccess) e = rfd::launch_expand(p, X, N, F, ldF, d, out, ldO, nullptr, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fold_flag, dim3(1), dim3(64), 0, st, sd.flag, own.flag);
    e = hipGetLastError();
  }
  p->dev = own;
  p->N = own_N;
  p->core_ready = own_ready;
  p->action_d = own_action;
  return e == hipSuccess ? RFD_OK : RFD_ERR_DEVICE;
}

}  // extern "C"
