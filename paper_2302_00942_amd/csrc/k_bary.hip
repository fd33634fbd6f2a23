// Elementwise steps of the Wasserstein-barycenter iteration (App. D, Alg. 1)
// around the two RFD integrations of each iteration. The k scaling vectors
// and fields are N x k row-major FP32 (channel i = distribution i), so one
// integration acts on all k at once. One thread per point; the channels of a
// point are handled in order, as the oracle does.
#include "rfd_internal.h"

namespace rfd {
namespace {

// Adds this wave's floored counts to the 64-bit counter (one atomic per wave;
// an integer sum, so the total does not depend on the order).
__device__ __forceinline__ void count_floored(unsigned n, unsigned long long* ctr) {
  for (int o = 32; o >= 1; o >>= 1) n += __shfl_xor(n, o);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(ctr, (unsigned long long)n);
}

// max(y, rho x) when the floor is on (rho >= 0), counting the floored entries
__device__ __forceinline__ float floored(float y, float x, float rho, unsigned& n) {
  if (rho < 0.f) return y;
  const float lo = rho * x;
  if (y < lo) {
    ++n;
    return lo;
  }
  return y;
}

}  // namespace

// v = 1, F = a (x) v, counter cleared (first step of a launch)
__global__ void k_bary_init(const float* __restrict__ a, int64_t N, int k, float* __restrict__ v, float* __restrict__ F,
                            unsigned long long* __restrict__ ctr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) *ctr = 0ull;
  if (p >= N) return;
  const float ap = a[p];
  for (int i = 0; i < k; ++i) {
    v[p * k + i] = 1.f;
    F[p * k + i] = ap;
  }
}

// step 1: w^i = mu^i / K(a v^i) (K floored at rho a v^i), then F = a (x) w
// for the second integration (F holds a v on entry)
__global__ void k_bary_ratio(const float* __restrict__ a, const float* __restrict__ mus, int64_t ldmu, int64_t N,
                             int k, float rho, const float* __restrict__ K, float* __restrict__ F,
                             unsigned long long* __restrict__ ctr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned n = 0;
  if (p < N) {
    const float ap = a[p];
    for (int i = 0; i < k; ++i) {
      const float y = floored(K[p * k + i], F[p * k + i], rho, n);
      F[p * k + i] = ap * (mus[p * ldmu + i] / y);
    }
  }
  count_floored(n, ctr);
}

// steps 2-4: d^i = v^i K(a w^i) (K floored at rho a w^i), mu = prod_i (d^i)^alpha_i,
// v^i = v^i mu / d^i, and F = a (x) v for the next iteration's first integration
__global__ void k_bary_update(const float* __restrict__ a, int64_t N, int k, const float* __restrict__ alpha,
                              float rho, const float* __restrict__ K, float* __restrict__ v, float* __restrict__ F,
                              float* __restrict__ mu_out, unsigned long long* __restrict__ ctr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned n = 0;
  if (p < N) {
    float d[kMaxBaryInputs];
    float mu = 1.f;
    for (int i = 0; i < k; ++i) {
      d[i] = v[p * k + i] * floored(K[p * k + i], F[p * k + i], rho, n);
      mu = mu * powf(d[i], alpha[i]);
    }
    const float ap = a[p];
    for (int i = 0; i < k; ++i) {
      const float vi = v[p * k + i] * mu / d[i];
      v[p * k + i] = vi;
      F[p * k + i] = ap * vi;
    }
    mu_out[p] = mu;
  }
  count_floored(n, ctr);
}

static dim3 bary_grid(int64_t N) { return dim3((unsigned)((N + 255) / 256 > 0 ? (N + 255) / 256 : 1)); }

hipError_t launch_bary_init(const float* a, int64_t N, int k, float* v, float* F, unsigned long long* ctr,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_bary_init, bary_grid(N), dim3(256), 0, st, a, N, k, v, F, ctr);
  return hipGetLastError();
}

hipError_t launch_bary_ratio(const float* a, const float* mus, int64_t ldmu, int64_t N, int k, float rho,
                             const float* K, float* F, unsigned long long* ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_bary_ratio, bary_grid(N), dim3(256), 0, st, a, mus, ldmu, N, k, rho, K, F, ctr);
  return hipGetLastError();
}

hipError_t launch_bary_update(const float* a, int64_t N, int k, const float* alpha, float rho, const float* K,
                              float* v, float* F, float* mu, unsigned long long* ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_bary_update, bary_grid(N), dim3(256), 0, st, a, N, k, alpha, rho, K, v, F, mu, ctr);
  return hipGetLastError();
}

}  // namespace rfd
