// Host side of the RFD library: parameter validation, the frequency sampler,
// importance weights, plan buffers and the single-cloud C ABI entry points.
//
// Built with -ffp-contract=off so that the sampler's float64 arithmetic is
// evaluated exactly as written (no fused multiply-adds).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "rfd_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
// First positive root of sin(u) - u cos(u): where the 3-D ball transform first
// changes sign. Main-lobe truncation radius = kU0 / (2 pi eps).
constexpr double kU0 = 4.493409457909064;
// Rejection sampling gives up after this many candidates (per frequency, plus
// a fixed allowance): a law whose truncation keeps almost no mass is refused.
constexpr int64_t kMaxCandidatesPerFrequency = 10000, kMaxCandidatesExtra = 1000000;

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): Weyl sequence with
// increment 0x9E3779B97F4A7C15, then the variant-13 mixer.
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

// Standard normals by Box-Muller on 53-bit uniforms: u1 in (0, 1],
// u2 in [0, 1); both outputs r cos(2 pi u2), r sin(2 pi u2) are used, in order.
struct Gaussian {
  SplitMix64 g;
  double spare = 0.0;
  bool has_spare = false;
  double next() {
    if (has_spare) {
      has_spare = false;
      return spare;
    }
    const uint64_t a = g.next(), b = g.next();
    const double u1 = (double)((a >> 11) + 1) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1));
    const double t = (2.0 * kPi) * u2;
    spare = r * sin(t);
    has_spare = true;
    return r * cos(t);
  }
};

// First positive zero of the Bessel function J_nu (nu >= 1/2): J_nu is
// positive on (0, j_{nu,1}) and j_{nu,1} > nu, so scan upward from nu in
// steps of 1/16 to the first sign change, then bisect it to the last bit.
double bessel_first_zero(double nu) {
  double a = nu, fa = std::cyl_bessel_j(nu, a);
  double b = a + 0.0625;
  while (std::cyl_bessel_j(nu, b) > 0.0) {
    a = b;
    b += 0.0625;
  }
  (void)fa;
  for (int i = 0; i < 200; ++i) {
    const double c = 0.5 * (a + b);
    if (c <= a || c >= b) break;
    if (std::cyl_bessel_j(nu, c) > 0.0) a = c;
    else b = c;
  }
  return 0.5 * (a + b);
}

void preset(const rfd_params& p, double* sigma, double* R) {
  if (p.sigma > 0.0 && p.radius > 0.0) {
    *sigma = p.sigma;
    *R = p.radius;
    return;
  }
  const int D = rfd::plan_dim(p);
  // main lobe of the ball: the first zero of its transform, j_{D/2,1} / (2 pi eps)
  const double r0 = (D == 3 ? kU0 : bessel_first_zero(0.5 * D)) / (2.0 * kPi);
  *R = (p.shape == RFD_BALL_L2) ? (r0 / p.eps) : (0.5 / p.eps);
  // R/3 in 3-D; R/sqrt(D + 6) in D dimensions (equal for D = 3), so that the
  // Gaussian's bulk, near radius sigma sqrt(D), stays inside R
  *sigma = D == 3 ? *R / 3.0 : *R / sqrt(D + 6.0);
}

// Fourier transform of the ball indicator 1[||z|| <= eps] in R^3 under
// f(z) = int exp(2 pi i w.z) tau(w) dw: (sin u - u cos u) / (2 pi^2 r^3),
// u = 2 pi eps r, with its Taylor series near the origin.
double tau_ball(double x, double y, double z, double eps) {
  const double r = sqrt(x * x + y * y + z * z);
  const double u = 2.0 * kPi * eps * r;
  const double vol = 4.0 * kPi * eps * eps * eps / 3.0;
  if (u < 1e-2) return vol * (1.0 - u * u / 10.0 + u * u * u * u / 280.0);
  return (sin(u) - u * cos(u)) / (2.0 * kPi * kPi * r * r * r);
}

// Transform of the box prod_i 1[|z_i| <= eps]: prod_i sin(2 pi eps w_i) / (pi w_i).
double tau_box(double x, double y, double z, double eps) {
  auto g = [eps](double w) {
    const double a = 2.0 * kPi * eps * w;
    if (fabs(a) < 1e-4) return 2.0 * eps * (1.0 - a * a / 6.0);
    return sin(a) / (kPi * w);
  };
  return g(x) * g(y) * g(z);
}

// P(N(0, I3) in the radius-t ball) (chi_3 CDF) or box (erf^3).
double trunc_mass(double t, int shape) {
  if (shape == RFD_BALL_L2) return erf(t / sqrt(2.0)) - sqrt(2.0 / kPi) * t * exp(-0.5 * t * t);
  const double e = erf(t / sqrt(2.0));
  return e * e * e;
}

// Regularised lower incomplete gamma P(a, x) = gamma(a, x) / Gamma(a):
// for x < a + 1 its power series x^a e^-x / Gamma(a + 1) sum_n x^n / ((a+1)..(a+n));
// otherwise 1 - Q(a, x) with Q from Legendre's continued fraction
// e^-x x^a / Gamma(a) * 1/(x + 1 - a - 1(1 - a)/(x + 3 - a - 2(2 - a)/(x + 5 - a - ...))),
// evaluated by the modified Lentz method.
double gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  const double lead = -x + a * log(x) - lgamma(a);
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 1000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (fabs(term) < fabs(sum) * 1e-17) break;
    }
    return sum * exp(lead);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 1000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return 1.0 - exp(lead) * h;
}

// Points in D dimensions. Transform of the D-ball indicator:
// eps^(D/2) J_{D/2}(2 pi eps r) / r^(D/2), the ball's volume
// pi^(D/2) eps^D / Gamma(D/2 + 1) at r = 0 and its two-term series for small u.
double tau_ball_nd(const double* w, int D, double eps) {
  double r2 = w[0] * w[0];
  for (int k = 1; k < D; ++k) r2 = r2 + w[k] * w[k];
  const double r = sqrt(r2), nu = 0.5 * D;
  const double u = 2.0 * kPi * eps * r;
  const double vol = pow(kPi, nu) * pow(eps, D) / tgamma(nu + 1.0);
  if (u < 1e-4) return vol * (1.0 - u * u / (4.0 * (nu + 1.0)));
  return pow(eps, nu) * std::cyl_bessel_j(nu, u) / pow(r, nu);
}
double tau_box_nd(const double* w, int D, double eps) {
  double t = 1.0;
  for (int k = 0; k < D; ++k) {
    const double a = 2.0 * kPi * eps * w[k];
    t *= fabs(a) < 1e-4 ? 2.0 * eps * (1.0 - a * a / 6.0) : sin(a) / (kPi * w[k]);
  }
  return t;
}
// P(N(0, I_D) in the radius-t ball): the chi_D CDF P(D/2, t^2/2); box: erf^D.
double trunc_mass_nd(double t, int shape, int D) {
  if (shape == RFD_BALL_L2) return gamma_p(0.5 * D, 0.5 * t * t);
  return pow(erf(t / sqrt(2.0)), D);
}

rfd_status check_params(const rfd_params* p) {
  if (!p) return RFD_ERR_INVALID_ARG;
  if (p->m < 2 || p->m > rfd::kMaxM || (p->m & 1)) return RFD_ERR_INVALID_ARG;
  if (!(p->eps > 0.0) || !isfinite(p->eps)) return RFD_ERR_INVALID_ARG;
  if (!isfinite(p->lambda)) return RFD_ERR_INVALID_ARG;
  if (p->shape != RFD_BALL_L2 && p->shape != RFD_BOX_LINF) return RFD_ERR_INVALID_ARG;
  if (p->precision != RFD_FP32 && p->precision != RFD_BF16) return RFD_ERR_INVALID_ARG;
  if (p->dim < 0 || p->dim > rfd::kMaxDim) return RFD_ERR_INVALID_ARG;
  const bool zs = p->sigma == 0.0, zr = p->radius == 0.0;
  if (zs != zr) return RFD_ERR_INVALID_ARG;
  if (!zs && !(p->sigma > 0.0 && p->radius > 0.0 && isfinite(p->sigma) && isfinite(p->radius)))
    return RFD_ERR_INVALID_ARG;
  return RFD_OK;
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc((void**)p, count * sizeof(T));
}

// Where a plan's buffers come from at creation: hipMalloc, or 256-byte
// aligned pieces of a caller's arena (base != nullptr; with base == nullptr
// and carving on, only the bytes are counted).
struct Source {
  bool carve = false;
  unsigned char* base = nullptr;
  size_t off = 0, cap = 0;
  template <class T>
  hipError_t get(T** p, size_t count) {
    if (!carve) return dalloc(p, count);
    *p = nullptr;
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    if (base && off + bytes > cap) return hipErrorOutOfMemory;
    if (base && count) *p = (T*)(base + off);
    off += bytes;
    return hipSuccess;
  }
};

void free_dev(rfd::PlanDev& d) {
  if (!d.external) {
    void* ptrs[] = {d.om, d.omD, d.cvec, d.svec, d.X, d.Mraw, d.H0, d.S64, d.T64, d.G32, d.Gt16, d.G64,
                    d.phi_ws, d.sdev, d.barrier, d.flag, d.lvl, d.partials};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
  }
  d = rfd::PlanDev{};
}

// Takes every fixed buffer of a plan with padded size M from `src`, and with
// an arena also the point copy and the partials for clouds of up to N_max
// points and fields of up to d_max channels (one-shot and resident passes).
hipError_t take_buffers(Source& src, rfd::PlanDev& d, int M, int prec, int64_t N_max, int d_max, int dim) {
  const int fp = M / 2;
  const size_t mm = (size_t)M * M;
  hipError_t e = hipSuccess;
  const auto ok = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  ok(src.get(&d.om, fp));
  if (dim != 3) ok(src.get(&d.omD, (size_t)fp * dim));
  ok(src.get(&d.cvec, M));
  ok(src.get(&d.svec, M));
  ok(src.get(&d.Mraw, mm));
  ok(src.get(&d.H0, (size_t)M * 64));
  ok(src.get(&d.S64, mm));
  ok(src.get(&d.T64, mm));
  ok(src.get(&d.G32, (size_t)M * 64));
  ok(src.get(&d.Gt16, (size_t)2 * M * 64));
  ok(src.get(&d.G64, (size_t)M * 32));
  ok(src.get(&d.phi_ws, rfd::phi1_ws_doubles(M)));
  ok(src.get(&d.sdev, 1));
  ok(src.get(&d.barrier, rfd::kBarrierWords));
  ok(src.get(&d.flag, 1));
  ok(src.get(&d.lvl, rfd::reduce_scratch_doubles(M)));
  if (src.carve) {
    const size_t pf = std::max(rfd::request_partial_floats(M, prec, N_max, d_max, true),
                               rfd::request_partial_floats(M, prec, N_max, d_max, false));
    if (dim == 3) ok(src.get(&d.X, (size_t)N_max * 3));  // no point copy in D != 3
    ok(src.get(&d.partials, pf));
    d.Xcap = N_max;
    d.partials_cap = pf;
    d.external = true;
  }
  return e;
}

// Frequencies (sampled from the seed, or taken from params->omega) and the
// weights w = tau / p at the float32 frequencies.
rfd_status sample_features(const rfd_params& prm, double sigma, double radius, std::vector<float>& omega,
                           std::vector<double>& w) {
  const int f = prm.m / 2;
  const int D = rfd::plan_dim(prm);
  omega.resize((size_t)f * D);
  if (prm.omega) {
    for (int i = 0; i < D * f; ++i) {
      if (!isfinite(prm.omega[i])) return RFD_ERR_INVALID_ARG;
      omega[i] = prm.omega[i];
    }
  } else if (D != 3) {
    // D normals per candidate, in stream order; squared norm summed in order
    Gaussian g{SplitMix64{prm.seed}};
    std::vector<double> cand(D);
    int k = 0;
    int64_t tries = 0;
    while (k < f) {
      if (++tries > kMaxCandidatesPerFrequency * f + kMaxCandidatesExtra) return RFD_ERR_INVALID_ARG;
      for (int i = 0; i < D; ++i) cand[i] = sigma * g.next();
      bool ok;
      if (prm.shape == RFD_BALL_L2) {
        double r2 = cand[0] * cand[0];
        for (int i = 1; i < D; ++i) r2 = r2 + cand[i] * cand[i];
        ok = r2 <= radius * radius;
      } else {
        double mx = 0.0;
        for (int i = 0; i < D; ++i) mx = std::max(mx, fabs(cand[i]));
        ok = mx <= radius;
      }
      if (ok) {
        for (int i = 0; i < D; ++i) omega[(size_t)k * D + i] = (float)cand[i];
        ++k;
      }
    }
  } else {
    Gaussian g{SplitMix64{prm.seed}};
    const double R = radius, sig = sigma;
    int k = 0;
    int64_t tries = 0;
    while (k < f) {
      if (++tries > kMaxCandidatesPerFrequency * f + kMaxCandidatesExtra) return RFD_ERR_INVALID_ARG;
      const double w0 = sig * g.next();
      const double w1 = sig * g.next();
      const double w2 = sig * g.next();
      bool ok;
      if (prm.shape == RFD_BALL_L2) ok = (w0 * w0 + w1 * w1) + w2 * w2 <= R * R;
      else ok = std::max(fabs(w0), std::max(fabs(w1), fabs(w2))) <= R;
      if (ok) {
        omega[3 * k] = (float)w0;
        omega[3 * k + 1] = (float)w1;
        omega[3 * k + 2] = (float)w2;
        ++k;
      }
    }
  }
  w.resize(f);
  if (D != 3) {
    const double C = trunc_mass_nd(radius / sigma, prm.shape, D);
    const double norm = pow(2.0 * kPi * sigma * sigma, -0.5 * D) / C;
    std::vector<double> wk(D);
    for (int k = 0; k < f; ++k) {
      double r2 = 0.0;
      for (int i = 0; i < D; ++i) {
        wk[i] = omega[(size_t)k * D + i];
        r2 += wk[i] * wk[i];
      }
      const double tau = prm.shape == RFD_BALL_L2 ? tau_ball_nd(wk.data(), D, prm.eps) : tau_box_nd(wk.data(), D, prm.eps);
      w[k] = tau / (norm * exp(-r2 / (2.0 * sigma * sigma)));
    }
    return RFD_OK;
  }
  const double C = trunc_mass(radius / sigma, prm.shape);
  const double norm = pow(2.0 * kPi * sigma * sigma, -1.5) / C;
  for (int k = 0; k < f; ++k) {
    const double x = omega[3 * k], y = omega[3 * k + 1], z = omega[3 * k + 2];
    const double tau = prm.shape == RFD_BALL_L2 ? tau_ball(x, y, z, prm.eps) : tau_box(x, y, z, prm.eps);
    const double pd = norm * exp(-(x * x + y * y + z * z) / (2.0 * sigma * sigma));
    w[k] = tau / pd;
  }
  return RFD_OK;
}

#define HIPCK(x)                           \
  do {                                     \
    if ((x) != hipSuccess) return RFD_ERR_DEVICE; \
  } while (0)

}  // namespace

// ------------------------------------------------------------------ internal helpers shared with the batch code
namespace rfd {

rfd_status ensure_partials(rfd_plan_s* p, size_t floats, hipStream_t st) {
  if (floats <= p->dev.partials_cap) return RFD_OK;
  if (p->dev.external) return RFD_ERR_OUT_OF_BUDGET;  // beyond the arena's sizing: never allocate
  if (p->dev.partials) {
    HIPCK(hipStreamSynchronize(st));
    HIPCK(hipFree(p->dev.partials));
    p->dev.partials = nullptr;
    p->dev.partials_cap = 0;
  }
  HIPCK(dalloc(&p->dev.partials, floats));
  p->dev.partials_cap = floats;
  return RFD_OK;
}

rfd_status ensure_x(rfd_plan_s* p, int64_t N, hipStream_t st) {
  if (N <= p->dev.Xcap) return RFD_OK;
  if (p->dev.external) return RFD_ERR_OUT_OF_BUDGET;
  if (p->dev.X) {
    HIPCK(hipStreamSynchronize(st));
    HIPCK(hipFree(p->dev.X));
    p->dev.X = nullptr;
    p->dev.Xcap = 0;
  }
  HIPCK(dalloc(&p->dev.X, (size_t)N * 3));
  p->dev.Xcap = N;
  return RFD_OK;
}

// Largest channel slice of one pass: fused Gram + B^T F keeps at most two
// channel blocks when m = 256 (register budget); otherwise four.
int slice_width(int dev_m, bool gram) { return (gram && dev_m == 256) ? 32 : 64; }

bool range_exceeded(const rfd_plan_s* p, int64_t N) {
  // ||lambda M||_2 <= |lambda| trace(|M|) = |lambda| N sum_k |w_k| / f, since
  // every feature pair contributes c_k^2 (cos^2 + sin^2) = |w_k| / f per point.
  return p->any_growth && fabs(p->params.lambda) * (double)N * p->wsum_abs / p->f > 700.0;
}

size_t partial_floats_needed(const rfd_plan_s* p, int64_t N, int d, bool gram) {
  return partial_floats_for(p->dev_m, p->params.precision, N, d, gram);
}

size_t partial_floats_for(int M, int prec, int64_t N, int d, bool gram) {
  return (size_t)bta_partials(N, M, d, gram, prec) * bta_partial_floats(M, d, gram);
}

size_t request_partial_floats(int M, int prec, int64_t N, int d, bool oneshot) {
  size_t need = 0;
  int c0 = 0;
  if (oneshot) {
    c0 = std::min(slice_width(M, true), d);
    need = partial_floats_for(M, prec, N, c0, true);
  }
  const int W = slice_width(M, false);
  for (; c0 < d; c0 += W) need = std::max(need, partial_floats_for(M, prec, N, std::min(W, d - c0), false));
  return need;
}

int padded_m(int m) { return m <= 64 ? 64 : (m <= 128 ? 128 : 256); }

rfd_status check_params(const rfd_params* p) { return ::check_params(p); }

void free_plan_device(rfd_plan_s* p) {
  free_dev(p->dev);
  delete p;
}

size_t plan_fixed_bytes(int M) {
  const size_t mm = (size_t)M * M;
  return sizeof(float4) * (M / 2) + 2 * sizeof(double) * M + 3 * sizeof(double) * mm +
         sizeof(double) * M * 64 + sizeof(float) * M * 64 + 2 * sizeof(__bf16) * M * 64 + sizeof(double) * M * 32 +
         sizeof(double) * phi1_ws_doubles(M) + 2 * sizeof(int) +
         sizeof(unsigned) * kBarrierWords + sizeof(double) * reduce_scratch_doubles(M);
}

size_t plan_device_bytes(const rfd_plan_s* p) {
  return plan_fixed_bytes(p->dev_m) + sizeof(float) * 3 * (size_t)p->dev.Xcap + sizeof(float) * p->dev.partials_cap;
}

// phi_1 either on the launch stream or, when `lane` is given, on the lane's
// stream between two event waits (the lane serialises the cooperative
// launches of concurrent requests).
static rfd_status enqueue_phi1(rfd_plan_s* p, hipStream_t st, const PhiLane* lane) {
  p->core_ready = true;
  if (!lane) {
    HIPCK(launch_phi1(p, st));
    return RFD_OK;
  }
  HIPCK(hipEventRecord(lane->before, st));
  HIPCK(hipStreamWaitEvent(lane->st, lane->before, 0));
  HIPCK(launch_phi1(p, lane->st));
  HIPCK(hipEventRecord(lane->after, lane->st));
  HIPCK(hipStreamWaitEvent(st, lane->after, 0));
  return RFD_OK;
}

rfd_status ensure_core(rfd_plan_s* p, hipStream_t st) {
  if (p->core_ready || p->N <= 0) return RFD_OK;
  return enqueue_phi1(p, st, nullptr);
}

rfd_status features_enqueue(rfd_plan_s* p, const float* X, int64_t N, hipStream_t st, const PhiLane* lane) {
  if (N < 0 || (N > 0 && !X)) return RFD_ERR_INVALID_ARG;
  if (range_exceeded(p, N)) return RFD_ERR_RANGE;
  p->N = N;
  if (N == 0) return RFD_OK;
  if (!plan_is_3d(p)) {
    // D-dimensional points: the Gram pass only (no point copy), then M and S
    rfd_status s = ensure_partials(p, partial_floats_needed(p, N, 0, true), st);
    if (s != RFD_OK) return s;
    HIPCK(launch_gram_nd(p, X, N, st));
    HIPCK(launch_reduce(p, N, 0, true, st));
    return enqueue_phi1(p, st, lane);
  }
  rfd_status s = ensure_x(p, N, st);
  if (s != RFD_OK) return s;
  s = ensure_partials(p, partial_floats_needed(p, N, 0, true), st);
  if (s != RFD_OK) return s;
  HIPCK(launch_bta(p, X, N, nullptr, 0, 0, true, st, p->dev.X));  // also copies X into the plan
  HIPCK(launch_reduce(p, N, 0, true, st));
  return enqueue_phi1(p, st, lane);
}

rfd_status integrate_enqueue(rfd_plan_s* p, const float* F, int64_t ldF, int d, float* out, int64_t ldO,
                             hipStream_t st, int first_channel_done, const float* rowscale) {
  if (!plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  const int M = p->dev_m;
  const int64_t N = p->N;
  const int W = slice_width(M, false);
  for (int c0 = first_channel_done; c0 < d; c0 += W) {
    const int dc = std::min(W, d - c0);
    rfd_status s = ensure_partials(p, partial_floats_needed(p, N, dc, false), st);
    if (s != RFD_OK) return s;
    HIPCK(launch_bta(p, p->dev.X, N, F + c0, ldF, dc, false, st));
    HIPCK(launch_reduce(p, N, dc, false, st));
    HIPCK(launch_gcore(p, dc, st));
    HIPCK(launch_expand(p, p->dev.X, N, F + c0, ldF, dc, out + c0, ldO, rowscale, st));
  }
  return RFD_OK;
}

rfd_status oneshot_enqueue(rfd_plan_s* p, const float* X, int64_t N, const float* F, int64_t ldF, int d,
                           float* out, int64_t ldO, hipStream_t st, const PhiLane* lane) {
  if (!plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  if (N < 0 || (N > 0 && !X)) return RFD_ERR_INVALID_ARG;
  rfd_status s = check_field_args(N, F, ldF, d, out, ldO);
  if (s != RFD_OK) return s;
  if (d == 0 || N == 0) return features_enqueue(p, X, N, st, lane);
  if (range_exceeded(p, N)) return RFD_ERR_RANGE;
  p->N = N;
  s = ensure_x(p, N, st);
  if (s != RFD_OK) return s;
  const int dc = std::min(slice_width(p->dev_m, true), d);
  s = ensure_partials(p, partial_floats_needed(p, N, dc, true), st);
  if (s != RFD_OK) return s;
  // pass 1 carries the Gram and the first channel slice of B^T F
  HIPCK(launch_bta(p, X, N, F, ldF, dc, true, st, p->dev.X));  // also copies X into the plan
  HIPCK(launch_reduce(p, N, dc, true, st));
  if (!lane && dc == d && d <= phi1_apply_max_width()) {
    // the whole field in one block: phi_1 in action form gives G directly
    HIPCK(launch_phi1_apply(p, d, st));
    p->core_ready = false;
  } else {
    s = enqueue_phi1(p, st, lane);
    if (s != RFD_OK) return s;
    HIPCK(launch_gcore(p, dc, st));
  }
  HIPCK(launch_expand(p, p->dev.X, N, F, ldF, dc, out, ldO, nullptr, st));
  return integrate_enqueue(p, F, ldF, d, out, ldO, st, dc, nullptr);
}

rfd_status check_field_args(int64_t N, const float* F, int64_t ldF, int d, const float* out, int64_t ldO) {
  if (d < 0 || d > kMaxD) return RFD_ERR_INVALID_ARG;
  if (d == 0 || N == 0) return RFD_OK;
  if (!F || !out || ldF < d || ldO < d) return RFD_ERR_INVALID_ARG;
  return RFD_OK;
}

}  // namespace rfd

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* rfd_status_string(rfd_status s) {
  switch (s) {
    case RFD_OK: return "ok";
    case RFD_ERR_INVALID_ARG: return "invalid argument";
    case RFD_ERR_RANGE: return "exp(lambda W) overflows float64";
    case RFD_ERR_OUT_OF_BUDGET: return "request does not fit the HBM budget";
    case RFD_ERR_NONFINITE: return "non-finite value in the input or the core";
    case RFD_ERR_DEVICE: return "HIP runtime error";
    case RFD_ERR_NOT_READY: return "not ready";
    case RFD_ERR_SHUTDOWN: return "server shut down";
  }
  return "unknown status";
}

}  // extern "C"

namespace {

rfd_status create_plan(const rfd_params* params, Source& src, int64_t N_max, int d_max, rfd_plan_t* out_plan) {
  if (!out_plan) return RFD_ERR_INVALID_ARG;
  *out_plan = nullptr;
  rfd_status st = check_params(params);
  if (st != RFD_OK) return st;
  rfd_plan_s* p = new (std::nothrow) rfd_plan_s();
  if (!p) return RFD_ERR_DEVICE;
  p->params = *params;
  p->m = params->m;
  p->f = params->m / 2;
  preset(*params, &p->sigma, &p->radius);
  const int f = p->f;
  st = sample_features(*params, p->sigma, p->radius, p->omega, p->w);
  if (st != RFD_OK) {
    delete p;
    return st;
  }
  p->wsum_abs = 0.0;
  p->any_growth = false;
  for (int k = 0; k < f; ++k) {
    p->wsum_abs += fabs(p->w[k]);
    if (params->lambda * p->w[k] > 0.0) p->any_growth = true;
  }

  const int M = rfd::padded_m(params->m);
  p->dev_m = M;
  const int fp = M / 2;
  (void)hipGetDevice(&p->device);
  rfd::PlanDev& d = p->dev;
  const int D = rfd::plan_dim(*params);
  const hipError_t te = take_buffers(src, d, M, params->precision, N_max, d_max, D);
  if (te != hipSuccess) {
    free_dev(d);
    delete p;
    return te == hipErrorOutOfMemory && src.carve ? RFD_ERR_OUT_OF_BUDGET : RFD_ERR_DEVICE;
  }
  bool ok = true;
  std::vector<float4> om(fp);
  std::vector<float> omD(D == 3 ? 0 : (size_t)fp * D, 0.f);  // padding rows stay zero
  std::vector<double> cv(M, 0.0), sv(M, 1.0);
  for (int k = 0; k < fp; ++k) {
    if (k < f && D != 3) {
      om[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int i = 0; i < D; ++i) omD[(size_t)k * D + i] = p->omega[(size_t)k * D + i];
      const double c = sqrt(fabs(p->w[k]) / f);
      cv[k] = c;
      cv[fp + k] = c;
      sv[k] = sv[fp + k] = p->w[k] < 0.0 ? -1.0 : 1.0;
    } else if (k < f) {
      om[k] = make_float4(p->omega[3 * k], p->omega[3 * k + 1], p->omega[3 * k + 2], 0.f);
      const double c = sqrt(fabs(p->w[k]) / f);
      cv[k] = c;
      cv[fp + k] = c;
      sv[k] = sv[fp + k] = p->w[k] < 0.0 ? -1.0 : 1.0;
    } else {
      om[k] = make_float4(0.f, 0.f, 0.f, 0.f);  // padding: zero-scaled columns
    }
  }
  int zero = 0;
  const std::vector<unsigned> zero_bar(rfd::kBarrierWords, 0u);
  ok = hipMemcpy(d.om, om.data(), sizeof(float4) * fp, hipMemcpyHostToDevice) == hipSuccess &&
       (D == 3 || hipMemcpy(d.omD, omD.data(), sizeof(float) * omD.size(), hipMemcpyHostToDevice) == hipSuccess) &&
       hipMemcpy(d.cvec, cv.data(), sizeof(double) * M, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.svec, sv.data(), sizeof(double) * M, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.flag, &zero, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.sdev, &zero, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
       // grid-barrier counters: zeroed once here; every phi_1 launch leaves them zero
       hipMemcpy(d.barrier, zero_bar.data(), sizeof(unsigned) * rfd::kBarrierWords, hipMemcpyHostToDevice) ==
           hipSuccess;
  if (!ok) {
    free_dev(d);
    delete p;
    return RFD_ERR_DEVICE;
  }
  *out_plan = p;
  return RFD_OK;
}

}  // namespace

extern "C" {

rfd_status rfd_plan_create(const rfd_params* params, rfd_plan_t* out_plan) {
  Source src;
  return create_plan(params, src, 0, 0, out_plan);
}

rfd_status rfd_plan_workspace_size(const rfd_params* params, int64_t N_max, int32_t d_max, size_t* bytes) {
  if (!bytes) return RFD_ERR_INVALID_ARG;
  *bytes = 0;
  rfd_status st = check_params(params);
  if (st != RFD_OK) return st;
  if (N_max < 0 || d_max < 0 || d_max > rfd::kMaxD) return RFD_ERR_INVALID_ARG;
  Source src;
  src.carve = true;
  rfd::PlanDev d;
  (void)take_buffers(src, d, rfd::padded_m(params->m), params->precision, N_max, d_max < 1 ? 1 : d_max,
                     rfd::plan_dim(*params));
  *bytes = src.off;
  return RFD_OK;
}

rfd_status rfd_plan_create_in(const rfd_params* params, void* arena_dev, size_t bytes, int64_t N_max, int32_t d_max,
                              rfd_plan_t* out_plan) {
  if (!out_plan) return RFD_ERR_INVALID_ARG;
  *out_plan = nullptr;
  if (!arena_dev || ((uintptr_t)arena_dev & 255) || N_max < 0 || d_max < 0 || d_max > rfd::kMaxD)
    return RFD_ERR_INVALID_ARG;
  Source src;
  src.carve = true;
  src.base = (unsigned char*)arena_dev;
  src.cap = bytes;
  return create_plan(params, src, N_max, d_max < 1 ? 1 : d_max, out_plan);
}

rfd_status rfd_params_frequencies(const rfd_params* params, float* omega_fx3, double* w_f) {
  rfd_status st = check_params(params);
  if (st != RFD_OK) return st;
  double sigma, R;
  preset(*params, &sigma, &R);
  std::vector<float> om;
  std::vector<double> w;
  st = sample_features(*params, sigma, R, om, w);
  if (st != RFD_OK) return st;
  if (omega_fx3) memcpy(omega_fx3, om.data(), sizeof(float) * om.size());
  if (w_f) memcpy(w_f, w.data(), sizeof(double) * w.size());
  return RFD_OK;
}

rfd_status rfd_plan_export(rfd_plan_t p, float* omega_fx3, double* w_f) {
  if (!p) return RFD_ERR_INVALID_ARG;
  if (omega_fx3) memcpy(omega_fx3, p->omega.data(), sizeof(float) * p->omega.size());
  if (w_f) memcpy(w_f, p->w.data(), sizeof(double) * p->w.size());
  return RFD_OK;
}

rfd_status rfd_features(rfd_plan_t p, const float* X_dev, int64_t N, rfd_stream_t stream) {
  if (!p) return RFD_ERR_INVALID_ARG;
  return rfd::features_enqueue(p, X_dev, N, (hipStream_t)stream, nullptr);
}

rfd_status rfd_features_sync(rfd_plan_t p, const float* X_dev, int64_t N, rfd_stream_t stream) {
  if (!p) return RFD_ERR_INVALID_ARG;
  const rfd_status s = rfd::features_enqueue(p, X_dev, N, (hipStream_t)stream, nullptr);
  if (s != RFD_OK) return s;
  return rfd_plan_check(p, stream);
}

rfd_status rfd_integrate(rfd_plan_t p, const float* F, int64_t ldF, int32_t d, float* out, int64_t ldO,
                         rfd_stream_t stream) {
  return rfd_integrate_scaled(p, F, ldF, d, out, ldO, nullptr, stream);
}

rfd_status rfd_integrate_scaled(rfd_plan_t p, const float* F, int64_t ldF, int32_t d, float* out, int64_t ldO,
                                const float* scale, rfd_stream_t stream) {
  if (!p || !rfd::plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  if (p->N < 0) return RFD_ERR_NOT_READY;
  rfd_status s = rfd::check_field_args(p->N, F, ldF, d, out, ldO);
  if (s != RFD_OK || d == 0 || p->N == 0) return s;
  s = rfd::ensure_core(p, (hipStream_t)stream);
  if (s != RFD_OK) return s;
  return rfd::integrate_enqueue(p, F, ldF, d, out, ldO, (hipStream_t)stream, 0, scale);
}

rfd_status rfd_integrate_oneshot(rfd_plan_t p, const float* X, int64_t N, const float* F, int64_t ldF, int32_t d,
                                 float* out, int64_t ldO, rfd_stream_t stream) {
  if (!p || !rfd::plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  return rfd::oneshot_enqueue(p, X, N, F, ldF, d, out, ldO, (hipStream_t)stream, nullptr);
}

rfd_status rfd_plan_check(rfd_plan_t p, rfd_stream_t stream) {
  if (!p) return RFD_ERR_INVALID_ARG;
  HIPCK(hipStreamSynchronize((hipStream_t)stream));
  int flag = 0, zero = 0;
  HIPCK(hipMemcpy(&flag, p->dev.flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) HIPCK(hipMemcpy(p->dev.flag, &zero, sizeof(int), hipMemcpyHostToDevice));
  if (flag & 1) return RFD_ERR_NONFINITE;
  if (flag & 2) return RFD_ERR_RANGE;
  if (flag & 4) return RFD_ERR_DEVICE;
  return RFD_OK;
}

rfd_status rfd_plan_core(rfd_plan_t p, double* M_out, double* S_out, int32_t* s_out, rfd_stream_t stream) {
  if (!p) return RFD_ERR_INVALID_ARG;
  if (p->N < 0) return RFD_ERR_NOT_READY;
  rfd_status st = rfd::ensure_core(p, (hipStream_t)stream);
  if (st != RFD_OK) return st;
  HIPCK(hipStreamSynchronize((hipStream_t)stream));
  const int M = p->dev_m, m = p->m, f = p->f, fp = M / 2;
  const size_t mm = (size_t)M * M;
  std::vector<double> raw(mm), S(mm);
  HIPCK(hipMemcpy(raw.data(), p->dev.Mraw, sizeof(double) * mm, hipMemcpyDeviceToHost));
  HIPCK(hipMemcpy(S.data(), p->dev.S64, sizeof(double) * mm, hipMemcpyDeviceToHost));
  int sv = 0;
  HIPCK(hipMemcpy(&sv, p->dev.sdev, sizeof(int), hipMemcpyDeviceToHost));
  // padded canonical index of real canonical index i: cos_k -> k, sin_k -> fp + k
  auto pidx = [&](int i) { return i < f ? i : fp + (i - f); };
  for (int i = 0; i < m; ++i) {
    const int wi = i < f ? i : i - f;
    const double ci = sqrt(fabs(p->w[wi]) / f);
    for (int j = 0; j < m; ++j) {
      const int wj = j < f ? j : j - f;
      const double cj = sqrt(fabs(p->w[wj]) / f), sj = p->w[wj] < 0.0 ? -1.0 : 1.0;
      const size_t q = (size_t)pidx(i) * M + pidx(j);
      if (M_out) M_out[(size_t)i * m + j] = p->N == 0 ? 0.0 : ci * raw[q] * cj * sj;
      if (S_out) S_out[(size_t)i * m + j] = S[q];
    }
  }
  if (s_out) *s_out = sv;
  return RFD_OK;
}

rfd_status rfd_plan_info(rfd_plan_t p, int64_t* N_out, int32_t* m_out, int32_t* padded_m_out) {
  if (!p) return RFD_ERR_INVALID_ARG;
  if (N_out) *N_out = p->N;
  if (m_out) *m_out = p->m;
  if (padded_m_out) *padded_m_out = p->dev_m;
  return RFD_OK;
}

rfd_status rfd_plan_action(rfd_plan_t p, double* H_out, double* G_out, int32_t* d_out, rfd_stream_t stream) {
  if (!p || !rfd::plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  if (p->N < 0 || p->action_d <= 0) return RFD_ERR_NOT_READY;
  HIPCK(hipStreamSynchronize((hipStream_t)stream));
  const int M = p->dev_m, m = p->m, f = p->f, fp = M / 2, d = p->action_d;
  constexpr int TW = 32;  // row pitch of G64
  std::vector<double> h0((size_t)M * d), g((size_t)M * TW);
  HIPCK(hipMemcpy(h0.data(), p->dev.H0, sizeof(double) * h0.size(), hipMemcpyDeviceToHost));
  HIPCK(hipMemcpy(g.data(), p->dev.G64, sizeof(double) * g.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < m; ++i) {
    const int k = i < f ? i : i - f;                  // frequency of canonical column i
    const int di = i < f ? 2 * k : 2 * k + 1;         // its device column
    const int pi = i < f ? i : fp + k;                // its padded canonical index
    const double c = sqrt(fabs(p->w[k]) / f);
    for (int j = 0; j < d; ++j) {
      if (H_out) H_out[(size_t)i * d + j] = c * h0[(size_t)di * d + j];
      if (G_out) G_out[(size_t)i * d + j] = g[(size_t)pi * TW + j];
    }
  }
  if (d_out) *d_out = d;
  return RFD_OK;
}

void rfd_plan_destroy(rfd_plan_t p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  free_dev(p->dev);
  delete p;
}

}  // extern "C"
