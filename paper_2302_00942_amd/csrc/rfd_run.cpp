// rfd_run: native driver of the C ABI for profiling runs.
//
//   rfd_run DIR STEPS [PREC]
//   rfd_run gw DIR STEPS [PREC]
//   rfd_run spectrum DIR STEPS M
//   rfd_run batch DIR STEPS [PREC]
//   rfd_run copy MIB
//
// DIR holds X.bin (N x 3 float32), F.bin (N x d float32) and meta.txt
// ("N d m eps lambda seed"), as written by `bench.py --dump-inputs DIR`.
// Runs STEPS one-shot integrations (PREC: bf16 or fp32, default bf16) on the
// default stream and prints the average milliseconds per step. The gw form
// reads Xc.bin (n x 3), Xd.bin (m x 3), T.bin (n x m) and meta_gw.txt
// ("n m feats eps lambda seed_c seed_d"), as written by `bench.py --dump-gw
// DIR`, and runs STEPS Gromov-Wasserstein loss matrices. The spectrum form
// reads Xs.bin (N x 3) and meta_spec.txt ("N k eps lambda seed"), as written
// by `bench.py --dump-spectrum DIR`, computes BF16 features with M features
// and runs STEPS spectrum calls (k smallest eigenvalues). The batch form
// reads Xb.bin and Fb.bin (the clouds' points and fields, concatenated) and
// meta_batch.txt ("count d m eps lambda", then "N seed" per cloud), as
// written by `bench.py --dump-batch DIR`, creates one batch over all clouds
// and times STEPS graph replays of it on a stream of its own. The copy form
// runs one device-to-device copy of MIB mebibytes (a reference kernel of
// known traffic for calibrating hardware byte counters).
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "rfd.h"

static bool read_file(const std::string& path, void* dst, size_t bytes) {
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) return false;
  const size_t got = fread(dst, 1, bytes, f);
  fclose(f);
  return got == bytes;
}

static int copy_mode(long long mib) {
  const size_t bytes = (size_t)mib << 20;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) return 1;
  if (hipMemset(a, 1, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 1;
  if (hipMemcpy(b, a, bytes, hipMemcpyDeviceToDevice) != hipSuccess) return 1;
  printf("rfd_run copy: %zu bytes\n", bytes);
  fflush(stdout);
  (void)hipFree(a);
  (void)hipFree(b);
  return 0;
}

static float* upload(const std::vector<float>& h) {
  float* d = nullptr;
  if (hipMalloc(&d, h.size() * 4) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), h.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return d;
}

static int gw_mode(const std::string& dir, int steps, int prec) {
  long long n = 0, m = 0;
  int feats = 0;
  double eps = 0, lam = 0;
  unsigned long long sc = 0, sd = 0;
  FILE* mf = fopen((dir + "/meta_gw.txt").c_str(), "r");
  if (!mf || fscanf(mf, "%lld %lld %d %lf %lf %llu %llu", &n, &m, &feats, &eps, &lam, &sc, &sd) != 7) {
    fprintf(stderr, "cannot read %s/meta_gw.txt\n", dir.c_str());
    return 1;
  }
  fclose(mf);
  if (n <= 0 || m <= 0 || steps <= 0) return 1;
  std::vector<float> Xc((size_t)n * 3), Xd((size_t)m * 3), T((size_t)n * m);
  if (!read_file(dir + "/Xc.bin", Xc.data(), Xc.size() * 4) || !read_file(dir + "/Xd.bin", Xd.data(), Xd.size() * 4) ||
      !read_file(dir + "/T.bin", T.data(), T.size() * 4)) {
    fprintf(stderr, "cannot read Xc.bin / Xd.bin / T.bin\n");
    return 1;
  }
  float *dXc = upload(Xc), *dXd = upload(Xd), *dT = upload(T), *dL = nullptr;
  if (!dXc || !dXd || !dT || hipMalloc(&dL, T.size() * 4) != hipSuccess) return 1;
  rfd_params p;
  memset(&p, 0, sizeof(p));
  p.m = feats;
  p.shape = RFD_BALL_L2;
  p.precision = prec;
  p.eps = eps;
  p.lambda = lam;
  rfd_plan_t pc = nullptr, pd = nullptr;
  rfd_gw_t g = nullptr;
  p.seed = sc;
  rfd_status st = rfd_plan_create(&p, &pc);
  p.seed = sd;
  if (st == RFD_OK) st = rfd_plan_create(&p, &pd);
  if (st == RFD_OK) st = rfd_features(pc, dXc, n, nullptr);
  if (st == RFD_OK) st = rfd_features(pd, dXd, m, nullptr);
  if (st == RFD_OK) st = rfd_gw_create(pc, pd, &g);
  if (st == RFD_OK) st = rfd_gw_loss(g, dT, m, dL, m, nullptr);  // untimed
  if (st == RFD_OK) st = rfd_plan_check(pc, nullptr);
  if (st != RFD_OK) {
    fprintf(stderr, "gw set-up: %s\n", rfd_status_string(st));
    return 1;
  }
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  (void)hipEventRecord(a, nullptr);
  for (int i = 0; i < steps && st == RFD_OK; ++i) st = rfd_gw_loss(g, dT, m, dL, m, nullptr);
  (void)hipEventRecord(b, nullptr);
  (void)hipEventSynchronize(b);
  if (st == RFD_OK) st = rfd_plan_check(pc, nullptr);
  if (st == RFD_OK) st = rfd_plan_check(pd, nullptr);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  printf("rfd_run gw n=%lld m=%lld feats=%d prec=%s steps=%d: %.4f ms/loss (%s)\n", n, m, feats,
         prec == RFD_BF16 ? "bf16" : "fp32", steps, ms / steps, rfd_status_string(st));
  fflush(stdout);
  rfd_gw_destroy(g);
  rfd_plan_destroy(pc);
  rfd_plan_destroy(pd);
  float* bufs[] = {dXc, dXd, dT, dL};
  for (float* q : bufs) (void)hipFree(q);
  return st == RFD_OK ? 0 : 1;
}

static int spectrum_mode(const std::string& dir, int steps, int m) {
  long long n = 0, k = 0;
  double eps = 0, lam = 0;
  unsigned long long seed = 0;
  FILE* mf = fopen((dir + "/meta_spec.txt").c_str(), "r");
  if (!mf || fscanf(mf, "%lld %lld %lf %lf %llu", &n, &k, &eps, &lam, &seed) != 5) {
    fprintf(stderr, "cannot read %s/meta_spec.txt\n", dir.c_str());
    return 1;
  }
  fclose(mf);
  if (n <= 0 || k <= 0 || k > n || steps <= 0 || m <= 0) return 1;
  std::vector<float> X((size_t)n * 3);
  if (!read_file(dir + "/Xs.bin", X.data(), X.size() * 4)) return 1;
  float* dX = upload(X);
  double* dOut = nullptr;
  if (!dX || hipMalloc(&dOut, sizeof(double) * k) != hipSuccess) return 1;
  rfd_params p;
  memset(&p, 0, sizeof(p));
  p.m = m;
  p.shape = RFD_BALL_L2;
  p.precision = RFD_BF16;
  p.eps = eps;
  p.lambda = lam;
  p.seed = seed;
  rfd_plan_t plan = nullptr;
  rfd_status st = rfd_plan_create(&p, &plan);
  if (st == RFD_OK) st = rfd_features(plan, dX, n, nullptr);
  if (st == RFD_OK) st = rfd_plan_spectrum(plan, 0, k, dOut, nullptr);  // untimed
  if (st == RFD_OK) st = rfd_plan_check(plan, nullptr);
  if (st != RFD_OK) {
    fprintf(stderr, "spectrum set-up: %s\n", rfd_status_string(st));
    return 1;
  }
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  (void)hipEventRecord(a, nullptr);
  for (int i = 0; i < steps && st == RFD_OK; ++i) st = rfd_plan_spectrum(plan, 0, k, dOut, nullptr);
  (void)hipEventRecord(b, nullptr);
  (void)hipEventSynchronize(b);
  if (st == RFD_OK) st = rfd_plan_check(plan, nullptr);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  printf("rfd_run spectrum N=%lld m=%d k=%lld steps=%d: %.4f ms/call (%s)\n", n, m, k, steps, ms / steps,
         rfd_status_string(st));
  fflush(stdout);
  rfd_plan_destroy(plan);
  (void)hipFree(dX);
  (void)hipFree(dOut);
  return st == RFD_OK ? 0 : 1;
}

static int batch_mode(const std::string& dir, int steps, int prec) {
  int count = 0, d = 0, m = 0;
  double eps = 0, lam = 0;
  FILE* mf = fopen((dir + "/meta_batch.txt").c_str(), "r");
  if (!mf || fscanf(mf, "%d %d %d %lf %lf", &count, &d, &m, &eps, &lam) != 5 || count <= 0 || d <= 0 || d > 64 ||
      steps <= 0) {
    fprintf(stderr, "cannot read %s/meta_batch.txt\n", dir.c_str());
    if (mf) fclose(mf);
    return 1;
  }
  std::vector<int64_t> Ns(count);
  std::vector<unsigned long long> seeds(count);
  long long total = 0;
  for (int i = 0; i < count; ++i) {
    long long n = 0;
    if (fscanf(mf, "%lld %llu", &n, &seeds[i]) != 2 || n <= 0) {
      fprintf(stderr, "bad cloud line %d\n", i);
      fclose(mf);
      return 1;
    }
    Ns[i] = n;
    total += n;
  }
  fclose(mf);
  std::vector<float> X((size_t)total * 3), F((size_t)total * d);
  if (!read_file(dir + "/Xb.bin", X.data(), X.size() * 4) || !read_file(dir + "/Fb.bin", F.data(), F.size() * 4)) {
    fprintf(stderr, "cannot read Xb.bin / Fb.bin\n");
    return 1;
  }
  float* dX = upload(X);
  float* dF = upload(F);
  float* dO = nullptr;
  if (!dX || !dF || hipMalloc(&dO, F.size() * 4) != hipSuccess) {
    fprintf(stderr, "device buffers failed\n");
    return 1;
  }
  std::vector<rfd_plan_t> plans(count, nullptr);
  std::vector<const float*> Xs(count), Fs(count);
  std::vector<float*> outs(count);
  std::vector<int64_t> lds(count, d);
  std::vector<int32_t> ds(count, d);
  size_t off = 0;
  rfd_status st = RFD_OK;
  for (int i = 0; i < count && st == RFD_OK; ++i) {
    rfd_params p;
    memset(&p, 0, sizeof(p));
    p.m = m;
    p.shape = RFD_BALL_L2;
    p.precision = prec;
    p.eps = eps;
    p.lambda = lam;
    p.seed = seeds[i];
    st = rfd_plan_create(&p, &plans[i]);
    Xs[i] = dX + off * 3;
    Fs[i] = dF + off * d;
    outs[i] = dO + off * d;
    off += (size_t)Ns[i];
  }
  rfd_batch_t batch = nullptr;
  if (st == RFD_OK)
    st = rfd_batch_create(plans.data(), Xs.data(), Ns.data(), Fs.data(), lds.data(), ds.data(), outs.data(),
                          lds.data(), count, &batch);
  hipStream_t s = nullptr;
  if (st == RFD_OK && hipStreamCreate(&s) != hipSuccess) st = RFD_ERR_DEVICE;
  // an eager launch, then the one that records the graph; the timed ones replay it
  for (int i = 0; i < 2 && st == RFD_OK; ++i) st = rfd_batch_launch(batch, s);
  if (st == RFD_OK && hipStreamSynchronize(s) != hipSuccess) st = RFD_ERR_DEVICE;
  float ms = 0.f;
  if (st == RFD_OK) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
    for (int i = 0; i < steps && st == RFD_OK; ++i) st = rfd_batch_launch(batch, s);
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  for (int i = 0; i < count && st == RFD_OK; ++i) st = rfd_plan_check(plans[i], s);
  printf("rfd_run batch clouds=%d points=%lld d=%d m=%d prec=%s steps=%d: %.4f ms/batch (%s)\n", count, total, d, m,
         prec == RFD_BF16 ? "bf16" : "fp32", steps, ms / steps, rfd_status_string(st));
  fflush(stdout);
  if (batch) rfd_batch_destroy(batch);
  for (rfd_plan_t p : plans)
    if (p) rfd_plan_destroy(p);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(dX);
  (void)hipFree(dF);
  (void)hipFree(dO);
  return st == RFD_OK ? 0 : 1;
}

// Where the library and the HIP runtime are mapped, so that frames of a
// crash report can be attributed to one of them (the symbols are looked up in
// the loaded libraries, not through this program's own call stubs).
static void print_load_addresses() {
  const char* libs[2][2] = {{"librfd.so", "rfd_plan_create"}, {"libamdhip64.so", "hipGetDeviceCount"}};
  for (auto& l : libs) {
    void* h = dlopen(l[0], RTLD_LAZY | RTLD_NOLOAD);
    void* sym = h ? dlsym(h, l[1]) : nullptr;
    Dl_info info{};
    if (sym && dladdr(sym, &info))
      fprintf(stderr, "rfd_run: %s mapped at %p\n", info.dli_fname, info.dli_fbase);
    if (h) dlclose(h);
  }
}

static int run(int argc, char** argv);

int main(int argc, char** argv) {
  print_load_addresses();
  const int rc = run(argc, argv);
  // nothing of the library's is left for the exit-time teardown
  rfd_library_release();
  fflush(stdout);
  fflush(stderr);
  return rc;
}

static int run(int argc, char** argv) {
  if (argc == 3 && strcmp(argv[1], "copy") == 0) return copy_mode(atoll(argv[2]));
  if (argc == 5 && strcmp(argv[1], "spectrum") == 0) return spectrum_mode(argv[2], atoi(argv[3]), atoi(argv[4]));
  if (argc >= 4 && strcmp(argv[1], "batch") == 0)
    return batch_mode(argv[2], atoi(argv[3]), (argc > 4 && strcmp(argv[4], "fp32") == 0) ? RFD_FP32 : RFD_BF16);
  if (argc >= 4 && strcmp(argv[1], "gw") == 0)
    return gw_mode(argv[2], atoi(argv[3]), (argc > 4 && strcmp(argv[4], "fp32") == 0) ? RFD_FP32 : RFD_BF16);
  if (argc < 3) {
    fprintf(stderr, "usage: %s DIR STEPS [bf16|fp32]\n", argv[0]);
    return 2;
  }
  const std::string dir = argv[1];
  const int steps = atoi(argv[2]);
  const int prec = (argc > 3 && strcmp(argv[3], "fp32") == 0) ? RFD_FP32 : RFD_BF16;
  long long N = 0;
  int d = 0, m = 0;
  double eps = 0, lam = 0;
  unsigned long long seed = 0;
  FILE* mf = fopen((dir + "/meta.txt").c_str(), "r");
  if (!mf || fscanf(mf, "%lld %d %d %lf %lf %llu", &N, &d, &m, &eps, &lam, &seed) != 6) {
    fprintf(stderr, "cannot read %s/meta.txt\n", dir.c_str());
    return 1;
  }
  fclose(mf);
  if (N <= 0 || d <= 0 || steps <= 0) {
    fprintf(stderr, "bad sizes\n");
    return 1;
  }
  std::vector<float> X((size_t)N * 3), F((size_t)N * d);
  if (!read_file(dir + "/X.bin", X.data(), X.size() * 4) || !read_file(dir + "/F.bin", F.data(), F.size() * 4)) {
    fprintf(stderr, "cannot read X.bin / F.bin\n");
    return 1;
  }
  float *dX = nullptr, *dF = nullptr, *dO = nullptr;
  if (hipMalloc(&dX, X.size() * 4) != hipSuccess || hipMalloc(&dF, F.size() * 4) != hipSuccess ||
      hipMalloc(&dO, F.size() * 4) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  if (hipMemcpy(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dF, F.data(), F.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "hipMemcpy failed\n");
    return 1;
  }
  rfd_params p;
  memset(&p, 0, sizeof(p));
  p.m = m;
  p.shape = RFD_BALL_L2;
  p.precision = prec;
  p.eps = eps;
  p.lambda = lam;
  p.seed = seed;
  rfd_plan_t plan = nullptr;
  rfd_status st = rfd_plan_create(&p, &plan);
  if (st != RFD_OK) {
    fprintf(stderr, "rfd_plan_create: %s\n", rfd_status_string(st));
    return 1;
  }
  // one untimed step (allocations), then the timed ones
  st = rfd_integrate_oneshot(plan, dX, N, dF, d, d, dO, d, nullptr);
  if (st == RFD_OK) st = rfd_plan_check(plan, nullptr);
  if (st != RFD_OK) {
    fprintf(stderr, "warm-up step: %s\n", rfd_status_string(st));
    return 1;
  }
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  (void)hipEventRecord(a, nullptr);
  for (int i = 0; i < steps && st == RFD_OK; ++i) st = rfd_integrate_oneshot(plan, dX, N, dF, d, d, dO, d, nullptr);
  (void)hipEventRecord(b, nullptr);
  (void)hipEventSynchronize(b);
  if (st == RFD_OK) st = rfd_plan_check(plan, nullptr);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  fflush(stderr);
  printf("rfd_run N=%lld d=%d m=%d prec=%s steps=%d: %.4f ms/step (%s)\n", N, d, m, prec == RFD_BF16 ? "bf16" : "fp32",
         steps, ms / steps, rfd_status_string(st));
  fflush(stdout);
  rfd_plan_destroy(plan);
  (void)hipFree(dX);
  (void)hipFree(dF);
  (void)hipFree(dO);
  return st == RFD_OK ? 0 : 1;
}
