// Autotuner of launch geometry. The knobs here change how work is spread over
// workgroups, never which operations a result is made of, so any setting
// gives bit-identical results; only speed differs. A process-wide table maps
// (knob, padded m, precision, channel blocks, floor(log2 N)) to the value
// measured fastest; entries come from rfd_autotune / rfd_batch_tune or from
// rfd_tune_import of a table exported on the same kind of device. Untuned
// keys fall back to fixed defaults.
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "rfd_internal.h"

namespace rfd {
namespace {

using Key = std::tuple<int, int, int, int, int>;

struct Table {
  std::mutex mu;
  std::map<Key, int> v;
};

Table& table() {
  static Table t;
  return t;
}

int log2_bucket(int64_t N) {
  int b = 0;
  while (N > 1) {
    N >>= 1;
    ++b;
  }
  return b;
}

}  // namespace

int tuned(int knob, int M, int prec, int DB, int64_t N, int fallback) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  auto it = t.v.find(Key{knob, M, prec, DB, log2_bucket(N)});
  return it == t.v.end() ? fallback : it->second;
}

void set_tuned(int knob, int M, int prec, int DB, int64_t N, int value) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  t.v[Key{knob, M, prec, DB, log2_bucket(N)}] = value;
}

// Default from tuning runs on MI355X: one tile per wave at every size and
// precision (the expansion keeps 8 waves per SIMD resident).
int default_expand_tiles_per_wave(int64_t N, int prec) {
  (void)N;
  (void)prec;
  return 1;
}
int default_batch_tiles_per_item() { return 64; }

}  // namespace rfd

#define HIPCK(x)                                  \
  do {                                            \
    if ((x) != hipSuccess) return RFD_ERR_DEVICE; \
  } while (0)

extern "C" {

rfd_status rfd_autotune(rfd_plan_t p, const float* F, int64_t ldF, int32_t d, float* out, int64_t ldO, int32_t reps,
                        rfd_stream_t stream) {
  if (!p || reps < 1 || !rfd::plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
  if (p->N < 0) return RFD_ERR_NOT_READY;
  rfd_status s = rfd::check_field_args(p->N, F, ldF, d, out, ldO);
  if (s != RFD_OK) return s;
  if (d == 0 || p->N == 0) return RFD_OK;
  if ((const float*)out == F) return RFD_ERR_INVALID_ARG;  // the expansion is re-run: out must not alias F
  hipStream_t st = (hipStream_t)stream;
  s = rfd::ensure_core(p, st);
  if (s != RFD_OK) return s;
  const int M = p->dev_m, prec = p->params.precision;
  const int64_t N = p->N;
  // G of the first channel slice, then each candidate expansion of that slice
  const int dc = d < rfd::slice_width(M, false) ? d : rfd::slice_width(M, false);
  s = rfd::ensure_partials(p, rfd::partial_floats_needed(p, N, dc, false), st);
  if (s != RFD_OK) return s;
  HIPCK(rfd::launch_bta(p, p->dev.X, N, F, ldF, dc, false, st));
  HIPCK(rfd::launch_reduce(p, N, dc, false, st));
  HIPCK(rfd::launch_gcore(p, dc, st));
  const int DB = rfd::dblocks(dc);
  const int prev = rfd::tuned(rfd::kTuneExpandTilesPerWave, M, prec, DB, N, rfd::default_expand_tiles_per_wave(N, prec));
  static const int cands[] = {1, 2, 4, 8, 16};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RFD_ERR_DEVICE;
  }
  int best = 0;
  float best_ms = 1e30f;
  bool ok = true;
  for (int c = 0; ok && c < (int)(sizeof(cands) / sizeof(cands[0])); ++c) {
    rfd::set_tuned(rfd::kTuneExpandTilesPerWave, M, prec, DB, N, cands[c]);
    ok = rfd::launch_expand(p, p->dev.X, N, F, ldF, dc, out, ldO, nullptr, st) == hipSuccess &&
         hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r)
      ok = rfd::launch_expand(p, p->dev.X, N, F, ldF, dc, out, ldO, nullptr, st) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && ms < best_ms) {
      best_ms = ms;
      best = cands[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  rfd::set_tuned(rfd::kTuneExpandTilesPerWave, M, prec, DB, N, ok && best ? best : prev);
  if (!ok || best == 0) return RFD_ERR_DEVICE;
  // fields of at most kValuMaxD channels: matrix-core or FMA arithmetic of the
  // expansion, whichever runs faster (this knob does change the rounding;
  // both paths are within the precision's bar, and single and batched calls
  // read the same entry)
  if (d <= rfd::kValuMaxD) {
    float path_ms[2] = {1e30f, 1e30f};
    const int path_prev = rfd::expand_path(M, prec, d);
    const int paths[2] = {rfd::kExpandMfma, rfd::kExpandValu};
    e0 = e1 = nullptr;
    ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    for (int q = 0; ok && q < 2; ++q) {
      rfd::set_tuned(rfd::kTuneExpandPath, M, prec, 1, (int64_t)1 << d, paths[q]);
      ok = rfd::launch_expand(p, p->dev.X, N, F, ldF, dc, out, ldO, nullptr, st) == hipSuccess &&
           hipEventRecord(e0, st) == hipSuccess;
      for (int r = 0; ok && r < reps; ++r)
        ok = rfd::launch_expand(p, p->dev.X, N, F, ldF, dc, out, ldO, nullptr, st) == hipSuccess;
      ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&path_ms[q], e0, e1) == hipSuccess;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    rfd::set_tuned(rfd::kTuneExpandPath, M, prec, 1, (int64_t)1 << d,
                   ok ? (path_ms[1] < path_ms[0] ? rfd::kExpandValu : rfd::kExpandMfma) : path_prev);
    if (!ok) return RFD_ERR_DEVICE;
  }
  // leave the full result in out
  return rfd::integrate_enqueue(p, F, ldF, d, out, ldO, st, 0, nullptr);
}

rfd_status rfd_autotune_phi1(rfd_plan_t p, int32_t reps, rfd_stream_t stream) {
  if (!p || reps < 1) return RFD_ERR_INVALID_ARG;
  if (p->N < 0) return RFD_ERR_NOT_READY;
  if (p->N == 0) return RFD_OK;
  hipStream_t st = (hipStream_t)stream;
  const int M = p->dev_m, nt = rfd::phi1_grid_workers_max(p);
  const int prev = rfd::tuned(rfd::kTunePhi1Workgroups, M, 0, 1, 0, nt);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RFD_ERR_DEVICE;
  }
  int best = 0;
  float best_ms = 1e30f;
  bool ok = true;
  // phi_1 reads the plan's core and rewrites S and T with the same values
  for (int nw = nt; ok && nw >= 2 && nw * 4 >= nt; nw = nw * 3 / 4) {
    rfd::set_tuned(rfd::kTunePhi1Workgroups, M, 0, 1, 0, nw);
    ok = rfd::launch_phi1(p, st) == hipSuccess && hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r) ok = rfd::launch_phi1(p, st) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && ms < best_ms) {
      best_ms = ms;
      best = nw;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  rfd::set_tuned(rfd::kTunePhi1Workgroups, M, 0, 1, 0, ok && best ? best : prev);
  if (ok) p->core_ready = true;  // the runs formed S and T
  return ok && best ? RFD_OK : RFD_ERR_DEVICE;
}

int32_t rfd_tune_export(char* buf, int32_t cap) {
  rfd::Table& t = rfd::table();
  std::string txt;
  {
    std::lock_guard<std::mutex> g(t.mu);
    char line[96];
    for (const auto& kv : t.v) {
      snprintf(line, sizeof(line), "%d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
               std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first), kv.second);
      txt += line;
    }
  }
  const int32_t need = (int32_t)txt.size() + 1;
  if (buf && cap >= need) memcpy(buf, txt.c_str(), (size_t)need);
  return need;
}

rfd_status rfd_tune_import(const char* text) {
  if (!text) return RFD_ERR_INVALID_ARG;
  std::map<rfd::Key, int> parsed;
  const char* q = text;
  while (*q) {
    int k, m, pr, db, nb, v, used = 0;
    while (*q == '\n' || *q == ' ') ++q;
    if (!*q) break;
    if (sscanf(q, "%d %d %d %d %d %d%n", &k, &m, &pr, &db, &nb, &v, &used) != 6) return RFD_ERR_INVALID_ARG;
    if (k < 0 || k >= rfd::kNumTuneKnobs || (m != 64 && m != 128 && m != 256) || (pr != 0 && pr != 1) ||
        (db != 1 && db != 2 && db != 4) || nb < 0 || nb > 62 || v < 1 || v > 4096)
      return RFD_ERR_INVALID_ARG;
    parsed[rfd::Key{k, m, pr, db, nb}] = v;
    q += used;
  }
  rfd::Table& t = rfd::table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const auto& kv : parsed) t.v[kv.first] = kv.second;
  return RFD_OK;
}

void rfd_tune_reset(void) {
  rfd::Table& t = rfd::table();
  std::lock_guard<std::mutex> g(t.mu);
  t.v.clear();
}

}  // extern "C"
