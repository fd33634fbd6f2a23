// Batched integration of many clouds: one launch per stage over a flattened
// (cloud, part) / (cloud, tile block) work list, recorded once into a
// hipGraph and replayed.
#include <string.h>

#include <algorithm>
#include <vector>

#include "rfd_internal.h"

struct rfd_batch_s {
  int n = 0, M = 0, prec = 0, DB = 1, dmax = 0, tpi = 64;
  int tpi_v = 64;  // tiles per item of the FMA-path expansion list (fixed at creation)
  bool aliased = false;  // some out aliases its F (the batch is then not re-runnable)
  int64_t total_n = 0;
  std::vector<int64_t> Ns;
  int exp_cap = 0;  // capacity of dwork_exp in items
  int max_parts = 0;  // largest split-N partition of the batch
  // phi_1 per cloud as the one-shot entry point takes it: in action form for
  // fields of at most phi1_apply_max_width() channels (no S), else S and G = S H
  int n_apply = 0, n_full = 0, dmax_full = 0;
  void* dargs_apply = nullptr;   // Phi1Args of the action-form clouds
  void* daargs = nullptr;        // their apply records
  rfd::CloudDesc* dcl_full = nullptr;  // descriptors of the other clouds (for G = S H)
  std::vector<bool> applied;     // per plan
  std::vector<rfd_plan_s*> plans;
  rfd::CloudDesc* dcl = nullptr;
  int2* dwork_bta = nullptr;
  int2* dwork_exp = nullptr;
  int2* dwork_expv = nullptr;    // expansion items of the clouds on the FMA path (expand_path)
  std::vector<bool> valu;        // per cloud: expansion on the FMA path
  int nwork_bta = 0, nwork_exp = 0, nwork_expv = 0;
  void* dargs = nullptr;
  int launches = 0;
  std::vector<const void*> bound;  // per plan: the X copy and partial buffers the work lists point into
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

#define HIPCK(x)                                  \
  do {                                            \
    if ((x) != hipSuccess) return RFD_ERR_DEVICE; \
  } while (0)

// Expansion work items: (cloud, first tile) every `tpi` tiles of 16 points,
// for the clouds whose flag in `on_valu` equals `valu`.
std::vector<int2> expand_work(const std::vector<int64_t>& Ns, int tpi, const std::vector<bool>& on_valu, bool valu) {
  std::vector<int2> we;
  for (int i = 0; i < (int)Ns.size(); ++i) {
    if (on_valu[i] != valu) continue;
    const int64_t ntiles = (Ns[i] + 15) / 16;
    for (int64_t t0 = 0; t0 < ntiles; t0 += tpi) we.push_back(make_int2(i, (int)t0));
  }
  return we;
}

// Reorders fixed-size records (and, with bsz > 0, a parallel record array)
// by descending N, ties in their original order.
void longest_first(std::vector<unsigned char>& a, size_t asz, std::vector<unsigned char>& b, size_t bsz,
                   const std::vector<int64_t>& Ns) {
  std::vector<int> idx(Ns.size());
  for (int i = 0; i < (int)idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return Ns[x] > Ns[y]; });
  std::vector<unsigned char> a2(a.size()), b2(b.size());
  for (size_t k = 0; k < idx.size(); ++k) {
    memcpy(a2.data() + k * asz, a.data() + idx[k] * asz, asz);
    if (bsz) memcpy(b2.data() + k * bsz, b.data() + idx[k] * bsz, bsz);
  }
  a.swap(a2);
  if (bsz) b.swap(b2);
}

void free_batch(rfd_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  void* ptrs[] = {b->dcl, b->dwork_bta, b->dwork_exp, b->dwork_expv, b->dargs, b->dargs_apply, b->daargs,
                  b->dcl_full};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete b;
}

rfd_status enqueue(rfd_batch_s* b, hipStream_t st) {
  HIPCK(rfd::launch_bta_batch(b->M, b->prec, b->DB, true, b->dcl, b->dwork_bta, b->nwork_bta, st));
  HIPCK(rfd::launch_reduce_batch(b->M, b->DB, true, b->dcl, b->n, b->max_parts, st));
  if (b->n_apply > 0) HIPCK(rfd::launch_phi1_apply_batch_dev(b->M, b->n_apply, b->dargs_apply, b->daargs, st));
  if (b->n_full > 0) {
    HIPCK(rfd::launch_phi1_batch_dev(b->M, b->n_full, b->dargs, st));
    HIPCK(rfd::launch_gcore_batch(b->M, b->dmax_full, b->dcl_full, b->n_full, st));
  }
  if (b->nwork_exp > 0)
    HIPCK(rfd::launch_expand_batch(b->M, b->prec, b->DB, b->dcl, b->dwork_exp, b->nwork_exp, b->tpi, st));
  if (b->nwork_expv > 0)
    HIPCK(rfd::launch_expand_valu_batch(b->M, b->prec, b->dcl, b->dwork_expv, b->nwork_expv, b->tpi_v, st));
  return RFD_OK;
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * src.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

}  // namespace

extern "C" {

rfd_status rfd_batch_create(const rfd_plan_t* plans, const float* const* Xs, const int64_t* Ns,
                            const float* const* Fs, const int64_t* ldFs, const int32_t* ds, float* const* outs,
                            const int64_t* ldOs, int32_t n, rfd_batch_t* out) {
  if (!out) return RFD_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 1 || !plans || !Xs || !Ns || !Fs || !ldFs || !ds || !outs || !ldOs) return RFD_ERR_INVALID_ARG;
  const int M = plans[0] ? plans[0]->dev_m : 0, prec = plans[0] ? plans[0]->params.precision : 0;
  int dmax = 0;
  for (int i = 0; i < n; ++i) {
    rfd_plan_s* p = plans[i];
    if (!p || p->dev_m != M || p->params.precision != prec || !rfd::plan_is_3d(p)) return RFD_ERR_INVALID_ARG;
    if (Ns[i] < 0 || ds[i] < 1 || ldFs[i] < ds[i] || ldOs[i] < ds[i]) return RFD_ERR_INVALID_ARG;
    if (Ns[i] > 0 && (!Xs[i] || !Fs[i] || !outs[i])) return RFD_ERR_INVALID_ARG;
    for (int j = 0; j < i; ++j)
      if (plans[j] == p) return RFD_ERR_INVALID_ARG;  // each cloud needs its own plan
    dmax = std::max(dmax, (int)ds[i]);
  }
  for (int i = 0; i < n; ++i)
    if (rfd::range_exceeded(plans[i], Ns[i])) return RFD_ERR_RANGE;
  if (dmax > rfd::slice_width(M, true)) return RFD_ERR_INVALID_ARG;
  rfd_batch_s* b = new (std::nothrow) rfd_batch_s();
  if (!b) return RFD_ERR_DEVICE;
  b->n = n;
  b->M = M;
  b->prec = prec;
  b->dmax = dmax;
  b->DB = rfd::dblocks(dmax);
  b->plans.assign(plans, plans + n);
  const size_t stride = rfd::bta_partial_floats(M, 16 * b->DB, true);
  for (int i = 0; i < n; ++i) {
    b->Ns.push_back(Ns[i]);
    b->total_n += Ns[i];
    if ((const float*)outs[i] == Fs[i]) b->aliased = true;
  }
  b->tpi = rfd::tuned(rfd::kTuneBatchExpandTilesPerItem, M, prec, b->DB, b->total_n,
                      rfd::default_batch_tiles_per_item());
  std::vector<rfd::CloudDesc> cl(n);
  std::vector<int2> wb;
  std::vector<unsigned char> args, args_apply, aargs;
  std::vector<rfd::CloudDesc> cl_full;
  std::vector<int64_t> Ns_apply, Ns_full;
  std::vector<unsigned char> aargs_none;
  const size_t PA = rfd::phi1_args_bytes(), AA = rfd::phi1_apply_args_bytes();
  for (int i = 0; i < n; ++i) {
    rfd_plan_s* p = plans[i];
    const int64_t N = Ns[i];
    const int np = rfd::bta_partials(N, M, ds[i], true, prec);
    b->max_parts = std::max(b->max_parts, np);
    rfd_status s = rfd::ensure_x(p, std::max<int64_t>(N, 1), nullptr);
    if (s == RFD_OK) s = rfd::ensure_partials(p, (size_t)np * stride, nullptr);
    if (s != RFD_OK) {
      free_batch(b);
      return s;
    }
    p->N = N;
    rfd::CloudDesc& c = cl[i];
    c.X = Xs[i];  // the kernels read the caller's points; the split-N pass copies them into the plan
    c.Xcopy = p->dev.X;
    c.N = N;
    c.om = p->dev.om;
    c.F = Fs[i];
    c.ldF = ldFs[i];
    c.out = outs[i];
    c.ldO = ldOs[i];
    c.partials = p->dev.partials;
    c.lvl = p->dev.lvl;
    c.Mraw = p->dev.Mraw;
    c.H0 = p->dev.H0;
    c.T64 = p->dev.T64;
    c.G32 = p->dev.G32;
    c.Gt16 = p->dev.Gt16;
    c.flag = p->dev.flag;
    c.d = ds[i];
    c.nparts = np;
    for (int q = 0; q < np; ++q) wb.push_back(make_int2(i, q));
    const bool ap = ds[i] <= rfd::phi1_apply_max_width();
    b->applied.push_back(ap);
    if (ap) {
      Ns_apply.push_back(N);
      args_apply.resize(args_apply.size() + PA);
      aargs.resize(aargs.size() + AA);
      rfd::phi1_fill_args(p, args_apply.data() + args_apply.size() - PA);
      rfd::phi1_fill_apply_args(p, ds[i], aargs.data() + aargs.size() - AA);
      ++b->n_apply;
    } else {
      Ns_full.push_back(N);
      args.resize(args.size() + PA);
      rfd::phi1_fill_args(p, args.data() + args.size() - PA);
      cl_full.push_back(c);
      b->dmax_full = std::max(b->dmax_full, (int)ds[i]);
      ++b->n_full;
    }
  }
  // phi_1 records largest cloud first. The per-cloud kernels run one
  // workgroup per cloud and, at m = 128 and 256, one workgroup per CU (LDS),
  // so the records queue for free CUs; the core's norm, and with it the
  // number of squarings, grows with N, so dispatching the large clouds first
  // leaves the short ones to fill the tail. Each record carries its own
  // pointers: the order changes no result.
  longest_first(args_apply, PA, aargs, AA, Ns_apply);
  longest_first(args, PA, aargs_none, 0, Ns_full);
  for (int i = 0; i < n; ++i) {
    b->bound.push_back(plans[i]->dev.X);
    b->bound.push_back(plans[i]->dev.partials);
  }
  // the expansion path of each cloud follows the single-cloud entry points
  // (expand_path of its field width), so every cloud keeps its bits
  for (int i = 0; i < n; ++i) b->valu.push_back(rfd::expand_path(M, prec, ds[i]) == rfd::kExpandValu);
  const std::vector<int2> we = expand_work(b->Ns, b->tpi, b->valu, false);
  b->tpi_v = b->tpi;
  const std::vector<int2> wv = expand_work(b->Ns, b->tpi_v, b->valu, true);
  b->nwork_bta = (int)wb.size();
  b->nwork_exp = (int)we.size();
  b->nwork_expv = (int)wv.size();
  b->exp_cap = b->nwork_exp;
  bool ok = upload(&b->dcl, cl) == hipSuccess &&
            upload(&b->dwork_bta, wb) == hipSuccess && upload(&b->dwork_exp, we) == hipSuccess &&
            upload(&b->dwork_expv, wv) == hipSuccess &&
            upload((unsigned char**)&b->dargs, args) == hipSuccess &&
            upload((unsigned char**)&b->dargs_apply, args_apply) == hipSuccess &&
            upload((unsigned char**)&b->daargs, aargs) == hipSuccess && upload(&b->dcl_full, cl_full) == hipSuccess;
  if (!ok) {
    free_batch(b);
    return RFD_ERR_DEVICE;
  }
  *out = b;
  return RFD_OK;
}

rfd_status rfd_batch_launch(rfd_batch_t b, rfd_stream_t stream) {
  if (!b) return RFD_ERR_INVALID_ARG;
  // a plan whose buffers were reallocated since creation (by a larger
  // standalone call) would leave the work lists pointing at freed memory
  for (int i = 0; i < b->n; ++i)
    if (b->plans[i]->dev.X != b->bound[2 * i] || b->plans[i]->dev.partials != b->bound[2 * i + 1])
      return RFD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < b->n; ++i) b->plans[i]->core_ready = !b->applied[i];  // S and T unless in action form
  // first launch eager (sets kernel attributes); the second records a graph
  // on a non-default stream; later launches replay it
  if (b->exec) {
    HIPCK(hipGraphLaunch(b->exec, st));
    return RFD_OK;
  }
  if (b->launches == 0 || st == nullptr) {
    ++b->launches;
    return enqueue(b, st);
  }
  rfd::set_capturing(true);
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
  rfd_status s = e == hipSuccess ? enqueue(b, st) : RFD_ERR_DEVICE;
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  rfd::set_capturing(false);
  if (s != RFD_OK || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return RFD_ERR_DEVICE;
  }
  b->graph = g;
  HIPCK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  ++b->launches;
  HIPCK(hipGraphLaunch(b->exec, st));
  return RFD_OK;
}

rfd_status rfd_batch_tune(rfd_batch_t b, int32_t reps, rfd_stream_t stream) {
  if (!b || reps < 1 || b->aliased) return RFD_ERR_INVALID_ARG;
  for (int i = 0; i < b->n; ++i)
    if (b->plans[i]->dev.X != b->bound[2 * i] || b->plans[i]->dev.partials != b->bound[2 * i + 1])
      return RFD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  // one full eager pass leaves every cloud's G in place; the expansion is
  // then re-run with each candidate geometry (it rewrites the same outputs)
  rfd_status s = enqueue(b, st);
  for (int i = 0; i < b->n; ++i) b->plans[i]->core_ready = !b->applied[i];
  if (s != RFD_OK || b->nwork_exp == 0) return s;
  static const int cands[] = {8, 16, 32, 64, 128, 256};
  const std::vector<int2> most = expand_work(b->Ns, cands[0], b->valu, false);
  int2* dw = nullptr;
  HIPCK(hipMalloc((void**)&dw, sizeof(int2) * most.size()));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = b->tpi;
  float best_ms = 1e30f;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  for (int c = 0; ok && c < (int)(sizeof(cands) / sizeof(cands[0])); ++c) {
    const std::vector<int2> we = expand_work(b->Ns, cands[c], b->valu, false);
    // (the previous candidate's launches have finished: its end event was waited on)
    ok = hipMemcpyAsync(dw, we.data(), sizeof(int2) * we.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess &&
         rfd::launch_expand_batch(b->M, b->prec, b->DB, b->dcl, dw, (int)we.size(), cands[c], st) == hipSuccess &&
         hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r)
      ok = rfd::launch_expand_batch(b->M, b->prec, b->DB, b->dcl, dw, (int)we.size(), cands[c], st) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && ms < best_ms) {
      best_ms = ms;
      best = cands[c];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(dw);
  if (!ok) return RFD_ERR_DEVICE;
  rfd::set_tuned(rfd::kTuneBatchExpandTilesPerItem, b->M, b->prec, b->DB, b->total_n, best);
  if (best != b->tpi) {
    const std::vector<int2> we = expand_work(b->Ns, best, b->valu, false);
    if ((int)we.size() > b->exp_cap) {
      (void)hipFree(b->dwork_exp);
      b->dwork_exp = nullptr;
      HIPCK(hipMalloc((void**)&b->dwork_exp, sizeof(int2) * we.size()));
      b->exp_cap = (int)we.size();
    }
    HIPCK(hipMemcpy(b->dwork_exp, we.data(), sizeof(int2) * we.size(), hipMemcpyHostToDevice));
    b->nwork_exp = (int)we.size();
    b->tpi = best;
    // the recorded graph holds the old geometry: record again on the next launch
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->launches = 1;
  }
  // the outputs hold the batch's result (every candidate rewrote them from the same G)
  return RFD_OK;
}

int32_t rfd_batch_tiles_per_item(rfd_batch_t b) { return b ? b->tpi : 0; }

void rfd_batch_destroy(rfd_batch_t b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_batch(b);
}

rfd_status rfd_integrate_batch(const rfd_plan_t* plans, const float* const* Xs, const int64_t* Ns,
                               const float* const* Fs, const int64_t* ldFs, const int32_t* ds, float* const* outs,
                               const int64_t* ldOs, int32_t n, rfd_stream_t stream) {
  rfd_batch_t b = nullptr;
  rfd_status s = rfd_batch_create(plans, Xs, Ns, Fs, ldFs, ds, outs, ldOs, n, &b);
  if (s != RFD_OK) return s;
  b->launches = 1;  // no graph for a single use
  s = enqueue(b, (hipStream_t)stream);
  for (int i = 0; i < b->n; ++i) b->plans[i]->core_ready = !b->applied[i];
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && s == RFD_OK) s = RFD_ERR_DEVICE;
  free_batch(b);
  return s;
}

}  // extern "C"
