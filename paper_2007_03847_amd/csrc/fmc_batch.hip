// fmc_batch.hip -- batched form of the method: many scenarios of different
// sizes, horizons, K and N advance together in time chunks ("ticks"); each
// tick is one persistent launch per size class over the work items of every
// scenario that still has steps, with the trajectory state kept on the device
// between ticks and the chunk's statistics rows merged after it.  All device
// work of a batch is captured once into a HIP graph and replayed while the
// batch keeps its shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "fmc_runtime.hpp"

namespace fmc {

namespace {

constexpr int64_t kBatchChunk = 250;     // steps per chunk (tick)
constexpr int64_t kBatchMaxItems = 512;  // work items per scenario
constexpr int64_t kTuneFill = 32768;     // tuner trial samples: two 64-trajectory tiles per CU

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(FMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

// Per-scenario plan of a batch.
struct Plan {
  const fmc_system* sys;
  const fmc_disturbance* dist;
  const fmc_params* par;
  fmc_outputs* out;
  int n, P, K, V;
  int64_t N, S, C, M;
  int vid;
  BatchVariantInfo bv;
  int64_t tiles, tiles_per_item, n_items, item0;
  int64_t Sc = 0, ticks = 0, lanes = 0;  // time chunk, chunks, state row stride
  double cost_tile;
  // device
  SetupDev sd{};
  NetDev nd{};
  bool kron = false;
  double *canon = nullptr, *phi = nullptr, *zeta = nullptr, *mean = nullptr, *var = nullptr;
  double2 *ybuf = nullptr, *kwork = nullptr, *part = nullptr;
  float *coef = nullptr, *w = nullptr, *state = nullptr;
  int32_t *strata = nullptr, *slot = nullptr;
  double* traj = nullptr;
  const int32_t* gen_d = nullptr;
  std::vector<double2> Yh, Yinfh;
  std::vector<int32_t> sloth;
};

std::string nm(int i, const char* what) { return "b" + std::to_string(i) + "_" + what; }

// Candidates of the batched integrator for (n, P): the three smallest lane
// variants that fit, then the smallest fitting matrix-core variant with the
// FP32 product (for n > 8, where the padded product is not mostly zeros).
// The BF16 x3 product variants run only when asked for by id: over long
// horizons their statistics drift past the reduced-precision tolerance
// (measured: 2e-4 of the mean and 5e-4 of the variance after 28 s, against
// 3e-5 and 5e-5 with the FP32 product).
std::vector<int> batch_candidates(int n, int P, int precision) {
  std::vector<int> lane, v;
  int mc[3] = {-1, -1, -1};
  for (int i = 0; i < n_batch_variants(); ++i) {
    const BatchVariantInfo b = batch_variant(i);
    if (!batch_fits(b, n, P, precision)) continue;
    if (b.prod == 0) {
      lane.push_back(i);
    } else if (n > 8 && (mc[b.prod] < 0 || b.NG < batch_variant(mc[b.prod]).NG)) {
      mc[b.prod] = i;
    }
  }
  std::stable_sort(lane.begin(), lane.end(),
                   [](int a, int b) { return batch_variant(a).NG < batch_variant(b).NG; });
  if (lane.size() > 3) lane.resize(3);
  v = lane;
  if (mc[1] >= 0) v.push_back(mc[1]);
  return v;
}

}  // namespace

bool batch_fits(const BatchVariantInfo& b, int n, int P, int precision) {
  return b.NG >= n && b.PM >= P && (b.prod != 2 || precision == FMC_BF16X3);
}

// Untuned choice: from 12 machines on the matrix-core class with the FP32
// product, measured faster than the lane variants there; otherwise the
// smallest lane variant that fits.
int default_batch_variant(int n, int P, int precision) {
  const bool mc = n >= 12;
  int vid = -1;
  for (int pass = 0; pass < 2 && vid < 0; ++pass)  // pass 1: whatever fits
    for (int i = 0; i < n_batch_variants(); ++i) {
      const BatchVariantInfo b = batch_variant(i);
      if (!batch_fits(b, n, P, precision) || b.prod == 2) continue;
      if (pass == 0 && (b.prod != 0) != mc) continue;
      if (vid < 0 || b.NG < batch_variant(vid).NG) vid = i;
    }
  return vid;
}

int run_batch_impl(Context* c, int32_t nsc, const fmc_scenario* scen, fmc_outputs* outs,
                   const int* forced_variant, double* t_out);

// Autotuner of the batched form: times the fitting variants on a one-scenario
// batch with a short horizon and caches the fastest under "B/" + key.
static int batch_pick(Context* c, const fmc_scenario& sc, int* vid) {
  const fmc_params* par = sc.par;
  const int n = sc.sys->n_gen, P = sc.dist->n_proc;
  const std::string key = "B/" + tune_key(n, P, par->N, par->precision);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    *vid = it->second;
    return FMC_OK;
  }
  std::vector<int> cand = batch_candidates(n, P, par->precision);
  if (cand.empty()) return fail(FMC_EINVAL, "no batched variant for n=" + std::to_string(n) + ", P=" + std::to_string(P));
  int best = cand[0];
  if (cand.size() > 1) {
    const int64_t S = (int64_t)std::llround(par->T / par->dt);
    const int64_t St = std::min<int64_t>(S, 48);
    fmc_params p2 = *par;
    p2.T = (double)St * par->dt;
    // A batch keeps the chip busy with its other scenarios, so a variant is
    // judged by its throughput on a full chip: the trial runs at least
    // kTuneFill samples (its own LHS design; a caller's zeta would be too
    // short).  A trial at a small N alone would favour the variants with the
    // smallest tiles, which lose once the chip is shared.
    if (p2.N < kTuneFill) {
      p2.N = kTuneFill;
      p2.zeta_in = nullptr;
    }
    fmc_scenario s2{sc.sys, sc.dist, &p2};
    const int V = 2 * n + P;
    void *m = nullptr, *v = nullptr;
    int rc;
    if ((rc = c->ensure("btune_mean", (size_t)(St + 1) * V * 8, &m))) return rc;
    if ((rc = c->ensure("btune_var", (size_t)(St + 1) * V * 8, &v))) return rc;
    double best_t = 0.0;
    for (int cv : cand) {
      fmc_outputs o{};
      o.mean = (double*)m;
      o.var = (double*)v;
      o.mem_kind = FMC_MEM_DEVICE;
      double t = 0.0;
      for (int r = 0; r < 2; ++r)
        if ((rc = run_batch_impl(c, 1, &s2, &o, &cv, &t)) && rc != FMC_ENONFINITE) return rc;
      if (cv == cand[0] || t < best_t) {
        best = cv;
        best_t = t;
      }
    }
  }
  c->tuned[key] = best;
  *vid = best;
  return FMC_OK;
}

int run_batch_impl(Context* c, int32_t nsc, const fmc_scenario* scen, fmc_outputs* outs,
                   const int* forced_variant, double* t_out) {
  if (nsc < 1 || !scen || !outs) return fail(FMC_EINVAL, "empty batch");
  HIPCHK(hipSetDevice(c->device));
  if (!c->bstream) HIPCHK(hipStreamCreateWithFlags(&c->bstream, hipStreamNonBlocking));
  for (int k = 0; k < kBatchClasses; ++k)
    if (!c->cstream[k]) HIPCHK(hipStreamCreateWithFlags(&c->cstream[k], hipStreamNonBlocking));
  for (auto& e : c->cev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipStream_t st = c->bstream;
  int rc;
  std::vector<Plan> plans(nsc);
  std::string shape_key;
  for (int i = 0; i < nsc; ++i) {
    Plan& p = plans[i];
    p.sys = scen[i].sys;
    p.dist = scen[i].dist;
    p.par = scen[i].par;
    p.out = &outs[i];
    if ((rc = validate(p.sys, p.dist, p.par, &p.S))) return fail(rc, "scenario " + std::to_string(i) + ": " + g_err);
    if (p.par->sampler == FMC_LHS_DECOR)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) +
                                  ": FMC_LHS_DECOR runs through fmc_run only");
    if (p.sys->event)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) + ": network events run through fmc_run only");
    if (p.out->rrf)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) + ": the fused RRF runs through fmc_run only");
    if (p.par->integrator != FMC_RK4)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) +
                                  ": the implicit trapezoid runs through fmc_run only");
    if (p.dist->sigma_mat)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) +
                                  ": a diffusion matrix runs through fmc_run only");
    if (p.dist->proc)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) +
                                  ": general Ito processes run through fmc_run only");
    if (p.sys->model != FMC_CLASSICAL)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) +
                                  ": the batched form runs classical machines (flux-decay "
                                  "systems go through fmc_run or fmc_submit)");
    if (p.par->precision == FMC_F64)
      return fail(FMC_EINVAL, "scenario " + std::to_string(i) + ": the batched form integrates in FP32 (FMC_F32 or FMC_BF16X3)");
    if (!p.out->mean || !p.out->var) return fail(FMC_EINVAL, "mean and var outputs are required");
    if (p.out->mem_kind != FMC_MEM_HOST && p.out->mem_kind != FMC_MEM_DEVICE)
      return fail(FMC_EINVAL, "unknown mem_kind");
    if (p.out->n_traj < 0 || (p.out->n_traj > 0 && (!p.out->traj_idx || !p.out->traj)))
      return fail(FMC_EINVAL, "n_traj > 0 needs traj_idx and traj");
    p.n = p.sys->n_gen;
    p.P = p.dist->n_proc;
    p.K = p.par->K;
    p.V = 2 * p.n + p.P;
    p.N = p.par->N;
    p.C = 2 * p.S + 1;
    p.M = (int64_t)p.P * p.K;
    if (forced_variant) {
      p.vid = *forced_variant;
    } else if (p.par->variant >= 0) {
      p.vid = p.par->variant;
    } else if ((rc = batch_pick(c, scen[i], &p.vid))) {
      return rc;
    }
    if (p.vid < 0 || p.vid >= n_batch_variants()) return fail(FMC_EINVAL, "no batched variant");
    p.bv = batch_variant(p.vid);
    if (!batch_fits(p.bv, p.n, p.P, p.par->precision))
      return fail(FMC_EINVAL, "batched variant does not fit the scenario (size, or a BF16 x3 "
                              "product for an FMC_F32 scenario)");
    p.tiles = (p.N + p.bv.TB - 1) / p.bv.TB;
    p.cost_tile = (double)p.S * p.bv.TB * (8.0 * p.bv.NG * p.bv.NG + 45.0 * p.bv.NG + 4.0 * p.P);
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%d,%d,%d,%lld,%lld,%.17g,%.17g,%llu,%d,%d,%d,%d,%d,%d,%d,%.17g,%.17g,%d,%d|",
                  p.n, p.P, p.K, (long long)p.N, (long long)p.S, p.par->T, p.par->dt,
                  (unsigned long long)p.par->seed, p.par->basis, p.par->sampler, p.par->precision,
                  p.par->ddof, p.vid, p.sys->infinite_bus, p.sys->Y_re ? 1 : (p.sys->net ? p.sys->net->n_bus : 0),
                  p.sys->V_inf, p.sys->f0_hz, p.out->n_traj, p.par->zeta_in ? 1 : 0);
    shape_key += buf;
    if (p.par->zeta_in) {
      char b2[64];
      std::snprintf(b2, sizeof(b2), "z%p|", (const void*)p.par->zeta_in);
      shape_key += b2;
    }
    if (!p.sys->Y_re) {
      const fmc_network* net = p.sys->net;
      char b3[96];
      std::snprintf(b3, sizeof(b3), "nb%d,%d,%d%d%d|", net->n_bus, net->n_branch, net->br_b ? 1 : 0,
                    net->load_g ? 1 : 0, net->load_b ? 1 : 0);
      shape_key += b3;
    }
    // which optional arrays are present decides the staging layout
    char b4[32];
    std::snprintf(b4, sizeof(b4), "o%d%d%d%d|", p.sys->delta0 ? 1 : 0, p.sys->Pm ? 1 : 0,
                  p.dist->xi0 ? 1 : 0, p.out->strata ? 1 : 0);
    shape_key += b4;
  }
  // ---- time chunks and work items.  Every scenario advances in chunks of
  // Sc steps (its time_chunk, else kBatchChunk); chunk k of every scenario
  // that still has steps left forms tick k of the batch.  A scenario is cut
  // into at most kBatchMaxItems items of consecutive tiles, fixed by the
  // scenario alone, so its statistics (merged per chunk, items in order) do
  // not depend on the other scenarios of the batch.
  int64_t n_ticks = 0, n_items = 0;
  for (auto& p : plans) {
    p.Sc = std::min<int64_t>(p.S, p.par->time_chunk > 0 ? p.par->time_chunk : kBatchChunk);
    p.ticks = (p.S + p.Sc - 1) / p.Sc;
    n_ticks = std::max(n_ticks, p.ticks);
    p.tiles_per_item = (p.tiles + kBatchMaxItems - 1) / kBatchMaxItems;
    p.n_items = (p.tiles + p.tiles_per_item - 1) / p.tiles_per_item;
    p.item0 = n_items;
    n_items += p.n_items;
    char b5[48];
    std::snprintf(b5, sizeof(b5), "c%lld|", (long long)p.Sc);
    shape_key += b5;
  }
  // ---- device buffers
  for (int i = 0; i < nsc; ++i) {
    Plan& p = plans[i];
    void* q = nullptr;
    const CanonLayout CL{p.n, p.P};
    if ((rc = c->ensure(nm(i, "canon").c_str(), (size_t)CL.size() * 8, &q))) return rc;
    p.canon = (double*)q;
    if ((rc = c->ensure(nm(i, "coef").c_str(), batch_coef_floats(p.bv) * 4, &q))) return rc;
    p.coef = (float*)q;
    if ((rc = c->ensure(nm(i, "phi").c_str(), (size_t)p.K * p.C * 8, &q))) return rc;
    p.phi = (double*)q;
    if (!p.par->zeta_in) {
      if ((rc = c->ensure(nm(i, "zeta").c_str(), (size_t)p.M * p.N * 8, &q))) return rc;
      p.zeta = (double*)q;
      if (p.out->strata) {
        if ((rc = c->ensure(nm(i, "strata").c_str(), (size_t)p.M * p.N * 4, &q))) return rc;
        p.strata = (int32_t*)q;
      }
    }
    if ((rc = c->ensure(nm(i, "w").c_str(), (size_t)(2 * p.Sc + 1) * p.P * p.N * 4, &q))) return rc;
    p.w = (float*)q;
    p.lanes = p.tiles * 64 * 4;
    if ((rc = c->ensure(nm(i, "state").c_str(), batch_state_floats(p.bv, p.tiles) * 4, &q))) return rc;
    p.state = (float*)q;
    if ((rc = c->ensure(nm(i, "part").c_str(), (size_t)p.n_items * (p.Sc + 1) * p.V * 16, &q))) return rc;
    p.part = (double2*)q;
    if ((rc = c->ensure(nm(i, "work").c_str(), (size_t)(3 * p.n * p.n + 8 * p.n + 64) * 8, &q))) return rc;
    p.sd.work = (double*)q;
    if (!p.sys->Y_re) {
      p.kron = true;
      if ((rc = c->ensure(nm(i, "ybuf").c_str(), (size_t)p.n * p.n * 16, &q))) return rc;
      p.ybuf = (double2*)q;
      // one work matrix per scenario: the reductions run side by side
      if ((rc = c->ensure(nm(i, "kwork").c_str(), kron_work_bytes(p.sys->net->n_bus, p.n), &q))) return rc;
      p.kwork = (double2*)q;
    }
    // the captured graph touches context buffers only; results are copied out
    // after each replay (caller pointers may change between calls)
    if ((rc = c->ensure(nm(i, "mean").c_str(), (size_t)(p.S + 1) * p.V * 8, &q))) return rc;
    p.mean = (double*)q;
    if ((rc = c->ensure(nm(i, "var").c_str(), (size_t)(p.S + 1) * p.V * 8, &q))) return rc;
    p.var = (double*)q;
    if (p.out->n_traj > 0) {
      if ((rc = c->ensure(nm(i, "traj").c_str(), (size_t)p.out->n_traj * (p.S + 1) * p.V * 8, &q))) return rc;
      p.traj = (double*)q;
    }
    if (p.out->n_traj > 0) {
      if ((rc = c->ensure(nm(i, "slot").c_str(), (size_t)p.N * 4, &q))) return rc;
      p.slot = (int32_t*)q;
      p.sloth.assign(p.N, -1);
      for (int t = 0; t < p.out->n_traj; ++t) {
        const int64_t idx = p.out->traj_idx[t];
        if (idx < 0 || idx >= p.N) return fail(FMC_EINVAL, "traj_idx out of range");
        if (p.sloth[idx] >= 0) return fail(FMC_EINVAL, "traj_idx has a duplicate");
        p.sloth[idx] = t;
      }
    }
  }
  void *status = nullptr, *counters = nullptr, *heads = nullptr;
  if ((rc = c->ensure("b_status", (size_t)nsc * 16, &status))) return rc;
  if ((rc = c->ensure("b_counters", (size_t)nsc * 16, &counters))) return rc;
  if ((rc = c->ensure("b_heads", (size_t)n_ticks * 16 * 4, &heads))) return rc;
  // ---- items (static) and, per tick and size class, the queue of the items
  // of the scenarios active in that tick (longest first)
  std::vector<BatchItem> items(n_items);
  std::vector<double> icost(n_items);
  std::vector<std::vector<int32_t>> by_cls(kBatchClasses);
  for (int i = 0; i < nsc; ++i) {
    Plan& p = plans[i];
    for (int64_t k = 0; k < p.n_items; ++k) {
      BatchItem& it = items[p.item0 + k];
      it.rows = p.part + k * (p.Sc + 1) * p.V;
      it.tile0 = k * p.tiles_per_item;
      it.tile1 = std::min<int64_t>(p.tiles, it.tile0 + p.tiles_per_item);
      it.scen = i;
      it.variant = p.vid;
      icost[p.item0 + k] = p.cost_tile / (double)p.S * (double)p.Sc * (double)(it.tile1 - it.tile0);
      by_cls[p.bv.cls].push_back((int32_t)(p.item0 + k));
    }
  }
  for (auto& o : by_cls)
    std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return icost[a] > icost[b]; });
  std::vector<int32_t> order_flat;
  std::vector<int64_t> ord_off((size_t)n_ticks * kBatchClasses + 1, 0);
  for (int64_t k = 0; k < n_ticks; ++k) {
    for (int cl = 0; cl < kBatchClasses; ++cl) {
      ord_off[k * kBatchClasses + cl] = (int64_t)order_flat.size();
      for (int32_t q : by_cls[cl])
        if (plans[items[q].scen].ticks > k) order_flat.push_back(q);
    }
  }
  ord_off[(size_t)n_ticks * kBatchClasses] = (int64_t)order_flat.size();
  // ---- one upload: scenario inputs, per-tick integrator arguments, items, queues
  Stager sg;
  std::vector<IntegArgs<float>> args((size_t)n_ticks * nsc);
  for (int i = 0; i < nsc; ++i) {
    Plan& p = plans[i];
    const fmc_system* s = p.sys;
    const fmc_disturbance* d = p.dist;
    p.sd.n = p.n;
    p.sd.P = p.P;
    if (s->Y_re) {
      p.Yh.resize((size_t)p.n * p.n);
      for (size_t q = 0; q < p.Yh.size(); ++q) p.Yh[q] = make_double2(s->Y_re[q], s->Y_im[q]);
    }
    if (s->infinite_bus) {
      p.Yinfh.resize(p.n);
      for (int k = 0; k < p.n; ++k) p.Yinfh[k] = make_double2(s->Yinf_re[k], s->Yinf_im[k]);
    }
    sg.add(s->H, p.n, &p.sd.H);
    sg.add(s->D, p.n, &p.sd.D);
    sg.add(s->E, p.n, &p.sd.E);
    sg.add(s->delta0, p.n, &p.sd.delta0);
    sg.add(s->Pm, p.n, &p.sd.Pm);
    sg.add(p.Yh.empty() ? nullptr : p.Yh.data(), p.Yh.size(), &p.sd.Y);
    sg.add(p.Yinfh.empty() ? nullptr : p.Yinfh.data(), p.Yinfh.size(), &p.sd.Yinf);
    sg.add(d->theta, p.P, &p.sd.theta);
    sg.add(d->sigma, p.P, &p.sd.sigma);
    sg.add(d->xi0, p.P, &p.sd.xi0);
    sg.add(d->gen, p.P, &p.gen_d);
    if (p.kron) {
      const fmc_network* net = s->net;
      p.nd.n_bus = net->n_bus;
      p.nd.n_branch = net->n_branch;
      p.nd.n_gen = net->n_gen;
      sg.add(net->br_from, net->n_branch, &p.nd.from);
      sg.add(net->br_to, net->n_branch, &p.nd.to);
      sg.add(net->br_r, net->n_branch, &p.nd.r);
      sg.add(net->br_x, net->n_branch, &p.nd.x);
      sg.add(net->br_b, net->n_branch, &p.nd.b);
      sg.add(net->load_g, net->n_bus, &p.nd.lg);
      sg.add(net->load_b, net->n_bus, &p.nd.lb);
      sg.add(net->gen_bus, net->n_gen, &p.nd.gen_bus);
      sg.add(net->gen_xdp, net->n_gen, &p.nd.xdp);
    }
    p.sd.inf_bus = s->infinite_bus ? 1 : 0;
    p.sd.V_inf = s->V_inf;
    p.sd.canon = p.canon;
    p.sd.status = (int*)status + 4 * i;  // [0]: setup, [1]: reduction
    for (int64_t k = 0; k < p.ticks; ++k) {
      IntegArgs<float>& a = args[(size_t)k * nsc + i];
      a.coef = p.coef;
      a.w = p.w;
      a.state = p.state;
      a.partial = nullptr;
      a.delta0 = p.canon + CanonLayout{p.n, p.P}.delta0();
      a.traj_slot = p.slot;
      a.traj = p.traj;
      a.nonfinite = (unsigned long long*)counters + 2 * i;
      a.first_bad = (long long*)counters + 2 * i + 1;
      a.n = p.n;
      a.P = p.P;
      a.V = p.V;
      a.N = p.N;
      a.S = p.S;
      a.s_begin = k * p.Sc;
      a.s_end = std::min<int64_t>(p.S, (k + 1) * p.Sc);
      a.c_base = 2 * a.s_begin;
      a.lanes = p.lanes;
      a.dt = (float)p.par->dt;
      a.wb = (float)(2.0 * M_PI * (s->f0_hz > 0.0 ? s->f0_hz : 60.0));
      a.recenter = s->infinite_bus ? 0 : 1;
      a.n_ref = p.n;
    }
  }
  const IntegArgs<float>* args_d = nullptr;
  const BatchItem* items_d = nullptr;
  const int32_t* order_d = nullptr;
  sg.add(args.data(), args.size(), &args_d);
  sg.add(items.data(), items.size(), &items_d);
  sg.add(order_flat.data(), order_flat.size(), &order_d);
  if ((rc = sg.upload(c, "b_inputs", st))) return rc;
  // trajectory slots (outside the graph)
  for (auto& p : plans) {
    if (p.sloth.empty()) continue;
    void* h = nullptr;
    const std::string hn = "bslot_" + std::to_string(&p - plans.data());
    if ((rc = c->host_stage(hn.c_str(), p.sloth.size() * 4, &h))) return rc;
    std::memcpy(h, p.sloth.data(), p.sloth.size() * 4);
    HIPCHK(hipMemcpyAsync(p.slot, h, p.sloth.size() * 4, hipMemcpyHostToDevice, st));
  }
  // ---- device work: captured once per batch shape, then replayed
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, c->device));
  int bpc[kBatchClasses];
  for (int k = 0; k < kBatchClasses; ++k) bpc[k] = persistent_blocks_per_cu(k);
  auto enqueue = [&]() -> int {
    HIPCHK(launch_fill_i64((int64_t*)status, 0, 2 * nsc, st));
    // per-scenario setup (reduction, operating point, packing, basis, design),
    // scenarios spread round-robin over the side streams
    {
      bool used[kBatchClasses] = {};
      HIPCHK(hipEventRecord(c->cev[kBatchClasses], st));
      for (int i = 0; i < nsc; ++i) {
        Plan& p = plans[i];
        const int x = i % kBatchClasses;
        const hipStream_t s = c->cstream[x];
        if (!used[x]) HIPCHK(hipStreamWaitEvent(s, c->cev[kBatchClasses], 0));
        used[x] = true;
        if (p.kron) {
          HIPCHK(launch_kron(p.nd, p.kwork, p.ybuf, (int*)status + 4 * i + 1, s));
          p.sd.Y = p.ybuf;
        }
        HIPCHK(launch_setup(p.sd, s));
        HIPCHK(launch_pack_batch(p.bv, p.canon, p.n, p.P, p.gen_d, p.coef, s));
        HIPCHK(launch_basis(p.par->basis, p.K, p.S, p.par->T, p.phi, s));
        if (!p.par->zeta_in)
          HIPCHK(launch_lhs(p.par->seed, (int32_t)p.M, p.N, p.par->sampler, p.strata, p.zeta, s));
      }
      for (int x = 0; x < kBatchClasses; ++x)
        if (used[x]) {
          HIPCHK(hipEventRecord(c->cev[x], c->cstream[x]));
          HIPCHK(hipStreamWaitEvent(st, c->cev[x], 0));
        }
    }
    // counters: (nonfinite = 0, first = max) per scenario; queue heads = 0
    for (int i = 0; i < nsc; ++i) {
      HIPCHK(launch_fill_i64((int64_t*)counters + 2 * i, 0, 1, st));
      HIPCHK(launch_fill_i64((int64_t*)counters + 2 * i + 1, LLONG_MAX, 1, st));
    }
    HIPCHK(launch_fill_i64((int64_t*)heads, 0, n_ticks * 8, st));
    for (int64_t k = 0; k < n_ticks; ++k) {
      // The tick's per-scenario launches of one phase (paths, merges) are
      // small: they are spread round-robin over the side streams (forked
      // from st, joined back) so that they run side by side.
      auto spread = [&](auto&& launch) -> int {
        bool used[kBatchClasses] = {};
        HIPCHK(hipEventRecord(c->cev[kBatchClasses], st));
        int j = 0;
        for (auto& p : plans) {
          if (p.ticks <= k) continue;
          const int x = j++ % kBatchClasses;
          if (!used[x]) HIPCHK(hipStreamWaitEvent(c->cstream[x], c->cev[kBatchClasses], 0));
          used[x] = true;
          HIPCHK(launch(p, c->cstream[x]));
        }
        for (int x = 0; x < kBatchClasses; ++x)
          if (used[x]) {
            HIPCHK(hipEventRecord(c->cev[x], c->cstream[x]));
            HIPCHK(hipStreamWaitEvent(st, c->cev[x], 0));
          }
        return FMC_OK;
      };
      rc = spread([&](Plan& p, hipStream_t s) {
        const int64_t s0 = k * p.Sc, s1 = std::min<int64_t>(p.S, s0 + p.Sc);
        const double* zeta = p.par->zeta_in ? p.par->zeta_in : p.zeta;
        return p.par->precision == FMC_F32
                   ? launch_kle_f64_to_f32(zeta, p.phi, p.C, p.P, p.K, p.N, 2 * (s1 - s0) + 1, 2 * s0, p.w, s)
                   : launch_kle_bf16x3(zeta, p.phi, p.C, p.P, p.K, p.N, 2 * (s1 - s0) + 1, 2 * s0, p.w, s);
      });
      if (rc) return rc;
      // the tick's size classes: one launch each; with more than one, each on
      // its own stream (fork after the paths, join before the merges) so that
      // the classes share the chip instead of each running partly filled
      int n_act = 0;
      for (int cl = 0; cl < kBatchClasses; ++cl)
        n_act += ord_off[k * kBatchClasses + cl + 1] > ord_off[k * kBatchClasses + cl];
      if (n_act > 1) HIPCHK(hipEventRecord(c->cev[kBatchClasses], st));
      for (int cl = 0; cl < kBatchClasses; ++cl) {
        const int64_t o0 = ord_off[k * kBatchClasses + cl], o1 = ord_off[k * kBatchClasses + cl + 1];
        if (o1 == o0) continue;
        const int grid = (int)std::min<int64_t>(o1 - o0, (int64_t)bpc[cl] * prop.multiProcessorCount);
        BatchArgs b{args_d + (size_t)k * nsc, items_d, order_d + o0, (int32_t)(o1 - o0),
                    (int32_t*)heads + k * 16 + 2 * cl};
        if (n_act > 1) {
          HIPCHK(hipStreamWaitEvent(c->cstream[cl], c->cev[kBatchClasses], 0));
          HIPCHK(launch_persistent(cl, b, grid, c->cstream[cl]));
          HIPCHK(hipEventRecord(c->cev[cl], c->cstream[cl]));
        } else {
          HIPCHK(launch_persistent(cl, b, grid, st));
        }
      }
      if (n_act > 1)
        for (int cl = 0; cl < kBatchClasses; ++cl)
          if (ord_off[k * kBatchClasses + cl + 1] > ord_off[k * kBatchClasses + cl])
            HIPCHK(hipStreamWaitEvent(st, c->cev[cl], 0));
      // rows completed by this tick: s0+1..s1 (and row 0 in the first chunk)
      rc = spread([&](Plan& p, hipStream_t s) {
        const int64_t s0 = k * p.Sc, s1 = std::min<int64_t>(p.S, s0 + p.Sc);
        const int64_t first = s0 == 0 ? 0 : s0 + 1;
        return launch_stats_merge_rows(p.part + (first - s0) * p.V, (p.Sc + 1) * p.V, p.n_items,
                                       (int)(p.tiles_per_item * p.bv.TB), p.N, s1 - first + 1, p.V,
                                       p.n, p.par->ddof, p.canon + CanonLayout{p.n, p.P}.delta0(),
                                       p.mean + first * p.V, p.var + first * p.V, s);
      });
      if (rc) return rc;
    }
    return FMC_OK;
  };
  hipEvent_t e0 = c->ev[0], e1 = c->ev[1];
  HIPCHK(hipEventRecord(e0, st));
  const std::string gkey = shape_key;
  auto git = c->graphs.find(gkey);
  if (git != c->graphs.end() && git->second.first == c->alloc_gen) {
    HIPCHK(hipGraphLaunch(git->second.second, st));
  } else {
    if (git != c->graphs.end()) {
      (void)hipGraphExecDestroy(git->second.second);
      c->graphs.erase(git);
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = enqueue();
    hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(FMC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    hipGraphExec_t ge = nullptr;
    hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(FMC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    if (c->graphs.size() > 32) {
      for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.second);
      c->graphs.clear();
    }
    c->graphs[gkey] = {c->alloc_gen, ge};
    HIPCHK(hipGraphLaunch(ge, st));
  }
  HIPCHK(hipEventRecord(e1, st));
  // ---- results
  for (auto& p : plans) {
    const hipMemcpyKind kind =
        p.out->mem_kind == FMC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const size_t sv = (size_t)(p.S + 1) * p.V * 8;
    HIPCHK(hipMemcpyAsync(p.out->mean, p.mean, sv, kind, st));
    HIPCHK(hipMemcpyAsync(p.out->var, p.var, sv, kind, st));
    if (p.out->n_traj > 0)
      HIPCHK(hipMemcpyAsync(p.out->traj, p.traj, (size_t)p.out->n_traj * sv, kind, st));
    if (p.out->zeta && p.zeta)
      HIPCHK(hipMemcpyAsync(p.out->zeta, p.zeta, (size_t)p.M * p.N * 8, kind, st));
    if (p.out->strata && p.strata)
      HIPCHK(hipMemcpyAsync(p.out->strata, p.strata, (size_t)p.M * p.N * 4, kind, st));
  }
  void* hb = nullptr;
  if ((rc = c->host_stage("b_readback", (size_t)nsc * 32, &hb))) return rc;
  int* st_h = (int*)hb;
  unsigned long long* cn_h = (unsigned long long*)((char*)hb + (size_t)nsc * 16);
  HIPCHK(hipMemcpyAsync(st_h, status, (size_t)nsc * 16, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(cn_h, counters, (size_t)nsc * 16, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  if (t_out) *t_out = ms * 1e-3;
  int64_t bad_total = 0;
  int first_err = FMC_OK;
  std::string first_msg;
  for (int i = 0; i < nsc; ++i) {
    Plan& p = plans[i];
    if (st_h[4 * i + 1] != 0 && first_err == FMC_OK) {
      first_err = FMC_EINVAL;
      first_msg = "scenario " + std::to_string(i) + ": network reduction failed";
    }
    if (st_h[4 * i] != 0 && first_err == FMC_OK) {
      first_err = FMC_ENOTCONV;
      first_msg = "scenario " + std::to_string(i) + ": operating-point Newton solve did not converge";
    }
    bad_total += (int64_t)cn_h[2 * i];
    if (p.out->report) {
      fmc_report* r = p.out->report;
      std::memset(r, 0, sizeof(*r));
      r->t_total_s = ms * 1e-3;
      r->t_integrate_s = ms * 1e-3;
      r->n_nonfinite = (int64_t)cn_h[2 * i];
      r->first_nonfinite = cn_h[2 * i] ? (int64_t)cn_h[2 * i + 1] : -1;
      r->variant_id = p.vid;
      r->lanes_per_traj = p.bv.L;
      r->tile = (int32_t)(p.tiles_per_item * p.bv.TB);
      r->time_chunk = (int32_t)p.Sc;
      r->hbm_peak_bytes = (int64_t)c->held;
    }
  }
  if (first_err) return fail(first_err, first_msg);
  if (bad_total) return fail(FMC_ENONFINITE, std::to_string(bad_total) + " sample paths became non-finite");
  return FMC_OK;
}

}  // namespace fmc

using namespace fmc;

extern "C" int fmc_run_batch(fmc_context* ctx, int32_t n, const fmc_scenario* scen,
                             fmc_outputs* outs) {
  if (!ctx) return fail(FMC_EINVAL, "ctx is NULL");
  Context* c = reinterpret_cast<Context*>(ctx);
  // work already queued on the caller's stream comes first
  if (c->bstream && c->bstream != c->stream) {
    (void)hipEventRecord(c->ev[2], c->stream);
    (void)hipStreamWaitEvent(c->bstream, c->ev[2], 0);
  }
  const int rc = run_batch_impl(c, n, scen, outs, nullptr, nullptr);
  if (rc != FMC_OK && rc != FMC_ENONFINITE && c->bstream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->bstream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c->bstream, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamSynchronize(c->bstream);
  }
  return rc;
}
