// fmc_run.hip -- one scenario through the whole method (Alg. 1) on the GPU:
// setup (network reduction, operating point) -> LHS design (step 1) -> basis
// -> per time chunk: KLE path contraction (step 2, on a second stream, one
// chunk ahead) and integration with fused per-wave statistics (step 3) ->
// ordered merge of the statistics (step 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fmc_runtime.hpp"

namespace fmc {

namespace {

struct EventPool {
  std::vector<hipEvent_t> ev;
  bool on = false;
  hipStream_t st = nullptr;
  ~EventPool() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  int record(hipStream_t on_stream = nullptr) {
    if (!on) return -1;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    (void)hipEventRecord(e, on_stream ? on_stream : st);
    ev.push_back(e);
    return (int)ev.size() - 1;
  }
  double secs(int a, int b) const {
    if (a < 0 || b < 0) return 0.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) return 0.0;
    return ms * 1e-3;
  }
};

struct ChunkTimes {
  std::vector<int> gemm0, gemm1, int0, int1;
  int st0 = -1, st1 = -1;  // the last chunk's statistics merge
};



// The general Ito processes as normalised rows (IntegArgs::sde), from the
// rows of Table I (rate theta scaling drift and squared diffusion) and the
// polynomial form of eq. 11; an OU spec becomes the polynomial form with
// drift -theta xi and constant diffusion sigma.  PM rows (the variant's
// process slots; rows past n_proc are zero: no drift, diffusion or
// injection).  False when every process is the plain OU of theta and sigma
// (no table).
static bool sde_table(const fmc_disturbance* dist, int basis, int PM, std::vector<double>& t) {
  if (!dist->proc) return false;
  const int P = dist->n_proc;
  t.assign((size_t)PM * kSdeCols, 0.0);
  // Wong-Zakai: the KLE ODE's limit is the Stratonovich solution; the Ito
  // process needs -sigma sigma'/2 in the drift, the one-hot basis (whose RK4
  // step carries (3/8) sigma sigma' of its own) -3/8.
  const double k =
      dist->calculus == FMC_ITO ? (basis == FMC_BASIS_EM ? 0.375 : 0.5) : 0.0;
  for (int p = 0; p < P; ++p) {
    const fmc_process& q = dist->proc[p];
    double* r = &t[(size_t)p * kSdeCols];
    const double th = q.theta, a = q.a, b = q.b;
    r[SDE_FORM] = 2.0;
    r[SDE_M1] = -th;
    switch (q.kind) {
      case FMC_PROC_OU:
        r[SDE_FORM] = 1.0;
        r[SDE_M1] = -dist->theta[p];
        r[SDE_C0] = dist->sigma[p];
        break;
      case FMC_PROC_GAUSS:  // mu = -theta (xi - a), sigma^2 = 2 theta b
        r[SDE_M0] = th * a;
        r[SDE_C0] = 2.0 * th * b;
        break;
      case FMC_PROC_BETA:  // mu = -theta (xi - a/(a+b)), sigma^2 = 2 theta xi (1 - xi)/(a+b)
        r[SDE_M0] = th * a / (a + b);
        r[SDE_C1] = 2.0 * th / (a + b);
        r[SDE_C2] = -2.0 * th / (a + b);
        break;
      case FMC_PROC_GAMMA:  // mu = -theta (xi - a/b), sigma^2 = 2 theta xi / b
        r[SDE_M0] = th * a / b;
        r[SDE_C1] = 2.0 * th / b;
        break;
      case FMC_PROC_LAPLACE:  // mu = -theta (xi - a), sigma^2 = theta (2b|xi - a| + 2b^2)
        r[SDE_M0] = th * a;
        r[SDE_C0] = 2.0 * th * b * b;
        r[SDE_C3] = 2.0 * th * b;
        r[SDE_R] = a;
        break;
      default:  // FMC_PROC_POLY
        r[SDE_FORM] = 1.0;
        for (int j = 0; j < 3; ++j) {
          r[SDE_M0 + j] = q.mu[j];
          r[SDE_C0 + j] = q.sg[j];
        }
        break;
    }
    r[SDE_K] = k;
    r[SDE_GAIN] = q.gain;
    r[SDE_REF] = q.ref;
  }
  return true;
}

template <typename R>
int run_chunks(Context* c, const fmc_params* par, int vid, int n, int P, int64_t S, int64_t N,
               double wb, const double* zeta, const double* phi, const R* coef,
               const double* delta0, double* partial, const int32_t* slot_d, double* traj_d,
               unsigned long long* cnt_d, int64_t Sc, double* mean_d, double* var_d,
               int recenter, bool trap, const void* const* s16, const R* coef_post,
               int64_t s_event, int n_ref_post, const double* rrf_w, double* rrf_acc,
               double* rrf_d, const R* sde, EventPool& evp, ChunkTimes& ct) {
  const VariantInfo& vi = variant(vid);
  const int V = 2 * n + P;
  const int64_t C = 2 * S + 1;
  const int64_t gs = vi.group_size();
  const int64_t n_groups = (N + gs - 1) / gs;
  const int64_t lanes = n_groups * 64 * vi.WPB;
  const int bw = (int)sizeof(R);
  // Two path buffers: the contraction of chunk k+1 runs on a second stream
  // while the integrator consumes chunk k (the integrator is bound by issue
  // latency at low occupancy, so the matrix-core contraction fits beside it).
  // The statistics rows of chunk k are merged on the second stream too, once
  // the integrator has finished chunk k, so only the last chunk's merge is
  // left after the integrator.
  void *w[2] = {nullptr, nullptr}, *state = nullptr;
  int rc;
  if ((rc = c->ensure("w", (size_t)(2 * Sc + 1) * P * N * bw, &w[0]))) return rc;
  if ((rc = c->ensure("w1", (size_t)(2 * Sc + 1) * P * N * bw, &w[1]))) return rc;
  if ((rc = c->ensure("state", (size_t)(2 * vi.NG + vi.PM + kOffsetRows) * lanes * bw, &state))) return rc;
  if ((rc = ensure_gstream(c))) return rc;
  hipStream_t ks = c->gstream;
  // merge of the rows completed by chunk [s0, s1] (row 0 with the first)
  auto merge = [&](int64_t s0, int64_t s1) -> hipError_t {
    const int64_t first = s0 == 0 ? 0 : s0 + 1;
    return launch_stats_merge_rows((const double2*)partial + first * V, (S + 1) * V, n_groups,
                                   (int)gs, N, s1 - first + 1, V, n, par->ddof, delta0,
                                   mean_d + first * V, var_d + first * V, ks);
  };
  // (ks is already ordered after the caller's earlier work, and the design
  // and basis are on it: the first contraction does not wait for the setup)
  IntegArgs<R> a{};
  a.coef = coef;
  a.state = (R*)state;
  a.partial = partial;
  a.delta0 = delta0;
  a.traj_slot = slot_d;
  a.traj = traj_d;
  a.nonfinite = cnt_d;
  a.first_bad = (long long*)(cnt_d + 1);
  a.notconv = cnt_d + 2;
  a.n = n;
  a.P = P;
  a.V = V;
  a.N = N;
  a.S = S;
  a.lanes = lanes;
  a.dt = (R)par->dt;
  a.wb = (R)wb;
  a.recenter = recenter;
  a.rrf_w = rrf_w;
  a.rrf_acc = rrf_acc;
  a.rrf = rrf_d;
  a.sde = sde;
  // With a network event, a chunk ends at the event step and the chunks from
  // there on run with the post-event coefficients.
  int64_t k = 0, prev0 = 0, last0 = 0;
  for (int64_t s0 = 0, s1 = 0; s0 < S; s0 = s1, ++k) {
    s1 = std::min<int64_t>(S, s0 + Sc);
    if (coef_post && s0 < s_event && s1 > s_event) s1 = s_event;
    const bool post = coef_post && s0 >= s_event;
    a.coef = post ? coef_post : coef;
    a.n_ref = post ? n_ref_post : n;
    const int64_t Cc = 2 * (s1 - s0) + 1;
    const int b = (int)(k & 1);
    hipError_t e = hipSuccess;
    if (k >= 2) e = hipStreamWaitEvent(ks, c->gev[2 + b], 0);  // chunk k-2 done with w[b]
    if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
    ct.gemm0.push_back(evp.record(ks));
    if (par->precision == FMC_F64)
      e = launch_kle_f64(zeta, phi, C, P, par->K, N, Cc, 2 * s0, (double*)w[b], ks);
    else if (par->precision == FMC_F32)
      e = launch_kle_f64_to_f32(zeta, phi, C, P, par->K, N, Cc, 2 * s0, (float*)w[b], ks);
    else  // BF16 x3 on the operands split once before the first chunk
      e = launch_kle_bf16x3_split(s16[0], s16[1], kle_kp(par->K), s16[2], s16[3], P, N, Cc,
                                  2 * s0, (float*)w[b], ks);
    if (e != hipSuccess) return fail(FMC_EDEVICE, std::string("KLE launch: ") + hipGetErrorString(e));
    ct.gemm1.push_back(evp.record(ks));
    if (hipEventRecord(c->gev[b], ks) != hipSuccess || hipStreamWaitEvent(c->stream, c->gev[b], 0) != hipSuccess)
      return fail(FMC_EDEVICE, "stream ordering failed");
    if (k >= 1) {  // chunk k-1's rows, after its integrator (queued behind the contraction)
      if (hipStreamWaitEvent(ks, c->gev[2 + (1 - b)], 0) != hipSuccess || merge(prev0, s0) != hipSuccess)
        return fail(FMC_EDEVICE, "statistics merge launch failed");
    }
    prev0 = s0;
    last0 = s0;
    a.w = (const R*)w[b];
    a.s_begin = s0;
    a.s_end = s1;
    a.c_base = 2 * s0;
    ct.int0.push_back(evp.record());
    if constexpr (sizeof(R) == 8)
      e = trap ? launch_trap_f64(vid, a, n_groups, c->stream)
               : launch_integrate_f64(vid, a, n_groups, c->stream);
    else
      e = launch_integrate_f32(vid, a, n_groups, c->stream);
    if (e != hipSuccess)
      return fail(FMC_EDEVICE, std::string("integrator launch: ") + hipGetErrorString(e));
    ct.int1.push_back(evp.record());
    if (hipEventRecord(c->gev[2 + b], c->stream) != hipSuccess)
      return fail(FMC_EDEVICE, "stream ordering failed");
  }
  // the last chunk's rows, then the main stream waits for every merge
  if (hipStreamWaitEvent(ks, c->gev[2 + (int)((k - 1) & 1)], 0) != hipSuccess)
    return fail(FMC_EDEVICE, "stream ordering failed");
  ct.st0 = evp.record(ks);
  if (merge(last0, S) != hipSuccess) return fail(FMC_EDEVICE, "statistics merge launch failed");
  ct.st1 = evp.record(ks);
  if (hipEventRecord(c->ev[6], ks) != hipSuccess || hipStreamWaitEvent(c->stream, c->ev[6], 0) != hipSuccess)
    return fail(FMC_EDEVICE, "stream ordering failed");
  return FMC_OK;
}

}  // namespace

// The second stream of fmc_run (LHS design, KLE contractions, statistics
// merges beside the integrator) and its ordering events.
int ensure_gstream(Context* c) {
  if (!c->gstream && hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess)
    return fail(FMC_EDEVICE, "cannot create the contraction stream");
  for (auto& e : c->gev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return fail(FMC_EDEVICE, "hipEventCreate failed");
  return FMC_OK;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(FMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

int run_single(Context* c, const fmc_system* sys, const fmc_disturbance* dist,
               const fmc_params* par, fmc_outputs* out) {
  int64_t S = 0;
  int rc = validate(sys, dist, par, &S);
  if (rc) return rc;
  if (!out->mean || !out->var) return fail(FMC_EINVAL, "mean and var outputs are required");
  if (out->mem_kind != FMC_MEM_HOST && out->mem_kind != FMC_MEM_DEVICE)
    return fail(FMC_EINVAL, "unknown mem_kind");
  if (out->n_traj < 0 || (out->n_traj > 0 && (!out->traj_idx || !out->traj)))
    return fail(FMC_EINVAL, "n_traj > 0 needs traj_idx and traj");
  HIPCHK(hipSetDevice(c->device));
  // a diffusion matrix is carried by the mixed design; the integrator sees sigma = 1
  UnitSigma unit_sigma;
  dist = unit_sigma.apply(dist);
  if (sys->model == FMC_FLUXDECAY_IEEET1) {
    if (out->rrf) return fail(FMC_EINVAL, "the fused RRF runs with the classical model");
    return run_fd(c, sys, dist, par, out, S);
  }
  const int n = sys->n_gen, P = dist->n_proc, K = par->K;
  const int64_t N = par->N, M = (int64_t)P * K, C = 2 * S + 1;
  const int V = 2 * n + P;
  const bool dev_out = out->mem_kind == FMC_MEM_DEVICE;
  const bool f64 = par->precision == FMC_F64;
  const int bw = f64 ? 8 : 4;
  // the implicit trapezoid runs on the shapes of the one-trajectory-per-lane
  // variants (the smallest that fits, or the one asked for); the general Ito
  // processes run on every variant, by default the one tuned for the shape
  const bool trap = par->integrator == FMC_TRAP;
  const bool lane_only = trap;
  int vid = par->variant >= 0 ? par->variant
                              : (lane_only ? -1 : pick_variant(c, n, P, N, par->precision));
  if (lane_only && vid < 0) {
    for (int i = 0; i < n_variants(); ++i) {
      const VariantInfo& v = variant(i);
      if (v.L != 1 || v.NG < n || v.PM < P || (trap && v.NG > kTrapMaxGen)) continue;
      if (vid < 0 || v.NG * v.NG + v.PM < variant(vid).NG * variant(vid).NG + variant(vid).PM) vid = i;
    }
  }
  if (vid < 0 || vid >= n_variants())
    return fail(FMC_EINVAL, "no integrator variant for n=" + std::to_string(n) + ", P=" + std::to_string(P));
  const VariantInfo& vi = variant(vid);
  if (vi.NG < n || vi.PM < P) return fail(FMC_EINVAL, "variant too small for the system");
  if (trap && (vi.L != 1 || vi.NG > kTrapMaxGen))
    return fail(FMC_EINVAL, "the implicit trapezoid runs on one-trajectory-per-lane variants of at "
                            "most 16 machines");
  const double f0 = sys->f0_hz > 0.0 ? sys->f0_hz : 60.0;
  const double wb = 2.0 * M_PI * f0;

  EventPool evp;
  evp.on = out->report != nullptr;
  evp.st = c->stream;
  const size_t held0 = c->held;
  const int ev_start = evp.record();
  // The second stream (design, basis, contractions, merges) starts after the
  // work already queued on the caller's stream, then runs beside the
  // reduction and setup below.
  if ((rc = ensure_gstream(c))) return rc;
  HIPCHK(hipEventRecord(c->ev[5], c->stream));
  HIPCHK(hipStreamWaitEvent(c->gstream, c->ev[5], 0));

  double* canon = nullptr;
  int32_t* gen_d = nullptr;
  int* status_d = nullptr;
  if ((rc = stage_scenario(c, sys, dist, "run", &canon, &gen_d, &status_d))) return rc;
  const CanonLayout CL{n, P};
  const double* delta0_d = canon + CL.delta0();

  void* coef = nullptr;
  const PackLayout PL{vi.NG, vi.PM};
  if ((rc = c->ensure("coef", (size_t)PL.size() * bw, &coef))) return rc;
  HIPCHK(f64 ? launch_pack<double>(canon, n, P, gen_d, vi.NG, vi.PM, (double*)coef, c->stream)
             : launch_pack<float>(canon, n, P, gen_d, vi.NG, vi.PM, (float*)coef, c->stream));

  // A network event: the post-event admittance (given, or the network reduced
  // with the tripped machine's internal node cut off by an infinite X'd), the
  // coefficients of the same operating point on it, and the processes at a
  // tripped machine injecting nowhere.
  void* coef_post = nullptr;
  int64_t s_event = 0;
  int n_ref_post = n;
  if (const fmc_event* ev = sys->event) {
    s_event = (int64_t)std::llround(ev->t / par->dt);
    const int g = ev->tripped;
    Stager sg;
    std::vector<double2> Yph, Yinfh;
    const double2 *Yp_d = nullptr, *Yinf_d = nullptr;
    if (ev->Y_re) {
      Yph.resize((size_t)n * n);
      for (size_t q = 0; q < Yph.size(); ++q) Yph[q] = make_double2(ev->Y_re[q], ev->Y_im[q]);
      sg.add(Yph.data(), Yph.size(), &Yp_d);
    }
    if (sys->infinite_bus) {
      const double *yr = ev->Yinf_re ? ev->Yinf_re : sys->Yinf_re;
      const double *yi = ev->Yinf_re ? ev->Yinf_im : sys->Yinf_im;
      Yinfh.resize(n);
      for (int i = 0; i < n; ++i) Yinfh[i] = make_double2(yr[i], yi[i]);
      sg.add(Yinfh.data(), Yinfh.size(), &Yinf_d);
    }
    std::vector<int32_t> genp(dist->gen, dist->gen + P);
    for (auto& q : genp)
      if (q == g) q = -1;
    const int32_t* genp_d = nullptr;
    sg.add(genp.data(), genp.size(), &genp_d);
    if ((rc = sg.upload(c, "stage_event"))) return rc;
    if (!ev->Y_re) {
      std::vector<double> xdp(sys->net->gen_xdp, sys->net->gen_xdp + n);
      xdp[g] = INFINITY;  // 1/(j X'd) = 0: the internal node is cut off
      fmc_network np = *sys->net;
      np.gen_xdp = xdp.data();
      void* yb = nullptr;
      if ((rc = c->ensure("yred_post", (size_t)n * n * sizeof(double2), &yb))) return rc;
      if ((rc = kron_on_device(c, &np, (double2*)yb, status_d + 3, "net_post"))) return rc;
      Yp_d = (const double2*)yb;
    }
    void* cp = nullptr;
    if ((rc = c->ensure("canon_post", (size_t)CL.size() * sizeof(double), &cp))) return rc;
    HIPCHK(launch_setup_post(canon, n, P, Yp_d, Yinf_d, sys->V_inf, g, (double*)cp, c->stream));
    if ((rc = c->ensure("coef_post", (size_t)PL.size() * bw, &coef_post))) return rc;
    HIPCHK(f64 ? launch_pack<double>((const double*)cp, n, P, genp_d, vi.NG, vi.PM, (double*)coef_post, c->stream)
               : launch_pack<float>((const double*)cp, n, P, genp_d, vi.NG, vi.PM, (float*)coef_post, c->stream));
    n_ref_post = n - (g >= 0 ? 1 : 0);
  }

  void* phi = nullptr;
  if ((rc = c->ensure("phi", (size_t)K * C * sizeof(double), &phi))) return rc;
  HIPCHK(launch_basis(par->basis, K, S, par->T, (double*)phi, c->gstream));

  // the design runs on the second stream, beside the setup work above; the
  // contractions follow it there
  const int ev_lhs0 = evp.record(c->gstream);
  const double* zeta = par->zeta_in;
  double* zeta_dev = nullptr;
  int32_t* dc_status = nullptr;  // correlation reduction of the design, if asked for
  int32_t* strata_dev = nullptr;
  if (!zeta) {
    void* p = nullptr;
    if (out->zeta && dev_out) {
      zeta_dev = out->zeta;
    } else {
      if ((rc = c->ensure("zeta", (size_t)M * N * sizeof(double), &p))) return rc;
      zeta_dev = (double*)p;
    }
    if (out->strata) {
      if (dev_out) {
        strata_dev = out->strata;
      } else {
        if ((rc = c->ensure("strata", (size_t)M * N * sizeof(int32_t), &p))) return rc;
        strata_dev = (int32_t*)p;
      }
    }
    const bool decor = par->sampler == FMC_LHS_DECOR;
    int32_t* lhs_strata = strata_dev;
    if (decor && !lhs_strata) {
      if ((rc = c->ensure("dc_strata", (size_t)M * N * sizeof(int32_t), &p))) return rc;
      lhs_strata = (int32_t*)p;
    }
    HIPCHK(launch_lhs(par->seed, (int32_t)M, N, decor ? FMC_LHS : par->sampler, lhs_strata,
                      zeta_dev, c->gstream));
    if (decor && (rc = decorrelate_design(c, (int32_t)M, N, zeta_dev, strata_dev, lhs_strata,
                                          &dc_status, c->gstream)))
      return rc;
    zeta = zeta_dev;
  }
  if (dist->sigma_mat && (rc = mix_design(c, dist, K, N, &zeta, c->gstream))) return rc;
  // BF16 x3: the basis and the design split into BF16 hi/lo planes once
  const void* s16[4] = {nullptr, nullptr, nullptr, nullptr};
  if (par->precision == FMC_BF16X3) {
    const int Kp = kle_kp(K);
    void *pp = nullptr, *zz = nullptr;
    if ((rc = c->ensure("phi16", (size_t)2 * C * Kp * 2, &pp))) return rc;
    if ((rc = c->ensure("zeta16", (size_t)2 * P * N * Kp * 2, &zz))) return rc;
    s16[0] = pp;
    s16[1] = (const char*)pp + (size_t)C * Kp * 2;
    s16[2] = zz;
    s16[3] = (const char*)zz + (size_t)P * N * Kp * 2;
    HIPCHK(launch_split_bf16((const double*)phi, C, K, C, Kp, 1, 0, 0, pp, (void*)s16[1],
                             c->gstream));
    HIPCHK(launch_split_bf16(zeta, N, K, N, Kp, P, (int64_t)K * N, N * Kp, zz, (void*)s16[3],
                             c->gstream));
  }
  const int ev_lhs1 = evp.record(c->gstream);

  // per-workgroup statistics partials, trajectory slots, counters
  const int64_t gsize = vi.group_size();
  const int64_t n_groups = (N + gsize - 1) / gsize;
  void *partial = nullptr, *cnt = nullptr;
  if ((rc = c->ensure("partial", (size_t)n_groups * (S + 1) * V * 2 * sizeof(double), &partial)))
    return rc;
  if ((rc = c->ensure("counters", 64, &cnt))) return rc;
  {
    void* h = nullptr;
    if ((rc = c->host_stage("counters", 64, &h))) return rc;
    unsigned long long* init = (unsigned long long*)h;
    init[0] = 0ULL;
    init[1] = (unsigned long long)LLONG_MAX;
    init[2] = 0ULL;
    HIPCHK(hipMemcpyAsync(cnt, init, 3 * sizeof(unsigned long long), hipMemcpyHostToDevice, c->stream));
  }
  int32_t* slot_d = nullptr;
  double* traj_d = nullptr;
  if (out->n_traj > 0) {
    std::vector<int32_t> slot(N, -1);
    for (int q = 0; q < out->n_traj; ++q) {
      const int64_t idx = out->traj_idx[q];
      if (idx < 0 || idx >= N) return fail(FMC_EINVAL, "traj_idx out of range");
      if (slot[idx] >= 0) return fail(FMC_EINVAL, "traj_idx has a duplicate");
      slot[idx] = q;
    }
    void *p = nullptr, *h = nullptr;
    if ((rc = c->ensure("traj_slot", (size_t)N * sizeof(int32_t), &p))) return rc;
    if ((rc = c->host_stage("traj_slot", (size_t)N * sizeof(int32_t), &h))) return rc;
    std::memcpy(h, slot.data(), (size_t)N * sizeof(int32_t));
    slot_d = (int32_t*)p;
    HIPCHK(hipMemcpyAsync(slot_d, h, (size_t)N * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    if (dev_out) {
      traj_d = out->traj;
    } else {
      if ((rc = c->ensure("traj", (size_t)out->n_traj * (S + 1) * V * sizeof(double), &p))) return rc;
      traj_d = (double*)p;
    }
  }

  // the RRF accumulated in the integrators' epilogue
  const double* rrf_wd = nullptr;
  double *rrf_acc = nullptr, *rrf_dev = nullptr;
  if (out->rrf) {
    if (!out->rrf_w) return fail(FMC_EINVAL, "rrf needs rrf_w");
    void *p = nullptr, *h = nullptr;
    if ((rc = c->ensure("rrf_w", (size_t)V * sizeof(double), &p))) return rc;
    if ((rc = c->host_stage("rrf_w", (size_t)V * sizeof(double), &h))) return rc;
    std::memcpy(h, out->rrf_w, (size_t)V * sizeof(double));
    HIPCHK(hipMemcpyAsync(p, h, (size_t)V * sizeof(double), hipMemcpyHostToDevice, c->stream));
    rrf_wd = (const double*)p;
    if ((rc = c->ensure("rrf_acc", (size_t)N * sizeof(double), &p))) return rc;
    rrf_acc = (double*)p;
    if (dev_out) {
      rrf_dev = out->rrf;
    } else {
      if ((rc = c->ensure("rrf_out", (size_t)N * sizeof(double), &p))) return rc;
      rrf_dev = (double*)p;
    }
  }
  // the general Ito processes' rows, in the integrator's arithmetic type
  const void* sde_d = nullptr;
  {
    std::vector<double> tab;
    if (sde_table(dist, par->basis, variant(vid).PM, tab)) {
      void *p = nullptr, *h = nullptr;
      const size_t bytes = tab.size() * bw;
      if ((rc = c->ensure("sde", bytes, &p))) return rc;
      if ((rc = c->host_stage("sde", bytes, &h))) return rc;
      for (size_t q = 0; q < tab.size(); ++q) {
        if (f64) ((double*)h)[q] = tab[q];
        else ((float*)h)[q] = (float)tab[q];
      }
      HIPCHK(hipMemcpyAsync(p, h, bytes, hipMemcpyHostToDevice, c->stream));
      sde_d = p;
    }
  }
  const int64_t Sc = par->time_chunk > 0 ? std::min<int64_t>(par->time_chunk, S)
                                         : auto_chunk(S, P, N, bw);
  double *mean_d = out->mean, *var_d = out->var;
  if (!dev_out) {
    void *pm = nullptr, *pv = nullptr;
    if ((rc = c->ensure("mean", (size_t)(S + 1) * V * sizeof(double), &pm))) return rc;
    if ((rc = c->ensure("var", (size_t)(S + 1) * V * sizeof(double), &pv))) return rc;
    mean_d = (double*)pm;
    var_d = (double*)pv;
  }
  ChunkTimes ct;
  if (f64)
    rc = run_chunks<double>(c, par, vid, n, P, S, N, wb, zeta, (const double*)phi,
                            (const double*)coef, delta0_d, (double*)partial, slot_d, traj_d,
                            (unsigned long long*)cnt, Sc, mean_d, var_d, sys->infinite_bus ? 0 : 1, trap, s16,
                            (const double*)coef_post, s_event, n_ref_post, rrf_wd, rrf_acc,
                            rrf_dev, (const double*)sde_d, evp, ct);
  else
    rc = run_chunks<float>(c, par, vid, n, P, S, N, wb, zeta, (const double*)phi,
                           (const float*)coef, delta0_d, (double*)partial, slot_d, traj_d,
                           (unsigned long long*)cnt, Sc, mean_d, var_d, sys->infinite_bus ? 0 : 1, trap, s16,
                           (const float*)coef_post, s_event, n_ref_post, rrf_wd, rrf_acc,
                           rrf_dev, (const float*)sde_d, evp, ct);
  if (rc) return rc;
  // statistics: merged per chunk on the second stream, joined into c->stream
  const int ev_end = evp.record();

  if (!dev_out) {
    const size_t sv = (size_t)(S + 1) * V * sizeof(double);
    HIPCHK(hipMemcpyAsync(out->mean, mean_d, sv, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(out->var, var_d, sv, hipMemcpyDeviceToHost, c->stream));
    if (traj_d)
      HIPCHK(hipMemcpyAsync(out->traj, traj_d, (size_t)out->n_traj * sv, hipMemcpyDeviceToHost, c->stream));
    if (rrf_dev)
      HIPCHK(hipMemcpyAsync(out->rrf, rrf_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (out->zeta && zeta_dev)
      HIPCHK(hipMemcpyAsync(out->zeta, zeta_dev, (size_t)M * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (out->strata && strata_dev)
      HIPCHK(hipMemcpyAsync(out->strata, strata_dev, (size_t)M * N * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  }
  void* hb = nullptr;
  if ((rc = c->host_stage("readback", 64, &hb))) return rc;
  // status: [0] operating point, [1] reduction, [3] post-event reduction
  // (from the device), [4] correlation reduction of the design
  int* status = (int*)hb;
  unsigned long long* cn = (unsigned long long*)((char*)hb + 32);
  status[4] = 0;
  HIPCHK(hipMemcpyAsync(status, status_d, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(cn, cnt, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  if (dc_status)
    HIPCHK(hipMemcpyAsync(status + 4, dc_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (status[1] != 0) return fail(FMC_EINVAL, "network reduction failed (singular Y_BB)");
  if (sys->event && status[3] != 0)
    return fail(FMC_EINVAL, "post-event network reduction failed (singular Y_BB)");
  if (status[4] != 0)
    return fail(FMC_EINVAL, "the design's sample covariance is not positive definite");
  if (status[0] != 0) return fail(FMC_ENOTCONV, "operating-point Newton solve did not converge");

  if (out->report) {
    fmc_report* r = out->report;
    std::memset(r, 0, sizeof(*r));
    r->t_total_s = evp.secs(ev_start, ev_end);
    r->t_lhs_s = evp.secs(ev_lhs0, ev_lhs1);
    for (size_t q = 0; q < ct.gemm0.size(); ++q) {
      r->t_gemm_s += evp.secs(ct.gemm0[q], ct.gemm1[q]);
      r->t_integrate_s += evp.secs(ct.int0[q], ct.int1[q]);
    }
    r->t_stats_s = evp.secs(ct.st0, ct.st1);  // the merge left after the integrator
    r->n_nonfinite = (int64_t)cn[0];
    r->first_nonfinite = cn[0] ? (int64_t)cn[1] : -1;
    r->variant_id = vid;
    r->lanes_per_traj = vi.L;
    r->tile = (int32_t)gsize;
    r->time_chunk = (int32_t)Sc;
    r->hbm_peak_bytes = (int64_t)std::max(c->held, held0);
  }
  if (cn[2] != 0)  // outputs are written from the last Newton iterates
    return fail(FMC_ENOTCONV, std::to_string(cn[2]) + " sample paths had a trapezoid step whose "
                                                      "Newton iteration did not converge");
  if (cn[0] != 0)
    return fail(FMC_ENONFINITE, std::to_string(cn[0]) + " sample paths became non-finite (first: " +
                                    std::to_string((long long)cn[1]) + ")");
  return FMC_OK;
}

}  // namespace fmc
