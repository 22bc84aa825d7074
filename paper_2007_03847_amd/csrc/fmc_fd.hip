// fmc_fd.hip -- one flux-decay scenario through the method (Alg. 1): the
// common setup (network reduction, operating point), the flux-decay operating
// point, LHS design, basis, then per time chunk the KLE path contraction, the
// matrix-core integrator over all tiles and the merge of the chunk's
// statistics rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fmc_runtime.hpp"

namespace fmc {

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(FMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

int fd_plan(int64_t N, int n_cu, FdPlan* p) {
  p->tiles = (N + 15) / 16;
  const int64_t slots = std::max(1, n_cu);  // one workgroup per CU (256 on MI355X)
  p->tiles_per_item = (p->tiles + slots - 1) / slots;
  p->n_items = (p->tiles + p->tiles_per_item - 1) / p->tiles_per_item;
  return FMC_OK;
}

int run_fd(Context* c, const fmc_system* sys, const fmc_disturbance* dist, const fmc_params* par,
           fmc_outputs* out, int64_t S) {
  const int n = sys->n_gen, P = dist->n_proc, K = par->K;
  const int64_t N = par->N, M = (int64_t)P * K, C = 2 * S + 1;
  const int V = 6 * n + P;
  const int n_pad = 16 * ((n + 15) / 16), NB = n_pad / 16;
  const bool dev_out = out->mem_kind == FMC_MEM_DEVICE;
  const double f0 = sys->f0_hz > 0.0 ? sys->f0_hz : 60.0;
  int rc;
  hipEvent_t e0 = c->ev[0], e1 = c->ev[1], e2 = c->ev[2];
  const size_t held0 = c->held;
  HIPCHK(hipEventRecord(e0, c->stream));

  double* canon = nullptr;
  int32_t* gen_d = nullptr;
  int* status_d = nullptr;
  if ((rc = stage_scenario(c, sys, dist, "run", &canon, &gen_d, &status_d))) return rc;
  // flux-decay data: E and the parameters
  Stager sg;
  const double *E_d = nullptr, *prm_d = nullptr;
  sg.add(sys->E, n, &E_d);
  sg.add(sys->model_params, (size_t)n * kFdParams, &prm_d);
  if ((rc = sg.upload(c, "fd_in", c->stream))) return rc;
  void *fd = nullptr, *coef = nullptr, *ap = nullptr;
  if ((rc = c->ensure("fd_block", (size_t)FdLayout{n}.size() * 8, &fd))) return rc;
  if ((rc = c->ensure("fd_coef", (size_t)FdPack{n_pad}.size() * 4, &coef))) return rc;
  if ((rc = c->ensure("fd_ap", (size_t)NB * (n_pad / 4) * 64 * sizeof(float2), &ap))) return rc;
  HIPCHK(launch_setup_fd(canon, n, P, E_d, prm_d, (double*)fd, c->stream));
  HIPCHK(launch_pack_fd(canon, n, P, prm_d, (const double*)fd, gen_d, n_pad, (float*)coef,
                        (float2*)ap, c->stream));
  // FMC_BF16X3: the network product in BF16 x3 on the matrix cores too
  const bool bf = fd_bf16_product(par);
  const int n_padk = 32 * ((n + 31) / 32);
  void* ap16 = nullptr;
  if (bf) {
    if ((rc = c->ensure("fd_ap16", fd_ap16_bytes(n_pad, n_padk), &ap16))) return rc;
    HIPCHK(launch_pack_fd_y16(canon, n, n_pad, n_padk, ap16, c->stream));
  }

  void* phi = nullptr;
  if ((rc = c->ensure("phi", (size_t)K * C * sizeof(double), &phi))) return rc;
  HIPCHK(launch_basis(par->basis, K, S, par->T, (double*)phi, c->stream));
  const double* zeta = par->zeta_in;
  double* zeta_dev = nullptr;
  int32_t* strata_dev = nullptr;
  int32_t* dc_status = nullptr;  // correlation reduction of the design, if asked for
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
                      zeta_dev, c->stream));
    if (decor && (rc = decorrelate_design(c, (int32_t)M, N, zeta_dev, strata_dev, lhs_strata,
                                          &dc_status, c->stream)))
      return rc;
    zeta = zeta_dev;
  }
  if (dist->sigma_mat && (rc = mix_design(c, dist, K, N, &zeta, c->stream))) return rc;

  // the plan is fixed (not taken from the device) so that a request gives the
  // same bits here and in the served form
  FdPlan pl{};
  fd_plan(N, kFdItems, &pl);
  // chunk: the paths of about 96 MB, and at most about 2 GB of per-tile rows
  const int64_t rows_cap = std::max<int64_t>(8, ((int64_t)1 << 31) / (pl.tiles * V * 16) - 1);
  const int64_t Sc = par->time_chunk > 0
                         ? std::min<int64_t>(par->time_chunk, S)
                         : std::min<int64_t>({S, auto_chunk(S, P, N, 4), rows_cap});
  void *w = nullptr, *state = nullptr, *xstate = nullptr, *rows = nullptr, *cnt = nullptr;
  if ((rc = c->ensure("w", (size_t)(2 * Sc + 1) * P * N * 4, &w))) return rc;
  // state: [tiles][waves][6 states x 8 machines][64 lanes], waves = ceil(NB/2)
  const int NW = (NB + 1) / 2;
  if ((rc = c->ensure("fd_state", (size_t)pl.tiles * NW * 48 * 64 * 4, &state))) return rc;
  if ((rc = c->ensure("fd_xstate", (size_t)pl.tiles * (kFdMaxProc + kFdOffsetRows) * 16 * 4, &xstate))) return rc;
  if ((rc = c->ensure("fd_rows", (size_t)pl.tiles * (Sc + 1) * V * 16, &rows))) return rc;
  if ((rc = c->ensure("counters", 64, &cnt))) return rc;
  HIPCHK(launch_fill_i64((int64_t*)cnt, 0, 1, c->stream));
  HIPCHK(launch_fill_i64((int64_t*)cnt + 1, LLONG_MAX, 1, c->stream));

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
  double *mean_d = out->mean, *var_d = out->var;
  if (!dev_out) {
    void *pm = nullptr, *pv = nullptr;
    if ((rc = c->ensure("mean", (size_t)(S + 1) * V * sizeof(double), &pm))) return rc;
    if ((rc = c->ensure("var", (size_t)(S + 1) * V * sizeof(double), &pv))) return rc;
    mean_d = (double*)pm;
    var_d = (double*)pv;
  }

  FdArgs a{};
  a.coef = (const float*)coef;
  a.ap = (const float2*)ap;
  a.ap16 = ap16;
  a.n_padk = n_padk;
  a.w = (const float*)w;
  a.state = (float*)state;
  a.xstate = (float*)xstate;
  a.off = (const double*)fd + FdLayout{n}.off();
  a.traj_slot = slot_d;
  a.traj = traj_d;
  a.nonfinite = (unsigned long long*)cnt;
  a.first_bad = (long long*)cnt + 1;
  a.rows = (double2*)rows;
  a.row_stride = (Sc + 1) * V;
  a.n = n;
  a.P = P;
  a.V = V;
  a.n_pad = n_pad;
  a.N = N;
  a.S = S;
  a.tiles = pl.tiles;
  a.tiles_per_item = pl.tiles_per_item;
  a.dt = (float)par->dt;
  a.wb = (float)(2.0 * M_PI * f0);
  a.recenter = sys->infinite_bus ? 0 : 1;
  double t_gemm = 0.0, t_int = 0.0;
  for (int64_t s0 = 0; s0 < S; s0 += Sc) {
    const int64_t s1 = std::min<int64_t>(S, s0 + Sc);
    const int64_t Cc = 2 * (s1 - s0) + 1;
    if (par->precision == FMC_F32)
      HIPCHK(launch_kle_f64_to_f32(zeta, (const double*)phi, C, P, K, N, Cc, 2 * s0, (float*)w,
                                   c->stream));
    else
      HIPCHK(launch_kle_bf16x3(zeta, (const double*)phi, C, P, K, N, Cc, 2 * s0, (float*)w,
                               c->stream));
    HIPCHK(hipEventRecord(e1, c->stream));
    a.s_begin = s0;
    a.s_end = s1;
    a.c_base = 2 * s0;
    a.row_base = s0;
    HIPCHK(launch_rk4_fd(a, pl.n_items, c->stream));
    HIPCHK(hipEventRecord(e2, c->stream));
    // rows completed by this chunk: s0+1..s1 (and row 0 in the first chunk)
    const int64_t first = s0 == 0 ? 0 : s0 + 1;
    HIPCHK(launch_stats_merge_rows((const double2*)rows + (first - s0) * V, (Sc + 1) * V,
                                   pl.tiles, 16, N, s1 - first + 1, V, 6 * n, par->ddof, a.off,
                                   mean_d + first * V, var_d + first * V, c->stream));
    if (out->report) {
      // per-chunk timing (the events are reused, so wait for them here)
      HIPCHK(hipEventSynchronize(e2));
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e1, e2) == hipSuccess) t_int += ms * 1e-3;
    }
  }
  (void)t_gemm;

  if (!dev_out) {
    const size_t sv = (size_t)(S + 1) * V * sizeof(double);
    HIPCHK(hipMemcpyAsync(out->mean, mean_d, sv, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(out->var, var_d, sv, hipMemcpyDeviceToHost, c->stream));
    if (traj_d)
      HIPCHK(hipMemcpyAsync(out->traj, traj_d, (size_t)out->n_traj * sv, hipMemcpyDeviceToHost, c->stream));
    if (out->zeta && zeta_dev)
      HIPCHK(hipMemcpyAsync(out->zeta, zeta_dev, (size_t)M * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (out->strata && strata_dev)
      HIPCHK(hipMemcpyAsync(out->strata, strata_dev, (size_t)M * N * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  }
  void* hb = nullptr;
  if ((rc = c->host_stage("readback", 64, &hb))) return rc;
  int* status = (int*)hb;
  unsigned long long* cn = (unsigned long long*)((char*)hb + 16);
  HIPCHK(hipMemcpyAsync(status, status_d, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(cn, cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  status[2] = 0;
  if (dc_status)
    HIPCHK(hipMemcpyAsync(status + 2, dc_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  hipEvent_t e3 = c->ev[3];
  HIPCHK(hipEventRecord(e3, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (status[1] != 0) return fail(FMC_EINVAL, "network reduction failed (singular Y_BB)");
  if (status[2] != 0)
    return fail(FMC_EINVAL, "the design's sample covariance is not positive definite");
  if (status[0] != 0) return fail(FMC_ENOTCONV, "operating-point Newton solve did not converge");
  if (out->report) {
    fmc_report* r = out->report;
    std::memset(r, 0, sizeof(*r));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e3) == hipSuccess) r->t_total_s = ms * 1e-3;
    r->t_integrate_s = t_int;
    r->n_nonfinite = (int64_t)cn[0];
    r->first_nonfinite = cn[0] ? (int64_t)cn[1] : -1;
    r->variant_id = bf ? 1 : 0;
    r->lanes_per_traj = 1;
    r->tile = (int32_t)(pl.tiles_per_item * 16);
    r->time_chunk = (int32_t)Sc;
    r->hbm_peak_bytes = (int64_t)std::max(c->held, held0);
  }
  if (cn[0] != 0)
    return fail(FMC_ENONFINITE, std::to_string(cn[0]) + " sample paths became non-finite (first: " +
                                    std::to_string((long long)cn[1]) + ")");
  return FMC_OK;
}

}  // namespace fmc
