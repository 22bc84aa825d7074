// k_trap.hip -- the implicit trapezoidal rule for the classical multimachine
// model (the integrator option of Alg. 1 step 3, applied to eq. 9 inside the
// swing equations), FP64, one trajectory per lane.
//
// Each step solves z = y + h/2 (f(y, w(t)) + f(z, w(t + h))) by Newton's
// method from the explicit Euler predictor z = y + h f(y, w(t)), with the
// Jacobian re-evaluated at every iterate, until the correction satisfies
// |dz|_inf <= 1e-13 (1 + |z|_inf) (z the absolute state), at most 20
// iterations; a trajectory that misses this in any step is counted (the
// caller reports FMC_ENOTCONV) and continues from the last iterate.
//
// The Newton matrix I - h/2 J has the block structure of the swing
// equations, so the correction is found from one n x n system: with
// h' = h/2, c_p = g_xi,p / (1 + h' theta_p) for the disturbances,
//   [diag(1 + h' D_i / 2H_i) + h'^2 w_b / 2H_i dPe_i/d delta_k] b
//       = g_w,i + h'/2H_i (sum_p B_ip c_p - sum_k dPe_i/d delta_k g_delta,k)
// for the speed deviations, and a = g_delta + h' w_b b for the angles (the
// Schur complement of the full system, the same solution).  The n x n matrix
// is diagonally dominant whenever the step resolves the swing modes
// (h'^2 w_b |dPe/d delta| << 2H), so it is factored without pivoting; a zero
// pivot ends the iteration unconverged.  Each lane keeps its matrix in its
// own column of LDS ([i][k][lane]: consecutive lanes, consecutive words).
#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"
#include "k_integrate.hpp"
#include "k_variants.hpp"

namespace fmc {

namespace {

constexpr int kTrapMaxIter = 20;
constexpr double kTrapTol = 1e-13;

// f(y) of the swing equations and OU processes in deviation form (as
// swing_rhs) and, if J is given, dPe_i/d delta_k at y into J[(i NG + k) 64].
template <int NG, int PM>
__device__ __forceinline__ void rhs_and_jac(const double* cfg, double wb, const double (&yd)[NG],
                                            const double (&yw)[NG], const double (&yx)[PM],
                                            const double (&wv)[PM], double (&kd)[NG],
                                            double (&kw)[NG], double (&kx)[PM], double* J) {
  constexpr PackLayout L{NG, PM};
  asm volatile("" : "+s"(cfg));
  const cptr<double> cf = (cptr<double>)cfg;
  double dc[NG], ds[NG];
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    double sh, ch;
    sincos_r_nb(yd[k] * 0.5, sh, ch);
    const double sd = 2.0 * sh * ch, omc = 2.0 * sh * sh;
    const double c0 = cf[L.c0() + k], s0 = cf[L.s0() + k];
    dc[k] = -(c0 * omc + s0 * sd);
    ds[k] = c0 * sd - s0 * omc;
  }
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    double ir = 0.0, ii = 0.0;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const double yr = cf[L.yre() + i * NG + k], yi = cf[L.yim() + i * NG + k];
      ir = fma(yr, dc[k], ir);
      ir = fma(-yi, ds[k], ir);
      ii = fma(yr, ds[k], ii);
      ii = fma(yi, dc[k], ii);
    }
    const double er_i = cf[L.c0() + i] + dc[i], ei_i = cf[L.s0() + i] + ds[i];
    const double dpe = dc[i] * cf[L.i0r() + i] + ds[i] * cf[L.i0i() + i] + er_i * ir + ei_i * ii;
    double F = cf[L.res() + i] - dpe - cf[L.dmp() + i] * yw[i];
#pragma unroll
    for (int p = 0; p < PM; ++p) F += cf[L.binc() + i * PM + p] * yx[p];
    kd[i] = wb * yw[i];
    kw[i] = F * cf[L.inv2h() + i];
    if (J) {
      // dPe_i/d delta_k = Re(E~_i conj(j Y_ik E~_k)), plus Re(j E~_i conj(I_i)) on the diagonal
      const double Ir = cf[L.i0r() + i] + ir, Ii = cf[L.i0i() + i] + ii;
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        const double yr = cf[L.yre() + i * NG + k], yi = cf[L.yim() + i * NG + k];
        const double er_k = cf[L.c0() + k] + dc[k], ei_k = cf[L.s0() + k] + ds[k];
        double v = yr * (ei_i * er_k - er_i * ei_k) - yi * (er_i * er_k + ei_i * ei_k);
        if (k == i) v += er_i * Ii - ei_i * Ir;
        J[(i * NG + k) * 64] = v;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PM; ++p) kx[p] = -cf[L.theta() + p] * yx[p] + cf[L.sigma() + p] * wv[p];
}

}  // namespace

template <int NG, int PM>
__global__ void __launch_bounds__(64) k_trap_lane(IntegArgs<double> a) {
  constexpr PackLayout L{NG, PM};
  constexpr int VM = 2 * NG + PM;
  __shared__ double tile[VM][65];
  __shared__ double mat[NG * NG * 64];
  const int lane = threadIdx.x;
  const int64_t gidx = (int64_t)blockIdx.x * 64 + lane;
  const int64_t N = a.N;
  const bool valid = gidx < N;
  const int64_t ns = valid ? gidx : N - 1;
  const int64_t rem = N - (int64_t)blockIdx.x * 64;
  const int cnt = rem < 64 ? (int)rem : 64;
  const int n = a.n, P = a.P;
  const double* __restrict__ cf = a.coef;
  const double* __restrict__ w = a.w;
  const int slot = (valid && a.traj_slot) ? a.traj_slot[ns] : -1;
  double* J = mat + lane;

  double yd[NG], yw[NG], yx[PM];
  double racc = 0.0;  // the epilogue's RRF sum (see IntegArgs::rrf_w)
  if (a.s_begin == 0) {
#pragma unroll
    for (int i = 0; i < NG; ++i) { yd[i] = 0.0; yw[i] = 0.0; }
#pragma unroll
    for (int p = 0; p < PM; ++p) yx[p] = cf[L.xi0() + p];
    emit_step<double, NG, PM>(a, tile, lane, cnt, 0, slot, 0.0, yd, yw, yx);
    if (a.rrf_w) {
      const double u = rrf_u_lane<double, NG, PM>(a, 0.0, yd, yw, yx);
      racc = 0.5 * u * u;
    }
  } else {
    if (a.rrf_w) racc = a.rrf_acc[ns];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      yd[i] = a.state[(int64_t)i * a.lanes + gidx];
      yw[i] = a.state[(int64_t)(NG + i) * a.lanes + gidx];
    }
#pragma unroll
    for (int p = 0; p < PM; ++p) yx[p] = a.state[(int64_t)(2 * NG + p) * a.lanes + gidx];
  }

  const double dt = a.dt, hh = 0.5 * a.dt, wb = a.wb;
  bool failed = false;
  for (int64_t s = a.s_begin; s < a.s_end; ++s) {
    const int64_t cl = 2 * s - a.c_base;
    double w0[PM], w2[PM];
#pragma unroll
    for (int p = 0; p < PM; ++p) {
      w0[p] = p < P ? w[(cl * P + p) * N + ns] : 0.0;
      w2[p] = p < P ? w[((cl + 2) * P + p) * N + ns] : 0.0;
    }
    double k1d[NG], k1w[NG], k1x[PM];
    rhs_and_jac<NG, PM>(cf, wb, yd, yw, yx, w0, k1d, k1w, k1x, nullptr);
    double zd[NG], zw[NG], zx[PM];
#pragma unroll
    for (int i = 0; i < NG; ++i) { zd[i] = yd[i] + dt * k1d[i]; zw[i] = yw[i] + dt * k1w[i]; }
#pragma unroll
    for (int p = 0; p < PM; ++p) zx[p] = yx[p] + dt * k1x[p];
    bool conv = false;
    for (int it = 0; it < kTrapMaxIter && !conv; ++it) {
      double fd[NG], fw[NG], fx[PM];
      rhs_and_jac<NG, PM>(cf, wb, zd, zw, zx, w2, fd, fw, fx, J);
      // residual g = -(z - y - h'(f(y) + f(z)))
      double gd[NG], gw[NG], gx[PM];
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        gd[i] = -(zd[i] - yd[i] - hh * (k1d[i] + fd[i]));
        gw[i] = -(zw[i] - yw[i] - hh * (k1w[i] + fw[i]));
      }
#pragma unroll
      for (int p = 0; p < PM; ++p) gx[p] = -(zx[p] - yx[p] - hh * (k1x[p] + fx[p]));
      // disturbances, then the reduced system for the speed deviations
      double cx[PM];
#pragma unroll
      for (int p = 0; p < PM; ++p) cx[p] = gx[p] / (1.0 + hh * cf[L.theta() + p]);
      double r[NG];
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const double ih = cf[L.inv2h() + i];
        double inj = 0.0, jg = 0.0;
#pragma unroll
        for (int p = 0; p < PM; ++p) inj += cf[L.binc() + i * PM + p] * cx[p];
#pragma unroll
        for (int k = 0; k < NG; ++k) jg += J[(i * NG + k) * 64] * gd[k];
        r[i] = gw[i] + hh * ih * (inj - jg);
        const double sc = hh * hh * wb * ih;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          const double m = sc * J[(i * NG + k) * 64] + (k == i ? 1.0 + hh * cf[L.dmp() + i] * ih : 0.0);
          J[(i * NG + k) * 64] = m;
        }
      }
      // LU without pivoting (diagonally dominant), forward elimination of r
      bool sing = false;
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        const double piv = J[(k * NG + k) * 64];
        if (piv == 0.0) sing = true;
        const double inv = 1.0 / piv;
#pragma unroll
        for (int i = k + 1; i < NG; ++i) {
          const double f = J[(i * NG + k) * 64] * inv;
#pragma unroll
          for (int j = k + 1; j < NG; ++j) J[(i * NG + j) * 64] -= f * J[(k * NG + j) * 64];
          r[i] -= f * r[k];
        }
      }
      double b[NG];
#pragma unroll
      for (int k = NG - 1; k >= 0; --k) {
        double acc = r[k];
#pragma unroll
        for (int j = k + 1; j < NG; ++j) acc -= J[(k * NG + j) * 64] * b[j];
        b[k] = acc / J[(k * NG + k) * 64];
      }
      if (sing) break;
      double dn = 0.0, zn = 0.0;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const double da = gd[i] + hh * wb * b[i];
        zd[i] += da;
        zw[i] += b[i];
        if (i < n) {
          dn = fmax(dn, fmax(fabs(da), fabs(b[i])));
          zn = fmax(zn, fmax(fabs(a.delta0[i] + zd[i]), fabs(zw[i])));
        }
      }
#pragma unroll
      for (int p = 0; p < PM; ++p) {
        zx[p] += cx[p];
        if (p < P) {
          dn = fmax(dn, fabs(cx[p]));
          zn = fmax(zn, fabs(zx[p]));
        }
      }
      conv = dn <= kTrapTol * (1.0 + zn);
    }
    failed |= !conv;
#pragma unroll
    for (int i = 0; i < NG; ++i) { yd[i] = zd[i]; yw[i] = zw[i]; }
#pragma unroll
    for (int p = 0; p < PM; ++p) yx[p] = zx[p];
    emit_step<double, NG, PM>(a, tile, lane, cnt, s + 1, slot, 0.0, yd, yw, yx);
    if (a.rrf_w) {
      const double u = rrf_u_lane<double, NG, PM>(a, 0.0, yd, yw, yx);
      racc += (s + 1 == a.S ? 0.5 : 1.0) * u * u;
    }
  }
  if (a.rrf_w && valid) {
    a.rrf_acc[gidx] = racc;
    if (a.s_end == a.S) a.rrf[gidx] = sqrt(racc / (double)a.S);
  }

#pragma unroll
  for (int i = 0; i < NG; ++i) {
    a.state[(int64_t)i * a.lanes + gidx] = yd[i];
    a.state[(int64_t)(NG + i) * a.lanes + gidx] = yw[i];
  }
#pragma unroll
  for (int p = 0; p < PM; ++p) a.state[(int64_t)(2 * NG + p) * a.lanes + gidx] = yx[p];
  if (valid && failed) atomicAdd(a.notconv, 1ULL);

  if (a.s_end == a.S && valid) {
    bool bad = false;
#pragma unroll
    for (int i = 0; i < NG; ++i) bad |= !isfinite(yd[i]) || !isfinite(yw[i]);
#pragma unroll
    for (int p = 0; p < PM; ++p) bad |= !isfinite(yx[p]);
    if (bad) {
      atomicAdd(a.nonfinite, 1ULL);
      atomicMin(a.first_bad, (long long)gidx);
    }
  }
}

// The trapezoid runs on the one-trajectory-per-lane variants of at most
// kTrapMaxGen machines (their (NG, PM) shapes and group size 64).
hipError_t launch_trap_f64(int variant_id, const IntegArgs<double>& a, int64_t n_groups,
                           hipStream_t st) {
  int id = 0;
#define FMC_X(NG, PM, L, WPB)                                                                 \
  if (variant_id == id) {                                                                     \
    if constexpr (L == 1 && NG <= kTrapMaxGen) {                                              \
      hipLaunchKernelGGL((k_trap_lane<NG, PM>), dim3((unsigned)n_groups), dim3(64), 0, st, a); \
      return hipGetLastError();                                                               \
    }                                                                                         \
    return hipErrorInvalidValue;                                                              \
  }                                                                                           \
  ++id;
  FMC_VARIANTS(FMC_X)
#undef FMC_X
  return hipErrorInvalidValue;
}

}  // namespace fmc
