// k_integrate.hpp -- batched fixed-step integrator of the classical
// multimachine model driven by the KLE-rebuilt OU disturbances (eq. 9 in the
// swing equations, Alg. 1 steps 2-3), with the cross-sample statistics of
// Alg. 1 step 4 fused into its epilogue.
//
// One trajectory per lane.  The machine data (reduced admittance, operating
// point) is identical for every lane of a wave, so it is read through uniform
// (scalar) loads and feeds the FMAs as scalar operands: no LDS or VGPR traffic
// for Y.
//
// The state is integrated as deviations from the operating point:
//   y = (d_delta_i, dw_i, xi_p).
// With E~_k = E~0_k exp(j d_delta_k), exp(j d) - 1 = -2 sin^2(d/2) + j sin d,
// so dE~ = E~0 (exp(j d) - 1) is formed from one sincos of d/2 without
// cancellation, and
//   Pe_i - Pe0_i = Re(dE~_i conj(I0_i)) + Re(E~_i conj(dI_i)),  dI = Y dE~,
// which keeps FP32 integration accurate to its own rounding of the deviation.
#pragma once

#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"

namespace fmc {

// Read-only machine data seen through the constant address space: uniform
// loads from it become scalar (SMEM) loads into SGPRs.
template <typename R>
using cptr = const __attribute__((address_space(4))) R*;

// sin and cos together (sincos_r_nb): Cody-Waite reduction x = k pi/2 + r,
// |r| <= pi/4, with pi/2 split into two (FP64) or three (FP32) parts applied
// by FMA (exact enough for |k| < 2^20, far beyond the angles met here), then
// the Taylor polynomials of sin and cos in r^2 (terms through r^15 / r^16 in
// FP64, r^9 / r^10 in FP32; truncation below half an ulp on |r| <= pi/4), and
// the quadrant of k.  When every active lane of the wave has |x| < 0.78 (the
// usual case: the argument is half an angle's deviation from the operating
// point), k is 0 for all of them, the reduction leaves r = x exactly and the
// quadrant step is the identity: sincos_many then skips both with one
// wave-uniform branch, with the same bits as the full path.
__device__ __forceinline__ bool sincos_all_small(bool small) {
  return __builtin_amdgcn_ballot_w64(!small) == 0;
}

// a*b + c as the three-operand FMA: the coefficients below stay in registers
// of their own, read but never overwritten (the two-operand form ties the
// addend to the result and costs a copy of the coefficient per use)
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// the polynomials on the reduced argument r; F3 selects the three-operand
// FMA for the Horner steps (the same rounding as fma(), so the same bits):
// worth it where the coefficients stay resident in vector registers, not
// where register pressure would have them rematerialised at every use
template <bool F3 = true>
__device__ __forceinline__ void sincos_poly(double r, double& sr, double& cr) {
  auto f = [](double a, double b, double c) { return F3 ? fma3(a, b, c) : fma(a, b, c); };
  const double r2 = r * r;
  double ps = -1.0 / 1307674368000.0;
  ps = f(ps, r2, 1.0 / 6227020800.0);
  ps = f(ps, r2, -1.0 / 39916800.0);
  ps = f(ps, r2, 1.0 / 362880.0);
  ps = f(ps, r2, -1.0 / 5040.0);
  ps = f(ps, r2, 1.0 / 120.0);
  ps = f(ps, r2, -1.0 / 6.0);
  sr = fma(r * r2, ps, r);
  double pc = 1.0 / 20922789888000.0;
  pc = f(pc, r2, -1.0 / 87178291200.0);
  pc = f(pc, r2, 1.0 / 479001600.0);
  pc = f(pc, r2, -1.0 / 3628800.0);
  pc = f(pc, r2, 1.0 / 40320.0);
  pc = f(pc, r2, -1.0 / 720.0);
  pc = f(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  cr = fma(r2, pc, 1.0);
}

__device__ __forceinline__ void sincos_poly(float r, float& sr, float& cr) {
  const float r2 = r * r;
  float ps = 1.0f / 362880.0f;
  ps = fmaf(ps, r2, -1.0f / 5040.0f);
  ps = fmaf(ps, r2, 1.0f / 120.0f);
  ps = fmaf(ps, r2, -1.0f / 6.0f);
  sr = fmaf(r * r2, ps, r);
  float pc = -1.0f / 3628800.0f;
  pc = fmaf(pc, r2, 1.0f / 40320.0f);
  pc = fmaf(pc, r2, -1.0f / 720.0f);
  pc = fmaf(pc, r2, 1.0f / 24.0f);
  pc = fmaf(pc, r2, -0.5f);
  cr = fmaf(r2, pc, 1.0f);
}

// The reduction always taken, with no branch: for callers that evaluate the
// sin/cos of several machines per lane back to back, where a branch per call
// would keep the compiler from interleaving them.
__device__ __forceinline__ void sincos_r_nb(double x, double& s, double& c) {
  const double k = rint(x * 0.63661977236758134308);  // 2/pi
  double r = fma(-k, 0x1.921fb54442d18p+0, x);
  r = fma(-k, 0x1.1a62633145c07p-54, r);
  double sr, cr;
  sincos_poly<false>(r, sr, cr);
  const int q = (int)k;
  const double a = (q & 1) ? cr : sr;
  const double b = (q & 1) ? sr : cr;
  s = (q & 2) ? -a : a;
  c = ((q + 1) & 2) ? -b : b;
}

__device__ __forceinline__ void sincos_r_nb(float x, float& s, float& c) {
  const float k = rintf(x * 0x1.45f306p-1f);  // 2/pi
  float r = fmaf(-k, 0x1.921fb6p+0f, x);
  r = fmaf(-k, -0x1.777a5cp-25f, r);
  r = fmaf(-k, -0x1.ee59dap-50f, r);
  float sr, cr;
  sincos_poly(r, sr, cr);
  const int q = (int)k;
  const float a = (q & 1) ? cr : sr;
  const float b = (q & 1) ? sr : cr;
  s = (q & 2) ? -a : a;
  c = ((q + 1) & 2) ? -b : b;
}

// sin and cos of a lane's N angles with one wave-uniform decision: the
// small-angle form for all of them when every active lane's angles are below
// 0.78 (the same bits as the full path), else the full path; in
// both branches the N evaluations are straight-line code the compiler can
// interleave.
template <typename R, int N>
__device__ __forceinline__ void sincos_many(const R (&x)[N], R (&s)[N], R (&c)[N]) {
  bool small = true;
#pragma unroll
  for (int k = 0; k < N; ++k) small = small && fabs(x[k]) < R(0.78);
  if (sincos_all_small(small)) [[likely]] {
#pragma unroll
    for (int k = 0; k < N; ++k) sincos_poly(x[k], s[k], c[k]);
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) sincos_r_nb(x[k], s[k], c[k]);
  }
}

// The FP64 common-angle offset in two state slots: the exact bits of the
// double (two 32-bit halves for an FP32 state array), so that a run split
// into time chunks gives the same bits as a run in one chunk.
__device__ __forceinline__ void store_offset(float* st, int64_t i0, int64_t i1, double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  reinterpret_cast<unsigned int*>(st)[i0] = (unsigned int)b;
  reinterpret_cast<unsigned int*>(st)[i1] = (unsigned int)(b >> 32);
}
__device__ __forceinline__ void store_offset(double* st, int64_t i0, int64_t, double v) {
  st[i0] = v;
}
__device__ __forceinline__ double load_offset(const float* st, int64_t i0, int64_t i1) {
  const unsigned long long lo = reinterpret_cast<const unsigned int*>(st)[i0];
  const unsigned long long hi = reinterpret_cast<const unsigned int*>(st)[i1];
  return __longlong_as_double((long long)(lo | (hi << 32)));
}
__device__ __forceinline__ double load_offset(const double* st, int64_t i0, int64_t) {
  return st[i0];
}

// d xi/dt of eq. 9 for a general Ito process (one row of IntegArgs::sde) at
// state x with white-noise surrogate value w, and the power it injects into
// its machine, gain (x - ref).
template <typename R, typename Ptr>
__device__ __forceinline__ R sde_rhs(Ptr q, R x, R w, R& inj) {
  const R mu = q[SDE_M0] + x * (q[SDE_M1] + x * q[SDE_M2]);
  R sg, ssp;  // sigma and sigma sigma'
  if (q[SDE_FORM] == R(2)) {
    const R d = x - q[SDE_R];
    const R g = q[SDE_C0] + x * (q[SDE_C1] + x * q[SDE_C2]) + q[SDE_C3] * fabs(d);
    const R sgn = d > R(0) ? R(1) : (d < R(0) ? R(-1) : R(0));
    const R dg = q[SDE_C1] + R(2) * q[SDE_C2] * x + q[SDE_C3] * sgn;
    const bool pos = g > R(0);
    sg = pos ? sqrt(g) : R(0);
    ssp = pos ? R(0.5) * dg : R(0);
  } else {
    sg = q[SDE_C0] + x * (q[SDE_C1] + x * q[SDE_C2]);
    ssp = sg * (q[SDE_C1] + R(2) * q[SDE_C2] * x);
  }
  inj = q[SDE_GAIN] * (x - q[SDE_REF]);
  return mu - q[SDE_K] * ssp + sg * w;
}

// Right-hand side of the swing equations + the disturbances in deviation
// form: OU from the packed theta and sigma, or (GEN) the general processes of
// sdeg.  GEN is a separate instantiation so that the OU kernels keep their
// register allocation.
template <typename R, int NG, int PM, bool GEN>
__device__ __forceinline__ void swing_rhs(const R* cfg, const R* sdeg, const R wb,
                                          const R (&yd)[NG], const R (&yw)[NG],
                                          const R (&yx)[PM], const R (&wv)[PM], R (&kd)[NG],
                                          R (&kw)[NG], R (&kx)[PM]) {
  constexpr PackLayout L{NG, PM};
  // Re-derive the pointer at every stage: the compiler then streams the
  // machine data through scalar loads instead of keeping it live in (spilled)
  // registers across stages and steps.
  asm volatile("" : "+s"(cfg));
  const cptr<R> cf = (cptr<R>)cfg;
  // general processes first: their injections feed the machines
  R xin[GEN ? PM : 1];
  if constexpr (GEN) {
    const cptr<R> sq = (cptr<R>)sdeg;
#pragma unroll
    for (int p = 0; p < PM; ++p) kx[p] = sde_rhs<R>(sq + p * kSdeCols, yx[p], wv[p], xin[p]);
  }
  R dc[NG], ds[NG];
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    // the branch-free form: a lane's machines are interleaved by the compiler
    // around the scalar loads of their data
    R sh, ch;
    sincos_r_nb(yd[k] * R(0.5), sh, ch);
    const R c0 = cf[L.c0() + k], s0 = cf[L.s0() + k];
    const R sd = R(2) * sh * ch;   // sin d
    const R omc = R(2) * sh * sh;  // 1 - cos d
    dc[k] = -(c0 * omc + s0 * sd);
    ds[k] = c0 * sd - s0 * omc;
  }
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    R ir = R(0), ii = R(0);
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const R yr = cf[L.yre() + i * NG + k];
      const R yi = cf[L.yim() + i * NG + k];
      // complex MAC as four FMAs (no intermediate products)
      ir = fma(yr, dc[k], ir);
      ir = fma(-yi, ds[k], ir);
      ii = fma(yr, ds[k], ii);
      ii = fma(yi, dc[k], ii);
    }
    const R dpe = dc[i] * cf[L.i0r() + i] + ds[i] * cf[L.i0i() + i] +
                  (cf[L.c0() + i] + dc[i]) * ir + (cf[L.s0() + i] + ds[i]) * ii;
    R F = cf[L.res() + i] - dpe - cf[L.dmp() + i] * yw[i];
#pragma unroll
    for (int p = 0; p < PM; ++p) {
      if constexpr (GEN)
        F += cf[L.binc() + i * PM + p] * xin[p];
      else
        F += cf[L.binc() + i * PM + p] * yx[p];
    }
    kd[i] = wb * yw[i];
    kw[i] = F * cf[L.inv2h() + i];
  }
  if constexpr (!GEN) {
#pragma unroll
    for (int p = 0; p < PM; ++p) kx[p] = -cf[L.theta() + p] * yx[p] + cf[L.sigma() + p] * wv[p];
  }
}

// u = sum_v w_v y_v of one trajectory held whole by one lane (absolute angles
// as the outputs store them), FP64.
template <typename R, int NG, int PM>
__device__ __forceinline__ double rrf_u_lane(const IntegArgs<R>& a, double coff, const R (&yd)[NG],
                                             const R (&yw)[NG], const R (&yx)[PM]) {
  const int n = a.n, P = a.P;
  double u = 0.0;  // in output order: angles, speed deviations, processes
#pragma unroll
  for (int i = 0; i < NG; ++i)
    if (i < n) u += a.rrf_w[i] * (a.delta0[i] + (coff + (double)yd[i]));
#pragma unroll
  for (int i = 0; i < NG; ++i)
    if (i < n) u += a.rrf_w[n + i] * (double)yw[i];
#pragma unroll
  for (int p = 0; p < PM; ++p)
    if (p < P) u += a.rrf_w[2 * n + p] * (double)yx[p];
  return u;
}

// Per-wave two-pass statistics of one output time through an LDS transpose:
// lane v of the wave reduces variable v over the wave's valid trajectories.
template <typename R, int NG, int PM>
__device__ __forceinline__ void emit_step(const IntegArgs<R>& a, double (*tile)[65], int lane,
                                          int cnt, int64_t s, int slot, double coff,
                                          const R (&yd)[NG], const R (&yw)[NG],
                                          const R (&yx)[PM]) {
  const int n = a.n, P = a.P, V = a.V;
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    if (i < n) {
      tile[i][lane] = coff + (double)yd[i];
      tile[n + i][lane] = (double)yw[i];
    }
  }
#pragma unroll
  for (int p = 0; p < PM; ++p)
    if (p < P) tile[2 * n + p][lane] = (double)yx[p];
  __syncthreads();
  const int64_t S1 = a.S + 1;
  for (int v = lane; v < V; v += 64) {
    double sm = 0.0;
    for (int j = 0; j < cnt; ++j) sm += tile[v][j];
    const double mu = sm / (double)cnt;
    double m2 = 0.0;
    for (int j = 0; j < cnt; ++j) {
      const double d = tile[v][j] - mu;
      m2 += d * d;
    }
    double2* dst = reinterpret_cast<double2*>(a.partial);
    dst[((int64_t)blockIdx.x * S1 + s) * V + v] = make_double2(mu, m2);
  }
  if (slot >= 0) {
    double* o = a.traj + ((int64_t)slot * S1 + s) * V;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      if (i < n) {
        o[i] = a.delta0[i] + (coff + (double)yd[i]);
        o[n + i] = (double)yw[i];
      }
    }
#pragma unroll
    for (int p = 0; p < PM; ++p)
      if (p < P) o[2 * n + p] = (double)yx[p];
  }
  __syncthreads();
}

template <typename R, int NG, int PM, bool GEN = false>
__global__ void __launch_bounds__(64) k_rk4_lane(IntegArgs<R> a) {
  constexpr PackLayout L{NG, PM};
  constexpr int VM = 2 * NG + PM;
  __shared__ double tile[VM][65];
  const int lane = threadIdx.x;
  const int64_t gidx = (int64_t)blockIdx.x * 64 + lane;
  const int64_t N = a.N;
  const bool valid = gidx < N;
  const int64_t ns = valid ? gidx : N - 1;
  const int64_t rem = N - (int64_t)blockIdx.x * 64;
  const int cnt = rem < 64 ? (int)rem : 64;
  const int P = a.P;
  const R* __restrict__ cf = a.coef;
  const R* __restrict__ w = a.w;
  const int slot = (valid && a.traj_slot) ? a.traj_slot[ns] : -1;

  R yd[NG], yw[NG], yx[PM];
  double coff = 0.0;  // common-angle offset of the trajectory (see IntegArgs::recenter)
  double racc = 0.0;  // the epilogue's RRF sum (see IntegArgs::rrf_w)
  if (a.s_begin == 0) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      yd[i] = R(0);
      yw[i] = R(0);
    }
#pragma unroll
    for (int p = 0; p < PM; ++p) yx[p] = cf[L.xi0() + p];
    emit_step<R, NG, PM>(a, tile, lane, cnt, 0, slot, coff, yd, yw, yx);
    if (a.rrf_w) {
      const double u = rrf_u_lane<R, NG, PM>(a, coff, yd, yw, yx);
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
    coff = load_offset(a.state, (int64_t)(2 * NG + PM) * a.lanes + gidx,
                       (int64_t)(2 * NG + PM + 1) * a.lanes + gidx);
  }

  const R dt = a.dt, h2 = a.dt * R(0.5), dt6 = a.dt / R(6), wb = a.wb;
  const R inv_n = R(1) / (R)a.n_ref;
  // KLE path values of the next step are loaded one step ahead.
  R w0[PM], w1[PM], w2[PM];
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    w0[p] = (p < P) ? w[(int64_t)p * N + ns] : R(0);
    w1[p] = (p < P) ? w[((int64_t)1 * P + p) * N + ns] : R(0);
    w2[p] = (p < P) ? w[((int64_t)2 * P + p) * N + ns] : R(0);
  }

  for (int64_t s = a.s_begin; s < a.s_end; ++s) {
    const int64_t cl = 2 * s - a.c_base;
    const bool more = s + 1 < a.s_end;
    R n1[PM], n2[PM];
#pragma unroll
    for (int p = 0; p < PM; ++p) {
      n1[p] = (more && p < P) ? w[((cl + 3) * P + p) * N + ns] : R(0);
      n2[p] = (more && p < P) ? w[((cl + 4) * P + p) * N + ns] : R(0);
    }
    R kd[NG], kw[NG], kx[PM];
    R ad[NG], aw[NG], ax[PM];
    R td[NG], tw[NG], tx[PM];
    // stage 1
    swing_rhs<R, NG, PM, GEN>(cf, GEN ? a.sde : nullptr, wb, yd, yw, yx, w0, kd, kw, kx);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      ad[i] = kd[i]; aw[i] = kw[i];
      td[i] = yd[i] + h2 * kd[i]; tw[i] = yw[i] + h2 * kw[i];
    }
#pragma unroll
    for (int p = 0; p < PM; ++p) { ax[p] = kx[p]; tx[p] = yx[p] + h2 * kx[p]; }
    // stage 2
    swing_rhs<R, NG, PM, GEN>(cf, GEN ? a.sde : nullptr, wb, td, tw, tx, w1, kd, kw, kx);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      ad[i] += R(2) * kd[i]; aw[i] += R(2) * kw[i];
      td[i] = yd[i] + h2 * kd[i]; tw[i] = yw[i] + h2 * kw[i];
    }
#pragma unroll
    for (int p = 0; p < PM; ++p) { ax[p] += R(2) * kx[p]; tx[p] = yx[p] + h2 * kx[p]; }
    // stage 3
    swing_rhs<R, NG, PM, GEN>(cf, GEN ? a.sde : nullptr, wb, td, tw, tx, w1, kd, kw, kx);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      ad[i] += R(2) * kd[i]; aw[i] += R(2) * kw[i];
      td[i] = yd[i] + dt * kd[i]; tw[i] = yw[i] + dt * kw[i];
    }
#pragma unroll
    for (int p = 0; p < PM; ++p) { ax[p] += R(2) * kx[p]; tx[p] = yx[p] + dt * kx[p]; }
    // stage 4
    swing_rhs<R, NG, PM, GEN>(cf, GEN ? a.sde : nullptr, wb, td, tw, tx, w2, kd, kw, kx);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      yd[i] += dt6 * (ad[i] + kd[i]);
      yw[i] += dt6 * (aw[i] + kw[i]);
    }
#pragma unroll
    for (int p = 0; p < PM; ++p) {
      yx[p] += dt6 * (ax[p] + kx[p]);
      w0[p] = w2[p];
      w1[p] = n1[p];
      w2[p] = n2[p];
    }
    if (a.recenter) {  // move the mean angle of the machines in service into the offset
      R sum = R(0);
#pragma unroll
      for (int i = 0; i < NG; ++i)
        if (i < a.n && (cf[L.c0() + i] != R(0) || cf[L.s0() + i] != R(0))) sum += yd[i];
      const R ref = sum * inv_n;
      coff += (double)ref;
#pragma unroll
      for (int i = 0; i < NG; ++i) yd[i] -= ref;
    }
    emit_step<R, NG, PM>(a, tile, lane, cnt, s + 1, slot, coff, yd, yw, yx);
    if (a.rrf_w) {
      const double u = rrf_u_lane<R, NG, PM>(a, coff, yd, yw, yx);
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
  store_offset(a.state, (int64_t)(2 * NG + PM) * a.lanes + gidx,
               (int64_t)(2 * NG + PM + 1) * a.lanes + gidx, coff);

  if (a.s_end == a.S && valid) {
    bool bad = !isfinite(coff);
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


// ---------------------------------------------------------------------------
// Group variant: L lanes share one trajectory (any L <= 64; a wave holds
// floor(64/L) trajectories and leaves the remaining lanes idle), lane g owns
// the G = ceil(NG/L) machines g*G .. g*G+G-1 and the rows of Y for them (held
// in registers, read once).  Per stage each lane rotates its own machines, the
// (dRe E~, dIm E~) pairs of a trajectory are exchanged through LDS (the lanes
// of a trajectory are in one wave, whose LDS operations complete in order, so
// only a compiler-level wavefront fence is needed), and each lane forms the
// network currents of its rows.  Every lane integrates the P disturbance
// processes of its trajectory (cheap) so that each can add the injections of
// its own machines.  A workgroup of WPB waves merges the statistics of its
// trajectories once per step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };

// Sizes of one group variant and the LDS it needs: the statistics tile (the
// values of up to D consecutive output steps, reduced together with two
// workgroup barriers per D steps), the exchange rows (NGP machine slots and PM
// process slots per trajectory; row TB is scratch for idle lanes) and the
// non-finite flags.
template <typename R, int NG, int PM, int L, int WPB, int D>
struct GroupShape {
  using R2 = typename vec2<R>::type;
  static constexpr int G = (NG + L - 1) / L;   // machines per lane
  static constexpr int PQ = (PM + L - 1) / L;  // processes per lane
  static constexpr int NGP = G * L;            // padded machine slots per trajectory
  static constexpr int XW = NGP + PM + 1;      // exchange row width (R2 entries)
  static constexpr int TW = 64 / L;            // trajectories per wave
  static constexpr int TB = TW * WPB;          // trajectories per workgroup
  static constexpr int VM = 2 * NG + PM;
  static constexpr size_t tile_bytes = (size_t)D * VM * (TB + 1) * sizeof(double);
  static constexpr size_t xch_bytes = (size_t)(TB + 1) * XW * sizeof(R2);
  static constexpr size_t lds_bytes = tile_bytes + xch_bytes + (TB + 1) * sizeof(int);
};

// Mean and sum of squared deviations of row[0, cnt) (cnt >= 1) in one pass
// over LDS: with the shift k = row[0] and d = x - k, mean = k + S1/cnt
// and M2 = S2 - S1^2/cnt (S1, S2 the sums of d and d^2, each in four partial
// sums over entries j mod 4, added in a fixed order).  The shift is one of the
// samples, so (mean - k)^2 <= (cnt - 1) M2 / cnt and the subtraction loses at
// most a factor cnt of relative accuracy (about 1e-14 here); equal entries
// give M2 = 0 exactly.
__device__ __forceinline__ void row_stats(const double* row, int cnt, double& mu, double& m2) {
  const double k = row[0];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
  int j = 0;
#pragma unroll 1
  for (; j + 3 < cnt; j += 4) {
    const double d0 = row[j] - k, d1 = row[j + 1] - k, d2 = row[j + 2] - k, d3 = row[j + 3] - k;
    s0 += d0; s1 += d1; s2 += d2; s3 += d3;
    q0 = fma(d0, d0, q0); q1 = fma(d1, d1, q1); q2 = fma(d2, d2, q2); q3 = fma(d3, d3, q3);
  }
  if (j < cnt) { const double d = row[j] - k; s0 += d; q0 = fma(d, d, q0); }
  if (j + 1 < cnt) { const double d = row[j + 1] - k; s1 += d; q1 = fma(d, d, q1); }
  if (j + 2 < cnt) { const double d = row[j + 2] - k; s2 += d; q2 = fma(d, d, q2); }
  const double S1 = (s0 + s1) + (s2 + s3), S2 = (q0 + q1) + (q2 + q3);
  const double dm = S1 / (double)cnt;
  mu = k + dm;
  m2 = fma(-S1, dm, S2);
}

// Where a group run leaves its statistics: rows[(s)*V + v] = (mean, M2) of the
// group's samples; prev > 0 means the rows already hold the statistics of prev
// earlier samples, and the group's are merged in with Chan's update (a fixed
// order, so results do not depend on scheduling).
struct GroupStats {
  double2* rows;
  int64_t prev;
};

// One workgroup integrates trajectories tile*TB .. tile*TB + TB - 1 of a
// scenario over the steps [s_begin, s_end) of a.  Lane g of a trajectory owns
// machines g*G .. g*G+G-1 (rows of Y in registers) and processes g, g+L, ...;
// per stage the lanes exchange the rotated EMF deviations of their machines
// and the stage values of their processes through LDS.  keep_state stores the
// state for a following chunk.  GEN: the processes are the general Ito
// processes of a.sde; the owner lane of a process evaluates its drift and
// diffusion and publishes the power it injects, gain (xi - ref), in the
// process's exchange slot (where the OU form publishes xi itself).
template <typename R, int NG, int PM, int L, int WPB, int D, bool GEN = false>
__device__ __forceinline__ void group_run(const IntegArgs<R>& a, int64_t tile,
                                          unsigned char* lds, GroupStats st, bool keep_state,
                                          const R* sde_rows = nullptr) {
  using Sh = GroupShape<R, NG, PM, L, WPB, D>;
  using R2 = typename Sh::R2;
  constexpr PackLayout Lp{NG, PM};
  constexpr int G = Sh::G, PQ = Sh::PQ, NGP = Sh::NGP, XW = Sh::XW, TW = Sh::TW, TB = Sh::TB,
                VM = Sh::VM;
  double (*tile_buf)[VM][TB + 1] = reinterpret_cast<double (*)[VM][TB + 1]>(lds);
  R2 (*xch)[XW] = reinterpret_cast<R2 (*)[XW]>(lds + Sh::tile_bytes);
  int* bad_t = reinterpret_cast<int*>(lds + Sh::tile_bytes + Sh::xch_bytes);
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  const bool lane_on = ln < TW * L;
  const int tl = lane_on ? wv * TW + ln / L : TB;
  const int g = lane_on ? ln % L : 0;
  const int64_t traj = tile * TB + tl;
  const int64_t N = a.N;
  const bool valid = lane_on && traj < N;
  const int64_t ns = valid ? traj : N - 1;
  const int64_t rem = N - tile * TB;
  const int cnt = rem < TB ? (int)rem : TB;
  const int n = a.n, P = a.P, V = a.V;
  const R* __restrict__ cf = a.coef;
  const R* __restrict__ w = a.w;
  const int slot = (valid && a.traj_slot) ? a.traj_slot[ns] : -1;

  // per-lane machine data (rows of Y and the operating point of my machines)
  R yr[G][NG], yi[G][NG], c0[G], s0[G], i0r[G], i0i[G], res[G], dmp[G], inv2h[G], binc[G][PM];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int i = g * G + q;
    const bool on = i < NG;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      yr[q][k] = on ? cf[Lp.yre() + i * NG + k] : R(0);
      yi[q][k] = on ? cf[Lp.yim() + i * NG + k] : R(0);
    }
    c0[q] = on ? cf[Lp.c0() + i] : R(0);
    s0[q] = on ? cf[Lp.s0() + i] : R(0);
    i0r[q] = on ? cf[Lp.i0r() + i] : R(0);
    i0i[q] = on ? cf[Lp.i0i() + i] : R(0);
    res[q] = on ? cf[Lp.res() + i] : R(0);
    dmp[q] = on ? cf[Lp.dmp() + i] : R(0);
    inv2h[q] = on ? cf[Lp.inv2h() + i] : R(0);
#pragma unroll
    for (int p = 0; p < PM; ++p) binc[q][p] = on ? cf[Lp.binc() + i * PM + p] : R(0);
  }
  bool live[G];
#pragma unroll
  for (int q = 0; q < G; ++q) live[q] = lane_on && (c0[q] != R(0) || s0[q] != R(0));
  // GEN: the gain and reference of my processes' injections
  R pgain[PQ], pref[PQ];
#pragma unroll
  for (int r = 0; r < PQ; ++r) {
    pgain[r] = R(0);
    pref[r] = R(0);
    if constexpr (GEN) {
      const int p = g + L * r;
      if (lane_on && p < a.P) {
        pgain[r] = a.sde[p * kSdeCols + SDE_GAIN];
        pref[r] = a.sde[p * kSdeCols + SDE_REF];
      }
    }
  }
  // my processes p = g + L r
  R theta[PQ], sigma[PQ];
  bool own[PQ];
  int64_t wofs[PQ];
#pragma unroll
  for (int r = 0; r < PQ; ++r) {
    const int p = g + L * r;
    own[r] = lane_on && p < P;
    theta[r] = own[r] ? cf[Lp.theta() + p] : R(0);
    sigma[r] = own[r] ? cf[Lp.sigma() + p] : R(0);
    wofs[r] = own[r] ? (int64_t)p * N + ns : 0;
  }

  // the process slots p >= P of my trajectory's exchange row stay zero
  if (g == 0) {
#pragma unroll
    for (int p = 0; p < PM; ++p) xch[tl][NGP + p] = R2{R(0), R(0)};
  }
  wave_lds_sync();

  auto rhs = [&](const R (&yd)[G], const R (&yw)[G], const R (&yx)[PQ], const R (&wv)[PQ],
                 R (&kd)[G], R (&kw)[G], R (&kx)[PQ]) {
    R dc[G], ds[G], hx[G], shs[G], chs[G];
    // idle lanes (whose exchange row is shared scratch) and machines without
    // EMF (padding, tripped) give dE = 0 at any angle: their angles are not
    // passed on, so they cannot push the wave off the small-angle branch
#pragma unroll
    for (int q = 0; q < G; ++q) hx[q] = live[q] ? yd[q] * R(0.5) : R(0);
    sincos_many(hx, shs, chs);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const R sh = shs[q], ch = chs[q];
      const R sd = R(2) * sh * ch;
      const R omc = R(2) * sh * sh;
      dc[q] = -(c0[q] * omc + s0[q] * sd);
      ds[q] = c0[q] * sd - s0[q] * omc;
      xch[tl][g * G + q] = R2{dc[q], ds[q]};
    }
    R gk[PQ];  // GEN: the processes' derivatives
#pragma unroll
    for (int r = 0; r < PQ; ++r) {
      R pub = yx[r];
      if constexpr (GEN) {
        // the injected power from registers (it feeds the exchange, on the
        // stage's critical path); the drift and diffusion come from the rows
        // staged in LDS (rows past P are zero; a lane that owns no process
        // reads row 0)
        const int p = g + L * r;
        R inj;
        gk[r] = sde_rhs<R>(sde_rows + (own[r] ? p : 0) * kSdeCols, yx[r], wv[r], inj);
        pub = pgain[r] * (yx[r] - pref[r]);
      }
      if (own[r]) xch[tl][NGP + g + L * r] = R2{pub, R(0)};
    }
    wave_lds_sync();
    // two accumulator pairs (even / odd columns) halve the FMA dependency chains
    R ir[G], ii[G], jr[G], ji[G];
#pragma unroll
    for (int q = 0; q < G; ++q) { ir[q] = R(0); ii[q] = R(0); jr[q] = R(0); ji[q] = R(0); }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      // keep at most 8 exchange loads in flight: bounds the registers the
      // scheduler would otherwise spend hoisting all NG loads
      if ((k & 7) == 0 && k > 0) asm volatile("" ::: "memory");
      const R2 e = xch[tl][k];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        // complex MAC as four FMAs (no intermediate products)
        if (k & 1) {
          jr[q] = fma(yr[q][k], e.x, jr[q]);
          jr[q] = fma(-yi[q][k], e.y, jr[q]);
          ji[q] = fma(yr[q][k], e.y, ji[q]);
          ji[q] = fma(yi[q][k], e.x, ji[q]);
        } else {
          ir[q] = fma(yr[q][k], e.x, ir[q]);
          ir[q] = fma(-yi[q][k], e.y, ir[q]);
          ii[q] = fma(yr[q][k], e.y, ii[q]);
          ii[q] = fma(yi[q][k], e.x, ii[q]);
        }
      }
    }
    R inj[G];
#pragma unroll
    for (int q = 0; q < G; ++q) inj[q] = R(0);
    // every process slot, the padding ones included (zero, as their columns
    // of binc): no branch on P between the exchange reads and their use
#pragma unroll
    for (int p = 0; p < PM; ++p) {
      const R xp = xch[tl][NGP + p].x;
#pragma unroll
      for (int q = 0; q < G; ++q) inj[q] += binc[q][p] * xp;
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < G; ++q) {
      ir[q] += jr[q];
      ii[q] += ji[q];
      const R dpe = dc[q] * i0r[q] + ds[q] * i0i[q] + (c0[q] + dc[q]) * ir[q] + (s0[q] + ds[q]) * ii[q];
      const R F = res[q] - dpe - dmp[q] * yw[q] + inj[q];
      kd[q] = a.wb * yw[q];
      kw[q] = F * inv2h[q];
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) {
      if constexpr (GEN)
        kx[r] = own[r] ? gk[r] : R(0);
      else
        kx[r] = -theta[r] * yx[r] + sigma[r] * wv[r];
    }
  };

  // RRF sum of trajectory tid of this tile (threads tid < TB; see IntegArgs::rrf_w)
  double racc = 0.0;
  if (a.rrf_w && a.s_begin > 0 && tid < cnt) racc = a.rrf_acc[tile * TB + tid];
  // Reduce the buffered steps [s_first, s_first + nb): thread q of the
  // workgroup takes rows (step, variable) q, q + 64 WPB, ...
  auto flush = [&](int64_t s_first, int nb) {
    __syncthreads();
    for (int rv = tid; rv < nb * V; rv += 64 * WPB) {
      const int b = rv / V, v = rv % V;
      double mu, m2;
      row_stats(tile_buf[b][v], cnt, mu, m2);
      double2* dst = st.rows + (s_first + b) * V + v;
      if (st.prev == 0) {
        *dst = make_double2(mu, m2);
      } else {
        const double2 old = *dst;
        const double na = (double)st.prev, nb2 = (double)cnt, tot = na + nb2;
        const double dl = mu - old.x;
        *dst = make_double2(old.x + dl * (nb2 / tot), old.y + m2 + dl * dl * (na * nb2 / tot));
      }
    }
    // the epilogue's RRF: thread j sums trajectory j's buffered steps in order
    if (a.rrf_w && tid < cnt) {
      for (int b = 0; b < nb; ++b) {
        const int64_t s = s_first + b;
        double u = 0.0;
        for (int v = 0; v < V; ++v) {
          const double y = tile_buf[b][v][tid];
          u += a.rrf_w[v] * (v < n ? a.delta0[v] + y : y);
        }
        racc += (s == 0 || s == a.S ? 0.5 : 1.0) * u * u;
      }
    }
    __syncthreads();
  };
  int nbuf = 0;
  int64_t s_first = 0;
  double coff = 0.0;  // common-angle offset of my trajectory (see IntegArgs::recenter)
  auto emit = [&](int64_t s, const R (&yd)[G], const R (&yw)[G], const R (&yx)[PQ]) {
    if (nbuf == 0) s_first = s;
    double (*tb)[TB + 1] = tile_buf[nbuf];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int i = g * G + q;
      if (lane_on && i < n) {
        tb[i][tl] = coff + (double)yd[q];
        tb[n + i][tl] = (double)yw[q];
      }
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r)
      if (own[r]) tb[2 * n + g + L * r][tl] = (double)yx[r];
    if (slot >= 0) {
      // every lane of a selected trajectory writes its own outputs
      double* o = a.traj + ((int64_t)slot * (a.S + 1) + s) * V;
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int i = g * G + q;
        if (i < n) {
          o[i] = a.delta0[i] + (coff + (double)yd[q]);
          o[n + i] = (double)yw[q];
        }
      }
#pragma unroll
      for (int r = 0; r < PQ; ++r)
        if (own[r]) o[2 * n + g + L * r] = (double)yx[r];
    }
    if (++nbuf == D) {
      flush(s_first, nbuf);
      nbuf = 0;
    }
  };

  R yd[G], yw[G], yx[PQ];
  const int64_t lane_id = tile * 64 * WPB + tid;
  if (a.s_begin == 0) {
#pragma unroll
    for (int q = 0; q < G; ++q) { yd[q] = R(0); yw[q] = R(0); }
#pragma unroll
    for (int r = 0; r < PQ; ++r) yx[r] = own[r] ? cf[Lp.xi0() + g + L * r] : R(0);
    emit(0, yd, yw, yx);
  } else {
#pragma unroll
    for (int q = 0; q < G; ++q) {
      yd[q] = a.state[(int64_t)q * a.lanes + lane_id];
      yw[q] = a.state[(int64_t)(G + q) * a.lanes + lane_id];
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) yx[r] = a.state[(int64_t)(2 * G + r) * a.lanes + lane_id];
    coff = load_offset(a.state, (int64_t)(2 * G + PQ) * a.lanes + lane_id,
                       (int64_t)(2 * G + PQ + 1) * a.lanes + lane_id);
  }

  const R dt = a.dt, h2 = a.dt * R(0.5), dt6 = a.dt / R(6);
  const R inv_n = R(1) / (R)a.n_ref;
  const int64_t colstride = (int64_t)P * N;
  // KLE path values of my processes: the two new stage columns of step s are
  // loaded one step ahead so their latency overlaps the previous step.
  R w0[PQ], w1[PQ], w2[PQ];
#pragma unroll
  for (int r = 0; r < PQ; ++r) {
    w0[r] = own[r] ? w[wofs[r]] : R(0);
    w1[r] = own[r] ? w[colstride + wofs[r]] : R(0);
    w2[r] = own[r] ? w[2 * colstride + wofs[r]] : R(0);
  }
  for (int64_t s = a.s_begin; s < a.s_end; ++s) {
    const int64_t cl = 2 * s - a.c_base;
    const bool more = s + 1 < a.s_end;
    R n1[PQ], n2[PQ];
#pragma unroll
    for (int r = 0; r < PQ; ++r) {
      n1[r] = (more && own[r]) ? w[(cl + 3) * colstride + wofs[r]] : R(0);
      n2[r] = (more && own[r]) ? w[(cl + 4) * colstride + wofs[r]] : R(0);
    }
    R kd[G], kw[G], kx[PQ], ad[G], aw[G], ax[PQ], td[G], tw[G], tx[PQ];
    rhs(yd, yw, yx, w0, kd, kw, kx);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      ad[q] = kd[q]; aw[q] = kw[q];
      td[q] = yd[q] + h2 * kd[q]; tw[q] = yw[q] + h2 * kw[q];
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) { ax[r] = kx[r]; tx[r] = yx[r] + h2 * kx[r]; }
    rhs(td, tw, tx, w1, kd, kw, kx);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      ad[q] += R(2) * kd[q]; aw[q] += R(2) * kw[q];
      td[q] = yd[q] + h2 * kd[q]; tw[q] = yw[q] + h2 * kw[q];
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) { ax[r] += R(2) * kx[r]; tx[r] = yx[r] + h2 * kx[r]; }
    rhs(td, tw, tx, w1, kd, kw, kx);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      ad[q] += R(2) * kd[q]; aw[q] += R(2) * kw[q];
      td[q] = yd[q] + dt * kd[q]; tw[q] = yw[q] + dt * kw[q];
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) { ax[r] += R(2) * kx[r]; tx[r] = yx[r] + dt * kx[r]; }
    rhs(td, tw, tx, w2, kd, kw, kx);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      yd[q] += dt6 * (ad[q] + kd[q]);
      yw[q] += dt6 * (aw[q] + kw[q]);
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) {
      yx[r] += dt6 * (ax[r] + kx[r]);
      w0[r] = w2[r];
      w1[r] = n1[r];
      w2[r] = n2[r];
    }
    if (a.recenter && ((s + 1) & 7) == 0) {
      // every eighth step (of the absolute step count, so time chunks keep the
      // bits; the common angle moves by milliradians in between):
      // the mean angle of the trajectory's machines in service (a tripped
      // machine has no EMF): each lane's sum over its machines through the
      // exchange row (free again: the last stage's reads ended with a wave
      // fence), added in lane order by every lane of the trajectory (the same
      // bits in each), then taken out of every angle
      R part = R(0);
#pragma unroll
      for (int q = 0; q < G; ++q)
        if (g * G + q < n && (c0[q] != R(0) || s0[q] != R(0))) part += yd[q];
      xch[tl][g] = R2{part, R(0)};
      wave_lds_sync();
      R sum = R(0);
      for (int k = 0; k < L; ++k) sum += xch[tl][k].x;
      wave_lds_sync();
      const R ref = sum * inv_n;
      coff += (double)ref;
#pragma unroll
      for (int q = 0; q < G; ++q) yd[q] -= ref;
    }
    emit(s + 1, yd, yw, yx);
  }

  if (nbuf > 0) flush(s_first, nbuf);  // nbuf is uniform over the workgroup
  if (a.rrf_w && tid < cnt) {
    a.rrf_acc[tile * TB + tid] = racc;
    if (a.s_end == a.S) a.rrf[tile * TB + tid] = sqrt(racc / (double)a.S);
  }

  if (keep_state) {
#pragma unroll
    for (int q = 0; q < G; ++q) {
      a.state[(int64_t)q * a.lanes + lane_id] = yd[q];
      a.state[(int64_t)(G + q) * a.lanes + lane_id] = yw[q];
    }
#pragma unroll
    for (int r = 0; r < PQ; ++r) a.state[(int64_t)(2 * G + r) * a.lanes + lane_id] = yx[r];
    store_offset(a.state, (int64_t)(2 * G + PQ) * a.lanes + lane_id,
                 (int64_t)(2 * G + PQ + 1) * a.lanes + lane_id, coff);
  }

  if (a.s_end == a.S) {  // uniform over the workgroup: the barriers below are safe
    bool bad = !isfinite(coff);
#pragma unroll
    for (int q = 0; q < G; ++q) bad |= !isfinite(yd[q]) || !isfinite(yw[q]);
#pragma unroll
    for (int r = 0; r < PQ; ++r) bad |= !isfinite(yx[r]);
    // one count per trajectory: the lanes of a trajectory combine through LDS
    if (lane_on && g == 0) bad_t[tl] = 0;
    __syncthreads();
    if (lane_on && bad) bad_t[tl] = 1;
    __syncthreads();
    if (valid && g == 0 && bad_t[tl] != 0) {
      atomicAdd(a.nonfinite, 1ULL);
      atomicMin(a.first_bad, (long long)traj);
    }
    __syncthreads();  // the flags may be reused by the workgroup's next run
  }
}

// At least two waves per SIMD (at most 256 registers per lane, VGPRs and
// AGPRs together): left to itself the compiler spends all 256 VGPRs plus a
// few AGPRs on the larger variants and drops them to one wave per SIMD.
#ifndef FMC_GROUP_MIN_WAVES
#define FMC_GROUP_MIN_WAVES 2
#endif
template <typename R, int NG, int PM, int L, int WPB>
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(FMC_GROUP_MIN_WAVES)))
k_rk4_group(IntegArgs<R> a) {
  constexpr int D = WPB == 1 ? 4 : 8;
  using Sh = GroupShape<R, NG, PM, L, WPB, D>;
  __shared__ __attribute__((aligned(16))) unsigned char lds[Sh::lds_bytes];
  GroupStats st{reinterpret_cast<double2*>(a.partial) + (int64_t)blockIdx.x * (a.S + 1) * a.V, 0};
  group_run<R, NG, PM, L, WPB, D>(a, blockIdx.x, lds, st, true);
}

// The same for general Ito processes (IntegArgs::sde), instantiated in their
// own translation units.
template <typename R, int NG, int PM, int L, int WPB>
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(FMC_GROUP_MIN_WAVES)))
k_rk4_group_gen(IntegArgs<R> a) {
  constexpr int D = WPB == 1 ? 4 : 8;
  using Sh = GroupShape<R, NG, PM, L, WPB, D>;
  __shared__ __attribute__((aligned(16))) unsigned char lds[Sh::lds_bytes];
  // the processes' rows (PM of them, zero past P) staged in LDS once: they
  // are read by the owner lanes at every stage
  __shared__ R sde_l[PM * kSdeCols];
  for (int i = threadIdx.x; i < PM * kSdeCols; i += 64 * WPB) sde_l[i] = a.sde[i];
  __syncthreads();
  GroupStats st{reinterpret_cast<double2*>(a.partial) + (int64_t)blockIdx.x * (a.S + 1) * a.V, 0};
  group_run<R, NG, PM, L, WPB, D, true>(a, blockIdx.x, lds, st, true, sde_l);
}

}  // namespace fmc
