// k_setup.hip -- scenario setup on the GPU (FP64): Kron reduction of the
// network equations, operating point, packed coefficients; and the ordered
// cross-sample merge of the per-group statistics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fmc_internal.hpp"

namespace fmc {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return sqrt(a.x * a.x + a.y * a.y); }

// ---------------------------------------------------------------------------
// Kron reduction (eq. 2 eliminated): one workgroup of 256 threads.  The
// augmented system [Y_BB | Y_BA] (n_bus rows, n_bus + n_gen columns) lives in
// LDS when it fits (else in the global work buffer).  Thread b assembles row b
// alone, scanning branches, loads and generators in index order, so the sums
// are deterministic.  Gaussian elimination with partial pivoting (pivot: the
// largest |a_rk|, lowest row on ties, found by wave shuffles), then back
// substitution gives X = Y_BB^-1 Y_BA and Y_red = Y_AA - Y_AB X.
// ---------------------------------------------------------------------------
constexpr int kKronLdsComplex = 4096;  // 64 KB of double2

__device__ __forceinline__ void kron_pivot_reduce(double& v, int& idx) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(v, off);
    const int i2 = __shfl_xor(idx, off);
    if (v2 > v || (v2 == v && i2 < idx)) {
      v = v2;
      idx = i2;
    }
  }
}

__global__ void __launch_bounds__(256) k_kron(NetDev net, double2* __restrict__ gwork,
                                              double2* __restrict__ Yred, int* status) {
  const int nb = net.n_bus, ng = net.n_gen, W = nb + ng;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double2 lds[kKronLdsComplex];
  __shared__ double s_val[4];
  __shared__ int s_idx[4];
  __shared__ int s_bad;
  double2* A = ((int64_t)nb * W <= kKronLdsComplex) ? lds : gwork;
  if (tid == 0) s_bad = 0;
  // assembly: thread b owns row b
  for (int b = tid; b < nb; b += nt) {
    double2* row = A + (int64_t)b * W;
    for (int c = 0; c < W; ++c) row[c] = make_double2(0.0, 0.0);
    for (int k = 0; k < net.n_branch; ++k) {
      const int f = net.from[k], t = net.to[k];
      if (f != b && t != b) continue;
      const double2 y = cdiv(make_double2(1.0, 0.0), make_double2(net.r[k], net.x[k]));
      const double2 sh = make_double2(0.0, net.b ? 0.5 * net.b[k] : 0.0);
      row[b] = cadd(row[b], cadd(y, sh));
      const int o = (f == b) ? t : f;
      row[o] = csub(row[o], y);
    }
    row[b] = cadd(row[b], make_double2(net.lg ? net.lg[b] : 0.0, net.lb ? net.lb[b] : 0.0));
    for (int g = 0; g < ng; ++g) {
      if (net.gen_bus[g] != b) continue;
      const double2 yg = make_double2(0.0, -1.0 / net.xdp[g]);  // 1/(j X'd)
      row[b] = cadd(row[b], yg);
      row[nb + g] = csub(row[nb + g], yg);  // Y_BA = -yg
    }
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    double best = -1.0;
    int bi = nb;
    for (int r = k + tid; r < nb; r += nt) {
      const double v = cabs2(A[(int64_t)r * W + k]);
      if (v > best || (v == best && r < bi)) { best = v; bi = r; }
    }
    kron_pivot_reduce(best, bi);
    if ((tid & 63) == 0) {
      s_val[tid >> 6] = best;
      s_idx[tid >> 6] = bi;
    }
    __syncthreads();
    double pv = s_val[0];
    int piv = s_idx[0];
    for (int w = 1; w < nt / 64; ++w)
      if (s_val[w] > pv || (s_val[w] == pv && s_idx[w] < piv)) { pv = s_val[w]; piv = s_idx[w]; }
    if (!(pv > 0.0)) {
      if (tid == 0) *status = -1;
      return;  // uniform: every thread saw the same pv
    }
    if (piv != k) {
      for (int c = k + tid; c < W; c += nt) {
        const double2 t = A[(int64_t)k * W + c];
        A[(int64_t)k * W + c] = A[(int64_t)piv * W + c];
        A[(int64_t)piv * W + c] = t;
      }
    }
    __syncthreads();
    const double2 akk = A[(int64_t)k * W + k];
    const int rows = nb - k - 1, cols = W - k - 1;
    for (int64_t q = tid; q < (int64_t)rows * cols; q += nt) {
      const int r = k + 1 + (int)(q / cols);
      const int c = k + 1 + (int)(q % cols);
      const double2 f = cdiv(A[(int64_t)r * W + k], akk);
      A[(int64_t)r * W + c] = csub(A[(int64_t)r * W + c], cmul(f, A[(int64_t)k * W + c]));
    }
    __syncthreads();
  }
  // back substitution on the n_gen right-hand columns
  for (int k = nb - 1; k >= 0; --k) {
    for (int g = tid; g < ng; g += nt) {
      double2 acc = A[(int64_t)k * W + nb + g];
      for (int j = k + 1; j < nb; ++j) acc = csub(acc, cmul(A[(int64_t)k * W + j], A[(int64_t)j * W + nb + g]));
      A[(int64_t)k * W + nb + g] = cdiv(acc, A[(int64_t)k * W + k]);
    }
    __syncthreads();
  }
  for (int q = tid; q < ng * ng; q += nt) {
    const int i = q / ng, k = q % ng;
    const double2 yg = make_double2(0.0, -1.0 / net.xdp[i]);
    double2 v = (i == k) ? yg : make_double2(0.0, 0.0);
    v = cadd(v, cmul(yg, A[(int64_t)net.gen_bus[i] * W + nb + k]));  // -(Y_AB X), Y_AB = -yg
    Yred[q] = v;
  }
  if (tid == 0) *status = s_bad;
}

// ---------------------------------------------------------------------------
// Large networks (the augmented system does not fit LDS): Kron's node
// elimination on the full admittance matrix of the buses and the generator
// internal nodes (W = n_bus + n_gen, buses first), one launch per eliminated
// bus k:  Y_ij -= Y_ik Y_kj / Y_kk  for all remaining i, j.  After the last bus
// the generator block is Y_red.  The buses are eliminated in index order
// without pivoting: the bus block of a network admittance matrix whose series
// branches share one R/X ratio and whose shunts are loads and transient
// reactances is diagonally dominant.  A zero pivot sets the status.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_kron_assemble(NetDev net, double2* __restrict__ A,
                                                       int* status) {
  const int nb = net.n_bus, ng = net.n_gen, W = nb + ng;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) *status = 0;  // the elimination steps only ever set -1
  if (r >= W) return;
  double2* row = A + (int64_t)r * W;  // zeroed before the launch
  if (r >= nb) {
    const int g = r - nb;
    const double2 yg = make_double2(0.0, -1.0 / net.xdp[g]);  // 1/(j X'd)
    row[r] = yg;
    row[net.gen_bus[g]] = make_double2(-yg.x, -yg.y);
    return;
  }
  for (int k = 0; k < net.n_branch; ++k) {
    const int f = net.from[k], t = net.to[k];
    if (f != r && t != r) continue;
    const double2 y = cdiv(make_double2(1.0, 0.0), make_double2(net.r[k], net.x[k]));
    const double2 sh = make_double2(0.0, net.b ? 0.5 * net.b[k] : 0.0);
    row[r] = cadd(row[r], cadd(y, sh));
    const int o = (f == r) ? t : f;
    row[o] = csub(row[o], y);
  }
  row[r] = cadd(row[r], make_double2(net.lg ? net.lg[r] : 0.0, net.lb ? net.lb[r] : 0.0));
  for (int g = 0; g < ng; ++g) {
    if (net.gen_bus[g] != r) continue;
    const double2 yg = make_double2(0.0, -1.0 / net.xdp[g]);
    row[r] = cadd(row[r], yg);
    row[nb + g] = csub(row[nb + g], yg);
  }
}

// One elimination step: block (64, 4) covers 64 columns; row k scaled by
// 1/Y_kk is formed once per block in LDS.
__global__ void __launch_bounds__(256) k_kron_elim(double2* __restrict__ A, int W, int k,
                                                   int* status) {
  __shared__ double2 sk[64];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int j = k + 1 + blockIdx.x * 64 + tx;
  const double2 akk = A[(int64_t)k * W + k];
  if (!(akk.x != 0.0 || akk.y != 0.0)) {  // uniform
    if (blockIdx.x == 0 && blockIdx.y == 0 && tx == 0 && ty == 0) *status = -1;
    return;
  }
  if (ty == 0) sk[tx] = j < W ? cdiv(A[(int64_t)k * W + j], akk) : make_double2(0.0, 0.0);
  __syncthreads();
  if (j >= W) return;
  const double2 s = sk[tx];
  for (int i = k + 1 + blockIdx.y * 4 + ty; i < W; i += gridDim.y * 4) {
    double2* a = A + (int64_t)i * W;
    a[j] = csub(a[j], cmul(a[k], s));
  }
}

__global__ void __launch_bounds__(256) k_kron_extract(const double2* __restrict__ A, int nb, int ng,
                                                      double2* __restrict__ Yred) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ng * ng) return;
  const int W = nb + ng, i = q / ng, k = q % ng;
  Yred[q] = A[(int64_t)(nb + i) * W + nb + k];
}

size_t kron_work_bytes(int n_bus, int n_gen) {
  const size_t W = (size_t)n_bus + n_gen;
  return W * W * sizeof(double2);
}

hipError_t launch_kron(const NetDev& net, double2* work, double2* Yred, int* status,
                       hipStream_t st) {
  const int nb = net.n_bus, ng = net.n_gen, W = nb + ng;
  if ((int64_t)nb * W <= kKronLdsComplex) {
    hipLaunchKernelGGL(k_kron, dim3(1), dim3(256), 0, st, net, work, Yred, status);
    return hipGetLastError();
  }
  hipError_t e = launch_fill_i64((int64_t*)work, 0, (int64_t)W * W * 2, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kron_assemble, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, st, net, work,
                     status);
  for (int k = 0; k < nb; ++k) {
    const int m = W - k - 1;
    const unsigned gx = (unsigned)((m + 63) / 64), gy = (unsigned)std::min(64, (m + 3) / 4);
    hipLaunchKernelGGL(k_kron_elim, dim3(gx, gy), dim3(64, 4), 0, st, work, W, k, status);
  }
  hipLaunchKernelGGL(k_kron_extract, dim3((unsigned)((ng * ng + 255) / 256)), dim3(256), 0, st,
                     work, nb, ng, Yred);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operating point.  Pe_i = Re{E~_i conj(I_i)}, I = Y E~ + Yinf V_inf.  Given
// delta0: Pm defaults to Pe(delta0) (equilibrium).  Without delta0 (infinite
// bus): Newton on Pe(delta) = Pm from delta = 0, dense LU with partial
// pivoting, serial in one thread (small n).
// ---------------------------------------------------------------------------
__device__ void op_currents(const SetupDev& s, const double* d, double2* Et, double2* I) {
  const int n = s.n;
  for (int k = 0; k < n; ++k) Et[k] = make_double2(s.E[k] * cos(d[k]), s.E[k] * sin(d[k]));
  for (int i = 0; i < n; ++i) {
    double2 c = (s.inf_bus && s.Yinf) ? make_double2(s.Yinf[i].x * s.V_inf, s.Yinf[i].y * s.V_inf)
                                      : make_double2(0.0, 0.0);
    for (int k = 0; k < n; ++k) c = cadd(c, cmul(s.Y[(int64_t)i * n + k], Et[k]));
    I[i] = c;
  }
}

__global__ void k_setup(SetupDev s) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = s.n, P = s.P;
  CanonLayout L{n, P};
  double* cn = s.canon;
  double* d = cn + L.delta0();
  double2* Et = (double2*)s.work;
  double2* I = Et + n;
  double* J = (double*)(I + n);
  double* rhs = J + (int64_t)n * n;
  int ok = 1;
  if (s.delta0) {
    for (int i = 0; i < n; ++i) d[i] = s.delta0[i];
  } else {
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    ok = 0;
    for (int it = 0; it < 100; ++it) {
      op_currents(s, d, Et, I);
      for (int i = 0; i < n; ++i) {
        const double pe = Et[i].x * I[i].x + Et[i].y * I[i].y;
        rhs[i] = s.Pm[i] - pe;
        for (int k = 0; k < n; ++k) {
          // d Pe_i / d delta_k
          const double2 yk = cmul(s.Y[(int64_t)i * n + k], make_double2(-Et[k].y, Et[k].x));
          double v = Et[i].x * yk.x + Et[i].y * yk.y;
          if (k == i) v += -Et[i].y * I[i].x + Et[i].x * I[i].y;
          J[(int64_t)i * n + k] = v;
        }
      }
      // solve J dx = rhs
      int sing = 0;
      for (int k = 0; k < n && !sing; ++k) {
        int piv = k;
        double best = fabs(J[(int64_t)k * n + k]);
        for (int r = k + 1; r < n; ++r)
          if (fabs(J[(int64_t)r * n + k]) > best) { best = fabs(J[(int64_t)r * n + k]); piv = r; }
        if (best == 0.0) { sing = 1; break; }
        if (piv != k) {
          for (int c = 0; c < n; ++c) {
            const double t = J[(int64_t)k * n + c];
            J[(int64_t)k * n + c] = J[(int64_t)piv * n + c];
            J[(int64_t)piv * n + c] = t;
          }
          const double t = rhs[k]; rhs[k] = rhs[piv]; rhs[piv] = t;
        }
        for (int r = k + 1; r < n; ++r) {
          const double f = J[(int64_t)r * n + k] / J[(int64_t)k * n + k];
          for (int c = k; c < n; ++c) J[(int64_t)r * n + c] -= f * J[(int64_t)k * n + c];
          rhs[r] -= f * rhs[k];
        }
      }
      if (sing) break;
      double nrm = 0.0;
      for (int k = n - 1; k >= 0; --k) {
        double acc = rhs[k];
        for (int j = k + 1; j < n; ++j) acc -= J[(int64_t)k * n + j] * rhs[j];
        rhs[k] = acc / J[(int64_t)k * n + k];
      }
      for (int i = 0; i < n; ++i) {
        d[i] += rhs[i];
        nrm = fmax(nrm, fabs(rhs[i]));
      }
      if (nrm <= 1e-15) { ok = 1; break; }
    }
  }
  op_currents(s, d, Et, I);
  for (int i = 0; i < n; ++i) {
    const double pe = Et[i].x * I[i].x + Et[i].y * I[i].y;
    const double pm = s.Pm ? s.Pm[i] : pe;
    cn[L.c0() + i] = Et[i].x;
    cn[L.s0() + i] = Et[i].y;
    cn[L.i0r() + i] = I[i].x;
    cn[L.i0i() + i] = I[i].y;
    cn[L.res() + i] = pm - pe;
    cn[L.dmp() + i] = s.D[i];
    cn[L.inv2h() + i] = 1.0 / (2.0 * s.H[i]);
    cn[L.pm() + i] = pm;
    for (int k = 0; k < n; ++k) {
      cn[L.yre() + (int64_t)i * n + k] = s.Y[(int64_t)i * n + k].x;
      cn[L.yim() + (int64_t)i * n + k] = s.Y[(int64_t)i * n + k].y;
    }
  }
  for (int p = 0; p < P; ++p) {
    cn[L.theta() + p] = s.theta[p];
    cn[L.sigma() + p] = s.sigma[p];
    cn[L.xi0() + p] = s.xi0 ? s.xi0[p] : 0.0;
  }
  *s.status = ok ? 0 : -6;
}

hipError_t launch_setup(const SetupDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, s);
  return hipGetLastError();
}

// Coefficients after a network event: the pre-event operating point (E~0,
// D, H, Pm, delta0, the processes) with the post-event admittance: I0 = Yp E~0
// + Yinf V_inf, res = Pm - Re(E~0 conj I0).  A tripped machine keeps no EMF,
// current, mechanical power or residual, so it neither drives nor sees the
// network (its row and column of Yp are zero) and only its damping acts.
__global__ void __launch_bounds__(256) k_setup_post(const double* __restrict__ pre, int n, int P,
                                                    const double2* __restrict__ Yp,
                                                    const double2* __restrict__ Yinf,
                                                    double V_inf, int tripped,
                                                    double* __restrict__ post) {
  const CanonLayout L{n, P};
  const int tid = threadIdx.x, bd = blockDim.x;
  for (int64_t q = tid; q < L.size(); q += bd) post[q] = pre[q];
  __syncthreads();
  for (int64_t q = tid; q < (int64_t)n * n; q += bd) {
    post[L.yre() + q] = Yp[q].x;
    post[L.yim() + q] = Yp[q].y;
  }
  for (int i = tid; i < n; i += bd) {
    double2 I = Yinf ? make_double2(Yinf[i].x * V_inf, Yinf[i].y * V_inf) : make_double2(0.0, 0.0);
    for (int k = 0; k < n; ++k)
      I = cadd(I, cmul(Yp[(int64_t)i * n + k], make_double2(pre[L.c0() + k], pre[L.s0() + k])));
    const double er = pre[L.c0() + i], ei = pre[L.s0() + i];
    const bool out = i == tripped;
    const double pm = out ? 0.0 : pre[L.pm() + i];
    const double pe = out ? 0.0 : er * I.x + ei * I.y;
    post[L.c0() + i] = out ? 0.0 : er;
    post[L.s0() + i] = out ? 0.0 : ei;
    post[L.i0r() + i] = out ? 0.0 : I.x;
    post[L.i0i() + i] = out ? 0.0 : I.y;
    post[L.res() + i] = pm - pe;
    post[L.pm() + i] = pm;
  }
}

hipError_t launch_setup_post(const double* pre, int n, int P, const double2* Yp,
                             const double2* Yinf, double V_inf, int tripped, double* post,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_setup_post, dim3(1), dim3(256), 0, st, pre, n, P, Yp, Yinf, V_inf, tripped,
                     post);
  return hipGetLastError();
}

// Packed, padded coefficients of a variant in its arithmetic type.
template <typename R>
__global__ void __launch_bounds__(256) k_pack(const double* __restrict__ cn, int n, int P,
                                              const int32_t* __restrict__ gen, int NG, int PM,
                                              R* __restrict__ coef) {
  CanonLayout C{n, P};
  PackLayout L{NG, PM};
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.size()) return;
  double v = 0.0;
  if (q < L.yim()) {
    const int i = q / NG, k = q % NG;
    if (i < n && k < n) v = cn[C.yre() + (int64_t)i * n + k];
  } else if (q < L.binc()) {
    const int e = q - L.yim(), i = e / NG, k = e % NG;
    if (i < n && k < n) v = cn[C.yim() + (int64_t)i * n + k];
  } else if (q < L.c0()) {
    const int e = q - L.binc(), i = e / PM, p = e % PM;
    v = (i < n && p < P && gen[p] == i) ? 1.0 : 0.0;
  } else if (q < L.theta()) {
    const int e = q - L.c0(), f = e / NG, i = e % NG;
    // fields c0, s0, i0r, i0i, res, dmp, inv2h in canonical order
    const int64_t base[7] = {C.c0(), C.s0(), C.i0r(), C.i0i(), C.res(), C.dmp(), C.inv2h()};
    if (i < n) v = cn[base[f] + i];
  } else {
    const int e = q - L.theta(), f = e / PM, p = e % PM;
    const int64_t base[3] = {C.theta(), C.sigma(), C.xi0()};
    if (p < P) v = cn[base[f] + p];
  }
  coef[q] = (R)v;
}

template <typename R>
hipError_t launch_pack(const double* canon, int n, int P, const int32_t* gen, int NG, int PM,
                       R* coef, hipStream_t st) {
  PackLayout L{NG, PM};
  hipLaunchKernelGGL(k_pack<R>, dim3((L.size() + 255) / 256), dim3(256), 0, st, canon, n, P, gen,
                     NG, PM, coef);
  return hipGetLastError();
}
template hipError_t launch_pack<double>(const double*, int, int, const int32_t*, int, int,
                                        double*, hipStream_t);
template hipError_t launch_pack<float>(const double*, int, int, const int32_t*, int, int, float*,
                                       hipStream_t);

// Ordered merge of per-group statistics into mean and variance (Alg. 1 step
// 4): partial[g * gstride + q] holds (mean, M2) of group g's samples for
// q = row * V + v (group_size samples per group, the last group the rest).
// A workgroup takes 64 consecutive q, one per lane, and splits the groups
// into kMergeSplit contiguous ranges, one per wave: each wave merges its
// range in group order with Chan's update (loads eight groups ahead, so
// that about 10 MB of partials are in flight over the workgroups), then
// the first wave merges the waves' results in wave order.  The order depends
// only on the sizes, so repeated runs give the same bits; every wave reads
// 64 consecutive pairs (1 KB) per group, and the workgroups together stream
// the partials once.  Angles get delta0 back (the integrators work in
// deviations).
constexpr int kMergeSplit = 16;

__device__ __forceinline__ void chan_merge(double& cnt, double& m, double& M2, double nb,
                                           double mb, double M2b) {
  const double tot = cnt + nb;
  const double dlt = mb - m;
  const double fb = tot > 0.0 ? nb / tot : 0.0;
  m += dlt * fb;
  M2 += M2b + dlt * dlt * (cnt * fb);
  cnt = tot;
}

__global__ void __launch_bounds__(64 * kMergeSplit) k_stats_merge(
    const double2* __restrict__ partial, int64_t gstride, int64_t n_groups, int group_size,
    int64_t N, int64_t SV, int V, int n, int ddof, const double* __restrict__ delta0,
    double* __restrict__ mean, double* __restrict__ var) {
  __shared__ double sh[3][kMergeSplit][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool on = q < SV;
  const int64_t per = (n_groups + kMergeSplit - 1) / kMergeSplit;
  const int64_t g0 = wv * per, g1 = g0 + per < n_groups ? g0 + per : n_groups;
  double cnt = 0.0, m = 0.0, M2 = 0.0;
  const double2* src = partial + (on ? q : 0);
  constexpr int D = 8;
  for (int64_t g = g0; g < g1; g += D) {
    double2 pt[D];
#pragma unroll
    for (int u = 0; u < D; ++u) pt[u] = (on && g + u < g1) ? src[(g + u) * gstride] : double2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < D; ++u) {
      if (g + u >= g1) break;
      const int64_t rem = N - (g + u) * group_size;
      chan_merge(cnt, m, M2, (double)(rem < group_size ? rem : group_size), pt[u].x, pt[u].y);
    }
  }
  sh[0][wv][lane] = cnt;
  sh[1][wv][lane] = m;
  sh[2][wv][lane] = M2;
  __syncthreads();
  if (wv != 0 || !on) return;
  for (int w = 1; w < kMergeSplit; ++w)
    chan_merge(cnt, m, M2, sh[0][w][lane], sh[1][w][lane], sh[2][w][lane]);
  const int v = (int)(q % V);
  mean[q] = m + (v < n ? delta0[v] : 0.0);
  var[q] = M2 / (double)(N - ddof);
}

hipError_t launch_stats_merge_rows(const double2* partial, int64_t gstride, int64_t n_groups,
                                   int group_size, int64_t N, int64_t rows, int V, int n,
                                   int ddof, const double* delta0, double* mean, double* var,
                                   hipStream_t st) {
  const int64_t SV = rows * V;
  if (SV <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_merge, dim3((unsigned)((SV + 63) / 64)), dim3(64 * kMergeSplit), 0,
                     st, partial, gstride, n_groups, group_size, N, SV, V, n, ddof, delta0, mean,
                     var);
  return hipGetLastError();
}

hipError_t launch_stats_merge(const double2* partial, int64_t n_groups, int group_size,
                              int64_t N, int64_t S, int V, int n, int ddof,
                              const double* delta0, double* mean, double* var, hipStream_t st) {
  return launch_stats_merge_rows(partial, (S + 1) * V, n_groups, group_size, N, S + 1, V, n, ddof,
                                 delta0, mean, var, st);
}

}  // namespace fmc
