// k_rrf.hip -- a scalar random response function (eq. 3) over stored
// trajectories: the RMS over the horizon of a linear combination of the
// outputs, u(t) = sum_v w_v y_v(t), sqrt((1/T) int_0^T u^2 dt) by the
// trapezoid rule on the grid t_s = s dt, T = S dt.  With w the inertia
// weights of the frequency deviations this is the RMS of the system
// (centre-of-inertia) frequency deviation, the RRF of Sec. V-B.
#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"

namespace fmc {

namespace {

// One workgroup per trajectory [S+1][V]; threads stride over the time points.
__global__ void __launch_bounds__(256) k_rrf_rms(const double* __restrict__ traj, int64_t S,
                                                 int32_t V, const double* __restrict__ w,
                                                 double dt, double* __restrict__ rrf) {
  const double* y = traj + (int64_t)blockIdx.x * (S + 1) * V;
  double acc = 0.0;
  for (int64_t s = threadIdx.x; s <= S; s += 256) {
    double u = 0.0;
    for (int v = 0; v < V; ++v) u += w[v] * y[s * V + v];
    const double h = (s == 0 || s == S) ? 0.5 : 1.0;
    acc += h * u * u;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) rrf[blockIdx.x] = sqrt(red[0] * dt / ((double)S * dt));
}

}  // namespace

hipError_t launch_rrf_rms(const double* traj, int64_t n, int64_t S, int32_t V, const double* w,
                          double dt, double* rrf, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rrf_rms, dim3((unsigned)n), dim3(256), 0, st, traj, S, V, w, dt, rrf);
  return hipGetLastError();
}

}  // namespace fmc
