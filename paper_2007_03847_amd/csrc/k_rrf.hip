// k_rrf.hip -- a scalar random response function (eq. 3) over stored
// trajectories: the RMS over the horizon of a linear combination of the
// outputs, u(t) = sum_v w_v y_v(t), sqrt((1/T) int_0^T u^2 dt) by the
// trapezoid rule on the grid t_s = s dt, T = S dt.  With w the inertia
// weights of the frequency deviations this is the RMS of the system
// (centre-of-inertia) frequency deviation, the RRF of Sec. V-B.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fmc_internal.hpp"

namespace fmc {

// Scratch of the allocation-free entry point (fmc_rrf_rms_noalloc): the
// device copy of the weights, at most kRrfStaticMaxV doubles.  Each device
// the library runs on holds its own copy until the process ends.  In host
// code the array's name is not a device address: host code uses the address
// hipGetSymbolAddress returned for the current device (rrf_scratch).
static __device__ __align__(256) double scratch[kRrfStaticMaxV];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

constexpr int kRrfLds = 2048;  // doubles of trajectory staged per tile (16 KB: several workgroups per CU)

// One workgroup per trajectory [S+1][V].  Tiles of whole time points are
// staged in LDS with coalesced loads (the rows are V doubles long, so a
// thread per time point reading global memory directly would stride by V);
// thread t then forms u for time point t of the tile.  Each thread holds its
// share of the next tile (at most kRrfLds / 256 doubles) in registers, loaded
// while the current tile is reduced, so that a workgroup keeps a tile of
// loads in flight beside its LDS work.
constexpr int kRrfPer = kRrfLds / 256;
__device__ __forceinline__ void rrf_fetch(const double* __restrict__ y, int64_t s0, int ne,
                                          int32_t V, double (&r)[kRrfPer]) {
#pragma unroll
  for (int i = 0; i < kRrfPer; ++i) {
    const int e = (int)threadIdx.x + i * 256;
    r[i] = e < ne ? y[s0 * V + e] : 0.0;
  }
}
__global__ void __launch_bounds__(256) k_rrf_rms(const double* __restrict__ traj, int64_t S,
                                                 int32_t V, int32_t pts,
                                                 const double* __restrict__ w, double dt,
                                                 double* __restrict__ rrf) {
  __shared__ double tile[kRrfLds];
  __shared__ double red[256];
  const double* y = traj + (int64_t)blockIdx.x * (S + 1) * V;
  double acc = 0.0;
  double r[kRrfPer];
  int np = (int)((S + 1) < pts ? (S + 1) : pts);
  rrf_fetch(y, 0, np * V, V, r);
  for (int64_t s0 = 0; s0 <= S; s0 += pts) {
    const int ne = np * V;
    __syncthreads();  // the previous tile has been read
#pragma unroll
    for (int i = 0; i < kRrfPer; ++i) {
      const int e = (int)threadIdx.x + i * 256;
      if (e < ne) tile[e] = r[i];
    }
    __syncthreads();
    const int64_t s1 = s0 + pts;
    const int np1 = s1 <= S ? (int)((S + 1 - s1) < pts ? (S + 1 - s1) : pts) : 0;
    if (np1 > 0) rrf_fetch(y, s1, np1 * V, V, r);
    for (int q = threadIdx.x; q < np; q += 256) {
      double u = 0.0;
      for (int v = 0; v < V; ++v) u += w[v] * tile[q * V + v];
      const int64_t s = s0 + q;
      const double h = (s == 0 || s == S) ? 0.5 : 1.0;
      acc += h * u * u;
    }
    np = np1;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) rrf[blockIdx.x] = sqrt(red[0] * dt / ((double)S * dt));
}

}  // namespace

// Once per device, with that device current (called by fmc_context_create):
// the device address of `scratch`.
hipError_t rrf_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (double*)p;
  return hipSuccess;
}

double* rrf_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_rrf_rms(const double* traj, int64_t n, int64_t S, int32_t V, const double* w,
                          double dt, double* rrf, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // whole time points per tile, at most 256 (one per thread) and kRrfLds doubles;
  // a row longer than the tile is beyond this kernel
  if (V > kRrfLds) return hipErrorInvalidValue;
  const int pts = V * 256 <= kRrfLds ? 256 : kRrfLds / V;
  hipLaunchKernelGGL(k_rrf_rms, dim3((unsigned)n), dim3(256), 0, st, traj, S, V, pts, w, dt, rrf);
  return hipGetLastError();
}

}  // namespace fmc
