// k_mfma_classical.hip -- classes 3-6 of the persistent batched integrator:
// classical machines with the network current on the matrix cores (the
// device code is in k_mfma_classical.hpp), and the packing of its
// coefficient block.
#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"
#include "k_mfma_classical.hpp"
#include "k_variants.hpp"

namespace fmc {

// Constants of a matrix-core variant from the canonical FP64 block: machine rows
// [n_pad][8] (zero for padding machines, which then stay at rest), then
// theta, sigma, xi0 and the driven machine of each process (as a float; -1
// for unused process slots).
__global__ void __launch_bounds__(256) k_pack_mc(const double* __restrict__ cn, int n, int P,
                                                 const int32_t* __restrict__ gen, int n_pad,
                                                 float* __restrict__ coef) {
  const CanonLayout C{n, P};
  const McPack K{n_pad};
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= K.consts()) return;
  float v = 0.0f;
  if (q < K.proc()) {
    const int m = q / McPack::kStride, f = q % McPack::kStride;
    const int64_t base[7] = {C.c0(), C.s0(), C.i0r(), C.i0i(), C.res(), C.dmp(), C.inv2h()};
    if (m < n && f < 7) v = (float)cn[base[f] + m];
  } else {
    const int e = q - K.proc(), f = e / kMcMaxProc, p = e % kMcMaxProc;
    if (f < 3) {
      const int64_t base[3] = {C.theta(), C.sigma(), C.xi0()};
      if (p < P) v = (float)cn[base[f] + p];
    } else {
      v = (p < P && gen[p] >= 0 && gen[p] < n) ? (float)gen[p] : -1.0f;
    }
  }
  coef[q] = v;
}

hipError_t launch_pack_mc(const double* canon, int n, int P, const int32_t* gen, int n_pad,
                          bool bf, float* coef, hipStream_t st) {
  const McPack K{n_pad};
  hipLaunchKernelGGL(k_pack_mc, dim3((unsigned)((K.consts() + 255) / 256)), dim3(256), 0, st,
                     canon, n, P, gen, n_pad, coef);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return bf ? launch_pack_fd_y16(canon, n, n_pad, K.n_padk(), coef + K.frag(), st)
            : launch_pack_fd_y(canon, n, n_pad, reinterpret_cast<float2*>(coef + K.frag()), st);
}

hipError_t launch_pack_batch(const BatchVariantInfo& b, const double* canon, int n, int P,
                             const int32_t* gen, float* coef, hipStream_t st) {
  if (b.prod != 0) return launch_pack_mc(canon, n, P, gen, b.NG, b.prod == 2, coef, st);
  return launch_pack<float>(canon, n, P, gen, b.NG, b.PM, coef, st);
}

// Persistent matrix-core kernels, one per block count NB (a kernel's register
// footprint is that of its largest variant, so the 32-machine variants get
// their own kernel and twice the waves per SIMD): workgroups pop work items
// (ranges of 64-trajectory tiles of one scenario) until the queue is empty,
// as the lane classes do.
#define FMC_MC_DISPATCH(NBV, BF)                                                    \
  if constexpr (NBV == NB)                                                          \
    if (it.variant == id)                                                           \
      for (int64_t t = it.tile0; t < it.tile1; ++t)                                 \
        mc_tile<BF != 0, NBV>(a, t, S, GroupStats{rows, (t - it.tile0) * mc::kTile}); \
  ++id;

// NB = 1 to 3 are held to 256 registers (two waves per SIMD; for NB = 3 at
// the cost of spills, measured faster: 38.8 -> 34.5 ms at 33 machines); NB = 4
// runs one wave per SIMD (two waves with its spills measured slower).
template <int NB>
__global__ void __launch_bounds__(64 * mc::kWaves)
    __attribute__((amdgpu_waves_per_eu(NB <= 3 ? 2 : 1))) k_rk4_persistent_mc(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) mc::Lds S;
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // everyone has read the previous s_item
    if (threadIdx.x == 0) s_item = atomicAdd(b.head, 1);
    __syncthreads();
    const int q = s_item;
    if (q >= b.n_items) break;  // uniform over the workgroup
    const BatchItem it = b.items[b.order[q]];
    const IntegArgs<float> a = b.scen[it.scen];
    // with a state buffer the rows hold the chunk's steps s_begin..s_end
    double2* rows = a.state ? it.rows - a.s_begin * a.V : it.rows;
    int id = batch_n_lane_variants();
    FMC_BATCH_MFMA(FMC_MC_DISPATCH)
  }
}
#undef FMC_MC_DISPATCH

template <int NB>
static int blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_persistent_mc<NB>, 64 * mc::kWaves,
                                                   0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int persistent_mc_blocks_per_cu(int nb) {
  return nb == 1   ? blocks_per_cu<1>()
         : nb == 2 ? blocks_per_cu<2>()
         : nb == 3 ? blocks_per_cu<3>()
                   : blocks_per_cu<4>();
}

hipError_t launch_persistent_mc(int nb, const BatchArgs& b, int grid, hipStream_t st) {
  const dim3 g((unsigned)grid), blk(64 * mc::kWaves);
  if (nb == 1)
    hipLaunchKernelGGL(k_rk4_persistent_mc<1>, g, blk, 0, st, b);
  else if (nb == 2)
    hipLaunchKernelGGL(k_rk4_persistent_mc<2>, g, blk, 0, st, b);
  else if (nb == 3)
    hipLaunchKernelGGL(k_rk4_persistent_mc<3>, g, blk, 0, st, b);
  else
    hipLaunchKernelGGL(k_rk4_persistent_mc<4>, g, blk, 0, st, b);
  return hipGetLastError();
}

}  // namespace fmc
