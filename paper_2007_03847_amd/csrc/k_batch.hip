// k_batch.hip -- persistent integrator of the batched form: one launch runs
// the work items of many scenarios of different sizes, horizons and N.
//
// A work item is (scenario, range of trajectory tiles).  Workgroups pop items
// from an atomic counter in a host-chosen order (longest first) until the
// queue is empty, which every workgroup reaches.  Each item runs its tiles one
// after another over the whole horizon with the scenario's compiled variant;
// the statistics of its tiles are merged into the item's own rows in tile
// order, and the items of a scenario are merged afterwards in item order, so
// the result does not depend on which workgroup ran what.
#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"
#include "k_integrate.hpp"
#include "k_variants.hpp"

namespace fmc {

constexpr int kBatchWPB = 4, kBatchD = 4;

template <int NG, int PM, int L>
constexpr size_t batch_lds() {
  return GroupShape<float, NG, PM, L, kBatchWPB, kBatchD>::lds_bytes;
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

template <int C>
struct BatchClass;

#define FMC_CLASS_LDS(NG, PM, L) m = cmax(m, batch_lds<NG, PM, L>());
template <>
struct BatchClass<0> {
  static constexpr size_t lds() { size_t m = 0; FMC_BATCH_CLASS0(FMC_CLASS_LDS) return m; }
};
template <>
struct BatchClass<1> {
  static constexpr size_t lds() { size_t m = 0; FMC_BATCH_CLASS1(FMC_CLASS_LDS) return m; }
};
template <>
struct BatchClass<2> {
  static constexpr size_t lds() { size_t m = 0; FMC_BATCH_CLASS2(FMC_CLASS_LDS) return m; }
};
#undef FMC_CLASS_LDS

template <int NG, int PM, int L>
__device__ __forceinline__ void batch_tiles(const IntegArgs<float>& a, const BatchItem& it,
                                            unsigned char* lds) {
  using Sh = GroupShape<float, NG, PM, L, kBatchWPB, kBatchD>;
  // With a state buffer the scenario runs in time chunks: the item's rows then
  // hold the chunk's steps s_begin..s_end, and the kernel addresses them by
  // global step.
  double2* rows = a.state ? it.rows - a.s_begin * a.V : it.rows;
  for (int64_t t = it.tile0; t < it.tile1; ++t) {
    GroupStats st{rows, (t - it.tile0) * Sh::TB};
    group_run<float, NG, PM, L, kBatchWPB, kBatchD>(a, t, lds, st, a.state != nullptr);
  }
}

// The variant ids are global (class 0 first); a class kernel dispatches the
// ids of its own variants.
#define FMC_DISPATCH(NG, PM, L)                                  \
  if (it.variant == id) batch_tiles<NG, PM, L>(a, it, lds);      \
  ++id;
#define FMC_COUNT(NG, PM, L) ++id;

template <int C>
__global__ void __launch_bounds__(64 * kBatchWPB) k_rk4_persistent(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[BatchClass<C>::lds()];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // everyone has read the previous s_item
    if (threadIdx.x == 0) s_item = atomicAdd(b.head, 1);
    __syncthreads();
    const int q = s_item;
    if (q >= b.n_items) break;  // uniform over the workgroup
    const BatchItem it = b.items[b.order[q]];
    const IntegArgs<float> a = b.scen[it.scen];
    int id = 0;
    if constexpr (C == 0) {
      FMC_BATCH_CLASS0(FMC_DISPATCH)
    } else if constexpr (C == 1) {
      FMC_BATCH_CLASS0(FMC_COUNT)
      FMC_BATCH_CLASS1(FMC_DISPATCH)
    } else {
      FMC_BATCH_CLASS0(FMC_COUNT)
      FMC_BATCH_CLASS1(FMC_COUNT)
      FMC_BATCH_CLASS2(FMC_DISPATCH)
    }
  }
}
#undef FMC_DISPATCH
#undef FMC_COUNT

int n_batch_variants() {
  int id = batch_n_lane_variants();
#define FMC_X(NB, BF) ++id;
  FMC_BATCH_MFMA(FMC_X)
#undef FMC_X
  return id;
}

BatchVariantInfo batch_variant(int i) {
  int id = 0, cls = 0;
#define FMC_X(NG, PM, L)                                                                       \
  if (i == id)                                                                                 \
    return BatchVariantInfo{id, NG, PM, L, GroupShape<float, NG, PM, L, kBatchWPB, kBatchD>::TB, \
                            cls};                                                              \
  ++id;
  FMC_BATCH_CLASS0(FMC_X)
  cls = 1;
  FMC_BATCH_CLASS1(FMC_X)
  cls = 2;
  FMC_BATCH_CLASS2(FMC_X)
#undef FMC_X
  // classes 3-6 (NB = 1 to 4): 16 NB machines, kMcMaxProc processes, 4 lanes
  // per trajectory in the state layout, 64-trajectory tiles
#define FMC_X(NB, BF)                                                                  \
  if (i == id) return BatchVariantInfo{id, 16 * NB, kMcMaxProc, 4, 64, 2 + NB, 1 + BF}; \
  ++id;
  FMC_BATCH_MFMA(FMC_X)
#undef FMC_X
  return BatchVariantInfo{-1, 0, 0, 0, 0, 0, 0};
}

hipError_t launch_persistent(int cls, const BatchArgs& b, int grid, hipStream_t st) {
  if (cls >= 3) return launch_persistent_mc(cls - 2, b, grid, st);
  if (cls == 0)
    hipLaunchKernelGGL(k_rk4_persistent<0>, dim3((unsigned)grid), dim3(64 * kBatchWPB), 0, st, b);
  else if (cls == 1)
    hipLaunchKernelGGL(k_rk4_persistent<1>, dim3((unsigned)grid), dim3(64 * kBatchWPB), 0, st, b);
  else
    hipLaunchKernelGGL(k_rk4_persistent<2>, dim3((unsigned)grid), dim3(64 * kBatchWPB), 0, st, b);
  return hipGetLastError();
}

int persistent_blocks_per_cu(int cls) {
  if (cls >= 3) return persistent_mc_blocks_per_cu(cls - 2);
  int nb = 0;
  hipError_t e;
  if (cls == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_persistent<0>, 64 * kBatchWPB, 0);
  else if (cls == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_persistent<1>, 64 * kBatchWPB, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_persistent<2>, 64 * kBatchWPB, 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace fmc
