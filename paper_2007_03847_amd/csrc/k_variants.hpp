// k_variants.hpp -- the compiled integrator variants X(NG, PM, L, WPB):
// NG machines and PM processes (a scenario with n <= NG and P <= PM runs on a
// variant padded with inert entries), L lanes per trajectory (L = 1: the lane
// kernel, machine data through scalar loads), WPB waves per workgroup.
#pragma once

#define FMC_VARIANTS(X) \
  X(1, 1, 1, 1)         \
  X(2, 4, 1, 1)         \
  X(4, 4, 1, 1)         \
  X(4, 8, 1, 1)         \
  X(6, 4, 1, 1)         \
  X(8, 4, 1, 1)         \
  X(8, 8, 1, 1)         \
  X(10, 4, 1, 1)        \
  X(12, 4, 1, 1)        \
  X(12, 8, 1, 1)        \
  X(16, 4, 1, 1)        \
  X(16, 8, 1, 1)        \
  X(20, 8, 1, 1)        \
  X(24, 8, 1, 1)        \
  X(32, 8, 1, 1)        \
  X(10, 4, 2, 1)        \
  X(10, 4, 4, 1)        \
  X(10, 4, 8, 1)        \
  X(10, 4, 16, 1)       \
  X(10, 4, 4, 4)        \
  X(10, 4, 8, 4)        \
  X(10, 4, 16, 4)       \
  X(10, 4, 10, 1)       \
  X(10, 4, 10, 2)       \
  X(10, 4, 10, 4)       \
  X(10, 4, 5, 1)        \
  X(10, 4, 5, 4)        \
  X(10, 4, 16, 2)       \
  X(10, 4, 10, 8)       \
  X(10, 4, 16, 8)       \
  X(16, 8, 16, 4)       \
  X(24, 8, 24, 4)       \
  X(32, 8, 32, 4)       \
  X(50, 8, 50, 4)

// Variants of the persistent batched integrator (FP32, 4 waves per
// workgroup): X(NG machines, PM processes, L lanes per trajectory), in three
// size classes compiled as separate persistent kernels (the register
// footprint of a kernel is that of its largest variant).
#define FMC_BATCH_CLASS0(X) \
  X(4, 8, 4)                \
  X(6, 8, 6)                \
  X(8, 8, 8)                \
  X(10, 8, 10)
#define FMC_BATCH_CLASS1(X) \
  X(12, 8, 12)              \
  X(16, 8, 16)              \
  X(20, 8, 20)              \
  X(24, 8, 24)
#define FMC_BATCH_CLASS2(X) \
  X(32, 8, 32)              \
  X(40, 8, 40)              \
  X(50, 8, 50)
#define FMC_BATCH_VARIANTS(X) FMC_BATCH_CLASS0(X) FMC_BATCH_CLASS1(X) FMC_BATCH_CLASS2(X)

// Matrix-core variants of the batched integrator (classes 3-6, one persistent
// kernel per NB): X(NB blocks of 16 machines, BF), BF = 1 for the BF16 x3
// product of the network current, 0 for FP32.  Ids follow the lane variants
// in this order (the 16-machine pair came last).
#define FMC_BATCH_MFMA(X) \
  X(2, 0)                 \
  X(3, 0)                 \
  X(4, 0)                 \
  X(2, 1)                 \
  X(3, 1)                 \
  X(4, 1)                 \
  X(1, 0)                 \
  X(1, 1)

// Number of lane (class 0-2) variants; the matrix-core ids follow them.
constexpr int batch_n_lane_variants() {
  int id = 0;
#define FMC_X(NG, PM, L) ++id;
  FMC_BATCH_VARIANTS(FMC_X)
#undef FMC_X
  return id;
}
