// k_variants.hpp -- the compiled integrator variants (one trajectory per
// lane): X(NG machines, PM processes).  A scenario with n <= NG machines and
// P <= PM processes runs on a variant padded with inert machines/processes.
#pragma once

#define FMC_LANE_VARIANTS(X) \
  X(1, 1)                    \
  X(2, 4)                    \
  X(4, 4)                    \
  X(4, 8)                    \
  X(6, 4)                    \
  X(8, 4)                    \
  X(8, 8)                    \
  X(10, 4)                   \
  X(12, 4)                   \
  X(12, 8)                   \
  X(16, 4)                   \
  X(16, 8)                   \
  X(20, 8)                   \
  X(24, 8)                   \
  X(32, 8)
