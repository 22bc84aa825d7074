// k_sample.hip -- LHS stratifier, KLE basis table and the KLE path
// contraction (MFMA) for gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fmc_device.hpp"
#include "fmc_internal.hpp"

namespace fmc {

// ---------------------------------------------------------------------------
// LHS (Sec. IV-B).  One thread per element (row i, sample n); sample-fastest
// so the stores coalesce.  Row i = p*K + j follows the reindexing of Sec. IV-A.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_lhs(uint64_t seed, int32_t M, int64_t N, int32_t sampler,
                                             int h, int32_t* __restrict__ strata,
                                             double* __restrict__ zeta) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  __shared__ uint64_t s_key[8];
  if (sampler == 0) {
    if (threadIdx.x < 8) s_key[threadIdx.x] = draw64(seed, (uint64_t)i, threadIdx.x, 0, kTagPerm);
    __syncthreads();
  }
  if (n >= N || i >= M) return;
  double z;
  int32_t s_out;
  if (sampler == 0) {
    uint64_t key[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) key[r] = s_key[r];
    const int64_t s = lhs_stratum(key, N, h, n);
    const double U = u01(draw64(seed, (uint64_t)i, (uint64_t)n, 0, kTagJitter));
    z = ppnd16(stratum_prob(s, U, N));
    s_out = (int32_t)s;
  } else {
    z = ppnd16(u01(draw64(seed, (uint64_t)i, (uint64_t)n, 0, kTagSrs)));
    s_out = -1;
  }
  const int64_t o = i * N + n;
  if (strata) strata[o] = s_out;
  zeta[o] = z;
}

hipError_t launch_lhs(uint64_t seed, int32_t M, int64_t N, int32_t sampler, int32_t* strata,
                      double* zeta, hipStream_t st) {
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)M);
  hipLaunchKernelGGL(k_lhs, grid, dim3(256), 0, st, seed, M, N, sampler, feistel_half_bits(N),
                     strata, zeta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Correlated disturbances (a diffusion matrix S, eq. 4): the noise driving
// process p is sum_q S[p][q] w_q, and since the KLE paths are linear in the
// coefficients, the coefficients are mixed instead of the paths:
// out[p*K + j][n] = sum_q S[p][q] in[q*K + j][n].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mix_design(const double* __restrict__ S, int32_t P,
                                                    int32_t K, int64_t N,
                                                    const double* __restrict__ in,
                                                    double* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int row = blockIdx.y, p = row / K, j = row % K;
  double s = 0.0;
  for (int q = 0; q < P; ++q) s += S[p * P + q] * in[(int64_t)(q * K + j) * N + n];
  out[(int64_t)row * N + n] = s;
}

hipError_t launch_mix_design(const double* S, int32_t P, int32_t K, int64_t N, const double* in,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mix_design, dim3((unsigned)((N + 255) / 256), (unsigned)(P * K)), dim3(256),
                     0, st, S, P, K, N, in, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// KLE basis (eq. 7) at the stage times t_c = c T/(2S).  The cosine argument is
// reduced exactly in integers: (j c) mod 4S for the paper basis,
// ((2j+1) c) mod 8S for the eigen basis, then cospi of the reduced fraction.
// Kind 2 is the one-hot basis of the Euler-Maruyama baseline (eq. 5): row j
// is 1.5 / sqrt(dt) at the midpoint stage c = 2j + 1 of step j, else 0.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_basis(int32_t kind, int32_t K, int64_t S, double T,
                                               double* __restrict__ phi) {
  const int64_t C = 2 * S + 1;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (c >= C || j >= K) return;
  const double a2 = sqrt(2.0 / T);
  double v;
  if (kind == 2) {
    v = c == 2 * j + 1 ? 1.5 / sqrt(T / (double)S) : 0.0;
  } else if (kind == 0) {
    if (j == 0) {
      v = sqrt(1.0 / T);
    } else {
      const int64_t q = (j * c) % (4 * S);
      v = a2 * cospi((double)q / (double)(2 * S));
    }
  } else {
    const int64_t q = ((2 * j + 1) * c) % (8 * S);
    v = a2 * cospi((double)q / (double)(4 * S));
  }
  phi[j * C + c] = v;
}

hipError_t launch_basis(int32_t kind, int32_t K, int64_t S, double T, double* phi,
                        hipStream_t st) {
  const int64_t C = 2 * S + 1;
  dim3 grid((unsigned)((C + 255) / 256), (unsigned)K);
  hipLaunchKernelGGL(k_basis, grid, dim3(256), 0, st, kind, K, S, T, phi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// KLE path contraction (eqs. 8-9): for each process p,
//   w[c][p][n] = sum_j phi[j][c0 + c] * zeta[p K + j][n],
// i.e. (Phi^T)[C x K] x Z_p[K x N].  Each wave owns a 16 (c) x 64 (n) output
// tile; four waves per workgroup stack along c.
//
// FP64: v_mfma_f64_16x16x4_f64.  Operand lanes: A[i][k] at lane 16k + i,
// B[k][j] at lane 16k + j; result register r of lane l is D[4r + l/16][l%16].
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

template <typename OutT>
__device__ __forceinline__ void kle_f64_tile(const double* __restrict__ zeta,
                                             const double* __restrict__ phi, int64_t phi_ld,
                                             int P, int K, int64_t N, int64_t C, int64_t c0,
                                             OutT* __restrict__ w, int64_t bx, int64_t by, int p) {
  const int lane = threadIdx.x & 63;
  const int64_t cb = (by * 4 + (threadIdx.x >> 6)) * 16;
  const int64_t n0 = bx * 64;
  if (cb >= C) return;  // uniform per wave
  const int li = lane & 15, lk = lane >> 4;
  const double* __restrict__ zp = zeta + (int64_t)p * K * N;
  d4_t acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = d4_t{0.0, 0.0, 0.0, 0.0};
  const int64_t ca = cb + li;
  for (int j0 = 0; j0 < K; j0 += 4) {
    const int j = j0 + lk;
    const bool jv = j < K;
    const double a = (jv && ca < C) ? phi[(int64_t)j * phi_ld + c0 + ca] : 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t n = n0 + 16 * b + li;
      const double bv = (jv && n < N) ? zp[(int64_t)j * N + n] : 0.0;
      acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t n = n0 + 16 * b + li;
    if (n >= N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t c = cb + 4 * r + lk;
      if (c < C) w[(c * P + p) * N + n] = (OutT)acc[b][r];
    }
  }
}

// The grid is a flat list of blocks striding over the (n, c, p) tiles, so a
// launch can use fewer workgroups than tiles (to run beside another kernel).
template <typename OutT>
__global__ void __launch_bounds__(256) k_kle_f64(const double* __restrict__ zeta,
                                                 const double* __restrict__ phi, int64_t phi_ld,
                                                 int P, int K, int64_t N, int64_t C, int64_t c0,
                                                 OutT* __restrict__ w) {
  const int64_t tx = (N + 63) / 64, ty = (C + 63) / 64, n_tiles = tx * ty * P;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
    kle_f64_tile<OutT>(zeta, phi, phi_ld, P, K, N, C, c0, w, tile % tx, (tile / tx) % ty,
                       (int)(tile / (tx * ty)));
}
template <typename OutT>
static hipError_t launch_kle_f64_t(const double* zeta, const double* phi, int64_t phi_ld, int P,
                                   int K, int64_t N, int64_t C, int64_t c0, OutT* w,
                                   hipStream_t st, int max_blocks) {
  if (C <= 0 || N <= 0 || P <= 0) return hipSuccess;
  int64_t tiles = ((N + 63) / 64) * ((C + 63) / 64) * P;
  if (max_blocks > 0) tiles = std::min<int64_t>(tiles, max_blocks);
  hipLaunchKernelGGL(k_kle_f64<OutT>, dim3((unsigned)tiles), dim3(256), 0, st, zeta, phi, phi_ld, P,
                     K, N, C, c0, w);
  return hipGetLastError();
}

hipError_t launch_kle_f64(const double* zeta, const double* phi, int64_t phi_ld, int P, int K,
                          int64_t N, int64_t C, int64_t c0, double* w, hipStream_t st,
                          int max_blocks) {
  return launch_kle_f64_t<double>(zeta, phi, phi_ld, P, K, N, C, c0, w, st, max_blocks);
}

hipError_t launch_kle_f64_to_f32(const double* zeta, const double* phi, int64_t phi_ld, int P,
                                 int K, int64_t N, int64_t C, int64_t c0, float* w,
                                 hipStream_t st, int max_blocks) {
  return launch_kle_f64_t<float>(zeta, phi, phi_ld, P, K, N, C, c0, w, st, max_blocks);
}

// ---------------------------------------------------------------------------
// BF16 hi+lo split (three products, FP32 accumulation) on
// v_mfma_f32_16x16x32_bf16.  x = hi + lo with hi = bf16(x), lo = bf16(x - hi);
// the product keeps hi*hi + hi*lo + lo*hi.  Operand lanes: A[i][8(l/16)+e] and
// B[8(l/16)+e][j] for e = 0..7 at lane l = 16(l/16) + i (resp. j); result
// register r of lane l is D[4(l/16) + r][l%16].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float xf = (float)x;
  hi = (__bf16)xf;
  lo = (__bf16)(xf - (float)hi);
}

__device__ __forceinline__ void kle_bf16x3_tile(const double* __restrict__ zeta,
                                                const double* __restrict__ phi, int64_t phi_ld,
                                                int P, int K, int64_t N, int64_t C, int64_t c0,
                                                float* __restrict__ w, int64_t bx, int64_t by,
                                                int p) {
  const int lane = threadIdx.x & 63;
  const int64_t cb = (by * 4 + (threadIdx.x >> 6)) * 16;
  const int64_t n0 = bx * 64;
  if (cb >= C) return;  // uniform per wave
  const int li = lane & 15, lk = lane >> 4;
  const double* __restrict__ zp = zeta + (int64_t)p * K * N;
  f4_t acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f4_t{0.f, 0.f, 0.f, 0.f};
  const int64_t ca = cb + li;
  for (int j0 = 0; j0 < K; j0 += 32) {
    bf8_t ahi, alo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = j0 + 8 * lk + e;
      const double a = (j < K && ca < C) ? phi[(int64_t)j * phi_ld + c0 + ca] : 0.0;
      __bf16 h, l;
      split_bf16(a, h, l);
      ahi[e] = h;
      alo[e] = l;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t n = n0 + 16 * b + li;
      bf8_t bhi, blo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = j0 + 8 * lk + e;
        const double z = (j < K && n < N) ? zp[(int64_t)j * N + n] : 0.0;
        __bf16 h, l;
        split_bf16(z, h, l);
        bhi[e] = h;
        blo[e] = l;
      }
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t n = n0 + 16 * b + li;
    if (n >= N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t c = cb + 4 * lk + r;
      if (c < C) w[(c * P + p) * N + n] = acc[b][r];
    }
  }
}

__global__ void __launch_bounds__(256) k_kle_bf16x3(const double* __restrict__ zeta,
                                                    const double* __restrict__ phi,
                                                    int64_t phi_ld, int P, int K, int64_t N,
                                                    int64_t C, int64_t c0,
                                                    float* __restrict__ w) {
  const int64_t tx = (N + 63) / 64, ty = (C + 63) / 64, n_tiles = tx * ty * P;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
    kle_bf16x3_tile(zeta, phi, phi_ld, P, K, N, C, c0, w, tile % tx, (tile / tx) % ty,
                    (int)(tile / (tx * ty)));
}

hipError_t launch_kle_bf16x3(const double* zeta, const double* phi, int64_t phi_ld, int P, int K,
                             int64_t N, int64_t C, int64_t c0, float* w, hipStream_t st,
                             int max_blocks) {
  if (C <= 0 || N <= 0 || P <= 0) return hipSuccess;
  int64_t tiles = ((N + 63) / 64) * ((C + 63) / 64) * P;
  if (max_blocks > 0) tiles = std::min<int64_t>(tiles, max_blocks);
  hipLaunchKernelGGL(k_kle_bf16x3, dim3((unsigned)tiles), dim3(256), 0, st, zeta, phi, phi_ld, P,
                     K, N, C, c0, w);
  return hipGetLastError();
}

}  // namespace fmc
