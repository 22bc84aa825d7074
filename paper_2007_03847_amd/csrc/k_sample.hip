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
// i.e. (Phi^T)[C x K] x Z_p[K x N].
//
// FP64: v_mfma_f64_16x16x4_f64.  Operand lanes: A[i][k] at lane 16k + i,
// B[k][j] at lane 16k + j; result register r of lane l is D[4r + l/16][l%16].
// Each wave owns a 32 (c) x 64 (n) output tile: 2 x 4 blocks of 16 x 16 in
// eight accumulators, so every k-step of four loads 2 + 4 operand fragments
// for 8 matrix operations; the fragments of the next k-step are loaded while
// the current one's operations run.  A workgroup's four waves lie along c (a
// 128 x 64 tile): they read the same zeta fragments, which the first brings
// into L1 for the others, so the design (tens to hundreds of MB, beyond the
// L2) is streamed C/128 times per chunk; Phi (a few hundred KB shared by
// every workgroup) stays in L2.
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kKleTC = 128, kKleTN = 64;  // workgroup tile (c, n): four waves along c

template <typename OutT, typename OffT>
__device__ __forceinline__ void kle_f64_tile(const double* __restrict__ zeta,
                                             const double* __restrict__ phi, int64_t phi_ld,
                                             int P, int K, int64_t N, int64_t C, int64_t c0,
                                             OutT* __restrict__ w, int64_t bx, int64_t by, int p) {
  const int lane = threadIdx.x & 63;
  const int64_t cb = by * kKleTC + (threadIdx.x >> 6) * 32;
  const int64_t n0 = bx * kKleTN;
  if (cb >= C) return;  // uniform per wave
  const int li = lane & 15, lk = lane >> 4;
  // Per-lane byte offsets inside a k-step of four rows, from a base that
  // moves with the step (the loads take a scalar base and a 32-bit offset).
  // Columns past the edge (c >= C, n >= N) read the last valid one: they
  // feed only output rows and columns that are never stored, so every load
  // is unconditional and the loop carries no branch.
  OffT ao[2], bo[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t c = cb + 16 * h + li;
    ao[h] = (OffT)(8 * (lk * phi_ld + (c < C ? c : C - 1)));
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t n = n0 + 16 * b + li;
    bo[b] = (OffT)(8 * (lk * N + (n < N ? n : N - 1)));
  }
  const char* __restrict__ A = (const char*)(phi + c0);                    // row j: + 8 j phi_ld
  const char* __restrict__ B = (const char*)(zeta + (int64_t)p * K * N);  // row j: + 8 j N
  d4_t acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[h][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  auto load = [&](int j0, double (&a)[2], double (&bv)[4]) {
    const char* Aj = A + 8 * (int64_t)j0 * phi_ld;
    const char* Bj = B + 8 * (int64_t)j0 * N;
#pragma unroll
    for (int h = 0; h < 2; ++h) a[h] = *(const double*)(Aj + ao[h]);
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = *(const double*)(Bj + bo[b]);
  };
  auto step = [&](const double (&a)[2], const double (&bv)[4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[h][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], bv[b], acc[h][b], 0, 0, 0);
  };
  // k-steps of four rows in pairs, with two fragment sets in turn: the next
  // step's fragments load while this step's products run.  A prefetch past
  // the last full step re-reads that step's rows and stays unused.
  const int K4 = K & ~3;
  double ax[2], bx4[4], ay[2], by4[4];
  if (K4 > 0) load(0, ax, bx4);
  int j0 = 0;
  for (; j0 + 8 <= K4; j0 += 8) {
    load(j0 + 4, ay, by4);
    step(ax, bx4);
    load(j0 + 8 < K4 ? j0 + 8 : K4 - 4, ax, bx4);
    step(ay, by4);
  }
  if (j0 < K4) step(ax, bx4);  // K4 mod 8 == 4: the fragments of row j0 are in x
  if (K4 < K) {  // the last K mod 4 rows; lanes of rows past K contribute zero
    const bool jv = K4 + lk < K;
    const int64_t dj = 8 * (int64_t)(jv ? K4 : K - 1 - lk);  // the lane's row, clamped to K - 1
    double a[2], bv[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double v = *(const double*)(A + dj * phi_ld + ao[h]);
      a[h] = jv ? v : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double v = *(const double*)(B + dj * N + bo[b]);
      bv[b] = jv ? v : 0.0;
    }
    step(a, bv);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t c = cb + 16 * h + 4 * r + lk;
      if (c >= C) continue;
      OutT* row = w + (c * P + p) * N;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t n = n0 + 16 * b + li;
        if (n < N) row[n] = (OutT)acc[h][b][r];
      }
    }
}

// Tile order of a launch with one workgroup per tile.  Workgroups are
// dealt to the eight XCDs in turn (block b to XCD b mod 8), each XCD with an
// L2 of its own, so block b takes tile number L(b) from a contiguous range
// per XCD; in that order the c-tiles of one (n-tile, process) are adjacent,
// so the workgroups that stream the same coefficient rows run on one XCD and
// share its L2.  Tile number L = ((p tx) + bx) ty + by.
__device__ __forceinline__ int64_t kle_xcd_tile(int64_t b, int64_t n_tiles) {
  const int64_t q = n_tiles / 8, r = n_tiles % 8, k = b % 8, j = b / 8;
  return k < r ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j;
}

// The grid is a flat list of blocks striding over the (n, c, p) tiles, so a
// launch can use fewer workgroups than tiles (to run beside another kernel).
// OffT is the type of the per-lane byte offsets: 32-bit while four rows of
// either operand span less than 4 GiB (the loads then take a scalar base and
// a 32-bit offset), else 64-bit.  Four waves per SIMD: eight accumulators
// of 16 x 16 doubles (64 registers) and two k-steps of fragments.
template <typename OutT, typename OffT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_kle_f64(const double* __restrict__ zeta, const double* __restrict__ phi, int64_t phi_ld, int P,
          int K, int64_t N, int64_t C, int64_t c0, OutT* __restrict__ w) {
  const int64_t tx = (N + kKleTN - 1) / kKleTN, ty = (C + kKleTC - 1) / kKleTC;
  const int64_t n_tiles = tx * ty * P;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t L = gridDim.x == n_tiles ? kle_xcd_tile(tile, n_tiles) : tile;
    kle_f64_tile<OutT, OffT>(zeta, phi, phi_ld, P, K, N, C, c0, w, (L / ty) % tx, L % ty,
                             (int)(L / (tx * ty)));
  }
}
template <typename OutT>
static hipError_t launch_kle_f64_t(const double* zeta, const double* phi, int64_t phi_ld, int P,
                                   int K, int64_t N, int64_t C, int64_t c0, OutT* w,
                                   hipStream_t st, int max_blocks) {
  if (C <= 0 || N <= 0 || P <= 0) return hipSuccess;
  int64_t tiles = ((N + kKleTN - 1) / kKleTN) * ((C + kKleTC - 1) / kKleTC) * P;
  if (max_blocks > 0) tiles = std::min<int64_t>(tiles, max_blocks);
  // largest byte offset of a lane inside a k-step: 8 (3 ld + ld - 1) < 32 ld
  const bool narrow = 32 * std::max<int64_t>(N, phi_ld) <= (int64_t)UINT32_MAX;
  if (narrow)
    hipLaunchKernelGGL((k_kle_f64<OutT, uint32_t>), dim3((unsigned)tiles), dim3(256), 0, st, zeta,
                       phi, phi_ld, P, K, N, C, c0, w);
  else
    hipLaunchKernelGGL((k_kle_f64<OutT, int64_t>), dim3((unsigned)tiles), dim3(256), 0, st, zeta,
                       phi, phi_ld, P, K, N, C, c0, w);
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

namespace fmc {

// ---------------------------------------------------------------------------
// BF16 x3 contraction on operands split once.  x -> hi = bf16(float(x)),
// lo = bf16(float(x) - float(hi)) as above, stored k-fastest: Phi as
// [column][Kp] and each process's coefficients as [sample][Kp] (Kp = K
// rounded up to 32, zero beyond K), so that a lane's eight consecutive k of
// an operand fragment are one 16-byte load and no split is left in the
// contraction's inner loop.
// ---------------------------------------------------------------------------

// X: rows k = 0..K-1 of `items` columns with leading dimension ld (process
// p's block at X + p xs); Y: [item][Kp] hi and lo planes (process p's block
// at + p ys).  A 32 (k) x 64 (item) tile is transposed through LDS so both
// the reads and the writes are coalesced.
__global__ void __launch_bounds__(256) k_split_bf16(const double* __restrict__ X, int64_t ld,
                                                    int K, int64_t items, int Kp, int64_t xs,
                                                    int64_t ys, __bf16* __restrict__ yh,
                                                    __bf16* __restrict__ yl) {
  __shared__ double tile[32][65];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int k0 = blockIdx.y * 32;
  const int p = blockIdx.z;
  const double* Xp = X + (int64_t)p * xs;
  for (int kk = tid >> 6; kk < 32; kk += 4) {
    const int k = k0 + kk;
    const int64_t it = i0 + (tid & 63);
    tile[kk][tid & 63] = (k < K && it < items) ? Xp[(int64_t)k * ld + it] : 0.0;
  }
  __syncthreads();
  const int item = tid >> 2, kq = (tid & 3) * 8;
  const int64_t it = i0 + item;
  if (it >= items) return;
  bf8_t h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float xf = (float)tile[kq + e][item];
    const __bf16 hh = (__bf16)xf;
    h[e] = hh;
    l[e] = (__bf16)(xf - (float)hh);
  }
  const int64_t o = (int64_t)p * ys + it * Kp + k0 + kq;
  *reinterpret_cast<bf8_t*>(yh + o) = h;
  *reinterpret_cast<bf8_t*>(yl + o) = l;
}

hipError_t launch_split_bf16(const double* X, int64_t ld, int K, int64_t items, int Kp, int P,
                             int64_t xs, int64_t ys, void* yh, void* yl, hipStream_t st) {
  if (items <= 0 || P <= 0 || Kp <= 0 || Kp % 32 != 0 || K > Kp) return hipErrorInvalidValue;
  dim3 grid((unsigned)((items + 63) / 64), (unsigned)(Kp / 32), (unsigned)P);
  hipLaunchKernelGGL(k_split_bf16, grid, dim3(256), 0, st, X, ld, K, items, Kp, xs, ys,
                     (__bf16*)yh, (__bf16*)yl);
  return hipGetLastError();
}

// w[c][p][n] = sum_k Phi[c0 + c][k] Z_p[n][k] as three BF16 products per
// pair (lo*hi + hi*lo + hi*hi, FP32 accumulation) on
// v_mfma_f32_16x16x32_bf16.  Each wave owns a 32 (c) x 64 (n) output tile (2 x
// 4 blocks, eight accumulators); a k-step of 32 loads 4 + 8 fragments of 16
// bytes for 24 matrix operations, and the next k-step's fragments are loaded
// while they run.  Four waves per workgroup along c, as for FP64.
__device__ __forceinline__ void kle_bf16s_tile(const __bf16* __restrict__ ph,
                                               const __bf16* __restrict__ pl, int Kp,
                                               const __bf16* __restrict__ zh,
                                               const __bf16* __restrict__ zl, int P, int64_t N,
                                               int64_t C, int64_t c0, float* __restrict__ w,
                                               int64_t bx, int64_t by, int p) {
  const int lane = threadIdx.x & 63;
  const int64_t cb = by * kKleTC + (threadIdx.x >> 6) * 32;
  const int64_t n0 = bx * kKleTN;
  if (cb >= C) return;  // uniform per wave
  const int li = lane & 15, ko = 8 * (lane >> 4);
  f4_t acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[h][b] = f4_t{0.f, 0.f, 0.f, 0.f};
  // Rows past the edge (c >= C, n >= N) read the last valid one: they feed
  // only outputs that are never stored, so every load is unconditional.
  int64_t ao[2], bo[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t c = cb + 16 * h + li;
    ao[h] = (c0 + (c < C ? c : C - 1)) * Kp + ko;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t n = n0 + 16 * b + li;
    bo[b] = ((int64_t)p * N + (n < N ? n : N - 1)) * Kp + ko;
  }
  struct frag {
    bf8_t ah[2], al[2], bh[4], bl[4];
  };
  auto load = [&](int k, frag& f) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f.ah[h] = *reinterpret_cast<const bf8_t*>(ph + ao[h] + k);
      f.al[h] = *reinterpret_cast<const bf8_t*>(pl + ao[h] + k);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      f.bh[b] = *reinterpret_cast<const bf8_t*>(zh + bo[b] + k);
      f.bl[b] = *reinterpret_cast<const bf8_t*>(zl + bo[b] + k);
    }
  };
  auto step = [&](const frag& f) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[h][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.al[h], f.bh[b], acc[h][b], 0, 0, 0);
        acc[h][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[h], f.bl[b], acc[h][b], 0, 0, 0);
        acc[h][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[h], f.bh[b], acc[h][b], 0, 0, 0);
      }
  };
  // One fragment set: the loads of a k-step wait for the previous step's
  // products, and the other waves of the SIMD cover that latency (the
  // products of a step are short next to the tile's loads and stores).
  for (int k = 0; k < Kp; k += 32) {
    frag f;
    load(k, f);
    step(f);
  }
  // result register r of lane l is D[4(l/16) + r][l%16]
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t c = cb + 16 * h + 4 * (lane >> 4) + r;
      if (c >= C) continue;
      float* row = w + (c * P + p) * N;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t n = n0 + 16 * b + li;
        if (n < N) row[n] = acc[h][b][r];
      }
    }
}

__global__ void __launch_bounds__(256) k_kle_bf16x3s(const __bf16* __restrict__ ph,
                                                     const __bf16* __restrict__ pl, int Kp,
                                                     const __bf16* __restrict__ zh,
                                                     const __bf16* __restrict__ zl, int P,
                                                     int64_t N, int64_t C, int64_t c0,
                                                     float* __restrict__ w) {
  const int64_t tx = (N + kKleTN - 1) / kKleTN, ty = (C + kKleTC - 1) / kKleTC;
  const int64_t n_tiles = tx * ty * P;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t L = gridDim.x == n_tiles ? kle_xcd_tile(tile, n_tiles) : tile;
    kle_bf16s_tile(ph, pl, Kp, zh, zl, P, N, C, c0, w, (L / ty) % tx, L % ty,
                   (int)(L / (tx * ty)));
  }
}

hipError_t launch_kle_bf16x3_split(const void* ph, const void* pl, int Kp, const void* zh,
                                   const void* zl, int P, int64_t N, int64_t C, int64_t c0,
                                   float* w, hipStream_t st) {
  if (C <= 0 || N <= 0 || P <= 0) return hipSuccess;
  if (Kp <= 0 || Kp % 32 != 0) return hipErrorInvalidValue;
  const int64_t tiles = ((N + kKleTN - 1) / kKleTN) * ((C + kKleTC - 1) / kKleTC) * P;
  hipLaunchKernelGGL(k_kle_bf16x3s, dim3((unsigned)tiles), dim3(256), 0, st, (const __bf16*)ph,
                     (const __bf16*)pl, Kp, (const __bf16*)zh, (const __bf16*)zl, P, N, C, c0, w);
  return hipGetLastError();
}

}  // namespace fmc
