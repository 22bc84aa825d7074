// k_decor.hip -- correlation-reducing permutation of an LHS design (Sec. IV-B,
// LHS Step 2: the rows may be permuted by any rule; the paper points to
// Cholesky-based correlation control).  The M rows of the design are taken as
// M variables observed in N samples.  Their sample covariance C is factored
// C = L L^T, the scores Z = L^{-1} (X - mean) have identity sample covariance,
// and each row of X is rearranged so that its values take the ranks of the
// same row of Z (one pass of rank-based correlation control towards the
// identity).  A row keeps its values; only their assignment to samples
// changes, so an LHS row still holds one value per stratum.
//
// Steps on the stream, all FP64:
//   k_dc_mean    row means                        M workgroups
//   k_dc_cov     lower-triangle 64x64 tiles of C  x sample slices, then k_dc_cov_sum
//   k_dc_chol    Cholesky by 32-column blocks     one workgroup (M <= 1024)
//   k_dc_whiten  substitution by 32-row blocks    residuals of 4-16 samples in LDS
//   k_dc_range .. k_dc_rank   ranks in each row   buckets + prefix sums, O(N) expected
//   k_dc_apply   rearrangement                    one thread per entry
// Ranks order equal values by the lower sample index and always form a
// permutation, so every gather stays in bounds whatever the values are.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fmc_internal.hpp"
#include "fmc_runtime.hpp"

namespace fmc {

namespace {

constexpr int kDcCovTile = 64;  // covariance tile edge (4x4 entries per thread)
constexpr int kDcChunk = 16;    // samples per LDS stage of the covariance
constexpr int kDcBlk = 32;      // block of the Cholesky factor and of the substitution
constexpr int kDcSlab = 64;     // rows of L staged at a time by the substitution
constexpr int kDcCholThreads = 1024;  // one thread per row below a block (M <= 1024)
constexpr int kDcPanelRows = 384;     // rows of a block of L held in LDS (101 KB)

__global__ void __launch_bounds__(256) k_dc_mean(int64_t N, const double* __restrict__ X,
                                                 double* __restrict__ mean) {
  const double* x = X + (int64_t)blockIdx.x * N;
  double s = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += 256) s += x[n];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[blockIdx.x] = red[0] / (double)N;
}

// Partial sample cross-products of the centred rows over one slice of the
// samples (blockIdx.y), for one 64x64 tile (ta, tb), ta >= tb, of C
// (blockIdx.x enumerates the lower-triangle tiles).  Thread (ty, tx) holds the
// 4x4 entries (ty + 16u, tx + 16v); chunks of 16 samples are staged in LDS.
__global__ void __launch_bounds__(256) k_dc_cov(int M, int64_t N, int64_t per,
                                                const double* __restrict__ X,
                                                const double* __restrict__ mean,
                                                double* __restrict__ P) {
  int t = blockIdx.x, ta = 0;
  while (t > ta) {
    t -= ta + 1;
    ++ta;
  }
  const int tb = t;
  const int64_t nb0 = (int64_t)blockIdx.y * per;
  const int64_t nb1 = std::min<int64_t>(N, nb0 + per);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  __shared__ double sa[kDcChunk][kDcCovTile + 1], sb[kDcChunk][kDcCovTile + 1];
  double acc[4][4] = {};
  for (int64_t n0 = nb0; n0 < nb1; n0 += kDcChunk) {
    __syncthreads();
    for (int q = threadIdx.x; q < kDcCovTile * kDcChunk; q += 256) {
      const int r = q / kDcChunk, k = q % kDcChunk;
      const int64_t n = n0 + k;
      const int ra = ta * kDcCovTile + r, rb = tb * kDcCovTile + r;
      sa[k][r] = (ra < M && n < nb1) ? X[(int64_t)ra * N + n] - mean[ra] : 0.0;
      sb[k][r] = (rb < M && n < nb1) ? X[(int64_t)rb * N + n] - mean[rb] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kDcChunk; ++k) {
      double va[4], vb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        va[u] = sa[k][ty + 16 * u];
        vb[u] = sb[k][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(va[u], vb[v], acc[u][v]);
    }
  }
  double* out = P + (int64_t)blockIdx.y * M * M;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ta * kDcCovTile + ty + 16 * u, b = tb * kDcCovTile + tx + 16 * v;
      if (a < M && b < M) out[(int64_t)a * M + b] = acc[u][v];
    }
}

// C = sum of the slices' partials (in slice order) / (N - 1), both triangles.
__global__ void __launch_bounds__(256) k_dc_cov_sum(int M, int64_t N, int n_slices,
                                                    const double* __restrict__ P,
                                                    double* __restrict__ Cv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * M) return;
  const int a = (int)(q / M), b = (int)(q % M);
  if (b > a) return;
  double s = 0.0;
  for (int z = 0; z < n_slices; ++z) s += P[(int64_t)z * M * M + q];
  const double v = s / (double)(N - 1);
  Cv[(int64_t)a * M + b] = v;
  Cv[(int64_t)b * M + a] = v;
}

// Cholesky of the M x M matrix A by blocks of 32 columns, one workgroup:
// the diagonal block is factored in LDS, the rows below it are solved one
// per thread, and the trailing matrix is updated one wave per row, from the
// rows' block of L in LDS once they fit (panel_rows rows).  L is
// written transposed to LT (LT[k][i] = L[i][k], the layout the substitution
// reads); A's lower triangle is overwritten.  A pivot of at most 1e-12 of its
// diagonal entry marks a row that is (to rounding) a combination of the rows
// before it: *status is set and LT is made the identity, so that the later
// steps leave the design as it is.
__global__ void __launch_bounds__(kDcCholThreads) k_dc_chol(int M, int panel_rows,
                                                            double* __restrict__ A,
                                                            double* __restrict__ LT,
                                                            int32_t* __restrict__ status) {
  extern __shared__ double s_panel[];  // [panel_rows][kDcBlk + 1] block of L below the diagonal
  __shared__ double s_d0[kDecorMaxM];
  __shared__ double s_D[kDcBlk][kDcBlk + 1];
  __shared__ double s_row[kDcCholThreads / 64][kDcBlk];  // one row of the block of L per wave
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64, n_waves = blockDim.x / 64;
  for (int i = tid; i < M; i += blockDim.x) s_d0[i] = A[(int64_t)i * M + i];
  if (tid == 0) s_bad = 0;
  for (int j0 = 0; j0 < M; j0 += kDcBlk) {
    const int nb = std::min(kDcBlk, M - j0);
    __syncthreads();
    for (int q = tid; q < kDcBlk * kDcBlk; q += blockDim.x) {
      const int r = q / kDcBlk, cc = q % kDcBlk;
      s_D[r][cc] = (r < nb && cc <= r) ? A[(int64_t)(j0 + r) * M + j0 + cc] : 0.0;
    }
    for (int c = 0; c < nb; ++c) {
      __syncthreads();
      if (tid == 0) {
        const double d = s_D[c][c];
        if (!(d > 1e-12 * s_d0[j0 + c])) s_bad = 1;
        s_D[c][c] = s_bad ? 1.0 : sqrt(d);
      }
      __syncthreads();
      if (s_bad) break;  // uniform: shared flag read after the barrier
      if (tid > c && tid < nb) s_D[tid][c] /= s_D[c][c];
      __syncthreads();
      for (int q = tid; q < kDcBlk * kDcBlk; q += blockDim.x) {
        const int r = q / kDcBlk, k = q % kDcBlk;
        if (k > c && k <= r && r < nb) s_D[r][k] -= s_D[r][c] * s_D[k][c];
      }
    }
    __syncthreads();
    if (s_bad) break;
    for (int q = tid; q < nb * nb; q += blockDim.x) {
      const int r = q / nb, cc = q % nb;
      if (cc <= r) LT[(int64_t)(j0 + cc) * M + j0 + r] = s_D[r][cc];
    }
    // rows below the block (at most 1023 of them): L[i][j0 + c] by
    // substitution against the block, one row per thread
    const int i = j0 + nb + tid;
    if (i < M) {
      double l[kDcBlk];
#pragma unroll
      for (int c = 0; c < kDcBlk; ++c) {
        if (c < nb) {
          double sv = A[(int64_t)i * M + j0 + c];
#pragma unroll
          for (int k = 0; k < c; ++k) sv -= l[k] * s_D[c][k];
          l[c] = sv / s_D[c][c];
          LT[(int64_t)(j0 + c) * M + i] = l[c];
          if (i - j0 - nb < panel_rows) s_panel[(i - j0 - nb) * (kDcBlk + 1) + c] = l[c];
        }
      }
    }
    __syncthreads();  // the block's columns of LT are complete
    const int base = j0 + nb;
    if (M - base <= panel_rows) {
      // trailing update from the rows' block of L held in LDS, one wave per row
      for (int i2 = base + wave; i2 < M; i2 += n_waves) {
        const double* pi = s_panel + (i2 - base) * (kDcBlk + 1);
        for (int k = base + lane; k <= i2; k += 64) {
          const double* pk = s_panel + (k - base) * (kDcBlk + 1);
          double acc = A[(int64_t)i2 * M + k];
          for (int c = 0; c < nb; ++c) acc -= pi[c] * pk[c];
          A[(int64_t)i2 * M + k] = acc;
        }
      }
      continue;
    }
    // trailing update, one wave per row i2: the row's block of L is staged in
    // the wave's slot of LDS, the 32 loads of each column k are issued at once
    double* li = s_row[wave];
    for (int i2 = j0 + nb + wave; i2 < M; i2 += n_waves) {
      if (lane < kDcBlk) li[lane] = lane < nb ? LT[(int64_t)(j0 + lane) * M + i2] : 0.0;
      __builtin_amdgcn_wave_barrier();
      for (int h = 0; h < nb; h += 16) {
        double lh[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) lh[c] = li[h + c];
        for (int k = j0 + nb + lane; k <= i2; k += 64) {
          double lk[16];
#pragma unroll
          for (int c = 0; c < 16; ++c)
            lk[c] = h + c < nb ? LT[(int64_t)(j0 + h + c) * M + k] : 0.0;
          double acc = A[(int64_t)i2 * M + k];
#pragma unroll
          for (int c = 0; c < 16; ++c) acc -= lh[c] * lk[c];
          A[(int64_t)i2 * M + k] = acc;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  if (s_bad) {
    for (int64_t q = tid; q < (int64_t)M * M; q += blockDim.x)
      LT[q] = (q / M == q % M) ? 1.0 : 0.0;
  }
  if (tid == 0) *status = s_bad;
}

// Z[:, n] = L^{-1} (X[:, n] - mean) by blocks of 32 rows: a workgroup holds
// the residuals of spw samples for every row in LDS ([M][spw]); within a block
// the scores z_k = s_k / L_kk are found one after another against the block's
// diagonal part of L (in LDS), then taken off every row below the block at
// once.  Thread t owns sample t % spw and rows (t / spw) + g * (256 / spw).
__global__ void __launch_bounds__(256) k_dc_whiten(int M, int64_t N, int spw,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ mean,
                                                   const double* __restrict__ LT,
                                                   double* __restrict__ Z) {
  extern __shared__ double s_dyn[];
  double* s_res = s_dyn;                       // [M][spw] residuals
  double* s_z = s_dyn + (size_t)M * spw;       // [kDcBlk][spw] the block's scores
  double* s_d = s_z + kDcBlk * spw;            // [kDcBlk][kDcBlk + 1] LT of the block
  double* s_slab = s_d + kDcBlk * (kDcBlk + 1);  // [kDcBlk][kDcSlab] LT below the block
  const int j = threadIdx.x % spw, g = threadIdx.x / spw, G = 256 / spw;
  const int64_t n = (int64_t)blockIdx.x * spw + j;
  const bool ok = n < N;
  for (int i = g; i < M; i += G) s_res[i * spw + j] = ok ? X[(int64_t)i * N + n] - mean[i] : 0.0;
  for (int b0 = 0; b0 < M; b0 += kDcBlk) {
    const int nb = std::min(kDcBlk, M - b0);
    __syncthreads();
    for (int q = threadIdx.x; q < kDcBlk * kDcBlk; q += 256) {
      const int k = q / kDcBlk, i = q % kDcBlk;
      s_d[k * (kDcBlk + 1) + i] =
          (k < nb && i < nb && i >= k) ? LT[(int64_t)(b0 + k) * M + b0 + i] : 0.0;
    }
    for (int k = 0; k < nb; ++k) {
      __syncthreads();
      const double zk = s_res[(b0 + k) * spw + j] / s_d[k * (kDcBlk + 1) + k];
      if (g == 0) s_z[k * spw + j] = zk;
      for (int i = k + 1 + g; i < nb; i += G)
        s_res[(b0 + i) * spw + j] -= s_d[k * (kDcBlk + 1) + i] * zk;
    }
    __syncthreads();
    // the block's scores go out here, not inside the steps above: a barrier
    // waits for the workgroup's outstanding stores
    for (int k = g; k < nb; k += G)
      if (ok) Z[(int64_t)(b0 + k) * N + n] = s_z[k * spw + j];
    // rows below the block, kDcSlab at a time: the block's columns of L for
    // those rows are staged in LDS with coalesced loads, then every thread
    // updates its rows from there
    for (int r0 = b0 + nb; r0 < M; r0 += kDcSlab) {
      const int nr = std::min(kDcSlab, M - r0);
      __syncthreads();  // the previous slab has been read
      for (int q = threadIdx.x; q < kDcBlk * kDcSlab; q += 256) {
        const int k = q / kDcSlab, i = q % kDcSlab;
        s_slab[k * kDcSlab + i] = (k < nb && i < nr) ? LT[(int64_t)(b0 + k) * M + r0 + i] : 0.0;
      }
      __syncthreads();
      for (int i = g; i < nr; i += G) {
        double acc = s_res[(r0 + i) * spw + j];
        for (int k = 0; k < nb; ++k) acc -= s_slab[k * kDcSlab + i] * s_z[k * spw + j];
        s_res[(r0 + i) * spw + j] = acc;
      }
    }
  }
}

// Total order on the bits of a double (negative values below positive ones,
// -0 taken as +0): the order of the values wherever they are comparable.
__device__ __forceinline__ uint64_t order_key(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v + 0.0);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Ranks of the entries of every row, by buckets: the finite range [lo, hi] of
// a row is cut into N equal buckets (a monotone map, so a lower bucket never
// holds a larger value), bucket offsets come from a prefix sum of the counts,
// and an entry's rank is its bucket's offset plus the entries of its own
// bucket that come before it (smaller key, or equal key and lower index).
// Expected O(N) per row for continuous values.  Non-finite values go to the
// end buckets (NaN to the first), so the ranks stay a permutation whatever
// the values are; the bucket of each entry is computed once and stored, so
// that the count, the placement and the rank see the same bucket.
__global__ void __launch_bounds__(256) k_dc_range(int64_t N, const double* __restrict__ V,
                                                  double2* __restrict__ lohi) {
  const double* v = V + (int64_t)blockIdx.x * N;
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t n = threadIdx.x; n < N; n += 256) {
    const double x = v[n];
    if (isfinite(x)) {
      lo = fmin(lo, x);
      hi = fmax(hi, x);
    }
  }
  __shared__ double s_lo[256], s_hi[256];
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
      s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lo = s_lo[0];
    hi = s_hi[0];
    const double span = hi - lo;
    // scale 0 (one bucket) if the row has no finite spread
    const double scale = (lo <= hi && span > 0.0 && span < INFINITY) ? (double)N / span : 0.0;
    lohi[blockIdx.x] = make_double2(lo <= hi ? lo : 0.0, scale);
  }
}

__global__ void __launch_bounds__(256) k_dc_zero(int64_t count, int32_t* __restrict__ a,
                                                 int32_t* __restrict__ b) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) {
    a[q] = 0;
    b[q] = 0;
  }
}

__global__ void __launch_bounds__(256) k_dc_bucket(int64_t N, const double* __restrict__ V,
                                                   const double2* __restrict__ lohi,
                                                   int32_t* __restrict__ bkt,
                                                   int32_t* __restrict__ cnt) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t row = (int64_t)blockIdx.y * N;
  const double2 ls = lohi[blockIdx.y];
  const double f = (V[row + n] - ls.x) * ls.y;
  int32_t b;
  if (!(f >= 0.0))
    b = 0;  // NaN, -inf
  else if (!(f < (double)N))
    b = (int32_t)(N - 1);  // +inf, the top of the range
  else
    b = (int32_t)f;
  bkt[row + n] = b;
  atomicAdd(&cnt[row + b], 1);
}

// Exclusive prefix sum of each row of cnt in place (one workgroup per row).
__global__ void __launch_bounds__(1024) k_dc_scan(int64_t N, int32_t* __restrict__ cnt) {
  int32_t* c = cnt + (int64_t)blockIdx.x * N;
  __shared__ int32_t s[1024];
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < N; c0 += 1024) {
    const int64_t q = c0 + threadIdx.x;
    const int32_t v = q < N ? c[q] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
      const int32_t add = (int)threadIdx.x >= w ? s[threadIdx.x - w] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (q < N) c[q] = carry + s[threadIdx.x] - v;
    carry += s[1023];
    __syncthreads();  // s is rewritten by the next chunk
  }
}

__global__ void __launch_bounds__(256) k_dc_place(int64_t N, const int32_t* __restrict__ bkt,
                                                  const int32_t* __restrict__ off,
                                                  int32_t* __restrict__ fill,
                                                  int32_t* __restrict__ perm) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t row = (int64_t)blockIdx.y * N;
  const int32_t b = bkt[row + n];
  const int32_t slot = off[row + b] + atomicAdd(&fill[row + b], 1);
  perm[row + slot] = (int32_t)n;
}

// R[i][n] = rank (if R), inv[i][rank] = n (if inv).
__global__ void __launch_bounds__(256) k_dc_rank(int64_t N, const double* __restrict__ V,
                                                 const int32_t* __restrict__ bkt,
                                                 const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ perm,
                                                 int32_t* __restrict__ R,
                                                 int32_t* __restrict__ inv) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t row = (int64_t)blockIdx.y * N;
  const int32_t b = bkt[row + n];
  const int32_t o0 = off[row + b];
  const int32_t o1 = b + 1 < N ? off[row + b + 1] : (int32_t)N;
  const uint64_t key = order_key(V[row + n]);
  int32_t r = o0;
  for (int32_t p = o0; p < o1; ++p) {
    const int32_t m = perm[row + p];
    const uint64_t km = order_key(V[row + m]);
    r += (km < key) || (km == key && m < n);
  }
  if (R) R[row + n] = r;
  if (inv) inv[row + r] = (int32_t)n;
}

// inv[i][strata[i][n]] = n for a design whose strata are known (an LHS
// design: the order of a row's values is the order of their strata).
__global__ void __launch_bounds__(256) k_dc_invert(int64_t N, const int32_t* __restrict__ strata,
                                                   int32_t* __restrict__ inv) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t row = (int64_t)blockIdx.y * N;
  inv[row + strata[row + n]] = (int32_t)n;
}

// out[i][n] = X[i][inv[i][Rz[i][n]]]: the entry whose row rank equals the
// score rank of (i, n); strata[i][n] = that rank.  After a failed
// factorisation (*status != 0) the design is copied as it is.
__global__ void __launch_bounds__(256) k_dc_apply(int64_t N, const double* __restrict__ X,
                                                  const int32_t* __restrict__ inv,
                                                  const int32_t* __restrict__ Rz,
                                                  const int32_t* __restrict__ status,
                                                  double* __restrict__ out,
                                                  int32_t* __restrict__ strata) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t row = (int64_t)blockIdx.y * N;
  const int32_t r = Rz[row + n];
  out[row + n] = *status ? X[row + n] : X[row + inv[row + r]];
  if (strata) strata[row + n] = r;
}

}  // namespace

namespace {

// Covariance launch: lower-triangle tiles times sample slices, about 1024
// workgroups in all, each slice a multiple of the LDS chunk and at least 256
// samples long.
struct CovPlan {
  unsigned n_tiles;
  int64_t per;
  int n_slices;
  CovPlan(int32_t M, int64_t N) {
    const int t1 = (M + kDcCovTile - 1) / kDcCovTile;
    n_tiles = (unsigned)(t1 * (t1 + 1) / 2);
    const int64_t want = std::max<int64_t>(1, 1024 / (int64_t)n_tiles);
    per = (N + want - 1) / want;
    per = std::max<int64_t>(256, (per + kDcChunk - 1) / kDcChunk * kDcChunk);
    n_slices = (int)((N + per - 1) / per);
  }
};

// Samples per substitution workgroup: the largest of 16, 8, 4 whose LDS
// (residuals, block scores, diagonal block, slab of L) stays within 80 KB.
size_t whiten_lds(int32_t M, int spw) {
  return ((size_t)M * spw + (size_t)kDcBlk * spw + (size_t)kDcBlk * (kDcBlk + 1) +
          (size_t)kDcBlk * kDcSlab) *
         sizeof(double);
}
int whiten_spw(int32_t M) {
  int spw = 16;
  while (spw > 4 && whiten_lds(M, spw) > 80 * 1024) spw /= 2;
  return spw;
}

struct RankBufs {
  double2* lohi;
  int32_t *bkt, *off, *fill, *perm;
};

// Ranks of the rows of V[M][N] (R and/or inv, see k_dc_rank).
void launch_rank(int32_t M, int64_t N, const double* V, const RankBufs& b, int32_t* R,
                 int32_t* inv, hipStream_t st) {
  const unsigned gs = (unsigned)((N + 255) / 256);
  const int64_t MN = (int64_t)M * N;
  hipLaunchKernelGGL(k_dc_range, dim3((unsigned)M), dim3(256), 0, st, N, V, b.lohi);
  hipLaunchKernelGGL(k_dc_zero, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, MN, b.off,
                     b.fill);
  hipLaunchKernelGGL(k_dc_bucket, dim3(gs, (unsigned)M), dim3(256), 0, st, N, V,
                     (const double2*)b.lohi, b.bkt, b.off);
  hipLaunchKernelGGL(k_dc_scan, dim3((unsigned)M), dim3(1024), 0, st, N, b.off);
  hipLaunchKernelGGL(k_dc_place, dim3(gs, (unsigned)M), dim3(256), 0, st, N,
                     (const int32_t*)b.bkt, (const int32_t*)b.off, b.fill, b.perm);
  hipLaunchKernelGGL(k_dc_rank, dim3(gs, (unsigned)M), dim3(256), 0, st, N, V,
                     (const int32_t*)b.bkt, (const int32_t*)b.off, (const int32_t*)b.perm, R, inv);
}

}  // namespace

size_t decorrelate_workspace(int32_t M, int64_t N) {
  const CovPlan cp(M, N);
  return (size_t)M * N * (sizeof(double) + 7 * sizeof(int32_t)) +
         ((size_t)cp.n_slices + 2) * M * M * sizeof(double) + 3 * (size_t)M * sizeof(double2) +
         7 * 256;
}

int decorrelate_design(Context* c, int32_t M, int64_t N, double* zeta, int32_t* strata,
                       const int32_t* lhs_strata, int32_t** status_out, hipStream_t st) {
  if (M < 1 || M > kDecorMaxM || N <= M || N > kDecorMaxN)
    return fail(FMC_EINVAL, "correlation reduction needs M <= 1024 and M < N < 2^31");
  const size_t MN = (size_t)M * N;
  const CovPlan cp(M, N);
  void *z, *rz, *inv, *bkt, *off, *fill, *perm, *part, *cv, *lt, *mean, *lohi, *sts;
  int rc;
  if ((rc = c->ensure("dc_z", MN * sizeof(double), &z))) return rc;
  if ((rc = c->ensure("dc_rz", MN * sizeof(int32_t), &rz))) return rc;
  if ((rc = c->ensure("dc_inv", MN * sizeof(int32_t), &inv))) return rc;
  if ((rc = c->ensure("dc_bkt", MN * sizeof(int32_t), &bkt))) return rc;
  if ((rc = c->ensure("dc_off", MN * sizeof(int32_t), &off))) return rc;
  if ((rc = c->ensure("dc_fill", MN * sizeof(int32_t), &fill))) return rc;
  if ((rc = c->ensure("dc_perm", MN * sizeof(int32_t), &perm))) return rc;
  if ((rc = c->ensure("dc_part", (size_t)cp.n_slices * M * M * sizeof(double), &part))) return rc;
  if ((rc = c->ensure("dc_c", (size_t)M * M * sizeof(double), &cv))) return rc;
  if ((rc = c->ensure("dc_lt", (size_t)M * M * sizeof(double), &lt))) return rc;
  if ((rc = c->ensure("dc_mean", (size_t)M * sizeof(double), &mean))) return rc;
  if ((rc = c->ensure("dc_lohi", (size_t)M * sizeof(double2), &lohi))) return rc;
  if ((rc = c->ensure("dc_status", 256, &sts))) return rc;
  double* Z = (double*)z;
  double* mu = (double*)mean;
  int32_t* status = (int32_t*)sts;
  const RankBufs rb{(double2*)lohi, (int32_t*)bkt, (int32_t*)off, (int32_t*)fill, (int32_t*)perm};
  const unsigned gs = (unsigned)((N + 255) / 256);
  const int spw = whiten_spw(M);
  hipLaunchKernelGGL(k_dc_mean, dim3((unsigned)M), dim3(256), 0, st, N, zeta, mu);
  hipLaunchKernelGGL(k_dc_cov, dim3(cp.n_tiles, (unsigned)cp.n_slices), dim3(256), 0, st, M, N,
                     cp.per, zeta, mu, (double*)part);
  hipLaunchKernelGGL(k_dc_cov_sum, dim3((unsigned)(((int64_t)M * M + 255) / 256)), dim3(256), 0, st,
                     M, N, cp.n_slices, (const double*)part, (double*)cv);
  const int panel_rows = std::min(M, kDcPanelRows);
  hipLaunchKernelGGL(k_dc_chol, dim3(1), dim3(kDcCholThreads),
                     (size_t)panel_rows * (kDcBlk + 1) * sizeof(double), st, M, panel_rows,
                     (double*)cv, (double*)lt, status);
  hipLaunchKernelGGL(k_dc_whiten, dim3((unsigned)((N + spw - 1) / spw)), dim3(256),
                     whiten_lds(M, spw), st, M, N, spw, zeta, mu, (const double*)lt, Z);
  launch_rank(M, N, Z, rb, (int32_t*)rz, nullptr, st);
  // the design's own ranks, kept only as their inverse (the entry of each
  // rank); an LHS design's strata are those ranks
  if (lhs_strata)
    hipLaunchKernelGGL(k_dc_invert, dim3(gs, (unsigned)M), dim3(256), 0, st, N, lhs_strata,
                       (int32_t*)inv);
  else
    launch_rank(M, N, zeta, rb, nullptr, (int32_t*)inv, st);
  // Z is free once its ranks are taken: it receives the rearranged design
  hipLaunchKernelGGL(k_dc_apply, dim3(gs, (unsigned)M), dim3(256), 0, st, N, zeta,
                     (const int32_t*)inv, (const int32_t*)rz, (const int32_t*)status, Z, strata);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(zeta, Z, MN * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  if (status_out) *status_out = status;
  return FMC_OK;
}

}  // namespace fmc
