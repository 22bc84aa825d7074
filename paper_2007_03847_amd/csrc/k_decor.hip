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
//   k_dc_cov     lower-triangle tiles of C        16x16 tiles, samples staged in LDS
//   k_dc_chol    right-looking Cholesky           one workgroup (M <= 1024)
//   k_dc_whiten  forward substitution             residuals of 8-16 samples in LDS
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

constexpr int kDcTile = 16;    // covariance tile edge
constexpr int kDcChunk = 64;   // samples per LDS stage of the covariance

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

// C[a][b] for the tile (ta, tb), ta >= tb; both triangles are written.
__global__ void __launch_bounds__(256) k_dc_cov(int M, int64_t N, const double* __restrict__ X,
                                                const double* __restrict__ mean,
                                                double* __restrict__ Cv) {
  const int tb = blockIdx.x, ta = blockIdx.y;
  if (tb > ta) return;  // uniform over the workgroup
  const int tx = threadIdx.x % kDcTile, ty = threadIdx.x / kDcTile;
  __shared__ double sa[kDcTile][kDcChunk + 1], sb[kDcTile][kDcChunk + 1];
  double acc = 0.0;
  for (int64_t n0 = 0; n0 < N; n0 += kDcChunk) {
    for (int q = threadIdx.x; q < kDcTile * kDcChunk; q += 256) {
      const int r = q / kDcChunk, k = q % kDcChunk;
      const int64_t n = n0 + k;
      const int ra = ta * kDcTile + r, rb = tb * kDcTile + r;
      sa[r][k] = (ra < M && n < N) ? X[(int64_t)ra * N + n] - mean[ra] : 0.0;
      sb[r][k] = (rb < M && n < N) ? X[(int64_t)rb * N + n] - mean[rb] : 0.0;
    }
    __syncthreads();
#pragma unroll 16
    for (int k = 0; k < kDcChunk; ++k) acc = fma(sa[ty][k], sb[tx][k], acc);
    __syncthreads();
  }
  const int a = ta * kDcTile + ty, b = tb * kDcTile + tx;
  if (a < M && b <= a) {
    const double v = acc / (double)(N - 1);
    Cv[(int64_t)a * M + b] = v;
    Cv[(int64_t)b * M + a] = v;
  }
}

// Cholesky of the M x M matrix A (right-looking, in place on the lower
// triangle), one workgroup; the finished column j is kept in LDS for the
// trailing update, and L is also written transposed to LT (LT[k][i] = L[i][k],
// the layout the substitution reads).  A pivot of at most 1e-12 of its
// diagonal entry marks a row that is (to rounding) a combination of the rows
// before it: *status is set and LT is made the identity, so that the later
// steps leave the design as it is.
__global__ void __launch_bounds__(1024) k_dc_chol(int M, double* __restrict__ A,
                                                  double* __restrict__ LT,
                                                  int32_t* __restrict__ status) {
  __shared__ double s_d0[kDecorMaxM];
  __shared__ double s_col[kDecorMaxM];
  __shared__ int s_bad;
  for (int i = threadIdx.x; i < M; i += blockDim.x) s_d0[i] = A[(int64_t)i * M + i];
  if (threadIdx.x == 0) s_bad = 0;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, n_waves = blockDim.x / 64;
  for (int j = 0; j < M; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double d = A[(int64_t)j * M + j];
      if (!(d > 1e-12 * s_d0[j])) s_bad = 1;
      s_col[j] = s_bad ? 1.0 : sqrt(d);
    }
    __syncthreads();
    if (s_bad) break;  // uniform: shared flag read after the barrier
    const double piv = s_col[j];
    for (int i = j + threadIdx.x; i < M; i += blockDim.x) {
      const double l = i == j ? piv : A[(int64_t)i * M + j] / piv;
      if (i > j) s_col[i] = l;
      LT[(int64_t)j * M + i] = l;
    }
    __syncthreads();
    // A[i][k] -= L[i][j] L[k][j] for j < k <= i: one wave per row
    for (int i = j + 1 + wave; i < M; i += n_waves) {
      const double li = s_col[i];
      for (int k = j + 1 + lane; k <= i; k += 64) A[(int64_t)i * M + k] -= li * s_col[k];
    }
  }
  __syncthreads();
  if (s_bad) {
    for (int64_t q = threadIdx.x; q < (int64_t)M * M; q += blockDim.x)
      LT[q] = (q / M == q % M) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) *status = s_bad;
}

// Z[:, n] = L^{-1} (X[:, n] - mean) by right-looking substitution: a workgroup
// holds the residuals of spw samples for every row in LDS ([M][spw]); at
// step k the score z_k = s_k / L_kk is final and is taken off the rows below.
// Thread t owns sample t % spw and rows (t / spw) + g * (256 / spw).
__global__ void __launch_bounds__(256) k_dc_whiten(int M, int64_t N, int spw,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ mean,
                                                   const double* __restrict__ LT,
                                                   double* __restrict__ Z) {
  extern __shared__ double s_res[];  // [M][spw]
  const int j = threadIdx.x % spw, g = threadIdx.x / spw, G = 256 / spw;
  const int64_t n = (int64_t)blockIdx.x * spw + j;
  const bool ok = n < N;
  for (int i = g; i < M; i += G) s_res[i * spw + j] = ok ? X[(int64_t)i * N + n] - mean[i] : 0.0;
  for (int k = 0; k < M; ++k) {
    __syncthreads();
    const double* lt = LT + (int64_t)k * M;
    const double zk = s_res[k * spw + j] / lt[k];
    if (g == 0 && ok) Z[(int64_t)k * N + n] = zk;
    for (int i = k + 1 + g; i < M; i += G) s_res[i * spw + j] -= lt[i] * zk;
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

size_t decorrelate_workspace(int32_t M, int64_t N) {
  return (size_t)M * N * (sizeof(double) + 6 * sizeof(int32_t)) +
         2 * (size_t)M * M * sizeof(double) + 3 * (size_t)M * sizeof(double2) + 6 * 256;
}

namespace {

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

int decorrelate_design(Context* c, int32_t M, int64_t N, double* zeta, int32_t* strata,
                       int32_t** status_out, hipStream_t st) {
  if (M < 1 || M > kDecorMaxM || N <= M || N > kDecorMaxN)
    return fail(FMC_EINVAL, "correlation reduction needs M <= 1024 and M < N < 2^31");
  const size_t MN = (size_t)M * N;
  void *z, *rz, *inv, *bkt, *off, *fill, *perm, *cv, *lt, *mean, *lohi, *sts;
  int rc;
  if ((rc = c->ensure("dc_z", MN * sizeof(double), &z))) return rc;
  if ((rc = c->ensure("dc_rz", MN * sizeof(int32_t), &rz))) return rc;
  if ((rc = c->ensure("dc_inv", MN * sizeof(int32_t), &inv))) return rc;
  if ((rc = c->ensure("dc_bkt", MN * sizeof(int32_t), &bkt))) return rc;
  if ((rc = c->ensure("dc_off", MN * sizeof(int32_t), &off))) return rc;
  if ((rc = c->ensure("dc_fill", MN * sizeof(int32_t), &fill))) return rc;
  if ((rc = c->ensure("dc_perm", MN * sizeof(int32_t), &perm))) return rc;
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
  const unsigned gt = (unsigned)((M + kDcTile - 1) / kDcTile);
  // samples per substitution workgroup: the residuals [M][spw] stay within 64 KB of LDS
  const int spw = M <= 512 ? 16 : 8;
  const size_t lds = (size_t)M * spw * sizeof(double);
  hipLaunchKernelGGL(k_dc_mean, dim3((unsigned)M), dim3(256), 0, st, N, zeta, mu);
  hipLaunchKernelGGL(k_dc_cov, dim3(gt, gt), dim3(256), 0, st, M, N, zeta, mu, (double*)cv);
  hipLaunchKernelGGL(k_dc_chol, dim3(1), dim3(1024), 0, st, M, (double*)cv, (double*)lt, status);
  hipLaunchKernelGGL(k_dc_whiten, dim3((unsigned)((N + spw - 1) / spw)), dim3(256), lds, st, M, N,
                     spw, zeta, mu, (const double*)lt, Z);
  launch_rank(M, N, Z, rb, (int32_t*)rz, nullptr, st);
  // the design's own ranks, kept only as their inverse (the entry of each rank)
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
