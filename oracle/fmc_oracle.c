/*
 * fmc_oracle.c -- plain, slow, FP64 CPU oracle for the fast Monte Carlo method
 * (Karhunen-Loeve expansion + Latin hypercube sampling) of Qiu, Lin, Chen, Liu
 * and Song, "Fast Monte Carlo Simulation of Dynamic Power Systems Under
 * Continuous Random Disturbances" (arXiv 2007.03847).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the GPU path.
 *
 * Everything is FP64, scalar loops, one sample at a time (OpenMP over samples
 * only).  Each function names the passage of the paper it follows.  Where the
 * paper is silent the reading taken is stated at the function.
 *
 * Pins (checked by the CPU tests against values fixed by mathematics or a
 * library routine, never against this file):
 *   philox         -> numpy.random.Philox (Philox-4x64-10)
 *   ppnd16         -> scipy.special.ndtri
 *   lhs            -> one sample per stratum, stratum bounds, bijection
 *   lhs_decorrelate -> rows keep their values (LHS rows: one per stratum), a
 *                     hand-worked 2 x 4 case, correlations reduced to the
 *                     level of a rank-exact whitening (statistical), a single
 *                     row left unchanged, invariance under scaling a row
 *   basis          -> orthonormality, Var W_K(t) closed form, eigen-KLE (Nystrom);
 *                     EM basis: one-hot rows, the eq. 5 increment of a unit
 *                     impulse, and the OU variance of EM paths (statistical)
 *   run (OU part)  -> OU closed-form mean/variance of the truncated KLE;
 *                     correlated disturbances: superposition of single-noise
 *                     runs (exact), a diagonal matrix equals the vector sigma,
 *                     cross-covariance against the truncated-KLE closed form
 *   run (swing)    -> SMIB linearised variance (Lyapunov / Van Loan), RK4 order
 *   kron           -> SMIB reduction to E V sin(delta)/X, symmetry, full solve
 *   rrf_rms        -> constant and full-period sine signals, scaling, a common
 *                     mode removed by centre-of-inertia weights
 *   run (general   -> Table I rows: the Ito mean and second-moment equations
 *   Ito processes)    (closed for linear drift), the stationary moments of the
 *                     named densities; the Stratonovich shift of the Gamma
 *                     row's mean; the wind model (eq. 11) against a plain
 *                     Euler-Maruyama simulation of eq. 5 (statistical)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENONFINITE -5
#define ORC_ENOTCONV -6

/* ------------------------------------------------------------------------- */
/* Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): counter-based; ten rounds of a multiply-xor      */
/* S-box with a Weyl-sequence key schedule.                                  */
/* ------------------------------------------------------------------------- */
static void mul_hi_lo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t h0, l0, h1, l1;
        mul_hi_lo(M0, x0, &h0, &l0);
        mul_hi_lo(M1, x2, &h1, &l1);
        uint64_t y0 = h1 ^ x1 ^ k0;
        uint64_t y1 = l1;
        uint64_t y2 = h0 ^ x3 ^ k1;
        uint64_t y3 = l0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter tags that keep the draws of the method apart. */
#define TAG_PERM   1ULL
#define TAG_JITTER 2ULL
#define TAG_SRS    3ULL

static uint64_t draw(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, uint64_t tag)
{
    uint64_t ctr[4] = {a, b, c, tag}, key[2] = {seed, 0}, o[4];
    orc_philox4x64_10(ctr, key, o);
    return o[0];
}

/* Uniform strictly inside (0,1): top 52 bits, centred.  Every step is exact. */
double orc_u01(uint64_t x)
{
    return ((double)(x >> 12) + 0.5) * 0x1.0p-52;
}

/* ------------------------------------------------------------------------- */
/* LHS Step 2 (Sec. IV-B): a random permutation of the N strata of each row.  */
/* The paper leaves the permutation algorithm open; the reading taken is a    */
/* counter-based bijection: an 8-round balanced Feistel network on 2h bits,   */
/* h = ceil(ceil(log2 N)/2) (at least 1), restricted to [0,N) by              */
/* cycle-walking.  Round r of row i uses the key k_{i,r} = one Philox draw    */
/* keyed on (i, r); its round function is the low h bits of the splitmix64    */
/* finaliser (Steele, Lea and Flood, OOPSLA 2014) of R xor k_{i,r}.           */
/* ------------------------------------------------------------------------- */
static int feistel_half_bits(int64_t N)
{
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < N) ++b;
    int h = (b + 1) / 2;
    return h < 1 ? 1 : h;
}

static uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int64_t orc_lhs_stratum(uint64_t seed, int64_t i, int64_t N, int64_t n)
{
    const int h = feistel_half_bits(N);
    const uint64_t mask = (1ULL << h) - 1ULL;
    uint64_t key[8];
    for (int r = 0; r < 8; ++r) key[r] = draw(seed, (uint64_t)i, (uint64_t)r, 0, TAG_PERM);
    uint64_t x = (uint64_t)n;
    do {
        uint64_t L = x >> h, R = x & mask;
        for (int r = 0; r < 8; ++r) {
            uint64_t f = splitmix64_mix(R ^ key[r]) & mask;
            uint64_t newL = R;
            uint64_t newR = L ^ f;
            L = newL;
            R = newR;
        }
        x = (L << h) | R;
    } while (x >= (uint64_t)N);
    return (int64_t)x;
}

/* ------------------------------------------------------------------------- */
/* Inverse of the standard normal CDF: Wichura, Algorithm AS 241 (PPND16),    */
/* Applied Statistics 37(3), 1988.  Rational approximations in three ranges;  */
/* about 1e-16 relative accuracy.                                             */
/* ------------------------------------------------------------------------- */
static double ratio8(const double *num, const double *den, double r)
{
    double a = num[7], b = den[7];
    for (int k = 6; k >= 0; --k) {
        a = a * r + num[k];
        b = b * r + den[k];
    }
    return a / b;
}

double orc_ppnd16(double p)
{
    static const double A[8] = {
        3.3871328727963666080e0, 1.3314166789178437745e+2, 1.9715909503065514427e+3,
        1.3731693765509461125e+4, 4.5921953931549871457e+4, 6.7265770927008700853e+4,
        3.3430575583588128105e+4, 2.5090809287301226727e+3};
    static const double B[8] = {
        1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
        5.3941960214247511077e+3, 2.1213794301586595867e+4, 3.9307895800092710610e+4,
        2.8729085735721942674e+4, 5.2264952788528545610e+3};
    static const double C[8] = {
        1.42343711074968357734e0, 4.63033784615654529590e0, 5.76949722146069140550e0,
        3.64784832476320460504e0, 1.27045825245236838258e0, 2.41780725177450611770e-1,
        2.27238449892691845833e-2, 7.74545014278341407640e-4};
    static const double D[8] = {
        1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
        6.89767334985100004550e-1, 1.48103976427480074590e-1, 1.51986665636164571966e-2,
        5.47593808499534494600e-4, 1.05075007164441684324e-9};
    static const double E[8] = {
        6.65790464350110377720e0, 5.46378491116411436990e0, 1.78482653991729133580e0,
        2.96560571828504891230e-1, 2.65321895265761230930e-2, 1.24266094738807843860e-3,
        2.71155556874348757815e-5, 2.01033439929228813265e-7};
    static const double F[8] = {
        1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
        1.48753612908506148525e-2, 7.86869131145613259100e-4, 1.84631831751005468180e-5,
        1.42151175831644588870e-7, 2.04426310338993978564e-15};

    if (!(p > 0.0 && p < 1.0)) {
        if (p == 0.0) return -INFINITY;
        if (p == 1.0) return INFINITY;
        return NAN;
    }
    double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q;
        return q * ratio8(A, B, r);
    }
    double r = q < 0.0 ? p : 1.0 - p;
    r = sqrt(-log(r));
    double val;
    if (r <= 5.0) {
        val = ratio8(C, D, r - 1.6);
    } else {
        val = ratio8(E, F, r - 5.0);
    }
    return q < 0.0 ? -val : val;
}

/* ------------------------------------------------------------------------- */
/* LHS Step 1 + Step 2 (Sec. IV-B; Alg. 1 step 1).  Row i of the M x N        */
/* sampling matrix is coefficient zeta_i (i = p*K + j, the reindexing of      */
/* Sec. IV-A); column n is sample n.  The N equiprobable CDF strata are        */
/* permuted, one uniform is drawn inside the chosen stratum, and the inverse  */
/* normal CDF maps it to zeta.  With sampler = 1 (simple random sampling)     */
/* the uniform is drawn on (0,1) and strata are reported as -1.               */
/* Only the columns listed in sel (all N if sel is NULL) are produced; the    */
/* output is [M][n_sel].                                                      */
/* ------------------------------------------------------------------------- */
static double lhs_p(int64_t s, double U, int64_t N)
{
    double p = ((double)s + U) / (double)N;
    if (p >= 1.0) p = 0x1.fffffffffffffp-1; /* keep the top stratum finite */
    return p;
}

static int lhs_plain(uint64_t seed, int32_t M, int64_t N, int32_t sampler, int64_t n_sel,
                     const int64_t *sel, int32_t *strata, double *zeta)
{
    if (M < 1 || N < 1) return ORC_EINVAL;
    if (!sel) n_sel = N;
    for (int64_t c = 0; c < n_sel; ++c) {
        int64_t n = sel ? sel[c] : c;
        if (n < 0 || n >= N) return ORC_EINVAL;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_sel; ++c) {
        int64_t n = sel ? sel[c] : c;
        for (int32_t i = 0; i < M; ++i) {
            double z;
            int32_t st;
            if (sampler == 0) {
                int64_t s = orc_lhs_stratum(seed, i, N, n);
                double U = orc_u01(draw(seed, (uint64_t)i, (uint64_t)n, 0, TAG_JITTER));
                z = orc_ppnd16(lhs_p(s, U, N));
                st = (int32_t)s;
            } else {
                double U = orc_u01(draw(seed, (uint64_t)i, (uint64_t)n, 0, TAG_SRS));
                z = orc_ppnd16(U);
                st = -1;
            }
            if (strata) strata[(int64_t)i * n_sel + c] = st;
            if (zeta) zeta[(int64_t)i * n_sel + c] = z;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* LHS Step 2 with correlation reduction (Sec. IV-B).  The paper leaves the   */
/* permutation of each row open and names Cholesky-based correlation control  */
/* as one choice.  Reading taken: one pass of rank-based correlation control  */
/* with the identity as its target (Iman and Conover, 1982).  The M rows of   */
/* the design are M variables observed in N samples:                          */
/*   1. their sample covariance C (divisor N - 1) is factored C = L L^T;      */
/*   2. the scores Z = L^{-1} (X - mean) have identity sample covariance;     */
/*   3. each row of X is rearranged so that its values take the ranks of the  */
/*      same row of Z: the sample with the r-th smallest score gets the r-th  */
/*      smallest value (equal scores: the lower sample index first).          */
/* A row keeps its values (for an LHS row, one per stratum); only their        */
/* assignment to samples changes.  Needs N > M, finite values and a positive   */
/* definite C, each pivot above 1e-12 of its diagonal entry (ORC_EINVAL        */
/* otherwise).  strata (optional, [M][N]) receives the  */
/* rank of each entry in its row, which for an LHS row is its stratum.         */
/* ------------------------------------------------------------------------- */
static int dbl_cmp(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

typedef struct {
    double v;
    int64_t n;
} keyed_t;

static int keyed_cmp(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    if (x->v < y->v) return -1;
    if (x->v > y->v) return 1;
    return (x->n > y->n) - (x->n < y->n);
}

int orc_lhs_decorrelate(int32_t M, int64_t N, double *zeta, int32_t *strata)
{
    if (M < 1 || N <= M || !zeta) return ORC_EINVAL;
    for (int64_t q = 0; q < (int64_t)M * N; ++q)
        if (!isfinite(zeta[q])) return ORC_EINVAL;
    double *mean = calloc(M, sizeof(double));
    double *Cv = calloc((size_t)M * M, sizeof(double));
    double *L = calloc((size_t)M * M, sizeof(double));
    double *Z = malloc(sizeof(double) * (size_t)M * N);
    int rc = ORC_OK;
    if (!mean || !Cv || !L || !Z) { rc = ORC_ENOMEM; goto done; }
    for (int a = 0; a < M; ++a) {
        double s = 0.0;
        for (int64_t n = 0; n < N; ++n) s += zeta[(int64_t)a * N + n];
        mean[a] = s / (double)N;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < M; ++a)
        for (int b = 0; b <= a; ++b) {
            double s = 0.0;
            for (int64_t n = 0; n < N; ++n)
                s += (zeta[(int64_t)a * N + n] - mean[a]) * (zeta[(int64_t)b * N + n] - mean[b]);
            Cv[(size_t)a * M + b] = Cv[(size_t)b * M + a] = s / (double)(N - 1);
        }
    /* Cholesky-Banachiewicz, row by row */
    for (int i = 0; i < M && rc == ORC_OK; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = Cv[(size_t)i * M + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * M + k] * L[(size_t)j * M + k];
            if (i == j) {
                /* a pivot of at most 1e-12 of its diagonal entry: the row is
                   (to rounding) a combination of the rows before it */
                if (!(s > 1e-12 * Cv[(size_t)i * M + i])) { rc = ORC_EINVAL; break; }
                L[(size_t)i * M + i] = sqrt(s);
            } else {
                L[(size_t)i * M + j] = s / L[(size_t)j * M + j];
            }
        }
    if (rc != ORC_OK) goto done;
    /* forward substitution L z = x - mean, one sample at a time */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < M; ++i) {
            double s = zeta[(int64_t)i * N + n] - mean[i];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * M + k] * Z[(int64_t)k * N + n];
            Z[(int64_t)i * N + n] = s / L[(size_t)i * M + i];
        }
    /* rearrangement, row by row */
#pragma omp parallel
    {
        keyed_t *zs = malloc(sizeof(keyed_t) * N);
        double *xs = malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < M; ++i) {
            if (!zs || !xs) continue;
            for (int64_t n = 0; n < N; ++n) {
                zs[n].v = Z[(int64_t)i * N + n];
                zs[n].n = n;
                xs[n] = zeta[(int64_t)i * N + n];
            }
            qsort(zs, N, sizeof(keyed_t), keyed_cmp);
            qsort(xs, N, sizeof(double), dbl_cmp);
            for (int64_t r = 0; r < N; ++r) {
                zeta[(int64_t)i * N + zs[r].n] = xs[r];
                if (strata) strata[(int64_t)i * N + zs[r].n] = (int32_t)r;
            }
        }
        if (!zs || !xs) rc = ORC_ENOMEM;
        free(zs);
        free(xs);
    }
done:
    free(mean);
    free(Cv);
    free(L);
    free(Z);
    return rc;
}

/* The design of Alg. 1 step 1.  sampler 0: LHS; 1: simple random sampling;  */
/* 2: LHS followed by the correlation reduction above (over all N samples,    */
/* then the selected columns are returned).                                   */
int orc_lhs(uint64_t seed, int32_t M, int64_t N, int32_t sampler, int64_t n_sel,
            const int64_t *sel, int32_t *strata, double *zeta)
{
    if (sampler == 0 || sampler == 1) return lhs_plain(seed, M, N, sampler, n_sel, sel, strata, zeta);
    if (sampler != 2 || M < 1 || N < 1) return ORC_EINVAL;
    if (!sel) n_sel = N;
    for (int64_t c = 0; c < n_sel; ++c) {
        int64_t n = sel ? sel[c] : c;
        if (n < 0 || n >= N) return ORC_EINVAL;
    }
    double *Zf = malloc(sizeof(double) * (size_t)M * N);
    int32_t *Sf = malloc(sizeof(int32_t) * (size_t)M * N);
    int rc = (Zf && Sf) ? lhs_plain(seed, M, N, 0, N, NULL, NULL, Zf) : ORC_ENOMEM;
    if (rc == ORC_OK) rc = orc_lhs_decorrelate(M, N, Zf, Sf);
    if (rc == ORC_OK)
        for (int32_t i = 0; i < M; ++i)
            for (int64_t c = 0; c < n_sel; ++c) {
                int64_t n = sel ? sel[c] : c;
                if (zeta) zeta[(int64_t)i * n_sel + c] = Zf[(int64_t)i * N + n];
                if (strata) strata[(int64_t)i * n_sel + c] = Sf[(int64_t)i * N + n];
            }
    free(Zf);
    free(Sf);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* KLE basis (Sec. IV-A, eq. 7) sampled on the half-step grid t_c = c*dt/2,   */
/* c = 0..2S (the RK4 stage times; the paper does not fix a grid).            */
/* kind 0: the paper's functions m_1 = sqrt(1/T), m_j = sqrt(2/T) cos((j-1)   */
/*         pi t / T) for j >= 2.                                              */
/* kind 1: the eigenfunctions of the Wiener covariance min(s,t), whose        */
/*         derivatives are sqrt(2/T) cos((j-1/2) pi t / T).                   */
/* The cosine argument is reduced exactly in integers before the call.        */
/* kind 2: the traditional Monte Carlo of eq. 5 written as a basis: row j is  */
/*         one step's white-noise sample, 1.5 / sqrt(dt) at the midpoint     */
/*         stage c = 2j + 1 of step j (RK4 weighs the two midpoint stages    */
/*         4/6 in all, so the step's increment is sigma sqrt(dt) zeta), and  */
/*         0 at every other stage; K = S.                                    */
/* Output Phi[j][c], j = 0..K-1 (row j is the paper's m_{j+1}).               */
/* ------------------------------------------------------------------------- */
int orc_basis(int32_t kind, int32_t K, int64_t S, double T, double *Phi)
{
    if (K < 1 || S < 1 || !(T > 0.0)) return ORC_EINVAL;
    const int64_t C = 2 * S + 1;
    const double a1 = sqrt(1.0 / T), a2 = sqrt(2.0 / T);
    for (int32_t j = 0; j < K; ++j) {
        for (int64_t c = 0; c < C; ++c) {
            double v;
            if (kind == 2) {
                v = (c == 2 * (int64_t)j + 1) ? 1.5 / sqrt(T / (double)S) : 0.0;
            } else if (kind == 0) {
                if (j == 0) {
                    v = a1;
                } else {
                    int64_t q = ((int64_t)j * c) % (4 * S);
                    v = a2 * cos(M_PI * (double)q / (double)(2 * S));
                }
            } else {
                int64_t q = ((int64_t)(2 * j + 1) * c) % (8 * S);
                v = a2 * cos(M_PI * (double)q / (double)(4 * S));
            }
            Phi[(int64_t)j * C + c] = v;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Dense linear algebra: Gaussian elimination with partial pivoting.          */
/* ------------------------------------------------------------------------- */
/* Solve A X = B in place: A is n x n, B is n x m (row-major). */
static int csolve(int n, int m, double complex *A, double complex *B)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = cabs(A[(int64_t)k * n + k]);
        for (int r = k + 1; r < n; ++r) {
            double v = cabs(A[(int64_t)r * n + k]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return ORC_EINVAL;
        if (piv != k) {
            for (int c = 0; c < n; ++c) {
                double complex t = A[(int64_t)k * n + c];
                A[(int64_t)k * n + c] = A[(int64_t)piv * n + c];
                A[(int64_t)piv * n + c] = t;
            }
            for (int c = 0; c < m; ++c) {
                double complex t = B[(int64_t)k * m + c];
                B[(int64_t)k * m + c] = B[(int64_t)piv * m + c];
                B[(int64_t)piv * m + c] = t;
            }
        }
        for (int r = k + 1; r < n; ++r) {
            double complex f = A[(int64_t)r * n + k] / A[(int64_t)k * n + k];
            if (f == 0.0) continue;
            for (int c = k; c < n; ++c) A[(int64_t)r * n + c] -= f * A[(int64_t)k * n + c];
            for (int c = 0; c < m; ++c) B[(int64_t)r * m + c] -= f * B[(int64_t)k * m + c];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int c = 0; c < m; ++c) {
            double complex acc = B[(int64_t)k * m + c];
            for (int j = k + 1; j < n; ++j) acc -= A[(int64_t)k * n + j] * B[(int64_t)j * m + c];
            B[(int64_t)k * m + c] = acc / A[(int64_t)k * n + k];
        }
    }
    return ORC_OK;
}

static int rsolve(int n, double *A, double *b)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(A[k * n + k]);
        for (int r = k + 1; r < n; ++r) {
            double v = fabs(A[r * n + k]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return ORC_EINVAL;
        if (piv != k) {
            for (int c = 0; c < n; ++c) {
                double t = A[k * n + c]; A[k * n + c] = A[piv * n + c]; A[piv * n + c] = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double f = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double acc = b[k];
        for (int j = k + 1; j < n; ++j) acc -= A[k * n + j] * b[j];
        b[k] = acc / A[k * n + k];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Network reduction.  The algebraic equations (eq. 2) of a constant-         */
/* impedance network are linear in the bus voltages, so they are eliminated   */
/* exactly: nodes are the n_gen generator internal EMFs (behind jX'd) and the */
/* n_bus buses; Y_red = Y_AA - Y_AB Y_BB^{-1} Y_BA.  Branch k contributes      */
/* 1/(r+jx) in series plus jb/2 at each end; loads are shunts g + jb.         */
/* ------------------------------------------------------------------------- */
int orc_kron(int32_t n_bus, int32_t n_br, const int32_t *from, const int32_t *to,
             const double *br_r, const double *br_x, const double *br_b,
             const double *load_g, const double *load_b, int32_t n_gen,
             const int32_t *gen_bus, const double *gen_xdp, double *Y_re, double *Y_im)
{
    if (n_bus < 1 || n_gen < 1 || n_br < 0) return ORC_EINVAL;
    const int nb = n_bus, ng = n_gen;
    double complex *Ybb = calloc((size_t)nb * nb, sizeof(double complex));
    double complex *Yba = calloc((size_t)nb * ng, sizeof(double complex));
    if (!Ybb || !Yba) { free(Ybb); free(Yba); return ORC_ENOMEM; }
    for (int k = 0; k < n_br; ++k) {
        int f = from[k], t = to[k];
        if (f < 0 || f >= nb || t < 0 || t >= nb || f == t) { free(Ybb); free(Yba); return ORC_EINVAL; }
        double complex y = 1.0 / (br_r[k] + I * br_x[k]);
        double complex sh = br_b ? I * br_b[k] / 2.0 : 0.0;
        Ybb[(int64_t)f * nb + f] += y + sh;
        Ybb[(int64_t)t * nb + t] += y + sh;
        Ybb[(int64_t)f * nb + t] -= y;
        Ybb[(int64_t)t * nb + f] -= y;
    }
    for (int b = 0; b < nb; ++b)
        Ybb[(int64_t)b * nb + b] += (load_g ? load_g[b] : 0.0) + I * (load_b ? load_b[b] : 0.0);
    for (int g = 0; g < ng; ++g) {
        int b = gen_bus[g];
        if (b < 0 || b >= nb || !(gen_xdp[g] > 0.0)) { free(Ybb); free(Yba); return ORC_EINVAL; }
        double complex yg = 1.0 / (I * gen_xdp[g]);
        Ybb[(int64_t)b * nb + b] += yg;
        Yba[(int64_t)b * ng + g] -= yg; /* Y_BA[b][g] = -yg */
    }
    int rc = csolve(nb, ng, Ybb, Yba); /* Yba <- Y_BB^{-1} Y_BA */
    if (rc == ORC_OK) {
        for (int i = 0; i < ng; ++i)
            for (int k = 0; k < ng; ++k) {
                double complex v = (i == k) ? 1.0 / (I * gen_xdp[i]) : 0.0; /* Y_AA */
                /* Y_AB[i][b] = -yg_i at b = gen_bus[i] */
                double complex yg = 1.0 / (I * gen_xdp[i]);
                v -= (-yg) * Yba[(int64_t)gen_bus[i] * ng + k];
                Y_re[i * ng + k] = creal(v);
                Y_im[i * ng + k] = cimag(v);
            }
    }
    free(Ybb);
    free(Yba);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* The problem: classical multimachine model (eqs. 1-2 instantiated as the    */
/* swing equations on the Kron-reduced network) driven by Ornstein-Uhlenbeck  */
/* disturbances (eq. 4 with mu = -theta xi, constant sigma; the Gaussian row  */
/* of Table I), whose Wiener drivers are replaced by the truncated KLE        */
/* (eqs. 8-9).                                                                */
/* ------------------------------------------------------------------------- */
typedef struct orc_problem {
    int32_t n_gen;
    double f0_hz;
    const double *H, *D, *E, *delta0, *Pm; /* [n]; delta0 NULL -> solve; Pm NULL -> equilibrium */
    const double *Y_re, *Y_im;             /* [n*n] reduced admittance */
    int32_t infinite_bus;
    double V_inf;
    const double *Yinf_re, *Yinf_im; /* [n] coupling to the infinite bus */
    int32_t n_proc;
    const int32_t *dist_gen;
    const double *theta, *sigma, *xi0;
    double T, dt;
    int32_t K;
    int64_t N;
    uint64_t seed;
    int32_t basis, sampler, integrator, ddof;
    int32_t model;               /* 0 classical, 1 flux decay + IEEE type-1 exciter */
    const double *model_params;  /* [n][9] for model 1 (order of FD_* below) */
    const double *sigma_mat;     /* NULL, or [P][P]: d xi_p = -theta_p xi_p dt +      */
                                 /* sum_q sigma_mat[p][q] dW_q (sigma is then unused) */
    /* A network event at t_event (> 0, a whole number of steps; 0: none): from  */
    /* then on the reduced admittance is Yp and the infinite-bus coupling Yinfp  */
    /* (NULL: unchanged), and machine `tripped` (>= 0) is disconnected: its      */
    /* mechanical power and the disturbances injected at it are removed (the     */
    /* caller's Yp has its row and column zero).                                 */
    double t_event;
    int32_t tripped;
    const double *Yp_re, *Yp_im, *Yinfp_re, *Yinfp_im;
    /* General scalar Ito disturbances (eq. 4 with state-dependent drift and   */
    /* diffusion; the rows of Table I and the wind model of eq. 11): NULL (every */
    /* process OU as above), or one spec per process.                           */
    const struct orc_process *proc;
    int32_t calculus; /* ORC_ITO or ORC_STRATONOVICH (below) */
} orc_problem;

/* One disturbance process.  Table I lists, per stationary density, the drift
 * and the squared diffusion of a unit-rate scalar Ito process; a rate theta
 * scales both (the stationary solution of the Fokker-Planck equation, which
 * depends on 2 mu / sigma^2 only, stays the named density):
 *   Gaussian(a, b)  mu = -theta (xi - a),          sigma^2 = 2 theta b
 *   Beta(a, b)      mu = -theta (xi - a/(a+b)),    sigma^2 = 2 theta xi (1 - xi)/(a+b)
 *   Gamma(a, b)     mu = -theta (xi - a/b),        sigma^2 = 2 theta xi / b
 *   Laplace(a, b)   mu = -theta (xi - a),          sigma^2 = theta (2 b |xi - a| + 2 b^2)
 * (b is the variance of the Gaussian row and the scale of the Laplace row;
 * a negative sigma^2 -- outside the support -- is taken as 0).  The wind model
 * (eq. 11) is the polynomial kind: mu = mu0 + mu1 xi + mu2 xi^2 and sigma =
 * sg0 + sg1 xi + sg2 xi^2.  An OU spec keeps theta[p], sigma[p] (or the
 * diffusion matrix).  The process enters its machine's power balance as
 * gain (xi - ref). */
typedef struct orc_process {
    int32_t kind;
    double a, b, theta;
    double mu[3], sg[3];
    double gain, ref;
} orc_process;
enum { ORC_PROC_OU = 0, ORC_PROC_GAUSS = 1, ORC_PROC_BETA = 2, ORC_PROC_GAMMA = 3,
       ORC_PROC_LAPLACE = 4, ORC_PROC_POLY = 5 };
/* The KLE paths of eq. 8 are smooth, so eq. 9 is an ordinary differential
 * equation whose solutions converge, as K grows, to the Stratonovich solution
 * of eq. 4 with the same coefficients (the Wong-Zakai limit), not to the Ito
 * solution.  ORC_ITO (default) integrates eq. 9 with the drift mu - c sigma
 * sigma', c = 1/2, whose Stratonovich solution is the Ito process of eq. 4;
 * ORC_STRATONOVICH integrates eq. 9 as written.  The two agree for additive
 * noise (OU and the Gaussian row).  The one-hot basis of the traditional
 * Monte Carlo baseline (eq. 5's normal of step j at that step's midpoint
 * stages, weight 3/(2 sqrt(dt))) is not smooth: expanding the RK4 step, its
 * increment is sigma sqrt(dt) zeta + (3/8) sigma sigma' zeta^2 dt + O(dt^1.5)
 * beside the drift, so its own noise-induced drift is (3/8) sigma sigma' and
 * ORC_ITO takes c = 3/8 there (the increments then converge to eq. 5's Ito
 * increments as dt -> 0). */
enum { ORC_ITO = 0, ORC_STRATONOVICH = 1 };

/* Flux-decay parameters per machine, in this order. */
enum { FD_XD, FD_XDP, FD_TDO, FD_KA, FD_TA, FD_KE, FD_TE, FD_KF, FD_TF, FD_NPARAM };

typedef struct {
    int n, P, V, ny;
    double wb;
    double *H, *D, *E, *d0, *Pm;
    double complex *Y, *Yinf;
    int inf;
    double Vinf;
    const int32_t *dgen;
    const double *theta, *sigma, *xi0;
    const double *sigma_mat; /* [P][P] or NULL */
    int fd;           /* flux-decay model */
    double *fdp;      /* [n][FD_NPARAM] */
    double *Vref;     /* [n] exciter reference */
    double *y0;       /* [ny] initial state (the operating point) */
    int tripped;      /* machine disconnected (post-event model), else -1 */
    const orc_process *proc; /* [P] or NULL */
    double ito_c;     /* drift correction -ito_c sigma sigma' (0: none) */
} model_t;

/* Diffusion term of process p driven by the white noises w (eq. 4): sigma_p */
/* w_p, or with a diffusion matrix (correlated disturbances, the m x n sigma */
/* of Sec. III, square here) sum_q sigma_pq w_q.                            */
static double diffusion(const model_t *m, int p, const double *w)
{
    if (!m->sigma_mat) return m->sigma[p] * w[p];
    double s = 0.0;
    for (int q = 0; q < m->P; ++q) s += m->sigma_mat[p * m->P + q] * w[q];
    return s;
}

/* Drift mu(xi), diffusion sigma(xi) and the product sigma(xi) sigma'(xi) of
 * a non-OU process (the table in the comment of orc_process).  For the rows
 * given by sigma^2 = g(xi): sigma = sqrt(g), sigma sigma' = g'/2 (0 where
 * g <= 0; |xi - a| has derivative sign(xi - a)). */
static void proc_terms(const orc_process *q, double xi, double *mu, double *sg, double *ssp)
{
    const double th = q->theta, a = q->a, b = q->b;
    double g = 0.0, dg = 0.0;
    switch (q->kind) {
    case ORC_PROC_GAUSS:
        *mu = -th * (xi - a);
        g = 2.0 * th * b;
        dg = 0.0;
        break;
    case ORC_PROC_BETA:
        *mu = -th * (xi - a / (a + b));
        g = 2.0 * th * xi * (1.0 - xi) / (a + b);
        dg = 2.0 * th * (1.0 - 2.0 * xi) / (a + b);
        break;
    case ORC_PROC_GAMMA:
        *mu = -th * (xi - a / b);
        g = 2.0 * th * xi / b;
        dg = 2.0 * th / b;
        break;
    case ORC_PROC_LAPLACE:
        *mu = -th * (xi - a);
        g = th * (2.0 * b * fabs(xi - a) + 2.0 * b * b);
        dg = 2.0 * th * b * (xi > a ? 1.0 : (xi < a ? -1.0 : 0.0));
        break;
    default: { /* ORC_PROC_POLY */
        *mu = q->mu[0] + q->mu[1] * xi + q->mu[2] * xi * xi;
        const double s = q->sg[0] + q->sg[1] * xi + q->sg[2] * xi * xi;
        *sg = s;
        *ssp = s * (q->sg[1] + 2.0 * q->sg[2] * xi);
        return;
    }
    }
    if (g > 0.0) {
        *sg = sqrt(g);
        *ssp = 0.5 * dg;
    } else {
        *sg = 0.0;
        *ssp = 0.0;
    }
}

/* d xi_p / dt of eq. 9 for process p at state xi with white-noise surrogate
 * values w (OU: -theta xi + the diffusion term above). */
static double proc_rhs(const model_t *m, int p, double xi, const double *w)
{
    const orc_process *q = m->proc ? &m->proc[p] : NULL;
    if (!q || q->kind == ORC_PROC_OU) return -m->theta[p] * xi + diffusion(m, p, w);
    double mu, sg, ssp;
    proc_terms(q, xi, &mu, &sg, &ssp);
    return mu - m->ito_c * ssp + sg * w[p];
}

/* Power that process p injects into its machine. */
static double proc_injection(const model_t *m, int p, double xi)
{
    const orc_process *q = m->proc ? &m->proc[p] : NULL;
    return q ? q->gain * (xi - q->ref) : xi;
}

/* Electrical power of every machine: Pe_i = Re{ E~_i conj(I_i) },
 * I = Y E~ (+ Yinf V_inf), E~_k = E_k exp(j delta_k). */
static void electrical_power(const model_t *m, const double *delta, double *Pe)
{
    const int n = m->n;
    double complex Et[512];
    for (int k = 0; k < n; ++k) Et[k] = m->E[k] * cexp(I * delta[k]);
    for (int i = 0; i < n; ++i) {
        double complex cur = m->inf ? m->Yinf[i] * m->Vinf : 0.0;
        for (int k = 0; k < n; ++k) cur += m->Y[(int64_t)i * n + k] * Et[k];
        Pe[i] = creal(Et[i] * conj(cur));
    }
}

/* d Pe_i / d delta_k (dense n x n). */
static void electrical_power_jac(const model_t *m, const double *delta, double *J)
{
    const int n = m->n;
    double complex Et[512];
    for (int k = 0; k < n; ++k) Et[k] = m->E[k] * cexp(I * delta[k]);
    for (int i = 0; i < n; ++i) {
        double complex cur = m->inf ? m->Yinf[i] * m->Vinf : 0.0;
        for (int k = 0; k < n; ++k) cur += m->Y[(int64_t)i * n + k] * Et[k];
        for (int k = 0; k < n; ++k) {
            double v = creal(Et[i] * conj(m->Y[(int64_t)i * n + k] * I * Et[k]));
            if (k == i) v += creal(I * Et[i] * conj(cur));
            J[i * n + k] = v;
        }
    }
}

/* Right-hand side. State y = (delta_1..n [rad, absolute], dw_1..n [pu],
 * xi_1..P); w[p] is the KLE white-noise surrogate of eq. 8 at this time. */
static void rhs_fd(const model_t *m, const double *y, const double *w, double *dy);

static void rhs(const model_t *m, const double *y, const double *w, double *dy)
{
    if (m->fd) {
        rhs_fd(m, y, w, dy);
        return;
    }
    const int n = m->n, P = m->P;
    double Pe[512];
    electrical_power(m, y, Pe);
    for (int i = 0; i < n; ++i) {
        double pm = m->Pm[i];
        for (int p = 0; p < P; ++p)
            if (m->dgen[p] == i && i != m->tripped) pm += proc_injection(m, p, y[2 * n + p]);
        dy[i] = m->wb * y[n + i];
        dy[n + i] = (pm - Pe[i] - m->D[i] * y[n + i]) / (2.0 * m->H[i]);
    }
    for (int p = 0; p < P; ++p) dy[2 * n + p] = proc_rhs(m, p, y[2 * n + p], w);
}

static void rhs_jac(const model_t *m, const double *y, double *J)
{
    const int n = m->n, P = m->P, ny = m->ny;
    double Jp[512 * 8];
    double *JP = (n * n <= 512 * 8) ? Jp : malloc(sizeof(double) * n * n);
    memset(J, 0, sizeof(double) * ny * ny);
    electrical_power_jac(m, y, JP);
    for (int i = 0; i < n; ++i) {
        J[i * ny + n + i] = m->wb;
        for (int k = 0; k < n; ++k) J[(n + i) * ny + k] = -JP[i * n + k] / (2.0 * m->H[i]);
        J[(n + i) * ny + n + i] = -m->D[i] / (2.0 * m->H[i]);
        for (int p = 0; p < P; ++p)
            if (m->dgen[p] == i && i != m->tripped) J[(n + i) * ny + 2 * n + p] += 1.0 / (2.0 * m->H[i]);
    }
    for (int p = 0; p < P; ++p) J[(2 * n + p) * ny + 2 * n + p] = -m->theta[p];
    if (JP != Jp) free(JP);
}

/* ------------------------------------------------------------------------- */
/* One-axis (flux-decay) machine with an IEEE type-1 exciter (no saturation,  */
/* no limits).  The paper's case study names this exciter type but gives no   */
/* equations; they are written here from the standard one-axis machine model */
/* with X'q = X'd (so E'd = 0 and E~' = E'q e^{j delta} behind jX'd) and the  */
/* IEEE (1968) type-1 block diagram:                                          */
/*   VR = KA/(1 + s TA) (Vref - Vt - VF),  Efd = VR/(KE + s TE),              */
/*   VF = s KF/(1 + s TF) Efd,  with the state RF = (KF/TF)/(1 + s TF) Efd.   */
/* State y = (delta, dw, E'q, Efd, VR, RF) per machine (blocks of n), then xi. */
/* ------------------------------------------------------------------------- */

/* Network quantities at (delta, E'q): I_i = sum_k Y_ik E~'_k + Yinf_i V_inf,
 * Id + jIq = j I e^{-j delta}, Pe = Re(E~' conj I), Vt = |E~' - j X'd I|. */
static void fd_network(const model_t *m, const double *delta, const double *eq, double *Pe,
                       double *Id, double *Vt)
{
    const int n = m->n;
    double complex Et[512];
    for (int k = 0; k < n; ++k) Et[k] = eq[k] * cexp(I * delta[k]);
    for (int i = 0; i < n; ++i) {
        double complex cur = m->inf ? m->Yinf[i] * m->Vinf : 0.0;
        for (int k = 0; k < n; ++k) cur += m->Y[(int64_t)i * n + k] * Et[k];
        const double complex dq = I * cur * cexp(-I * delta[i]); /* Id + j Iq */
        Pe[i] = creal(Et[i] * conj(cur));
        Id[i] = creal(dq);
        Vt[i] = cabs(Et[i] - I * m->fdp[i * FD_NPARAM + FD_XDP] * cur);
    }
}

static void rhs_fd(const model_t *m, const double *y, const double *w, double *dy)
{
    const int n = m->n, P = m->P;
    const double *delta = y, *dw = y + n, *eq = y + 2 * n, *efd = y + 3 * n, *vr = y + 4 * n,
                 *rf = y + 5 * n, *xi = y + 6 * n;
    double Pe[512], Id[512], Vt[512];
    fd_network(m, delta, eq, Pe, Id, Vt);
    for (int i = 0; i < n; ++i) {
        const double *q = m->fdp + i * FD_NPARAM;
        double pm = m->Pm[i];
        for (int p = 0; p < P; ++p)
            if (m->dgen[p] == i) pm += proc_injection(m, p, xi[p]);
        dy[i] = m->wb * dw[i];
        dy[n + i] = (pm - Pe[i] - m->D[i] * dw[i]) / (2.0 * m->H[i]);
        dy[2 * n + i] = (-eq[i] - (q[FD_XD] - q[FD_XDP]) * Id[i] + efd[i]) / q[FD_TDO];
        dy[3 * n + i] = (-q[FD_KE] * efd[i] + vr[i]) / q[FD_TE];
        dy[5 * n + i] = (-rf[i] + q[FD_KF] / q[FD_TF] * efd[i]) / q[FD_TF];
        dy[4 * n + i] = (-vr[i] + q[FD_KA] * rf[i] - q[FD_KA] * q[FD_KF] / q[FD_TF] * efd[i] +
                         q[FD_KA] * (m->Vref[i] - Vt[i])) / q[FD_TA];
    }
    for (int p = 0; p < P; ++p) dy[6 * n + p] = proc_rhs(m, p, xi[p], w);
}

/* Exciter and field states at the operating point (delta0, E'q0 = E): every
 * derivative vanishes. */
static int fd_operating_point(model_t *m)
{
    const int n = m->n;
    double Pe[512], Id[512], Vt[512];
    for (int i = 0; i < n; ++i) {
        const double *q = m->fdp + i * FD_NPARAM;
        if (!(q[FD_XDP] > 0.0) || !(q[FD_TDO] > 0.0) || !(q[FD_TA] > 0.0) || !(q[FD_TE] > 0.0) ||
            !(q[FD_TF] > 0.0) || q[FD_KA] < 0.0)
            return ORC_EINVAL;
    }
    fd_network(m, m->d0, m->E, Pe, Id, Vt);
    for (int i = 0; i < n; ++i) {
        const double *q = m->fdp + i * FD_NPARAM;
        const double efd = m->E[i] + (q[FD_XD] - q[FD_XDP]) * Id[i];
        const double vr = q[FD_KE] * efd;
        m->y0[i] = m->d0[i];
        m->y0[n + i] = 0.0;
        m->y0[2 * n + i] = m->E[i];
        m->y0[3 * n + i] = efd;
        m->y0[4 * n + i] = vr;
        m->y0[5 * n + i] = q[FD_KF] / q[FD_TF] * efd;
        m->Vref[i] = Vt[i] + (q[FD_KA] > 0.0 ? vr / q[FD_KA] : 0.0);
    }
    return ORC_OK;
}

/* Operating point.  With delta0 given, Pm_i := Pe_i(delta0) (equilibrium by
 * construction).  Without it (infinite-bus systems), delta0 solves
 * Pe(delta) = Pm by Newton's method from delta = 0. */
static int setup_model(const orc_problem *pb, model_t *m)
{
    const int n = pb->n_gen, P = pb->n_proc;
    memset(m, 0, sizeof(*m));
    m->tripped = -1;
    if (n < 1 || n > 512 || P < 0) return ORC_EINVAL;
    m->fd = pb->model == 1;
    if (pb->model != 0 && pb->model != 1) return ORC_EINVAL;
    if (m->fd && !pb->model_params) return ORC_EINVAL;
    m->n = n; m->P = P;
    m->ny = m->V = (m->fd ? 6 * n : 2 * n) + P;
    m->y0 = calloc(m->ny, sizeof(double));
    m->Vref = calloc(n, sizeof(double));
    m->fdp = calloc((size_t)n * FD_NPARAM, sizeof(double));
    if (m->fd) memcpy(m->fdp, pb->model_params, sizeof(double) * n * FD_NPARAM);
    m->wb = 2.0 * M_PI * pb->f0_hz;
    m->H = malloc(sizeof(double) * n); m->D = malloc(sizeof(double) * n);
    m->E = malloc(sizeof(double) * n); m->d0 = malloc(sizeof(double) * n);
    m->Pm = malloc(sizeof(double) * n);
    m->Y = malloc(sizeof(double complex) * n * n);
    m->Yinf = malloc(sizeof(double complex) * n);
    for (int i = 0; i < n; ++i) {
        m->H[i] = pb->H[i]; m->D[i] = pb->D[i]; m->E[i] = pb->E[i];
        if (!(pb->H[i] > 0.0)) return ORC_EINVAL;
        m->Yinf[i] = pb->infinite_bus ? pb->Yinf_re[i] + I * pb->Yinf_im[i] : 0.0;
    }
    for (int k = 0; k < n * n; ++k) m->Y[k] = pb->Y_re[k] + I * pb->Y_im[k];
    m->inf = pb->infinite_bus;
    m->Vinf = pb->V_inf;
    m->dgen = pb->dist_gen; m->theta = pb->theta; m->sigma = pb->sigma; m->xi0 = pb->xi0;
    m->sigma_mat = pb->sigma_mat;
    m->proc = pb->proc;
    m->ito_c = pb->calculus == ORC_ITO ? (pb->basis == 2 ? 0.375 : 0.5) : 0.0;
    if (pb->calculus != ORC_ITO && pb->calculus != ORC_STRATONOVICH) return ORC_EINVAL;
    if (pb->proc)
        for (int p = 0; p < P; ++p) {
            const orc_process *q = &pb->proc[p];
            const double v[10] = {q->a, q->b, q->theta, q->mu[0], q->mu[1], q->mu[2],
                                  q->sg[0], q->sg[1], q->sg[2], q->gain + q->ref};
            for (int k = 0; k < 10; ++k)
                if (!isfinite(v[k])) return ORC_EINVAL;
            if (q->kind < ORC_PROC_OU || q->kind > ORC_PROC_POLY) return ORC_EINVAL;
            if (q->kind >= ORC_PROC_GAUSS && q->kind <= ORC_PROC_LAPLACE && !(q->theta >= 0.0))
                return ORC_EINVAL;
            if ((q->kind == ORC_PROC_BETA || q->kind == ORC_PROC_GAMMA) && !(q->a > 0.0 && q->b > 0.0))
                return ORC_EINVAL;
            if ((q->kind == ORC_PROC_GAUSS || q->kind == ORC_PROC_LAPLACE) && !(q->b >= 0.0))
                return ORC_EINVAL;
            /* state-dependent diffusion has no column in the diffusion matrix */
            if (pb->sigma_mat && q->kind != ORC_PROC_OU) return ORC_EINVAL;
        }
    if (pb->sigma_mat)
        for (int q = 0; q < P * P; ++q)
            if (!isfinite(pb->sigma_mat[q])) return ORC_EINVAL;
    for (int p = 0; p < P; ++p) {
        if (pb->dist_gen[p] < 0 || pb->dist_gen[p] >= n) return ORC_EINVAL;
        if (pb->theta[p] < 0.0 || pb->sigma[p] < 0.0) return ORC_EINVAL;
    }
    if (pb->delta0) {
        for (int i = 0; i < n; ++i) m->d0[i] = pb->delta0[i];
        if (pb->Pm) {
            for (int i = 0; i < n; ++i) m->Pm[i] = pb->Pm[i];
        } else {
            electrical_power(m, m->d0, m->Pm);
        }
    } else {
        if (!pb->Pm || !pb->infinite_bus) return ORC_EINVAL;
        for (int i = 0; i < n; ++i) { m->Pm[i] = pb->Pm[i]; m->d0[i] = 0.0; }
        double *J = malloc(sizeof(double) * n * n), *r = malloc(sizeof(double) * n);
        double Pe[512];
        int ok = 0;
        for (int it = 0; it < 100; ++it) {
            electrical_power(m, m->d0, Pe);
            electrical_power_jac(m, m->d0, J);
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) r[i] = m->Pm[i] - Pe[i];
            if (rsolve(n, J, r) != ORC_OK) break;
            for (int i = 0; i < n; ++i) { m->d0[i] += r[i]; nrm = fmax(nrm, fabs(r[i])); }
            if (nrm <= 1e-15) { ok = 1; break; }
        }
        free(J); free(r);
        if (!ok) return ORC_ENOTCONV;
    }
    if (m->fd) return fd_operating_point(m);
    for (int i = 0; i < n; ++i) m->y0[i] = m->d0[i];
    for (int p = 0; p < P; ++p) m->y0[2 * n + p] = pb->xi0 ? pb->xi0[p] : 0.0;
    return ORC_OK;
}

static void free_model(model_t *m)
{
    free(m->H); free(m->D); free(m->E); free(m->d0); free(m->Pm); free(m->Y); free(m->Yinf);
    free(m->y0); free(m->Vref); free(m->fdp);
}

/* The model after a network event: a shallow copy of m with the event's
 * reduced admittance and infinite-bus coupling, and the mechanical power of
 * a tripped machine removed (its injections are skipped by rhs).  The
 * classical model only. */
static int post_model(const orc_problem *pb, const model_t *m, model_t *mp)
{
    if (m->fd || !pb->Yp_re || !pb->Yp_im || pb->tripped < -1 || pb->tripped >= m->n)
        return ORC_EINVAL;
    *mp = *m;
    mp->Y = malloc(sizeof(double complex) * m->n * m->n);
    mp->Yinf = malloc(sizeof(double complex) * m->n);
    mp->Pm = malloc(sizeof(double) * m->n);
    for (int k = 0; k < m->n * m->n; ++k) mp->Y[k] = pb->Yp_re[k] + I * pb->Yp_im[k];
    for (int i = 0; i < m->n; ++i) {
        mp->Yinf[i] = pb->Yinfp_re ? pb->Yinfp_re[i] + I * pb->Yinfp_im[i] : m->Yinf[i];
        mp->Pm[i] = i == pb->tripped ? 0.0 : m->Pm[i];
    }
    mp->tripped = pb->tripped;
    return ORC_OK;
}

static void free_post(model_t *mp)
{
    free(mp->Y); free(mp->Yinf); free(mp->Pm);
}

/* White-noise surrogate of eq. 8 for every process at stage column c:
 * w_p(t_c) = sum_j zeta[p*K + j] * m_{j+1}(t_c). */
static void kle_forcing(const double *zcol, int64_t zstride, const double *Phi, int K,
                        int64_t C, int P, int64_t c, double *w)
{
    for (int p = 0; p < P; ++p) {
        double acc = 0.0;
        for (int j = 0; j < K; ++j)
            acc += zcol[(int64_t)(p * K + j) * zstride] * Phi[(int64_t)j * C + c];
        w[p] = acc;
    }
}

/* One sample path (Alg. 1 steps 2-3): rebuild the disturbance from zeta via
 * eq. 9 and integrate the swing equations over [0, T].  Integrator 0 is the
 * classical fourth-order Runge-Kutta method with the forcing taken at the
 * stage times; integrator 1 is the implicit trapezoidal rule solved by full
 * Newton iterations.  Writes out[(S+1)][V]: delta (absolute), dw, xi. */
static int simulate_one(const model_t *m0, const model_t *mpost, int64_t s_event,
                        const double *zcol, int64_t zstride, const double *Phi, int K, int64_t S,
                        double dt, int integrator, double *out)
{
    const model_t *m = m0;
    const int P = m->P, ny = m->ny;
    const int64_t C = 2 * S + 1;
    double *y = calloc(ny * 8 + ny * ny + 4 * P + 8, sizeof(double));
    double *k1 = y + ny, *k2 = k1 + ny, *k3 = k2 + ny, *k4 = k3 + ny, *tmp = k4 + ny;
    double *z = tmp + ny, *g = z + ny, *J = g + ny;
    double *w0 = J + ny * ny, *w1 = w0 + P, *w2 = w1 + P;
    int rc = ORC_OK;
    memcpy(y, m->y0, sizeof(double) * ny);
    for (int p = 0; p < P; ++p) y[ny - P + p] = m->xi0 ? m->xi0[p] : 0.0;
    memcpy(out, y, sizeof(double) * ny);
    for (int64_t s = 0; s < S; ++s) {
        m = (mpost && s >= s_event) ? mpost : m0; /* the network after the event */
        kle_forcing(zcol, zstride, Phi, K, C, P, 2 * s, w0);
        kle_forcing(zcol, zstride, Phi, K, C, P, 2 * s + 2, w2);
        if (integrator == 0) {
            kle_forcing(zcol, zstride, Phi, K, C, P, 2 * s + 1, w1);
            rhs(m, y, w0, k1);
            for (int q = 0; q < ny; ++q) tmp[q] = y[q] + 0.5 * dt * k1[q];
            rhs(m, tmp, w1, k2);
            for (int q = 0; q < ny; ++q) tmp[q] = y[q] + 0.5 * dt * k2[q];
            rhs(m, tmp, w1, k3);
            for (int q = 0; q < ny; ++q) tmp[q] = y[q] + dt * k3[q];
            rhs(m, tmp, w2, k4);
            for (int q = 0; q < ny; ++q)
                y[q] += dt / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        } else {
            /* z = y + dt/2 (f(y, w0) + f(z, w2)) */
            rhs(m, y, w0, k1);
            for (int q = 0; q < ny; ++q) z[q] = y[q] + dt * k1[q];
            int conv = 0;
            for (int it = 0; it < 20; ++it) {
                rhs(m, z, w2, k2);
                for (int q = 0; q < ny; ++q) g[q] = -(z[q] - y[q] - 0.5 * dt * (k1[q] + k2[q]));
                rhs_jac(m, z, J);
                for (int a = 0; a < ny * ny; ++a) J[a] = -0.5 * dt * J[a];
                for (int q = 0; q < ny; ++q) J[q * ny + q] += 1.0;
                if (rsolve(ny, J, g) != ORC_OK) break;
                double dn = 0.0, zn = 0.0;
                for (int q = 0; q < ny; ++q) {
                    z[q] += g[q];
                    dn = fmax(dn, fabs(g[q]));
                    zn = fmax(zn, fabs(z[q]));
                }
                if (dn <= 1e-13 * (1.0 + zn)) { conv = 1; break; }
            }
            if (!conv) rc = ORC_ENOTCONV;
            memcpy(y, z, sizeof(double) * ny);
        }
        memcpy(out + (s + 1) * ny, y, sizeof(double) * ny);
    }
    free(y);
    return rc;
}

/* Neumaier-compensated sum. */
typedef struct { double s, c; } ksum_t;
static void kadd(ksum_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
    a->s = t;
}

/* ------------------------------------------------------------------------- */
/* The whole method (Alg. 1): LHS set (step 1), paths by eq. 9 (step 2),      */
/* simulation (step 3), expectation and variance of the response at every     */
/* output time (step 4; two passes with compensated sums, divisor N - ddof). */
/* zeta_in (if given) replaces step 1 and is [M][n_sel] for the selected     */
/* samples.  sel lists the samples of the design to run (all N if NULL); the  */
/* statistics are over those samples.  traj (optional) is [n_sel][S+1][V].    */
/* ------------------------------------------------------------------------- */
int orc_run(const orc_problem *pb, const double *zeta_in, int64_t n_sel, const int64_t *sel,
            double *mean, double *var, double *traj, int64_t *n_nonfinite, int64_t *n_notconv,
            double *pm_out, double *delta0_out)
{
    if (!(pb->dt > 0.0) || !(pb->T > 0.0) || pb->K < 1 || pb->N < 1) return ORC_EINVAL;
    const int64_t S = (int64_t)llround(pb->T / pb->dt);
    if (S < 1 || fabs((double)S * pb->dt - pb->T) > 1e-9 * pb->T) return ORC_EINVAL;
    const int64_t C = 2 * S + 1;
    if (pb->model == 1 && pb->integrator != 0) return ORC_EINVAL; /* RK4 only */
    if (pb->proc && pb->integrator != 0) return ORC_EINVAL;       /* RK4 only */
    model_t m;
    int rc = setup_model(pb, &m);
    if (rc != ORC_OK) { free_model(&m); return rc; }
    if (pm_out) memcpy(pm_out, m.Pm, sizeof(double) * m.n);
    if (delta0_out) memcpy(delta0_out, m.d0, sizeof(double) * m.n);
    /* the post-event model (the same machines and operating point, the       */
    /* event's network, a tripped machine's mechanical power removed)          */
    model_t mp;
    int64_t s_event = 0;
    const int has_event = pb->t_event > 0.0;
    if (has_event) {
        s_event = (int64_t)llround(pb->t_event / pb->dt);
        if (s_event < 1 || s_event >= S || fabs((double)s_event * pb->dt - pb->t_event) > 1e-9 * pb->T ||
            post_model(pb, &m, &mp) != ORC_OK) {
            free_model(&m);
            return ORC_EINVAL;
        }
    }
    if (!sel) n_sel = pb->N;
    const int M = m.P * pb->K;
    const int V = m.V;
    double *Phi = malloc(sizeof(double) * pb->K * C);
    orc_basis(pb->basis, pb->K, S, pb->T, Phi);
    double *Z = NULL;
    const double *Zuse = zeta_in;
    if (!zeta_in && M > 0) {
        Z = malloc(sizeof(double) * (size_t)M * n_sel);
        rc = orc_lhs(pb->seed, M, pb->N, pb->sampler, n_sel, sel, NULL, Z);
        if (rc != ORC_OK) { free(Phi); free(Z); if (has_event) free_post(&mp); free_model(&m); return rc; }
        Zuse = Z;
    }
    double *tr = traj;
    if (!tr) tr = malloc(sizeof(double) * (size_t)n_sel * (S + 1) * V);
    if (!tr) { free(Phi); free(Z); if (has_event) free_post(&mp); free_model(&m); return ORC_ENOMEM; }
    int64_t nonfin = 0, notconv = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nonfin, notconv)
    for (int64_t c = 0; c < n_sel; ++c) {
        double *o = tr + (size_t)c * (S + 1) * V;
        int r = simulate_one(&m, has_event ? &mp : NULL, s_event, Zuse ? Zuse + c : NULL, n_sel,
                             Phi, pb->K, S, pb->dt, pb->integrator, o);
        if (r == ORC_ENOTCONV) notconv++;
        int bad = 0;
        for (int64_t q = 0; q < (S + 1) * V; ++q)
            if (!isfinite(o[q])) { bad = 1; break; }
        nonfin += bad;
    }
    if (mean || var) {
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < (S + 1) * V; ++q) {
            ksum_t a = {0.0, 0.0};
            for (int64_t c = 0; c < n_sel; ++c) kadd(&a, tr[(size_t)c * (S + 1) * V + q]);
            double mu = (a.s + a.c) / (double)n_sel;
            ksum_t b = {0.0, 0.0};
            for (int64_t c = 0; c < n_sel; ++c) {
                double d = tr[(size_t)c * (S + 1) * V + q] - mu;
                kadd(&b, d * d);
            }
            if (mean) mean[q] = mu;
            if (var) var[q] = (n_sel - pb->ddof > 0) ? (b.s + b.c) / (double)(n_sel - pb->ddof) : NAN;
        }
    }
    if (!traj) free(tr);
    free(Phi);
    free(Z);
    if (has_event) free_post(&mp);
    free_model(&m);
    if (n_nonfinite) *n_nonfinite = nonfin;
    if (n_notconv) *n_notconv = notconv;
    if (notconv) return ORC_ENOTCONV;
    return nonfin ? ORC_ENONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* A scalar RRF (eq. 3; Sec. V-B uses the RMS of the system frequency         */
/* deviation over the horizon): for each trajectory y [S+1][V] on the grid    */
/* t_s = s dt, the RMS over [0, T], T = S dt, of the linear combination       */
/* u(t) = sum_v w_v y_v(t):  sqrt( (1/T) int_0^T u(t)^2 dt ), the integral by */
/* the trapezoid rule on the stored points.  With w_v = H_i / sum H on the    */
/* frequency deviations this is the RMS of the centre-of-inertia (system)     */
/* frequency deviation.  traj [n][S+1][V], w [V], rrf [n].                    */
/* ------------------------------------------------------------------------- */
int orc_rrf_rms(const double *traj, int64_t n, int64_t S, int32_t V, const double *w, double dt,
                double *rrf)
{
    if (n < 0 || S < 1 || V < 1 || !(dt > 0.0)) return ORC_EINVAL;
    for (int64_t c = 0; c < n; ++c) {
        double acc = 0.0;
        for (int64_t s = 0; s <= S; ++s) {
            double u = 0.0;
            for (int v = 0; v < V; ++v) u += w[v] * traj[(c * (S + 1) + s) * V + v];
            const double h = (s == 0 || s == S) ? 0.5 : 1.0;
            acc += h * u * u;
        }
        rrf[c] = sqrt(acc * dt / ((double)S * dt));
    }
    return ORC_OK;
}

/* Right-hand side at one state, for tests of the model itself. */
int orc_rhs(const orc_problem *pb, const double *y, const double *w, double *dy)
{
    model_t m;
    int rc = setup_model(pb, &m);
    if (rc == ORC_OK) rhs(&m, y, w, dy);
    free_model(&m);
    return rc;
}

/* Right-hand side of the post-event model at one state. */
int orc_rhs_post(const orc_problem *pb, const double *y, const double *w, double *dy)
{
    model_t m, mp;
    int rc = setup_model(pb, &m);
    if (rc == ORC_OK && (rc = post_model(pb, &m, &mp)) == ORC_OK) {
        rhs(&mp, y, w, dy);
        free_post(&mp);
    }
    free_model(&m);
    return rc;
}

/* Jacobian d rhs / d y ([ny][ny], row = equation) of the classical model at
 * one state, for tests of the model itself (the trapezoid's Newton matrix is
 * built from it). */
int orc_rhs_jac(const orc_problem *pb, const double *y, double *J)
{
    model_t m;
    int rc = setup_model(pb, &m);
    if (rc == ORC_OK && (m.fd || m.proc)) rc = ORC_EINVAL; /* classical OU model only */
    if (rc == ORC_OK) rhs_jac(&m, y, J);
    free_model(&m);
    return rc;
}

/* The operating point (initial state, [ny]) and, for the flux-decay model,
 * the exciter references Vref [n] (may be NULL). */
int orc_initial_state(const orc_problem *pb, double *y0, double *vref)
{
    model_t m;
    int rc = setup_model(pb, &m);
    if (rc == ORC_OK) {
        memcpy(y0, m.y0, sizeof(double) * m.ny);
        if (vref) memcpy(vref, m.Vref, sizeof(double) * m.n);
    }
    free_model(&m);
    return rc;
}

/* Threads of the OpenMP loops over samples (for the single-thread baseline). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
