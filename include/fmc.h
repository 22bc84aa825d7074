/*
 * fmc.h -- C ABI of an MI355X (gfx950) library for the fast Monte Carlo method
 * of Qiu, Lin, Chen, Liu and Song, "Fast Monte Carlo Simulation of Dynamic
 * Power Systems Under Continuous Random Disturbances" (arXiv 2007.03847).
 *
 * The method (Alg. 1 of the paper): model each continuous disturbance as an
 * Ito process (eq. 4: Ornstein-Uhlenbeck by default, or the general scalar
 * processes of fmc_process: Table I's rows and the wind model of eq. 11),
 * replace each driving Wiener increment by its Karhunen-Loeve expansion
 * truncated at order K (eqs. 6-8), draw the M = P*K standard-normal
 * coefficients by Latin hypercube sampling (Sec. IV-B), rebuild every
 * disturbance path from the ODE with random coefficients (eq. 9), simulate the
 * power system under it (eqs. 1-2, the classical swing equations on the
 * Kron-reduced network), and take the expectation and variance of the response
 * across the N samples at every output time (Alg. 1 step 4).
 *
 * Conventions shared by every entry point
 *  - Status: FMC_OK (0) or a negative FMC_E* code; the message of the last
 *    failure on the calling thread is returned by fmc_last_error() and stays
 *    valid until the next call on that thread.  No C++ exception crosses the ABI.
 *  - Ownership: the caller owns every buffer it passes.  Inputs are read only
 *    during the call (fmc_submit copies its inputs before it returns).  The
 *    library allocates device memory only inside a context, within the HBM
 *    budget given at creation; it is released by fmc_context_destroy().
 *  - Pointers: descriptor arrays (network, system, disturbance data, traj_idx)
 *    are host memory.  Bulk arrays are device memory unless a mem_kind field
 *    says otherwise.
 *  - Layouts are row-major.  The time grid is t_s = s*dt, s = 0..S with
 *    S = T/dt; stage times are t_c = c*dt/2, c = 0..2S.  The outputs of a
 *    classical system with n machines and P disturbances are V = 2n + P
 *    variables per time: delta_1..n (absolute rotor angle, rad), dw_1..n
 *    (speed deviation, pu), xi_1..P (disturbance, pu); a flux-decay system
 *    has V = 6n + P (see FMC_FD_*).
 *  - Streams: all work of a context is enqueued on the stream given at
 *    creation (or set by fmc_set_stream); calls that return results to host
 *    memory synchronise that stream.
 *  - Threading: one context per device and thread, except fmc_submit,
 *    fmc_poll, fmc_wait and fmc_cancel, which are thread-safe.
 */
#ifndef FMC_H
#define FMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMC_ABI_VERSION 4

/* Status codes. */
#define FMC_OK 0
#define FMC_EINVAL -1       /* invalid argument (see each entry point) */
#define FMC_ENOMEM -2       /* the request can never fit the context's HBM budget */
#define FMC_EBUSY -3        /* the request does not fit the budget free right now */
#define FMC_EDEVICE -4      /* a HIP runtime call failed */
#define FMC_ENONFINITE -5   /* some sample paths became non-finite; outputs written */
#define FMC_ENOTCONV -6     /* a Newton solve did not converge */
#define FMC_ECANCELLED -7   /* the ticket was cancelled */
#define FMC_EAGAIN -8       /* the ticket is still pending */
#define FMC_ETIMEDOUT -9    /* fmc_wait ran out of time */

/* Arithmetic of the path. */
#define FMC_F64 0    /* everything in FP64 */
#define FMC_F32 1    /* KLE paths and integration in FP32; statistics in FP64 */
#define FMC_BF16X3 2 /* KLE paths as BF16 hi+lo split products (3 MFMA, FP32
                        accumulate); integration FP32; statistics FP64 */

/* KLE basis (Sec. IV-A). */
#define FMC_BASIS_PAPER 0 /* eq. 7: m_1 = sqrt(1/T), m_j = sqrt(2/T) cos((j-1) pi t/T) */
#define FMC_BASIS_EIGEN 1 /* Wiener eigenfunctions: sqrt(2/T) cos((j-1/2) pi t/T) */
/* Traditional Monte Carlo (eq. 5, Euler-Maruyama increments) through the same
 * path contraction: K must equal S, and m_j is 1.5/sqrt(dt) at the midpoint
 * stage t = (j + 1/2) dt of step j and 0 at every other stage time, so the
 * coefficient zeta_{p,j} is step j's standard normal and enters the RK4 step
 * through its two midpoint stages (weight 4/6), giving the increment
 * sigma sqrt(dt) zeta_{p,j} of eq. 5 up to O(theta dt) terms of the drift.
 * It is the baseline of the paper's comparison, not a tuned path: the
 * contraction multiplies by a one-hot basis. */
#define FMC_BASIS_EM 2

/* Sampler of the KLE coefficients (Sec. IV-B). */
#define FMC_LHS 0 /* Latin hypercube: one draw per stratum, permuted per row */
#define FMC_SRS 1 /* simple random sampling (plain Monte Carlo of the coefficients) */
/* Latin hypercube followed by the correlation-reducing permutation of
 * fmc_lhs_decorrelate over all N samples: the same values in every row,
 * reassigned to samples so that the rows are close to uncorrelated (LHS
 * Step 2 of Sec. IV-B, with Cholesky-based correlation control).  Needs
 * M = n_proc*K <= 1024 and M < N < 2^31 (FMC_EINVAL otherwise); the ranks
 * are found by bucketing, O(N) expected work per row.  fmc_run only: the
 * batched and served forms reject it. */
#define FMC_LHS_DECOR 2

/* Time integrator. */
#define FMC_RK4 0  /* classical Runge-Kutta, forcing taken at the stage times */
#define FMC_TRAP 1 /* implicit trapezoidal rule, Newton-solved */

/* Generator model. */
#define FMC_CLASSICAL 0        /* constant EMF behind X'd, swing equations */
#define FMC_FLUXDECAY_IEEET1 1 /* one-axis flux decay + IEEE type-1 exciter */

/* Memory kind of output arrays. */
#define FMC_MEM_HOST 0
#define FMC_MEM_DEVICE 1

typedef struct fmc_context fmc_context;

/* Network data for the reduction of eq. 2: buses, series branches (with
 * optional total line charging b), constant-impedance load shunts g + jb (pu
 * admittance at each bus, NULL = none), and each generator's internal node
 * behind jX'd at bus gen_bus[g].  All arrays host memory. */
typedef struct fmc_network {
    int32_t n_bus, n_branch, n_gen;
    const int32_t *br_from, *br_to; /* [n_branch], bus indices 0..n_bus-1 */
    const double *br_r, *br_x;      /* [n_branch] series impedance, pu */
    const double *br_b;             /* [n_branch] or NULL */
    const double *load_g, *load_b;  /* [n_bus] or NULL */
    const int32_t *gen_bus;         /* [n_gen] */
    const double *gen_xdp;          /* [n_gen] transient reactance, pu */
} fmc_network;

/* A network event (the case study of Sec. V-B trips a generator at t = 1 s):
 * from step t/dt on, the reduced admittance is the post-event one, and
 * machine `tripped` (if >= 0) is disconnected: its internal node leaves the
 * network and its mechanical power and the disturbances injected at it are
 * removed (it keeps turning, d dw/dt = -D dw / 2H).  The post-event
 * admittance is Y_re/Y_im when given (host [n*n]; with a tripped machine, its
 * row and column must be zero, and so its entry of Yinf), else the system's
 * network reduced without the tripped machine's internal node (a network
 * system and tripped >= 0).  Yinf_re/Yinf_im: the post-event infinite-bus
 * coupling (host [n]) or NULL (unchanged).  t must be a whole number of steps
 * in (0, T).  fmc_run with the classical model only: the batched and served
 * forms and the flux-decay model reject an event. */
typedef struct fmc_event {
    double t;
    int32_t tripped;                 /* machine index, or -1 */
    const double *Y_re, *Y_im;       /* [n_gen*n_gen] or NULL */
    const double *Yinf_re, *Yinf_im; /* [n_gen] or NULL */
} fmc_event;

/* Machine data (eq. 1 instantiated as the swing equations
 *   d delta_i/dt = w_b dw_i,  2 H_i d dw_i/dt = Pm_i + sum_{p: gen[p]=i} xi_p
 *                                              - Pe_i - D_i dw_i,
 *   Pe_i = Re{ E~_i conj( sum_k Y_ik E~_k + Yinf_i V_inf ) },  E~_k = E_k e^{j delta_k},
 * w_b = 2 pi f0).  Give either (delta0, Pm = NULL): Pm is set to Pe(delta0), an
 * equilibrium by construction; or (delta0 = NULL, Pm) on an infinite-bus
 * system: delta0 solves Pe(delta0) = Pm.  Give either the reduced admittance
 * (Y_re, Y_im) or a network (net) to reduce.  All arrays host memory. */
typedef struct fmc_system {
    int32_t n_gen;
    double f0_hz;                 /* 60 if <= 0 */
    const double *H, *D, *E;      /* [n_gen] inertia (s), damping (pu), EMF (pu) */
    const double *delta0, *Pm;    /* [n_gen] or NULL, see above */
    const double *Y_re, *Y_im;    /* [n_gen*n_gen] or NULL */
    const fmc_network *net;       /* used when Y_re is NULL */
    int32_t infinite_bus;         /* nonzero: Yinf and V_inf are used */
    double V_inf;                 /* infinite-bus voltage at angle 0 */
    const double *Yinf_re, *Yinf_im; /* [n_gen] */
    int32_t model;                /* FMC_CLASSICAL or FMC_FLUXDECAY_IEEET1 */
    const double *model_params;   /* [n_gen][FMC_FD_NPARAM] for the flux-decay
                                     model, NULL for the classical model */
    const fmc_event *event;       /* a network event, or NULL */
} fmc_system;

/* One-axis (flux-decay) machine with an IEEE type-1 exciter, per machine, in
 * this order (no saturation, no regulator limits).  With E~'_k = E'q_k
 * e^{j delta_k} behind jX'd on the reduced network, I = Y E~' + Yinf V_inf,
 * Id + jIq = j I e^{-j delta}, Pe = E'q Iq, Vt = |E~' - jX'd I|:
 *   d delta/dt = w_b dw,      2H d dw/dt = Pm + xi - Pe - D dw,
 *   T'do dE'q/dt = -E'q - (Xd - X'd) Id + Efd,
 *   TE dEfd/dt = -KE Efd + VR,
 *   TF dRF/dt = -RF + (KF/TF) Efd,
 *   TA dVR/dt = -VR + KA RF - (KA KF/TF) Efd + KA (Vref - Vt).
 * E is E'q at t = 0; Efd, VR, RF and Vref are set so that t = 0 is an
 * equilibrium.  Outputs per time: delta, dw, E'q, Efd, VR, RF (n each), xi. */
#define FMC_FD_XD 0    /* synchronous reactance Xd */
#define FMC_FD_XDP 1   /* transient reactance X'd (the one behind E~') */
#define FMC_FD_TDO 2   /* open-circuit transient time constant T'do (s) */
#define FMC_FD_KA 3    /* regulator gain */
#define FMC_FD_TA 4    /* regulator time constant (s) */
#define FMC_FD_KE 5    /* exciter constant */
#define FMC_FD_TE 6    /* exciter time constant (s) */
#define FMC_FD_KF 7    /* rate-feedback gain */
#define FMC_FD_TF 8    /* rate-feedback time constant (s) */
#define FMC_FD_NPARAM 9

/* General scalar Ito disturbances (eq. 4 with state-dependent drift mu and
 * diffusion sigma; Sec. III, Table I; the wind model of eq. 11).  Table I gives,
 * per stationary density, the drift and squared diffusion of a unit-rate
 * process; the rate theta (>= 0) scales both, which keeps the named density
 * stationary:
 *   FMC_PROC_GAUSS   (a, b >= 0): mu = -theta (xi - a),        sigma^2 = 2 theta b
 *   FMC_PROC_BETA    (a, b > 0):  mu = -theta (xi - a/(a+b)),  sigma^2 = 2 theta xi (1 - xi)/(a+b)
 *   FMC_PROC_GAMMA   (a, b > 0):  mu = -theta (xi - a/b),      sigma^2 = 2 theta xi / b
 *   FMC_PROC_LAPLACE (a, b >= 0): mu = -theta (xi - a),        sigma^2 = theta (2b |xi - a| + 2b^2)
 * (b is the Gaussian row's variance and the Laplace row's scale; where
 * sigma^2 < 0, outside the support, sigma is 0), and
 *   FMC_PROC_POLY: mu = mu[0] + mu[1] xi + mu[2] xi^2,  sigma = sg[0] + sg[1] xi + sg[2] xi^2
 * (eq. 11 is of this form).  FMC_PROC_OU keeps theta[p] and sigma[p] of
 * fmc_disturbance (or its sigma_mat).  Every process enters the power balance
 * of machine gen[p] as gain (xi - ref): gain 1 and ref 0 give the OU
 * convention.  Fields a kind does not use are ignored (they must be finite). */
#define FMC_PROC_OU 0
#define FMC_PROC_GAUSS 1
#define FMC_PROC_BETA 2
#define FMC_PROC_GAMMA 3
#define FMC_PROC_LAPLACE 4
#define FMC_PROC_POLY 5
typedef struct fmc_process {
    int32_t kind;
    double a, b, theta;
    double mu[3], sg[3];
    double gain, ref;
} fmc_process;

/* Which solution of eq. 4 the paths approximate.  The KLE paths (eq. 8) are
 * smooth, so eq. 9 is an ordinary differential equation whose solutions
 * converge, as K grows, to the Stratonovich solution of eq. 4 (the
 * Wong-Zakai limit).  FMC_ITO integrates eq. 9 with the drift mu - c sigma
 * sigma', c = 1/2, whose Stratonovich solution is the Ito process of eq. 4;
 * with the one-hot basis FMC_BASIS_EM, whose RK4 step carries a noise-induced
 * drift of (3/8) sigma sigma' of its own, c = 3/8.  FMC_STRATONOVICH
 * integrates eq. 9 as written.  The two agree for additive noise (OU and the
 * Gaussian row). */
#define FMC_ITO 0
#define FMC_STRATONOVICH 1

/* The disturbances: by default Ornstein-Uhlenbeck processes (eq. 4 with
 * mu = -theta xi, constant sigma): d xi_p = -theta_p xi_p dt + sigma_p dW_p,
 * added to Pm of machine gen[p]; proc makes any of them a general process
 * (fmc_process above).  Host arrays of length n_proc. */
typedef struct fmc_disturbance {
    int32_t n_proc;
    const int32_t *gen;
    const double *theta, *sigma;
    const double *xi0; /* NULL: 0 */
    /* NULL, or host [n_proc][n_proc] diffusion matrix (correlated
     * disturbances, the matrix sigma of eq. 4 / Sec. III made square):
     * d xi_p = -theta_p xi_p dt + sum_q sigma_mat[p][q] dW_q, with sigma then
     * unused (may be NULL).  The design's rows stay the KLE coefficients of the
     * independent W_q.  fmc_run only: the batched and served forms reject it. */
    const double *sigma_mat;
    /* NULL (every process OU), or host [n_proc] process specs (fmc_process).
     * fmc_run with FMC_RK4 and the classical model only: the implicit
     * trapezoid, the flux-decay model and the batched and served forms
     * reject them, as does sigma_mat with a non-OU process. */
    const fmc_process *proc;
    int32_t calculus; /* FMC_ITO (0) or FMC_STRATONOVICH */
} fmc_disturbance;

/* Alg. 1 inputs: truncation order K, sample size N, horizon T and step dt. */
typedef struct fmc_params {
    double T, dt;            /* S = T/dt must be an integer within 1e-9 S */
    int32_t K;               /* KLE truncation order per process, >= 1 */
    int64_t N;               /* samples, >= 2 */
    uint64_t seed;           /* LHS design seed */
    int32_t basis, sampler, integrator, precision;
    int32_t ddof;            /* variance divisor N - ddof (1: unbiased) */
    int32_t variant;         /* integrator kernel variant; -1 = choose (autotuner).
                                Flux-decay systems: -1 or 0 = network product in
                                FP32; 1 (FMC_BF16X3 only) = network product as
                                BF16 hi+lo split products, faster but with larger
                                error (measured over 30 s: 1.5e-3 of the mean,
                                6e-3 of the variance, against 4e-5 and 3e-4 in
                                FP32).  Batched form: ids 14-16 and 18 (FMC_BF16X3
                                only) likewise take the classical network
                                product in BF16 split products; the tuner never
                                picks them. */
    int32_t time_chunk;      /* steps per chunk; 0 = choose */
    const double *zeta_in;   /* device [M][N] FP64 coefficients replacing the
                                sampler (M = n_proc*K), or NULL */
} fmc_params;

typedef struct fmc_report {
    double t_total_s, t_lhs_s, t_gemm_s, t_integrate_s, t_stats_s; /* HIP events */
    int64_t n_nonfinite;     /* samples whose path became non-finite */
    int64_t first_nonfinite; /* smallest such sample index, -1 if none */
    int32_t variant_id, lanes_per_traj, tile, time_chunk;
    int64_t hbm_peak_bytes;  /* device bytes held for the call */
    double queue_wait_s;     /* serving: admission delay */
    double latency_s;        /* serving: submit to completion */
} fmc_report;

/* Results.  mean/var are [(S+1)][V] FP64; traj (optional) is
 * [n_traj][S+1][V] FP64 for the samples listed in traj_idx (host); strata
 * and zeta (optional) are the [M][N] design (int32 / FP64).  mem_kind applies
 * to mean, var, traj, strata and zeta. */
typedef struct fmc_outputs {
    double *mean, *var;
    int32_t n_traj;
    const int64_t *traj_idx;
    double *traj;
    int32_t *strata;
    double *zeta;
    int32_t mem_kind;
    fmc_report *report; /* host, optional */
    /* A scalar random response function accumulated while integrating (eq. 3;
     * Sec. V-B evaluates the RMS of the system frequency deviation): rrf [N]
     * (mem_kind) receives for every sample sqrt((1/T) int_0^T u(t)^2 dt), the
     * integral by the trapezoid rule on the output grid, of u = sum_v rrf_w[v]
     * y_v(t) (rrf_w host [V]; y the outputs, absolute angles) -- what
     * fmc_rrf_rms gives for the sample's trajectory, without storing it.
     * NULL: none.  fmc_run with the classical model only. */
    double *rrf;
    const double *rrf_w;
} fmc_outputs;

typedef struct fmc_scenario {
    const fmc_system *sys;
    const fmc_disturbance *dist;
    const fmc_params *par;
} fmc_scenario;

/* ABI version of the loaded library (FMC_ABI_VERSION). */
int fmc_abi_version(void);

/* Message of the last failure on this thread ("" if none). */
const char *fmc_last_error(void);

/* Create a context on HIP device `device`.  hbm_budget bounds the device
 * memory the context may hold (0: 90% of the free memory).  stream is a
 * hipStream_t or NULL (the null stream).  FMC_EDEVICE if the device cannot be
 * used, FMC_EINVAL for a NULL out. */
int fmc_context_create(int device, size_t hbm_budget, void *stream, fmc_context **out);
int fmc_context_destroy(fmc_context *ctx);
int fmc_set_stream(fmc_context *ctx, void *stream);

/* Kron reduction of the network equations (eq. 2 eliminated for a
 * constant-impedance network), FP64 on the GPU: Y_red = Y_AA - Y_AB Y_BB^-1
 * Y_BA with the generator internal nodes kept.  Y_re/Y_im: host
 * [n_gen*n_gen].  FMC_EINVAL on bad indices, non-positive X'd or a singular
 * Y_BB. */
int fmc_kron_reduce(fmc_context *ctx, const fmc_network *net, double *Y_re, double *Y_im);

/* LHS (Sec. IV-B, Alg. 1 step 1) of M coefficients over N samples: row i
 * (i = p*K + j) is a Feistel-permuted assignment of the N equiprobable strata
 * of the standard normal CDF, one uniform draw inside each, mapped by the
 * inverse CDF.  strata (int32, may be NULL; -1 for FMC_SRS) and zeta (FP64)
 * are device [M][N].  Bit-exact with the published counter-based definitions
 * (Philox-4x64-10, AS 241). */
int fmc_lhs(fmc_context *ctx, uint64_t seed, int32_t M, int64_t N, int32_t sampler,
            int32_t *strata, double *zeta);

/* Correlation-reducing permutation of a design (Sec. IV-B, LHS Step 2: the
 * permutation of each row is free; the paper points to Cholesky-based
 * correlation control).  The M rows of zeta (device [M][N] FP64, in place)
 * are M variables observed in N samples.  Their sample covariance C (divisor
 * N - 1) is factored C = L L^T; the scores Z = L^-1 (X - mean) have identity
 * covariance; each row is rearranged so that its values take the ranks of
 * the same row of Z (equal scores: lower sample index first).  A row keeps
 * its values, so an LHS row still holds one value per stratum.  strata
 * (device [M][N] int32, may be NULL) receives each entry's rank in its row,
 * which for an LHS row is its stratum.  Workspace: about M*N*16 + M*M*8
 * bytes held by the context.  Synchronises the context's stream.
 * FMC_EINVAL: M < 1, M > 1024, N <= M, N >= 2^31, or the covariance is not
 * positive definite (a Cholesky pivot at most 1e-12 of its diagonal entry, a
 * repeated row, a non-finite value): the design is then left unchanged and
 * strata is unspecified. */
int fmc_lhs_decorrelate(fmc_context *ctx, int32_t M, int64_t N, double *zeta, int32_t *strata);

/* A scalar random response function (eq. 3) of stored trajectories: for each
 * of the n trajectories in traj (device [n][S+1][V] FP64, the layout fmc_run
 * writes for sampled trajectories, grid t_s = s dt), the RMS over the horizon
 * T = S dt of u(t) = sum_v w[v] y_v(t), sqrt((1/T) int_0^T u(t)^2 dt), the
 * integral by the trapezoid rule on the S+1 points.  With w[n_gen + i] =
 * H_i / sum H on the frequency deviations (classical layout) this is the RMS
 * of the system (centre-of-inertia) frequency deviation, the RRF of Sec. V-B.
 * w: host [V]; rrf: device [n] FP64 (traj and rrf may be NULL when n = 0).
 * Synchronises the context's stream.  FMC_EINVAL: NULL pointers, n < 0,
 * n >= 2^31, S < 1, V < 1, V > 2048, dt <= 0. */
int fmc_rrf_rms(fmc_context *ctx, const double *traj, int64_t n, int64_t S, int32_t V,
                const double *w, double dt, double *rrf);

/* fmc_rrf_rms without any allocation, for callers that cannot allocate
 * device or pinned host memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and
 * errors as fmc_rrf_rms, bit for bit, except that V is limited to 2048 by
 * the library's static per-device scratch (the device copy of w), which
 * every call on a device shares: calls that overlap on one device race.
 * w is copied from host memory on the context's stream; the call
 * synchronises that stream.  FMC_EINVAL also for V > 2048. */
int fmc_rrf_rms_noalloc(fmc_context *ctx, const double *traj, int64_t n, int64_t S, int32_t V,
                        const double *w, double dt, double *rrf);

/* KLE basis (eq. 7, or the eigen basis) on the stage grid: phi device
 * [K][2S+1] FP64. */
int fmc_basis(fmc_context *ctx, int32_t basis, int32_t K, int64_t S, double T, double *phi);

/* KLE path reconstruction (eqs. 8-9): w[c][p][n] = sum_j zeta[p*K+j][n] *
 * phi[j][c0+c] for c = 0..C-1, p = 0..P-1, n = 0..N-1, as a dense
 * contraction on the matrix cores.  zeta: device [P*K][N] FP64; phi: device
 * [K][phi_ld] FP64; w: device [C][P][N], FP64 for FMC_F64, FP32 for FMC_F32
 * and FMC_BF16X3 (BF16 hi+lo split products, FP32 accumulation). */
int fmc_kle_paths(fmc_context *ctx, int32_t precision, int32_t P, int32_t K, int64_t N,
                  int64_t C, int64_t c0, const double *zeta, const double *phi, int64_t phi_ld,
                  void *w);

/* The whole method (Alg. 1) for one scenario: LHS, basis, KLE paths,
 * integration of every sample, mean and variance at every output time.
 * FMC_EINVAL: dt <= 0, T/dt not an integer, K < 1, N < 2, theta < 0,
 * sigma < 0, H <= 0, a machine index out of range, ddof outside [0, N).
 * FMC_ENONFINITE: outputs are written, NaN propagates into the statistics,
 * the report counts the samples. */
int fmc_run(fmc_context *ctx, const fmc_system *sys, const fmc_disturbance *dist,
            const fmc_params *par, fmc_outputs *out);

/* Batched form: n scenarios of different sizes, horizons, K and N in one
 * persistent launch; outs[i] receives scenario i (same results as fmc_run of
 * scenario i alone, to the tolerance of its precision). */
int fmc_run_batch(fmc_context *ctx, int32_t n, const fmc_scenario *scen, fmc_outputs *outs);

/* Served form (continuous batching).  A server thread of the context runs
 * every admitted request together: each tick rebuilds the next time chunk of
 * KLE paths (par->time_chunk steps, 0: 200) of every active request and runs
 * all of their work items in one persistent integrator launch per size class,
 * with the trajectory state resident on the device between ticks; requests
 * submitted meanwhile join at the next tick.  A request's result depends only
 * on the request (the same alone and in any mix, bit for bit).
 *
 * fmc_submit validates the scenario (as fmc_run; precision FMC_F32 or
 * FMC_BF16X3, zeta_in NULL, outputs mean and var only: n_traj 0, strata and
 * zeta NULL), copies its inputs, and admits it if its footprint (see
 * fmc_footprint) fits the free part of the context's serving arena and one of
 * 256 slots is free: FMC_EBUSY otherwise, FMC_ENOMEM if it is larger than the
 * whole arena.  The arena is taken from the HBM budget at the first submit:
 * the environment variable FMC_SERVE_ARENA_BYTES, else half of the free budget
 * up to 32 GiB.  outs (mean, var, report) must stay valid until completion is
 * reported; the report's queue_wait_s and latency_s are measured from the
 * submit.  Returns a ticket.
 *
 * fmc_poll returns FMC_EAGAIN while the request runs, then its final status
 * once (FMC_OK, or FMC_ENONFINITE / FMC_ENOTCONV / FMC_EINVAL (singular
 * network) / FMC_ECANCELLED / FMC_EDEVICE); after that the ticket is unknown
 * (FMC_EINVAL).  fmc_wait blocks until then (timeout_s < 0: no limit;
 * FMC_ETIMEDOUT leaves the ticket pending).  fmc_cancel marks a pending
 * ticket; it leaves at the next tick boundary and reports FMC_ECANCELLED.
 * These four calls are thread-safe.  fmc_context_destroy stops the server;
 * no call on the context may be in progress then. */
int fmc_submit(fmc_context *ctx, const fmc_scenario *scen, fmc_outputs *out, uint64_t *ticket);
int fmc_poll(fmc_context *ctx, uint64_t ticket);
int fmc_wait(fmc_context *ctx, uint64_t ticket, double timeout_s);
int fmc_cancel(fmc_context *ctx, uint64_t ticket);

/* Autotuner: times every compiled integrator variant that fits the scenario
 * (machines, processes; lanes per trajectory and workgroup size differ) on a
 * short horizon (three time chunks, whole run timed) at the scenario's N and
 * precision, caches the fastest for the
 * (n, P, N bucket, precision) key in the context (used by every later call
 * with variant = -1), appends it to the JSON file named by the environment
 * variable FMC_TUNE_CACHE if set, and returns it in *variant. */
int fmc_autotune(fmc_context *ctx, const fmc_scenario *scen, int32_t *variant);

/* Device bytes a scenario needs while it runs.  FMC_F32 / FMC_BF16X3: the
 * admission footprint of the served form (staged inputs, design, basis, one
 * time chunk of paths, state, statistics rows, results); FMC_F64,
 * FMC_LHS_DECOR or a diffusion matrix: the single-run form's working set.
 * Validation as fmc_run. */
int fmc_footprint(const fmc_scenario *scen, int64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* FMC_H */
