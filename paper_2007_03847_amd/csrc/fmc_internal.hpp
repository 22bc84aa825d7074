// fmc_internal.hpp -- launch interface between the host runtime and the
// gfx950 kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmc {

// Layout of the FP64 operating-point block written by the setup kernel
// ("canonical" coefficients; n machines, P processes, unpadded):
//   [0, 2n^2)      Y_red re | im            (row-major n x n)
//   c0[n] s0[n]    E_k cos(delta0_k), E_k sin(delta0_k)
//   i0r[n] i0i[n]  I0 = Y E~0 + Yinf V_inf
//   res[n]         Pm - Pe(delta0)
//   dmp[n]         D
//   inv2h[n]       1/(2H)
//   delta0[n] pm[n]
//   theta[P] sigma[P] xi0[P]
struct CanonLayout {
  int64_t n, P;
  __host__ __device__ int64_t yre() const { return 0; }
  __host__ __device__ int64_t yim() const { return n * n; }
  __host__ __device__ int64_t c0() const { return 2 * n * n; }
  __host__ __device__ int64_t s0() const { return c0() + n; }
  __host__ __device__ int64_t i0r() const { return s0() + n; }
  __host__ __device__ int64_t i0i() const { return i0r() + n; }
  __host__ __device__ int64_t res() const { return i0i() + n; }
  __host__ __device__ int64_t dmp() const { return res() + n; }
  __host__ __device__ int64_t inv2h() const { return dmp() + n; }
  __host__ __device__ int64_t delta0() const { return inv2h() + n; }
  __host__ __device__ int64_t pm() const { return delta0() + n; }
  __host__ __device__ int64_t theta() const { return pm() + n; }
  __host__ __device__ int64_t sigma() const { return theta() + P; }
  __host__ __device__ int64_t xi0() const { return sigma() + P; }
  __host__ __device__ int64_t size() const { return xi0() + P; }
};

// Packed coefficients of one integrator variant (NG machines, PM processes,
// padded with inert entries), in the variant's arithmetic type.
struct PackLayout {
  int NG, PM;
  __host__ __device__ constexpr int yre() const { return 0; }
  __host__ __device__ constexpr int yim() const { return NG * NG; }
  __host__ __device__ constexpr int binc() const { return 2 * NG * NG; }  // [NG][PM] 0/1 injection
  __host__ __device__ constexpr int c0() const { return binc() + NG * PM; }
  __host__ __device__ constexpr int s0() const { return c0() + NG; }
  __host__ __device__ constexpr int i0r() const { return s0() + NG; }
  __host__ __device__ constexpr int i0i() const { return i0r() + NG; }
  __host__ __device__ constexpr int res() const { return i0i() + NG; }
  __host__ __device__ constexpr int dmp() const { return res() + NG; }
  __host__ __device__ constexpr int inv2h() const { return dmp() + NG; }
  __host__ __device__ constexpr int theta() const { return inv2h() + NG; }
  __host__ __device__ constexpr int sigma() const { return theta() + PM; }
  __host__ __device__ constexpr int xi0() const { return sigma() + PM; }
  __host__ __device__ constexpr int size() const { return xi0() + PM; }
};

// Arguments of one time chunk of the batched integrator.
template <typename R>
struct IntegArgs {
  const R* coef;            // PackLayout block
  const R* w;               // [cols][P][N] KLE white-noise paths of this chunk
  R* state;                 // [2*NG + PM][lanes] state between chunks
  double* partial;          // [n_groups][S+1][V] (mean, M2) pairs
  const double* delta0;     // [n] FP64 operating point (for trajectories)
  const int32_t* traj_slot; // [N] output slot of each sample or -1 (may be null)
  double* traj;             // [n_traj][S+1][V]
  unsigned long long* nonfinite;
  long long* first_bad;
  unsigned long long* notconv;  // implicit trapezoid: trajectories whose Newton solve failed
  int n, P, V;
  int64_t N, S;
  int64_t s_begin, s_end;   // steps [s_begin, s_end) of this chunk
  int64_t c_base;           // global stage column of w's first column
  int64_t lanes;            // state row stride
  R dt, wb;
  // Nonzero for systems without an infinite bus, whose electrical powers
  // depend on rotor-angle differences only: after every step (every eighth
  // step of the absolute count in the group kernel, whose lanes share the
  // sum through LDS) the mean angle deviation of the machines is moved out of
  // every machine's angle state
  // into a per-trajectory FP64 offset, so the reduced-precision state holds
  // the small angles relative to the mean rather than the common angle (a
  // neutral mode that drifts by radians over long horizons, whose rounding
  // would otherwise land on the relative angles that drive the powers).  The
  // offset is kept in two state rows after the variant's own rows (the bits
  // of the double).
  int recenter;
  int n_ref;  // machines in service (their mean angle is the reference; a
              // tripped machine, whose EMF the post-event coefficients zero, is not)
  // A scalar RRF accumulated in the epilogue (eq. 3; Sec. V-B's RMS of the
  // system frequency deviation): with rrf_w set, each trajectory sums
  // h_s u(t_s)^2 over its output steps in step order, u = sum_v rrf_w[v] y_v
  // with y the outputs (absolute angles), h_s = 1/2 at s = 0 and s = S and 1
  // otherwise; rrf_acc keeps the sums between chunks and the last chunk writes
  // rrf[n] = sqrt(sum / S), the RMS over the horizon by the trapezoid rule.
  const double* rrf_w;  // [V] or null
  double* rrf_acc;      // [N]
  double* rrf;          // [N]
  // General Ito disturbances (eq. 4 with state-dependent drift and diffusion):
  // null (every process OU, from the packed theta and sigma), or [P][kSdeCols]
  // rows of the normalised form below, one per process.
  const R* sde;
};
// A process row: form (1: sigma = c0 + c1 xi + c2 xi^2; 2: sigma = sqrt(g),
// g = c0 + c1 xi + c2 xi^2 + c3 |xi - r|, sigma = 0 where g <= 0), drift
// m0 + m1 xi + m2 xi^2, the drift correction -k sigma sigma' (k = 1/2, 3/8
// or 0 by calculus and basis), and the injection gain (xi - ref).
constexpr int kSdeCols = 12;
enum SdeCol { SDE_FORM, SDE_M0, SDE_M1, SDE_M2, SDE_C0, SDE_C1, SDE_C2, SDE_C3, SDE_R, SDE_K,
              SDE_GAIN, SDE_REF };
// State rows of the per-trajectory common-angle offset: the two 32-bit
// halves of the FP64 offset and, in the flux-decay state, the mean angle
// left by the last step (taken out at the next step).
constexpr int kOffsetRows = 2;
constexpr int kFdOffsetRows = 3;

// ---- launchers (each returns hipError_t of the launch) ----
// Static scratch of fmc_rrf_rms_noalloc (weights, doubles) and its per-device
// address (rrf_scratch_init once per device with the device current).
constexpr int kRrfStaticMaxV = 2048;
constexpr int kMaxDevices = 64;
hipError_t rrf_scratch_init(int device);
double* rrf_scratch(int device);
hipError_t launch_rrf_rms(const double* traj, int64_t n, int64_t S, int32_t V, const double* w,
                          double dt, double* rrf, hipStream_t st);
hipError_t launch_mix_design(const double* S, int32_t P, int32_t K, int64_t N, const double* in,
                             double* out, hipStream_t st);
hipError_t launch_lhs(uint64_t seed, int32_t M, int64_t N, int32_t sampler, int32_t* strata,
                      double* zeta, hipStream_t st);
hipError_t launch_basis(int32_t kind, int32_t K, int64_t S, double T, double* phi, hipStream_t st);
// max_blocks > 0 caps the workgroups (they then stride over the tiles).
hipError_t launch_kle_f64(const double* zeta, const double* phi, int64_t phi_ld, int P, int K,
                          int64_t N, int64_t C, int64_t c0, double* w, hipStream_t st,
                          int max_blocks = 0);
hipError_t launch_kle_f64_to_f32(const double* zeta, const double* phi, int64_t phi_ld, int P,
                                 int K, int64_t N, int64_t C, int64_t c0, float* w,
                                 hipStream_t st, int max_blocks = 0);
hipError_t launch_kle_bf16x3(const double* zeta, const double* phi, int64_t phi_ld, int P, int K,
                             int64_t N, int64_t C, int64_t c0, float* w, hipStream_t st,
                             int max_blocks = 0);
// The BF16 x3 contraction on operands split once (hi and lo BF16 planes,
// k-fastest, Kp = K rounded up to 32): launch_split_bf16 writes them from
// FP64 rows X[k][ld] (P blocks of stride xs into blocks of stride ys).
inline int kle_kp(int K) { return 32 * ((K + 31) / 32); }
hipError_t launch_split_bf16(const double* X, int64_t ld, int K, int64_t items, int Kp, int P,
                             int64_t xs, int64_t ys, void* yh, void* yl, hipStream_t st);
hipError_t launch_kle_bf16x3_split(const void* ph, const void* pl, int Kp, const void* zh,
                                   const void* zl, int P, int64_t N, int64_t C, int64_t c0,
                                   float* w, hipStream_t st);

// Network reduction: device network arrays -> Y_red as (re, im) pairs [n_gen^2].
struct NetDev {
  int32_t n_bus, n_branch, n_gen;
  const int32_t *from, *to, *gen_bus;
  const double *r, *x, *b, *lg, *lb, *xdp;  // b, lg, lb may be null
};
hipError_t launch_kron(const NetDev& net, double2* work, double2* Yred, int* status,
                       hipStream_t st);
size_t kron_work_bytes(int n_bus, int n_gen);  // device work buffer of launch_kron

// Operating point and canonical coefficients.
struct SetupDev {
  int32_t n, P;
  const double2* Y;           // [n*n]
  const double *H, *D, *E;    // [n]
  const double *delta0, *Pm;  // [n] or null
  int32_t inf_bus;
  double V_inf;
  const double2* Yinf;        // [n] or null
  const double *theta, *sigma, *xi0;  // [P], xi0 may be null
  double* work;               // >= 3 n^2 + 8 n doubles
  double* canon;              // CanonLayout
  int* status;                // 0 ok, -6 Newton failure
};
hipError_t launch_setup(const SetupDev& s, hipStream_t st);
// Coefficients after a network event (CanonLayout): the operating point of
// `pre` with the post-event admittance Yp ([n*n]) and infinite-bus coupling
// Yinf ([n] or null) at V_inf; a tripped machine (>= 0) gets no EMF, current,
// mechanical power or residual.
hipError_t launch_setup_post(const double* pre, int n, int P, const double2* Yp,
                             const double2* Yinf, double V_inf, int tripped, double* post,
                             hipStream_t st);

template <typename R>
hipError_t launch_pack(const double* canon, int n, int P, const int32_t* gen, int NG, int PM,
                       R* coef, hipStream_t st);

hipError_t launch_stats_merge(const double2* partial, int64_t n_groups, int group_size,
                              int64_t N, int64_t S, int V, int n, int ddof,
                              const double* delta0, double* mean, double* var, hipStream_t st);
// The same over `rows` consecutive rows: partial points at the first row of
// group 0, groups are gstride elements apart; mean/var point at the first row.
hipError_t launch_stats_merge_rows(const double2* partial, int64_t gstride, int64_t n_groups,
                                   int group_size, int64_t N, int64_t rows, int V, int n,
                                   int ddof, const double* delta0, double* mean, double* var,
                                   hipStream_t st);

// Integrator variants: NG machines, PM processes, L lanes per trajectory,
// WPB waves per workgroup; a workgroup integrates group_size() trajectories.
struct VariantInfo {
  int id, NG, PM, L, WPB;
  int group_size() const { return (64 / L) * WPB; }
  int G() const { return (NG + L - 1) / L; }
};
int n_variants();
const VariantInfo& variant(int i);
hipError_t launch_integrate_f64(int variant_id, const IntegArgs<double>& a, int64_t n_groups,
                                hipStream_t st);
// General Ito processes (IntegArgs::sde set): every variant, compiled
// separately.
hipError_t launch_integrate_gen_f64(int variant_id, const IntegArgs<double>& a, int64_t n_groups,
                                    hipStream_t st);
hipError_t launch_integrate_gen_f32(int variant_id, const IntegArgs<float>& a, int64_t n_groups,
                                    hipStream_t st);
hipError_t launch_integrate_f32(int variant_id, const IntegArgs<float>& a, int64_t n_groups,
                                hipStream_t st);
// Implicit trapezoid (FP64, classical machines) on the shape of a
// one-trajectory-per-lane variant with at most kTrapMaxGen machines.
constexpr int kTrapMaxGen = 16;
hipError_t launch_trap_f64(int variant_id, const IntegArgs<double>& a, int64_t n_groups,
                           hipStream_t st);

// Persistent batched integrator (FP32).
struct BatchItem {
  double2* rows;        // statistics rows of this item: [S+1][V], or [chunk+1][V]
                        // (steps s_begin..s_end) when the scenario has a state buffer
  int64_t tile0, tile1; // trajectory tiles [tile0, tile1) of the scenario
  int32_t scen, variant;
};
struct BatchArgs {
  const IntegArgs<float>* scen;  // one per scenario (this launch's steps)
  const BatchItem* items;
  const int32_t* order;          // queue position -> item
  int32_t n_items;
  int32_t* head;                 // queue counter, zero before the launch
};
// prod: how a variant forms the network current: 0 lanes and FMAs (classes
// 0-2), 1 FP32 matrix cores, 2 BF16 x3 matrix cores (classes 3-6, one per
// count of 16-machine blocks: 1, 2, 3, 4).
struct BatchVariantInfo {
  int id, NG, PM, L, TB, cls, prod;
};
constexpr int kBatchClasses = 7;
// Correlation reduction of the design (FMC_LHS_DECOR): the Cholesky factor is
// computed by one workgroup with the diagonal in LDS, and ranks are int32.
constexpr int kDecorMaxM = 1024;
constexpr int64_t kDecorMaxN = 2147483647;
int n_batch_variants();
BatchVariantInfo batch_variant(int i);
int persistent_blocks_per_cu(int cls);
hipError_t launch_persistent(int cls, const BatchArgs& b, int grid, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t st);

// Matrix-core classical variants (classes 3-6): up to kMcMaxGen machines and
// kMcMaxProc processes, 64 trajectories per workgroup tile.
constexpr int kMcMaxGen = 64;
constexpr int kMcMaxProc = 8;
// Coefficient block of a matrix-core variant (n_pad machines): machine-major
// constants [n_pad][8] = C0 S0 I0R I0I | RES DMP INV2H 0 (two 16-byte groups),
// the process block theta, sigma, xi0, machine index [4][kMcMaxProc], then Y
// in the A-operand order of the variant's product (the FP32 pairs of
// k_pack_fd_y or the BF16 hi/lo vectors of k_pack_fd_y16).
struct McPack {
  int n_pad;
  static constexpr int kStride = 8;
  static constexpr int kMaxConsts = kMcMaxGen * kStride + 4 * kMcMaxProc;
  __host__ __device__ constexpr int n_padk() const { return 32 * ((n_pad + 31) / 32); }
  __host__ __device__ constexpr int at(int m, int f) const { return m * kStride + f; }
  __host__ __device__ constexpr int proc() const { return n_pad * kStride; }
  __host__ __device__ constexpr int consts() const { return n_pad * kStride + 4 * kMcMaxProc; }
  __host__ __device__ constexpr int frag() const { return consts(); }  // 16-byte aligned
  __host__ __device__ constexpr int size(bool bf) const {
    return frag() + (bf ? (n_pad / 16) * (n_padk() / 32) * 64 * 16 : (n_pad / 16) * (n_pad / 4) * 64 * 2);
  }
};
hipError_t launch_pack_mc(const double* canon, int n, int P, const int32_t* gen, int n_pad, bool bf,
                          float* coef, hipStream_t st);
// nb: 16-machine blocks of the class (1 to 4)
int persistent_mc_blocks_per_cu(int nb);
hipError_t launch_persistent_mc(int nb, const BatchArgs& b, int grid, hipStream_t st);
// State buffer of a batched variant (floats) for `tiles` trajectory tiles:
// 2 G + PQ rows (G = ceil(NG / L), PQ = ceil(PM / L)) of 256 lanes per tile;
// the lane classes address it [row][lanes], classes 3-6 [tile][wave][row][64].
inline size_t batch_state_floats(const BatchVariantInfo& b, int64_t tiles) {
  const int G = (b.NG + b.L - 1) / b.L, PQ = (b.PM + b.L - 1) / b.L;
  return (size_t)(2 * G + PQ + kOffsetRows) * (size_t)tiles * 64 * 4;
}
// Coefficient block size (floats) and packing of a batched variant.
inline size_t batch_coef_floats(const BatchVariantInfo& b) {
  return b.prod != 0 ? (size_t)McPack{b.NG}.size(b.prod == 2) : (size_t)PackLayout{b.NG, b.PM}.size();
}
hipError_t launch_pack_batch(const BatchVariantInfo& b, const double* canon, int n, int P,
                             const int32_t* gen, float* coef, hipStream_t st);

// ---- flux-decay machines with IEEE type-1 exciters ----
// Parameter order per machine (as in the C ABI).
constexpr int kFdXd = 0, kFdXdp = 1, kFdTdo = 2, kFdKa = 3, kFdTa = 4, kFdKe = 5, kFdTe = 6,
              kFdKf = 7, kFdTf = 8, kFdParams = 9;
constexpr int kFdMaxProc = 32;  // processes per flux-decay system
constexpr int kFdMaxGen = 256;  // machines (16 per wave, 16 waves per workgroup)

// FP64 operating point block of the flux-decay model (n machines):
// e^{j delta0}, J0 = I0 e^{-j delta0}, Vt0 = E~0 - jX'd I0 and |Vt0|, then the
// output offsets [6n] (delta0, 0, E, Efd0, VR0, RF0 per block of n).
struct FdLayout {
  int64_t n;
  __host__ __device__ int64_t u0r() const { return 0; }
  __host__ __device__ int64_t u0i() const { return n; }
  __host__ __device__ int64_t j0r() const { return 2 * n; }
  __host__ __device__ int64_t j0i() const { return 3 * n; }
  __host__ __device__ int64_t vt0r() const { return 4 * n; }
  __host__ __device__ int64_t vt0i() const { return 5 * n; }
  __host__ __device__ int64_t vt0a() const { return 6 * n; }
  __host__ __device__ int64_t off() const { return 7 * n; }
  __host__ __device__ int64_t size() const { return 13 * n; }
};

// FP32 constants of the flux-decay integrator, machine-major [n_pad][kStride]
// in six groups of four fields read together (one 16-byte LDS read each); the
// stride of 28 floats keeps rows 16-byte aligned and puts the four machines a
// wave reads at once on distinct LDS banks.  Then the process block theta,
// sigma, xi0, machine index [4][kFdMaxProc].
struct FdPack {
  enum Field {
    C0, S0, U0R, U0I,        // E~0 and e^{j delta0}
    I0R, I0I, J0R, J0I,      // I0 and I0 e^{-j delta0}
    XDP, VT0R, VT0I, VT0A,   // X'd, Vt0 and |Vt0|
    RES, DMP, INV2H, ITDO,   // Pm - Pe0, D, 1/(2H), 1/T'do
    XDD_T, KE_TE, ITE, ITF,  // (Xd - X'd)/T'do, KE/TE, 1/TE, 1/TF
    KF_TF2, KA_TA, ITA, KAKF,  // KF/TF^2, KA/TA, 1/TA, KA KF/(TF TA)
    NFIELD
  };
  static constexpr int kStride = 28;
  int n_pad;
  __host__ __device__ int at(int m, int f) const { return m * kStride + f; }
  __host__ __device__ int proc() const { return n_pad * kStride; }
  __host__ __device__ int size() const { return n_pad * kStride + 4 * kFdMaxProc; }
};

struct FdArgs {
  const float* coef;          // FdPack block
  const float2* ap;           // (Yr, Yi) in A-operand order [n_pad/16][n_pad/4][64]
  const void* ap16;           // BF16 x3 product: Y hi/lo [n_pad/16][n_padk/32][64][4] x 16 B,
                              // or null for the FP32 product
  int n_padk;                 // n rounded up to 32 (K dimension of the BF16 product)
  const float* w;             // [cols][P][N] KLE paths of this chunk
  float* state;               // [tiles][ceil(NB/2)][48][64] deviations between chunks
  float* xstate;              // [tiles][kFdMaxProc + kFdOffsetRows][16]: processes, then the
                              // common-angle offset (two 32-bit halves) and the pending
                              // mean angle of each trajectory
  const double* off;          // [6n] FP64 output offsets
  const int32_t* traj_slot;   // [N] or null
  double* traj;               // [n_traj][S+1][V]
  unsigned long long* nonfinite;
  long long* first_bad;
  double2* rows;              // statistics rows [tiles][row_stride] (mean, M2 per tile)
  int64_t row_stride;         // elements between tiles' rows ((chunk + 1) * V)
  int64_t row_base;           // step held by the first row
  int n, P, V, n_pad;
  int64_t N, S, s_begin, s_end, c_base;
  int64_t tiles, tiles_per_item;
  float dt, wb;
  int recenter;               // as IntegArgs::recenter
};
hipError_t launch_setup_fd(const double* canon, int n, int P, const double* E, const double* prm,
                           double* fd, hipStream_t st);
hipError_t launch_pack_fd(const double* canon, int n, int P, const double* prm, const double* fd,
                          const int32_t* gen, int n_pad, float* coef, float2* ap, hipStream_t st);
size_t fd_lds_bytes(int n_pad, int n_padk, bool bf16, int P);
constexpr size_t kFdMaxLds = 160 * 1024;  // LDS of a gfx950 CU
hipError_t launch_rk4_fd(const FdArgs& a, int64_t n_items, hipStream_t st);
hipError_t launch_pack_fd_y16(const double* canon, int n, int n_pad, int n_padk, void* ap16,
                              hipStream_t st);
hipError_t launch_pack_fd_y(const double* canon, int n, int n_pad, float2* ap, hipStream_t st);
inline size_t fd_ap16_bytes(int n_pad, int n_padk) {
  return (size_t)(n_pad / 16) * (n_padk / 32) * 64 * 64;
}

}  // namespace fmc
