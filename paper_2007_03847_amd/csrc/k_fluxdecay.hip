// k_fluxdecay.hip -- one-axis (flux-decay) machines with IEEE type-1 exciters
// (FP32 integration, FP64 setup and statistics).
//
// Model (per machine, X'q = X'd so the machine is E~' = E'q e^{j delta}
// behind jX'd on the reduced network; IEEE type-1 exciter without saturation
// or limits):
//   d delta/dt = w_b dw,  2H d dw/dt = Pm + xi - Pe - D dw,
//   T'do dE'q/dt = -E'q - (Xd - X'd) Id + Efd,   TE dEfd/dt = -KE Efd + VR,
//   TF dRF/dt = -RF + (KF/TF) Efd,
//   TA dVR/dt = -VR + KA RF - (KA KF/TF) Efd + KA (Vref - Vt),
// with I = Y E~' + Yinf V_inf, Id + jIq = j I e^{-j delta}, Pe = Re(E~' conj I),
// Vt = |E~' - jX'd I|.  The OU disturbances and their KLE paths are those of
// the classical model.
//
// The integrator works in deviations from the operating point.  Per RK4 stage
// the network current deviation of a tile of 16 trajectories is one dense
// product dI = Y dE' (n x n complex by n x 16), done on the matrix cores as a
// real product [Re dI; Im dI] = [Yr -Yi; Yi Yr] [Re dE'; Im dE'] with
// v_mfma_f32_16x16x4f32.  Wave w of a workgroup computes the 16 x 16 output
// blocks of the machine blocks 2w and 2w+1 (16 machines each; one LDS
// fragment feeds four products), and the accumulator layout (lane l holds
// rows 4(l/16)+r, r = 0..3, of column l%16) makes lane l the owner of
// machines 16b + 4(l/16) + r of trajectory l%16: the lane that receives a
// current also holds that machine's state.  Y is
// packed once into the A-operand order of each wave and streamed from L2;
// the dE' tile (the B operand) lives in LDS.  Each lane's RK4 sums live in
// LDS too: with 8 machines a lane holds 48 state values and 48 stage values
// in registers, and the sums would not fit beside them.
#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"
#include "k_integrate.hpp"

namespace fmc {

namespace {

constexpr int kT = 16;  // trajectories per tile

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// FP64 operating point of the flux-decay machines (one thread per machine),
// after the common setup kernel has solved delta0 and I0 = Y E~0 + Yinf V:
//   J0 = I0 e^{-j delta0}, Id0 = -Im J0, Vt0 = E~0 - jX'd I0,
//   Efd0 = E + (Xd - X'd) Id0, VR0 = KE Efd0, RF0 = (KF/TF) Efd0,
// and the FP64 output offsets (delta0, 0, E, Efd0, VR0, RF0 per block).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_setup_fd(const double* __restrict__ canon, int n, int P,
                                                  const double* __restrict__ E,
                                                  const double* __restrict__ prm,
                                                  double* __restrict__ fd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CanonLayout C{n, P};
  const FdLayout F{n};
  const double* q = prm + (int64_t)i * kFdParams;
  const double d0 = canon[C.delta0() + i];
  const double ur = cos(d0), ui = sin(d0);
  const double i0r = canon[C.i0r() + i], i0i = canon[C.i0i() + i];
  const double j0r = i0r * ur + i0i * ui, j0i = i0i * ur - i0r * ui;  // I0 e^{-j d0}
  const double id0 = -j0i;
  const double c0 = canon[C.c0() + i], s0 = canon[C.s0() + i];
  const double xdp = q[kFdXdp];
  const double vtr = c0 + xdp * i0i, vti = s0 - xdp * i0r;  // E~0 - j X'd I0
  const double efd0 = E[i] + (q[kFdXd] - xdp) * id0;
  fd[F.u0r() + i] = ur;
  fd[F.u0i() + i] = ui;
  fd[F.j0r() + i] = j0r;
  fd[F.j0i() + i] = j0i;
  fd[F.vt0r() + i] = vtr;
  fd[F.vt0i() + i] = vti;
  fd[F.vt0a() + i] = sqrt(vtr * vtr + vti * vti);
  fd[F.off() + i] = d0;
  fd[F.off() + n + i] = 0.0;
  fd[F.off() + 2 * n + i] = E[i];
  fd[F.off() + 3 * n + i] = efd0;
  fd[F.off() + 4 * n + i] = q[kFdKe] * efd0;
  fd[F.off() + 5 * n + i] = q[kFdKf] / q[kFdTf] * efd0;
}

// FP32 constants [n_pad][kStride] (padding machines are zero except |Vt0| = 1,
// hence inert)
// and the per-process block (theta, sigma, xi0, machine index).
__global__ void __launch_bounds__(256) k_pack_fd(const double* __restrict__ canon, int n, int P,
                                                 const double* __restrict__ prm,
                                                 const double* __restrict__ fd,
                                                 const int32_t* __restrict__ gen, int n_pad,
                                                 float* __restrict__ cf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const CanonLayout C{n, P};
  const FdLayout F{n};
  const FdPack K{n_pad};
  if (i < n_pad) {
    const bool on = i < n;
    const double* q = prm + (int64_t)(on ? i : 0) * kFdParams;
    auto put = [&](int field, double v) { cf[K.at(i, field)] = on ? (float)v : 0.0f; };
    put(FdPack::C0, on ? canon[C.c0() + i] : 0.0);
    put(FdPack::S0, on ? canon[C.s0() + i] : 0.0);
    put(FdPack::U0R, on ? fd[F.u0r() + i] : 0.0);
    put(FdPack::U0I, on ? fd[F.u0i() + i] : 0.0);
    put(FdPack::I0R, on ? canon[C.i0r() + i] : 0.0);
    put(FdPack::I0I, on ? canon[C.i0i() + i] : 0.0);
    put(FdPack::J0R, on ? fd[F.j0r() + i] : 0.0);
    put(FdPack::J0I, on ? fd[F.j0i() + i] : 0.0);
    put(FdPack::VT0R, on ? fd[F.vt0r() + i] : 0.0);
    put(FdPack::VT0I, on ? fd[F.vt0i() + i] : 0.0);
    cf[K.at(i, FdPack::VT0A)] = on ? (float)fd[F.vt0a() + i] : 1.0f;  // padding: no 0/0 below
    put(FdPack::RES, on ? canon[C.res() + i] : 0.0);
    put(FdPack::DMP, on ? canon[C.dmp() + i] : 0.0);
    put(FdPack::INV2H, on ? canon[C.inv2h() + i] : 0.0);
    put(FdPack::XDP, q[kFdXdp]);
    put(FdPack::XDD_T, (q[kFdXd] - q[kFdXdp]) / q[kFdTdo]);
    put(FdPack::ITDO, 1.0 / q[kFdTdo]);
    put(FdPack::KE_TE, q[kFdKe] / q[kFdTe]);
    put(FdPack::ITE, 1.0 / q[kFdTe]);
    put(FdPack::ITF, 1.0 / q[kFdTf]);
    put(FdPack::KF_TF2, q[kFdKf] / q[kFdTf] / q[kFdTf]);
    put(FdPack::KA_TA, q[kFdKa] / q[kFdTa]);
    put(FdPack::ITA, 1.0 / q[kFdTa]);
    put(FdPack::KAKF, q[kFdKa] * q[kFdKf] / q[kFdTf] / q[kFdTa]);
  }
  if (i < P) {
    cf[K.proc() + i] = (float)canon[C.theta() + i];
    cf[K.proc() + kFdMaxProc + i] = (float)canon[C.sigma() + i];
    cf[K.proc() + 2 * kFdMaxProc + i] = (float)canon[C.xi0() + i];
    cf[K.proc() + 3 * kFdMaxProc + i] = (float)gen[i];  // exact for any machine index < 2^24
  }
}

// Y in the A-operand order of v_mfma_f32_16x16x4f32: for machine block b,
// k-step s < n_pad/4 and lane l, the pair (Yr, Yi)[16b + l%16][4s + l/16].
// The real product [Yr -Yi; Yi Yr][Re dE'; Im dE'] uses each pair twice: as
// (Yr, Yi) against the Re dE' rows 4s.. and as (-Yi, Yr) against the Im dE'
// rows n_pad + 4s.., so Y is read once per stage.
__global__ void __launch_bounds__(256) k_pack_fd_y(const double* __restrict__ canon, int n,
                                                   int n_pad, float2* __restrict__ ap) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int KH = n_pad / 4;
  const int64_t total = (int64_t)(n_pad / 16) * KH * 64;
  if (q >= total) return;
  const int l = (int)(q % 64);
  const int s = (int)((q / 64) % KH);
  const int b = (int)(q / (64 * KH));
  const int i = 16 * b + l % 16;
  const int k = 4 * s + l / 16;
  float yr = 0.0f, yi = 0.0f;
  if (i < n && k < n) {
    yr = (float)canon[(int64_t)i * n + k];
    yi = (float)canon[(int64_t)n * n + (int64_t)i * n + k];
  }
  ap[q] = make_float2(yr, yi);
}

// Y for the BF16 x3 product on v_mfma_f32_16x16x32_bf16 (x = hi + lo, hi =
// bf16(x), lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi): for machine
// block b, k-step s < n_padk/32 and lane l, the vectors Yr hi, Yr lo, Yi hi,
// Yi lo of the 8 entries [16b + l%16][32s + 8(l/16) + e], e = 0..7.
__global__ void __launch_bounds__(256) k_pack_fd_y16(const double* __restrict__ canon, int n,
                                                     int n_pad, int n_padk,
                                                     u32x4* __restrict__ ap) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int KS = n_padk / 32;
  const int64_t total = (int64_t)(n_pad / 16) * KS * 64;
  if (q >= total) return;
  const int l = (int)(q % 64);
  const int s = (int)((q / 64) % KS);
  const int b = (int)(q / (64 * KS));
  const int i = 16 * b + l % 16;
  bf8_t rh, rl, ih, il;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 32 * s + 8 * (l / 16) + e;
    float yr = 0.0f, yi = 0.0f;
    if (i < n && k < n) {
      yr = (float)canon[(int64_t)i * n + k];
      yi = (float)canon[(int64_t)n * n + (int64_t)i * n + k];
    }
    rh[e] = (__bf16)yr;
    rl[e] = (__bf16)(yr - (float)rh[e]);
    ih[e] = (__bf16)yi;
    il[e] = (__bf16)(yi - (float)ih[e]);
  }
  ap[4 * q + 0] = __builtin_bit_cast(u32x4, rh);
  ap[4 * q + 1] = __builtin_bit_cast(u32x4, rl);
  ap[4 * q + 2] = __builtin_bit_cast(u32x4, ih);
  ap[4 * q + 3] = __builtin_bit_cast(u32x4, il);
}

// Sum over the 16 lanes of a row (lanes l with equal l/16) with DPP moves:
// pairs (quad_perm 1,0,3,2), quads (quad_perm 2,3,0,1), half rows
// (row_half_mirror), rows (row_mirror).  Every step adds two values in both
// orders, so all 16 lanes end with the same bits.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_id) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  switch (ctrl_id) {
    case 0:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 2:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
      break;
  }
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  v += dpp_f64(v, 2);
  v += dpp_f64(v, 3);
  return v;
}

// Mean and M2 of a row's 16 values (invalid lanes excluded), stored by the
// row's first lane: every tile has rows of its own, so nothing is read back.
__device__ __forceinline__ void row_stats(double x, bool valid, double inv_cnt, bool writer,
                                          double2* dst) {
  const double mu = row16_sum(valid ? x : 0.0) * inv_cnt;
  const double d = valid ? x - mu : 0.0;
  const double m2 = row16_sum(d * d);
  if (writer) *dst = make_double2(mu, m2);
}

}  // namespace

// ---------------------------------------------------------------------------
// Integrator.  Grid: one workgroup per work item (a contiguous range of
// tiles, run one after another); block: NW = ceil(NB/2) waves, wave w owning
// the machine blocks 2w and 2w+1 (NB = n_pad/16 blocks of 16 machines).  Lane
// l of wave w owns machines 16(2w+j) + 4(l/16) + r (j = 0..1, r = 0..3) of
// trajectory l%16, slot q = 4j + r, and process (64w + l)/16 if that is < P.
// ---------------------------------------------------------------------------
constexpr int kQ = 8;  // machines per lane

// B tile of the BF16 x3 product: hi and lo planes [16 trajectories][BS] with
// BS = 2 n_padk + 8 (Re dE' rows, then Im dE' rows, then a bank skew).
__host__ __device__ inline int fd_bs(int n_padk) { return 2 * n_padk + 8; }
__host__ __device__ inline size_t fd_btile_bytes(int n_pad, int n_padk, bool bf) {
  return bf ? (size_t)2 * 16 * fd_bs(n_padk) * 2 : (size_t)2 * n_pad * 16 * 4;
}

template <bool BF>
__global__ void __launch_bounds__(512) k_rk4_fd(FdArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int n_pad = a.n_pad, n = a.n, P = a.P, V = a.V;
  const int NB = n_pad / 16, NW = (NB + 1) / 2, KH = n_pad / 4;
  const int n_padk = a.n_padk, KS16 = n_padk / 32, BS = fd_bs(n_padk);
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, g = l >> 4, t = l & 15;
  const bool two = 2 * wv + 1 < NB;  // wave-uniform: the second block exists
  const FdPack K{n_pad};
  // LDS: constants + process block, the dE' tile, xi stage values (2 buffers
  // of [P][16]), flags [16], each wave's sum of the angle deviations of its
  // machines per trajectory (2 buffers of [NW][16]), then the RK4 sums of
  // every lane [NW][6 kQ][64] (kept here rather than in registers)
  float* cst = reinterpret_cast<float*>(smem);
  unsigned char* btile = smem + (size_t)K.size() * 4;
  float* bs = reinterpret_cast<float*>(btile);          // FP32 product: [2 n_pad][16]
  __bf16* bh = reinterpret_cast<__bf16*>(btile);        // BF16 product: hi plane
  __bf16* bl = bh + 16 * BS;                            //               lo plane
  float* xs = reinterpret_cast<float*>(btile + fd_btile_bytes(n_pad, n_padk, BF));
  int* bad_t = reinterpret_cast<int*>(xs + 2 * P * kT);
  float* refb = reinterpret_cast<float*>(bad_t + kT);
  float* accl = refb + 2 * NW * kT + (int64_t)wv * 6 * kQ * 64 + l;
  for (int q = tid; q < K.size(); q += blockDim.x) cst[q] = a.coef[q];
  // the tile's padding rows (machines n_pad..n_padk) are never written: zero
  for (int q = tid; q < (int)(fd_btile_bytes(n_pad, n_padk, BF) / 4); q += blockDim.x)
    reinterpret_cast<float*>(btile)[q] = 0.0f;
  __syncthreads();

  auto mach = [&](int q) { return 16 * (2 * wv + (q >> 2)) + 4 * g + (q & 3); };
  const float dt = a.dt, h2 = 0.5f * a.dt, dt6 = a.dt / 6.0f, wb = a.wb;
  const float inv_n = 1.0f / (float)n;
  // mean over the waves' published sums of trajectory t (buffer b), in wave order
  auto mean_angle = [&](int b) {
    float sum = 0.0f;
    for (int ww = 0; ww < NW; ++ww) sum += refb[(b * NW + ww) * kT + t];
    return sum * inv_n;
  };
  const int item = blockIdx.x;
  const int64_t tile0 = (int64_t)item * a.tiles_per_item;
  const int64_t tile1 = tile0 + a.tiles_per_item < a.tiles ? tile0 + a.tiles_per_item : a.tiles;
  const int pg = (wv * 64 + l) >> 4;
  const bool proc = pg < P;  // uniform over a row of 16 lanes
  const float th = proc ? cst[K.proc() + pg] : 0.0f;
  const float sg = proc ? cst[K.proc() + kFdMaxProc + pg] : 0.0f;
  const int64_t colstride = (int64_t)P * a.N;
  const float2* apw = a.ap + (int64_t)(2 * wv) * KH * 64 + l;
  const float* B0 = bs + (l >> 4) * kT + (l & 15);
  const u32x4* aq = reinterpret_cast<const u32x4*>(a.ap16) + ((int64_t)(2 * wv) * KS16 * 64 + l) * 4;
  const int bfo = t * BS + 8 * g;  // B fragment of lane l: column t, rows 8(l/16)..
  int buf = 0;

  for (int64_t tile = tile0; tile < tile1; ++tile) {
    const int64_t traj = tile * kT + t;
    const bool valid = traj < a.N;
    const int64_t ns = valid ? traj : a.N - 1;
    const int64_t rem = a.N - tile * kT;
    const double cnt = (double)(rem < kT ? rem : kT);
    const double inv_cnt = 1.0 / cnt;  // one division per tile, not per variable
    double2* rows = a.rows + tile * a.row_stride;  // this tile's statistics rows
    const int slot = (valid && a.traj_slot) ? a.traj_slot[ns] : -1;
    // state: deviations of (delta, dw, E'q, Efd, VR, RF) of my machines; xi
    float y[6][kQ], x = 0.0f;
    double coff = 0.0;  // common-angle offset of trajectory t (see FdArgs::recenter)
    float pend = 0.0f;  // the mean angle left by the previous step
    const int64_t sbase = ((tile * NW + wv) * 6 * kQ) * 64 + l;
    const int64_t xrow = tile * (kFdMaxProc + kFdOffsetRows);
    const int64_t xbase = (xrow + (proc ? pg : 0)) * kT + t;
    const int64_t obase = (xrow + kFdMaxProc) * kT + t;
    if (a.s_begin == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int q = 0; q < kQ; ++q) y[c][q] = 0.0f;
      x = proc ? cst[K.proc() + 2 * kFdMaxProc + pg] : 0.0f;
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int q = 0; q < kQ; ++q) y[c][q] = a.state[sbase + (c * kQ + q) * 64];
      if (proc) x = a.xstate[xbase];
      coff = load_offset(a.xstate, obase, obase + kT);
      pend = a.xstate[obase + 2 * kT];
    }
    const int64_t wofs = (int64_t)(proc ? pg : 0) * a.N + ns;

    // statistics and sampled outputs of step s (deviations + FP64 offsets)
    auto emit = [&](int64_t s) {
      // n and the offset table pass through an empty asm so that the
      // compiler recomputes the (c, machine) addresses here instead of
      // keeping 48 loop-invariant 64-bit addresses live across the steps
      int nl = n;
      const double* offl = a.off;
      asm volatile("" : "+s"(nl), "+s"(offl));
      double2* row = rows + (s - a.row_base) * V;
      double* o = slot >= 0 ? a.traj + ((int64_t)slot * (a.S + 1) + s) * V : nullptr;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int m = mach(q);  // uniform over the row of 16 lanes
        if (m < nl) {
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const double yv = c == 0 ? coff + (double)y[0][q] : (double)y[c][q];
            row_stats(yv, valid, inv_cnt, t == 0, row + c * nl + m);
            if (o) o[c * nl + m] = offl[c * nl + m] + yv;
          }
        }
      }
      if (proc) {
        row_stats((double)x, valid, inv_cnt, t == 0, row + 6 * n + pg);
        if (o) o[6 * n + pg] = (double)x;
      }
    };
    if (a.s_begin == 0) emit(0);

    const float* w = a.w;
    float w0 = proc ? w[wofs] : 0.0f, w1 = proc ? w[colstride + wofs] : 0.0f,
          w2 = proc ? w[2 * colstride + wofs] : 0.0f;
    for (int64_t s = a.s_begin; s < a.s_end; ++s) {
      const int64_t cl = 2 * s - a.c_base;
      const bool more = s + 1 < a.s_end;
      const float n1 = (more && proc) ? w[(cl + 3) * colstride + wofs] : 0.0f;
      const float n2 = (more && proc) ? w[(cl + 4) * colstride + wofs] : 0.0f;
      float ys[6][kQ], xsg = x, ax = 0.0f;
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int q = 0; q < kQ; ++q) ys[c][q] = y[c][q];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        // RK4 weights: stage st enters the sum with wgt, the next stage's input
        // is y + hn k
        const float wgt = (st == 0 || st == 3) ? 1.0f : 2.0f;
        const float hn = st < 2 ? h2 : dt;
        const float wst = st == 0 ? w0 : (st == 3 ? w2 : w1);
        float* Bw = bs;
        float* X = xs + buf * (P * kT);
        // -- before the product: EMF deviations, the derivatives that do not
        //    need the network current, and the parts of those that do
        float omc[kQ], sd[kQ], dEr[kQ], dEi[kQ], pw[kQ], pe[kQ], pv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          if (q >= 4 && !two) continue;
          const int m = mach(q);
          int mo = K.at(m, 0), bo = m * kT + t;
          asm volatile("" : "+v"(mo), "+v"(bo));  // recompute, do not keep live
          const float4* cm = reinterpret_cast<const float4*>(cst + mo);
          const float4 g0 = cm[0], g3 = cm[3], g4 = cm[4], g5 = cm[5];
          float sh, ch;
          sincos_r_nb(0.5f * ys[0][q], sh, ch);
          sd[q] = 2.0f * sh * ch;   // sin d
          omc[q] = 2.0f * sh * sh;  // 1 - cos d
          const float c0 = g0.x, s0 = g0.y, ur = g0.z, ui = g0.w;
          const float de = ys[2][q];
          // dE' = E~0 (e^{jd} - 1) + dE'q e^{j delta}
          dEr[q] = -c0 * omc[q] - s0 * sd[q] + de * (ur * (1.0f - omc[q]) - ui * sd[q]);
          dEi[q] = c0 * sd[q] - s0 * omc[q] + de * (ui * (1.0f - omc[q]) + ur * sd[q]);
          // padding machines contribute exact zeros (Y's padding columns are
          // zero, and 0 * NaN would still poison the product)
          if constexpr (BF) {
            const float er = m < n ? dEr[q] : 0.0f, ei = m < n ? dEi[q] : 0.0f;
            const __bf16 rh = (__bf16)er, ih = (__bf16)ei;
            const int o = t * BS + m;
            bh[o] = rh;
            bl[o] = (__bf16)(er - (float)rh);
            bh[o + n_padk] = ih;
            bl[o + n_padk] = (__bf16)(ei - (float)ih);
          } else {
            Bw[bo] = m < n ? dEr[q] : 0.0f;
            Bw[bo + n_pad * kT] = m < n ? dEi[q] : 0.0f;
          }
          // g3 = (RES, DMP, INV2H, ITDO), g4 = (XDD_T, KE_TE, ITE, ITF),
          // g5 = (KF_TF2, KA_TA, ITA, KAKF)
          const float kd = wb * ys[1][q];
          const float kf = -g4.y * ys[3][q] + g4.z * ys[4][q];
          const float kr = -g4.w * ys[5][q] + g5.x * ys[3][q];
          pw[q] = g3.x - g3.y * ys[1][q];
          pe[q] = (ys[3][q] - ys[2][q]) * g3.w;
          pv[q] = -g5.z * ys[4][q] + g5.y * ys[5][q] - g5.w * ys[3][q];
          accl[(0 * kQ + q) * 64] = st == 0 ? kd : accl[(0 * kQ + q) * 64] + wgt * kd;
          accl[(3 * kQ + q) * 64] = st == 0 ? kf : accl[(3 * kQ + q) * 64] + wgt * kf;
          accl[(5 * kQ + q) * 64] = st == 0 ? kr : accl[(5 * kQ + q) * 64] + wgt * kr;
          if (st < 3) {
            ys[0][q] = y[0][q] + hn * kd;
            ys[3][q] = y[3][q] + hn * kf;
            ys[5][q] = y[5][q] + hn * kr;
          }
        }
        if (proc) X[pg * kT + t] = xsg;
        __syncthreads();
        // -- dI = Y dE' for my machine blocks over the tile's 16 trajectories
        f32x4 ar0 = {0.f, 0.f, 0.f, 0.f}, ai0 = ar0, ar1 = ar0, ai1 = ar0;
        const float* bp = B0;
        if constexpr (BF) {
          // three BF16 products per real product (lo*hi, hi*lo, hi*hi), the
          // sign of Yi flipped in its bits for the -Yi block
          const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
          for (int k = 0; k < KS16; ++k) {
            const bf8_t rh_ = *reinterpret_cast<const bf8_t*>(bh + bfo + 32 * k);
            const bf8_t rl_ = *reinterpret_cast<const bf8_t*>(bl + bfo + 32 * k);
            const bf8_t ih_ = *reinterpret_cast<const bf8_t*>(bh + bfo + n_padk + 32 * k);
            const bf8_t il_ = *reinterpret_cast<const bf8_t*>(bl + bfo + n_padk + 32 * k);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              if (j == 1 && !two) break;
              const u32x4* av = aq + (int64_t)(j * KS16 + k) * 64 * 4;
              const u32x4 u0 = av[0], u1 = av[1], u2 = av[2], u3 = av[3];
              const bf8_t yrh = __builtin_bit_cast(bf8_t, u0), yrl = __builtin_bit_cast(bf8_t, u1);
              const bf8_t yih = __builtin_bit_cast(bf8_t, u2), yil = __builtin_bit_cast(bf8_t, u3);
              const bf8_t nih = __builtin_bit_cast(bf8_t, u2 ^ sgn), nil = __builtin_bit_cast(bf8_t, u3 ^ sgn);
              f32x4& ar = j == 0 ? ar0 : ar1;
              f32x4& ai = j == 0 ? ai0 : ai1;
              ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrl, rh_, ar, 0, 0, 0);
              ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, rl_, ar, 0, 0, 0);
              ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, rh_, ar, 0, 0, 0);
              ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yil, rh_, ai, 0, 0, 0);
              ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yih, rl_, ai, 0, 0, 0);
              ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yih, rh_, ai, 0, 0, 0);
              ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, ih_, ar, 0, 0, 0);
              ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, il_, ar, 0, 0, 0);
              ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, ih_, ar, 0, 0, 0);
              ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrl, ih_, ai, 0, 0, 0);
              ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, il_, ai, 0, 0, 0);
              ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, ih_, ai, 0, 0, 0);
            }
          }
        } else if (two) {
          constexpr int PF = 4;
          float2 p0[PF], p1[PF];
#pragma unroll
          for (int u = 0; u < PF; ++u) {
            p0[u] = apw[(int64_t)u * 64];
            p1[u] = apw[(int64_t)(KH + u) * 64];
          }
          for (int k0 = 0; k0 < KH; k0 += PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
              const int k = k0 + u;
              const float2 a0 = p0[u], a1 = p1[u];
              if (k + PF < KH) {
                p0[u] = apw[(int64_t)(k + PF) * 64];
                p1[u] = apw[(int64_t)(KH + k + PF) * 64];
              }
              const float br = bp[k * 4 * kT], bi = bp[(k * 4 + n_pad) * kT];
              ar0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, br, ar0, 0, 0, 0);
              ai0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, br, ai0, 0, 0, 0);
              ar1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, br, ar1, 0, 0, 0);
              ai1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, br, ai1, 0, 0, 0);
              ar0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-a0.y, bi, ar0, 0, 0, 0);
              ai0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, bi, ai0, 0, 0, 0);
              ar1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-a1.y, bi, ar1, 0, 0, 0);
              ai1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, bi, ai1, 0, 0, 0);
            }
          }
        } else {
          constexpr int PF = 4;
          float2 p0[PF];
#pragma unroll
          for (int u = 0; u < PF; ++u) p0[u] = apw[(int64_t)u * 64];
          for (int k0 = 0; k0 < KH; k0 += PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
              const int k = k0 + u;
              const float2 a0 = p0[u];
              if (k + PF < KH) p0[u] = apw[(int64_t)(k + PF) * 64];
              const float br = bp[k * 4 * kT], bi = bp[(k * 4 + n_pad) * kT];
              ar0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, br, ar0, 0, 0, 0);
              ai0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, br, ai0, 0, 0, 0);
              ar0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-a0.y, bi, ar0, 0, 0, 0);
              ai0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, bi, ai0, 0, 0, 0);
            }
          }
        }
        __syncthreads();  // every wave is done reading the dE' tile
        // -- after the product: injections, dPe, dId, d|Vt|
        // injections sum_p [gen(p) = m] xi_p as a small product on the
        // matrix cores: the 0/1 matrix [machine][process] in A-operand order
        // (lane l: machine 16 blk + l%16, process 4s + l/16) against the
        // processes' stage values (B: process 4s + l/16 of trajectory l%16);
        // the result lands on the lanes that own the machines
        f32x4 aj0 = {0.f, 0.f, 0.f, 0.f}, aj1 = aj0;
        for (int s4 = 0; s4 < (P + 3) / 4; ++s4) {
          const int p = 4 * s4 + g;
          const int gm = p < P ? (int)cst[K.proc() + 3 * kFdMaxProc + p] : -1;
          const float xb = p < P ? X[p * kT + t] : 0.0f;
          aj0 = __builtin_amdgcn_mfma_f32_16x16x4f32(gm == 32 * wv + t ? 1.0f : 0.0f, xb, aj0, 0, 0, 0);
          if (two)  // wave-uniform
            aj1 = __builtin_amdgcn_mfma_f32_16x16x4f32(gm == 32 * wv + 16 + t ? 1.0f : 0.0f, xb, aj1,
                                                      0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          if (q >= 4 && !two) continue;
          const int m = mach(q);
          int mo = K.at(m, 0);
          asm volatile("" : "+v"(mo));
          const float4* cm = reinterpret_cast<const float4*>(cst + mo);
          const float4 g0 = cm[0], g1 = cm[1], g2 = cm[2], g3 = cm[3], g4 = cm[4], g5 = cm[5];
          const int r = q & 3;
          const float dIr = q < 4 ? ar0[r] : ar1[r], dIi = q < 4 ? ai0[r] : ai1[r];
          const float c0 = g0.x, s0 = g0.y, ur = g0.z, ui = g0.w;
          const float i0r = g1.x, i0i = g1.y, j0r = g1.z, j0i = g1.w;
          // dPe = Re(dE' conj I0) + Re(E~' conj dI)
          const float dpe = dEr[q] * i0r + dEi[q] * i0i + (c0 + dEr[q]) * dIr + (s0 + dEi[q]) * dIi;
          // dId = -Im(J0 (e^{-jd} - 1) + dI e^{-j delta0} e^{-jd})
          const float djr = dIr * ur + dIi * ui, dji = dIi * ur - dIr * ui;
          const float did = j0i * omc[q] + j0r * sd[q] - dji * (1.0f - omc[q]) + djr * sd[q];
          // d|Vt| with dVt = dE' - j X'd dI
          const float xdp = g2.x;
          const float vr_ = dEr[q] + xdp * dIi, vi_ = dEi[q] - xdp * dIr;
          const float v0r = g2.y, v0i = g2.z;
          const float vr1 = v0r + vr_, vi1 = v0i + vi_;
          // |Vt| and the quotient through the hardware reciprocal square root
          // and reciprocal (about 1 ulp each; |Vt| only scales the small
          // deviation here, and the sum of squares is kept above zero for
          // the padding machines, whose |Vt| is 0)
          const float vs = fmaxf(vr1 * vr1 + vi1 * vi1, 1e-30f);
          const float va = vs * __builtin_amdgcn_rsqf(vs);
          const float dva = (2.0f * (v0r * vr_ + v0i * vi_) + vr_ * vr_ + vi_ * vi_) *
                            __builtin_amdgcn_rcpf(va + g2.w);
          const float kw = (pw[q] - dpe + (q < 4 ? aj0[r] : aj1[r])) * g3.z;
          const float ke = pe[q] - g4.x * did;
          const float kv = pv[q] - g5.y * dva;
          accl[(1 * kQ + q) * 64] = st == 0 ? kw : accl[(1 * kQ + q) * 64] + wgt * kw;
          accl[(2 * kQ + q) * 64] = st == 0 ? ke : accl[(2 * kQ + q) * 64] + wgt * ke;
          accl[(4 * kQ + q) * 64] = st == 0 ? kv : accl[(4 * kQ + q) * 64] + wgt * kv;
          if (st < 3) {
            ys[1][q] = y[1][q] + hn * kw;
            ys[2][q] = y[2][q] + hn * ke;
            ys[4][q] = y[4][q] + hn * kv;
          }
        }
        const float kx = -th * xsg + sg * wst;
        ax = st == 0 ? kx : ax + wgt * kx;
        if (st < 3) xsg = x + hn * kx;
        buf ^= 1;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int q = 0; q < kQ; ++q)
          if (q < 4 || two) y[c][q] += dt6 * accl[(c * kQ + q) * 64];
      x += dt6 * ax;
      w0 = w2; w1 = n1; w2 = n2;
      if (a.recenter) {
        // The mean angle of trajectory t's machines as the previous step left
        // it (from the waves' sums published in LDS at the end of that step,
        // visible after this step's barriers; at the first step of a chunk,
        // carried in the state; 0 before the first step) is taken out of
        // every angle.  A common shift leaves the network quantities
        // unchanged whenever it is taken, as long as all machines of a
        // trajectory take the same one.  Then this wave publishes its sum of
        // trajectory t's angles (lanes t, t + 16, t + 32, t + 48, in order).
        const int rb = (int)(s & 1);
        const float ref = s == a.s_begin ? pend : mean_angle(rb ^ 1);
        coff += (double)ref;
        float part = 0.0f;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          y[0][q] -= ref;
          if ((q < 4 || two) && mach(q) < n) part += y[0][q];
        }
        float wsum = __shfl(part, t, 64);
        wsum += __shfl(part, t + 16, 64);
        wsum += __shfl(part, t + 32, 64);
        wsum += __shfl(part, t + 48, 64);
        if (g == 0) refb[(rb * NW + wv) * kT + t] = wsum;
      }
      emit(s + 1);
    }

    if (a.state) {
      float pnext = 0.0f;  // the mean angle the next chunk starts by taking out
      if (a.recenter) {
        __syncthreads();  // every wave has published the last step's sums
        pnext = mean_angle((int)((a.s_end - 1) & 1));
      }
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int q = 0; q < kQ; ++q) a.state[sbase + (c * kQ + q) * 64] = y[c][q];
      if (proc) a.xstate[xbase] = x;
      if (wv == 0 && g == 0) {
        store_offset(a.xstate, obase, obase + kT, coff);
        a.xstate[obase + 2 * kT] = pnext;
      }
    }
    if (a.s_end == a.S) {  // uniform over the workgroup
      bool bad = (proc && !isfinite(x)) || !isfinite(coff);
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int q = 0; q < kQ; ++q) bad |= (mach(q) < n) && !isfinite(y[c][q]);
      if (tid < kT) bad_t[tid] = 0;
      __syncthreads();
      if (bad) bad_t[t] = 1;
      __syncthreads();
      if (tid < kT && tile * kT + tid < a.N && bad_t[tid] != 0) {
        atomicAdd(a.nonfinite, 1ULL);
        atomicMin(a.first_bad, (long long)(tile * kT + tid));
      }
    }
    __syncthreads();  // LDS buffers and flags are reused by the next tile
  }
}

hipError_t launch_setup_fd(const double* canon, int n, int P, const double* E, const double* prm,
                           double* fd, hipStream_t st) {
  hipLaunchKernelGGL(k_setup_fd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, canon, n, P,
                     E, prm, fd);
  return hipGetLastError();
}

hipError_t launch_pack_fd(const double* canon, int n, int P, const double* prm, const double* fd,
                          const int32_t* gen, int n_pad, float* coef, float2* ap,
                          hipStream_t st) {
  const int m = n_pad > P ? n_pad : P;
  hipLaunchKernelGGL(k_pack_fd, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, canon, n, P,
                     prm, fd, gen, n_pad, coef);
  const int64_t total = (int64_t)(n_pad / 16) * (n_pad / 4) * 64;
  hipLaunchKernelGGL(k_pack_fd_y, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, canon,
                     n, n_pad, ap);
  return hipGetLastError();
}

size_t fd_lds_bytes(int n_pad, int n_padk, bool bf, int P) {
  const FdPack K{n_pad};
  const int nw = (n_pad / 16 + 1) / 2;
  return (size_t)K.size() * 4 + fd_btile_bytes(n_pad, n_padk, bf) + (size_t)2 * P * kT * 4 +
         kT * 4 + (size_t)2 * nw * kT * 4 + (size_t)nw * 6 * kQ * 64 * 4;
}

template <bool BF>
static hipError_t launch_rk4_fd_t(const FdArgs& a, int64_t n_items, hipStream_t st) {
  const size_t lds = fd_lds_bytes(a.n_pad, a.n_padk, BF, a.P);
  static size_t lds_set = 0;  // dynamic LDS above 64 KB must be allowed explicitly
  if (lds > lds_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_rk4_fd<BF>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    lds_set = lds;
  }
  const int nw = (a.n_pad / 16 + 1) / 2;
  hipLaunchKernelGGL(k_rk4_fd<BF>, dim3((unsigned)n_items), dim3((unsigned)(nw * 64)), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_rk4_fd(const FdArgs& a, int64_t n_items, hipStream_t st) {
  return a.ap16 ? launch_rk4_fd_t<true>(a, n_items, st) : launch_rk4_fd_t<false>(a, n_items, st);
}

hipError_t launch_pack_fd_y(const double* canon, int n, int n_pad, float2* ap, hipStream_t st) {
  const int64_t total = (int64_t)(n_pad / 16) * (n_pad / 4) * 64;
  hipLaunchKernelGGL(k_pack_fd_y, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, canon,
                     n, n_pad, ap);
  return hipGetLastError();
}

hipError_t launch_pack_fd_y16(const double* canon, int n, int n_pad, int n_padk, void* ap16,
                              hipStream_t st) {
  const int64_t total = (int64_t)(n_pad / 16) * (n_padk / 32) * 64;
  hipLaunchKernelGGL(k_pack_fd_y16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, canon,
                     n, n_pad, n_padk, (u32x4*)ap16);
  return hipGetLastError();
}

}  // namespace fmc
