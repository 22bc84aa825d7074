// k_mfma_classical.hpp -- classical machines with the network current on the
// matrix cores (the batched and served forms' size classes for larger systems).
//
// Same deviation form as the lane-per-machine integrators: per RK4 stage
// dE~ = E~0 (e^{j dd} - 1), dPe = Re(dE~ conj I0) + Re(E~ conj dI) with
// dI = Y dE~, and the swing equations.  Here a wave owns a tile of 16
// trajectories and computes dI for all of them as the real product
// [Re dI; Im dI] = [Yr -Yi; Yi Yr][Re dE~; Im dE~] on v_mfma_f32_16x16x4f32
// (or, for BF16 x3 scenarios, three BF16 products per real product on
// v_mfma_f32_16x16x32_bf16), with dE~ in the wave's own LDS tile and Y read
// in A-operand order from the scenario's coefficient block (L2).  The
// accumulator layout (lane l holds rows 4(l/16)+r of column l%16) makes lane l
// the owner of machines 16b + 4(l/16) + r of trajectory l%16, for blocks
// b < n_pad/16.  The four waves of a workgroup run independently; per step
// their statistics are reduced across each row's 16 lanes (DPP), combined over
// the four waves in LDS and stored per 64-trajectory tile.
#pragma once

#include <hip/hip_runtime.h>

#include "fmc_internal.hpp"
#include "k_integrate.hpp"

namespace fmc {

namespace mc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;            // trajectories per wave
constexpr int kWaves = 4;         // waves per workgroup
constexpr int kTile = kT * kWaves;
constexpr int kNP = kMcMaxGen;    // largest n_pad
constexpr int kVM = 2 * kNP + kMcMaxProc;

// Static LDS of the class: constants, per-wave dE~ tiles (the larger of the
// FP32 and BF16 forms), two buffers of per-wave statistics, per-trajectory
// flags.
constexpr int kBtileFloats = (2 * kNP * kT > 16 * (2 * kNP + 8)) ? 2 * kNP * kT : 16 * (2 * kNP + 8);
struct Lds {
  float cst[McPack::kMaxConsts];
  float btile[kWaves][kBtileFloats];
  double2 part[2][kWaves][kVM];
  int bad[kTile];
  double cw[2][kWaves];  // Chan weights of the tile's in-order wave merge
  double pw[2];          // and of its merge into the item's earlier tiles
};

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

// Sum over the 16 lanes of a row; every lane ends with the same bits.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  v += dpp_f64(v, 2);
  v += dpp_f64(v, 3);
  return v;
}

}  // namespace mc

// One 64-trajectory tile of a scenario (trajectories 64 tile .. 64 tile + 63)
// over the steps [s_begin, s_end) of a, with the machines padded to 16 NB.
// st.rows is addressed by global step; st.prev trajectories of the work item
// are already merged into it.
template <bool BF, int NB>
__device__ __forceinline__ void mc_tile(const IntegArgs<float>& a, int64_t tile, mc::Lds& S,
                                        GroupStats st) {
  using namespace mc;
  constexpr int n_pad = 16 * NB, KH = n_pad / 4, kQ = 4 * NB;
  constexpr int n_padk = 32 * ((n_pad + 31) / 32), KS16 = n_padk / 32, BS = 2 * n_padk + 8;
  constexpr McPack K{n_pad};
  const int n = a.n, P = a.P, V = a.V;
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, g = l >> 4, t = l & 15;
  const int64_t N = a.N;
  const int64_t traj = tile * kTile + wv * kT + t;
  const bool valid = traj < N;
  const int64_t ns = valid ? traj : N - 1;
  auto wave_count = [&](int w) {  // valid trajectories of wave w of this tile
    const int64_t r = N - (tile * kTile + w * kT);
    return (double)(r <= 0 ? 0 : (r < kT ? r : kT));
  };
  const double wcnt = wave_count(wv);
  const double winv = wcnt > 0.0 ? 1.0 / wcnt : 0.0;

  const int slot = (valid && a.traj_slot) ? a.traj_slot[ns] : -1;

  __syncthreads();  // every reader of the previous tile's constants is done
  for (int q = tid; q < K.consts(); q += blockDim.x) S.cst[q] = a.coef[q];
  if (tid == 0) {
    // Chan weights (the same at every step of the tile): merging wave w into
    // waves 0..w-1 uses nb / tot and cnt nb / tot, then the tile into the
    // item's st.prev earlier samples; computed once rather than divided at
    // every step
    double cnt = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      const double nb = wave_count(w), tot = cnt + nb;
      S.cw[0][w] = tot > 0.0 ? nb / tot : 0.0;
      S.cw[1][w] = tot > 0.0 ? cnt * nb / tot : 0.0;
      cnt = tot;
    }
    const double ptot = (double)st.prev + cnt;
    S.pw[0] = cnt / ptot;
    S.pw[1] = (double)st.prev * cnt / ptot;
  }
  __syncthreads();

  auto mach = [&](int q) { return 16 * (q >> 2) + 4 * g + (q & 3); };
  // processes g and g + 4 of trajectory t
  const bool own0 = g < P, own1 = g + 4 < P;
  const float th0 = own0 ? S.cst[K.proc() + g] : 0.0f;
  const float sg0 = own0 ? S.cst[K.proc() + kMcMaxProc + g] : 0.0f;
  const float th1 = own1 ? S.cst[K.proc() + g + 4] : 0.0f;
  const float sg1 = own1 ? S.cst[K.proc() + kMcMaxProc + g + 4] : 0.0f;
  // The injections sum_p [gen(p) = m] xi_p of a tile are one more product on
  // the matrix cores: the 0/1 matrix [machine][process] in A-operand order
  // (lane l: machine 16b + l%16, process 4s + l/16) against the stage values
  // of the processes, which lane l holds itself as the B operand (process
  // 4s + l/16 of trajectory l%16); the result lands on the lanes that own
  // the machines, like the network current.
  float ainj[NB][2];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = 4 * h + g;
      ainj[b][h] = (p < P && (int)S.cst[K.proc() + 3 * kMcMaxProc + p] == 16 * b + t) ? 1.0f : 0.0f;
    }

  // State between time chunks: [tile][wave][kRows][64], rows dd (kQ), dw
  // (kQ), the two process slots, the common-angle offset (hi, lo); kRows =
  // 2 G + PQ + kOffsetRows of the host's allocation with G = n_pad / 4 and
  // PQ = kMcMaxProc / 4 (4 lanes per trajectory).
  constexpr int kRows = 2 * kQ + kMcMaxProc / 4 + kOffsetRows;
  static_assert(kMcMaxProc / 4 == 2, "two process slots per lane");
  float yd[kQ], yw[kQ], x0, x1;
  double coff = 0.0;  // common-angle offset of trajectory t (see IntegArgs::recenter)
  const int64_t sbase = (tile * kWaves + wv) * kRows * 64 + l;
  if (a.s_begin == 0) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) { yd[q] = 0.0f; yw[q] = 0.0f; }
    x0 = own0 ? S.cst[K.proc() + 2 * kMcMaxProc + g] : 0.0f;
    x1 = own1 ? S.cst[K.proc() + 2 * kMcMaxProc + g + 4] : 0.0f;
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      yd[q] = a.state[sbase + q * 64];
      yw[q] = a.state[sbase + (kQ + q) * 64];
    }
    x0 = a.state[sbase + (2 * kQ) * 64];
    x1 = a.state[sbase + (2 * kQ + 1) * 64];
    coff = load_offset(a.state, sbase + (2 * kQ + 2) * 64, sbase + (2 * kQ + 3) * 64);
  }

  int pbuf = 0;
  // Statistics of step s: exact two-pass (mean, M2) of each wave's trajectories
  // (sums over the 16 lanes of a row), the four waves combined in order with
  // Chan's update, then merged into the item's row.
  auto emit = [&](int64_t s) {
    // n and the operating point pass through an empty asm so that the
    // machine addresses are recomputed here rather than kept live (with
    // the loaded delta0 values) across the whole run
    int nl = n;
    const double* d0 = a.delta0;
    asm volatile("" : "+v"(nl), "+v"(d0));
    double2* part = S.part[pbuf][wv];
    double* o = slot >= 0 ? a.traj + ((int64_t)slot * (a.S + 1) + s) * V : nullptr;
    const double inv = winv;
    auto one = [&](double xv, int v) {
      const double mu = row16_sum(valid ? xv : 0.0) * inv;
      const double d = valid ? xv - mu : 0.0;
      const double m2 = row16_sum(d * d);
      if (t == 0) part[v] = make_double2(mu, m2);
    };
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int m = mach(q);  // uniform over a row of 16 lanes
      if (m < nl) {
        one(coff + (double)yd[q], m);
        one((double)yw[q], nl + m);
        if (o) {
          o[m] = d0[m] + (coff + (double)yd[q]);
          o[nl + m] = (double)yw[q];
        }
      }
    }
    if (own0) {
      one((double)x0, 2 * nl + g);
      if (o) o[2 * nl + g] = (double)x0;
    }
    if (own1) {
      one((double)x1, 2 * nl + g + 4);
      if (o) o[2 * nl + g + 4] = (double)x1;
    }
    __syncthreads();
    double2* dst = st.rows + s * V;
    for (int v = tid; v < V; v += blockDim.x) {
      // wave 0 always has valid trajectories (a tile exists only if it does)
      double mu = S.part[pbuf][0][v].x, M2 = S.part[pbuf][0][v].y;
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        if (wave_count(w) == 0.0) continue;  // the tile's trailing empty waves
        const double2 pt = S.part[pbuf][w][v];
        const double dl = pt.x - mu;
        mu += dl * S.cw[0][w];
        M2 += pt.y + dl * dl * S.cw[1][w];
      }
      if (st.prev == 0) {
        dst[v] = make_double2(mu, M2);
      } else {
        const double2 old = dst[v];
        const double dl = mu - old.x;
        dst[v] = make_double2(old.x + dl * S.pw[0], old.y + M2 + dl * dl * S.pw[1]);
      }
    }
    pbuf ^= 1;  // the next step fills the other buffer: one barrier per step suffices
  };
  if (a.s_begin == 0) emit(0);

  float* B = S.btile[wv];
  __bf16* bh = reinterpret_cast<__bf16*>(B);
  __bf16* bl = bh + 16 * BS;
  const float* Bf = B + g * kT + t;
  const int bfo = t * BS + 8 * g;
  if constexpr (BF) {
    // rows n_pad .. n_padk of the tile are never written: zero them
    for (int q = l; q < 16 * BS; q += 64) B[q] = 0.0f;
    wave_lds_sync();
  }

  const float dt = a.dt, h2 = 0.5f * a.dt, dt6 = a.dt / 6.0f, wb = a.wb;
  const float inv_n = 1.0f / (float)n;
  const int64_t colstride = (int64_t)P * N;
  const float* w = a.w;
  const int64_t wo0 = (int64_t)(own0 ? g : 0) * N + ns, wo1 = (int64_t)(own1 ? g + 4 : 0) * N + ns;
  const int64_t cb = 2 * a.s_begin - a.c_base;
  float w00 = own0 ? w[cb * colstride + wo0] : 0.f;
  float w01 = own0 ? w[(cb + 1) * colstride + wo0] : 0.f;
  float w02 = own0 ? w[(cb + 2) * colstride + wo0] : 0.f;
  float w10 = own1 ? w[cb * colstride + wo1] : 0.f;
  float w11 = own1 ? w[(cb + 1) * colstride + wo1] : 0.f;
  float w12 = own1 ? w[(cb + 2) * colstride + wo1] : 0.f;

  for (int64_t s = a.s_begin; s < a.s_end; ++s) {
    const int64_t cl = 2 * s - a.c_base;
    const bool more = s + 1 < a.s_end;
    const float n01 = (more && own0) ? w[(cl + 3) * colstride + wo0] : 0.f;
    const float n02 = (more && own0) ? w[(cl + 4) * colstride + wo0] : 0.f;
    const float n11 = (more && own1) ? w[(cl + 3) * colstride + wo1] : 0.f;
    const float n12 = (more && own1) ? w[(cl + 4) * colstride + wo1] : 0.f;
    float sd_[kQ], sw_[kQ], ad[kQ], aw[kQ];
    float sx0 = x0, sx1 = x1, ax0 = 0.f, ax1 = 0.f;
#pragma unroll
    for (int q = 0; q < kQ; ++q) { sd_[q] = yd[q]; sw_[q] = yw[q]; ad[q] = 0.f; aw[q] = 0.f; }
#pragma unroll 1
    for (int sg = 0; sg < 4; ++sg) {
      const float wgt = (sg == 0 || sg == 3) ? 1.0f : 2.0f;
      const float hn = sg < 2 ? h2 : dt;
      const float wa = sg == 0 ? w00 : (sg == 3 ? w02 : w01);
      const float wc = sg == 0 ? w10 : (sg == 3 ? w12 : w11);
      // rotated EMF deviations of my machines into the wave's tile
      float dEr[kQ], dEi[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int m = mach(q);
        int mo = K.at(m, 0);
        asm volatile("" : "+v"(mo));  // reread the constants, do not keep them live
        const float4 c = *reinterpret_cast<const float4*>(S.cst + mo);  // C0 S0 I0R I0I
        float sh, ch;
        // the branch-free form: the four or eight machines of a lane are
        // interleaved by the compiler (a padding machine, E~0 = 0, gives dE = 0
        // at any angle)
        sincos_r_nb(0.5f * sd_[q], sh, ch);
        const float sdd = 2.0f * sh * ch, omc = 2.0f * sh * sh;
        dEr[q] = -(c.x * omc + c.y * sdd);  // zero for padding machines (E~0 = 0)
        dEi[q] = c.x * sdd - c.y * omc;
        if constexpr (BF) {
          const __bf16 rh = (__bf16)dEr[q], ih = (__bf16)dEi[q];
          const int o = t * BS + m;
          bh[o] = rh;
          bl[o] = (__bf16)(dEr[q] - (float)rh);
          bh[o + n_padk] = ih;
          bl[o + n_padk] = (__bf16)(dEi[q] - (float)ih);
        } else {
          B[m * kT + t] = dEr[q];
          B[(n_pad + m) * kT + t] = dEi[q];
        }
      }
      wave_lds_sync();
      // dI = Y dE~ for my machine blocks.  With one block the lane's Y
      // fragments (8 or 16 registers) stay in registers for the whole tile;
      // with more, the coefficient pointer passes an empty asm so that Y is
      // streamed from the cache at every stage instead of being hoisted into
      // (spilled) registers.
      const float* cf = a.coef;
      if constexpr (NB > 1) asm volatile("" : "+v"(cf));
      const float2* ap = reinterpret_cast<const float2*>(cf + K.frag()) + l;
      const u32x4* aq = reinterpret_cast<const u32x4*>(cf + K.frag()) + (int64_t)l * 4;
      f32x4 ar[NB], ai[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) { ar[b] = f32x4{0.f, 0.f, 0.f, 0.f}; ai[b] = ar[b]; }
      if constexpr (BF) {
        const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
#pragma unroll
        for (int k = 0; k < KS16; ++k) {
          const bf8_t rh_ = *reinterpret_cast<const bf8_t*>(bh + bfo + 32 * k);
          const bf8_t rl_ = *reinterpret_cast<const bf8_t*>(bl + bfo + 32 * k);
          const bf8_t ih_ = *reinterpret_cast<const bf8_t*>(bh + bfo + n_padk + 32 * k);
          const bf8_t il_ = *reinterpret_cast<const bf8_t*>(bl + bfo + n_padk + 32 * k);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const u32x4* av = aq + (int64_t)(b * KS16 + k) * 64 * 4;
            const u32x4 u0 = av[0], u1 = av[1], u2 = av[2], u3 = av[3];
            const bf8_t yrh = __builtin_bit_cast(bf8_t, u0), yrl = __builtin_bit_cast(bf8_t, u1);
            const bf8_t yih = __builtin_bit_cast(bf8_t, u2), yil = __builtin_bit_cast(bf8_t, u3);
            const bf8_t nih = __builtin_bit_cast(bf8_t, u2 ^ sgn);
            const bf8_t nil = __builtin_bit_cast(bf8_t, u3 ^ sgn);
            // Re dI = Yr Re dE - Yi Im dE, Im dI = Yi Re dE + Yr Im dE, each
            // product as hi*lo + lo*hi + hi*hi
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrl, rh_, ar[b], 0, 0, 0);
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, rl_, ar[b], 0, 0, 0);
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, rh_, ar[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yil, rh_, ai[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yih, rl_, ai[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yih, rh_, ai[b], 0, 0, 0);
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, ih_, ar[b], 0, 0, 0);
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, il_, ar[b], 0, 0, 0);
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, ih_, ar[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrl, ih_, ai[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, il_, ai[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yrh, ih_, ai[b], 0, 0, 0);
          }
        }
      } else {
#pragma unroll 4
        for (int k = 0; k < KH; ++k) {
          const float br = Bf[k * 4 * kT], bi = Bf[(k * 4 + n_pad) * kT];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const float2 av = ap[(int64_t)(b * KH + k) * 64];
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, br, ar[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, br, ai[b], 0, 0, 0);
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av.y, bi, ar[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bi, ai[b], 0, 0, 0);
          }
        }
      }
      // injections of my machines (the matrix cores, as above)
      f32x4 aj[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        aj[b] = f32x4{0.f, 0.f, 0.f, 0.f};
        aj[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ainj[b][0], own0 ? sx0 : 0.0f, aj[b], 0, 0, 0);
        if (P > 4)  // uniform
          aj[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ainj[b][1], own1 ? sx1 : 0.0f, aj[b], 0, 0, 0);
      }
      wave_lds_sync();  // the tile is read: the next stage may overwrite it
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        int mo = K.at(mach(q), 0);
        asm volatile("" : "+v"(mo));
        const float4 c = *reinterpret_cast<const float4*>(S.cst + mo);      // C0 S0 I0R I0I
        const float4 e = *reinterpret_cast<const float4*>(S.cst + mo + 4);  // RES DMP INV2H -
        const float dIr = ar[q >> 2][q & 3], dIi = ai[q >> 2][q & 3];
        const float dpe = dEr[q] * c.z + dEi[q] * c.w + (c.x + dEr[q]) * dIr + (c.y + dEi[q]) * dIi;
        const float kd = wb * sw_[q];
        const float kw = (e.x - dpe - e.y * sw_[q] + aj[q >> 2][q & 3]) * e.z;
        ad[q] += wgt * kd;
        aw[q] += wgt * kw;
        if (sg < 3) {
          sd_[q] = yd[q] + hn * kd;
          sw_[q] = yw[q] + hn * kw;
        }
      }
      const float kx0 = -th0 * sx0 + sg0 * wa, kx1 = -th1 * sx1 + sg1 * wc;
      ax0 += wgt * kx0;
      ax1 += wgt * kx1;
      if (sg < 3) {
        sx0 = x0 + hn * kx0;
        sx1 = x1 + hn * kx1;
      }
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      yd[q] += dt6 * ad[q];
      yw[q] += dt6 * aw[q];
    }
    x0 += dt6 * ax0;
    x1 += dt6 * ax1;
    if (a.recenter) {
      // the mean angle of trajectory t's machines (lanes t, t + 16, t + 32,
      // t + 48 hold them), summed in that order by each of the four lanes
      float part = 0.0f;
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (mach(q) < n) part += yd[q];
      float sum = __shfl(part, t, 64);
      sum += __shfl(part, t + 16, 64);
      sum += __shfl(part, t + 32, 64);
      sum += __shfl(part, t + 48, 64);
      const float ref = sum * inv_n;
      coff += (double)ref;
#pragma unroll
      for (int q = 0; q < kQ; ++q) yd[q] -= ref;
    }
    w00 = w02; w01 = n01; w02 = n02;
    w10 = w12; w11 = n11; w12 = n12;
    emit(s + 1);
  }

  if (a.state) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      a.state[sbase + q * 64] = yd[q];
      a.state[sbase + (kQ + q) * 64] = yw[q];
    }
    a.state[sbase + (2 * kQ) * 64] = x0;
    a.state[sbase + (2 * kQ + 1) * 64] = x1;
    store_offset(a.state, sbase + (2 * kQ + 2) * 64, sbase + (2 * kQ + 3) * 64, coff);
  }
  if (a.s_end == a.S) {  // uniform over the workgroup
    bool bad = (own0 && !isfinite(x0)) || (own1 && !isfinite(x1)) || !isfinite(coff);
#pragma unroll
    for (int q = 0; q < kQ; ++q)
      bad |= mach(q) < n && (!isfinite(yd[q]) || !isfinite(yw[q]));
    if (g == 0) S.bad[wv * kT + t] = 0;
    __syncthreads();
    if (bad) S.bad[wv * kT + t] = 1;
    __syncthreads();
    if (g == 0 && valid && S.bad[wv * kT + t] != 0) {
      atomicAdd(a.nonfinite, 1ULL);
      atomicMin(a.first_bad, (long long)traj);
    }
  }
}

}  // namespace fmc
