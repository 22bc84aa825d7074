// fmc_runtime.hip -- host runtime behind the C ABI (include/fmc.h): argument
// validation, device memory of a context, scenario staging, variant choice,
// time chunking and the launch sequence of the method (Alg. 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fmc.h"
#include "fmc_internal.hpp"
#include "fmc_runtime.hpp"
#include "k_variants.hpp"

namespace fmc {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------------------
// Variant table: the lane integrator compiled for (NG, PM) pairs.
// ---------------------------------------------------------------------------
static const std::vector<VariantInfo>& lane_table() {
  static const std::vector<VariantInfo> t = [] {
    std::vector<VariantInfo> v;
    int id = 0;
#define FMC_X(NG, PM, L, WPB) v.push_back(VariantInfo{id++, NG, PM, L, WPB});
    FMC_VARIANTS(FMC_X)
#undef FMC_X
    return v;
  }();
  return t;
}

int n_variants() { return (int)lane_table().size(); }
const VariantInfo& variant(int i) { return lane_table()[i]; }

// Choice used when no tuned one is cached.  A lanes-per-trajectory variant
// with one machine per lane (L >= NG >= n) and at most as many padding
// machines as real ones comes first: the fewest padding machines, then four
// waves per workgroup (measured on the 10-machine
// workload at N = 1e4: L = 10 x 4 waves 9.9 ms per FP64 pass, the other
// L = 10 shapes 12.3-12.7, L = 16 17-23, two machines per lane 11.9, one
// trajectory per lane 102).  Otherwise a cost model: per-step work of one
// workgroup-wave times the number of waves that run back to back on the
// busiest SIMD (1024 SIMDs, occupancy ignored), plus a padding penalty.
int choose_variant(int n, int P, int64_t N) {
  int best = -1;
  for (const auto& v : lane_table()) {
    if (v.L == 1 || v.G() != 1 || v.NG < n || v.NG > 2 * n || v.PM < std::max(P, 1)) continue;
    if (best < 0) {
      best = v.id;
      continue;
    }
    const VariantInfo& b = lane_table()[best];
    const bool better = v.NG < b.NG || (v.NG == b.NG && v.L < b.L) ||
                        (v.NG == b.NG && v.L == b.L && v.WPB == 4 && b.WPB != 4);
    if (better) best = v.id;
  }
  if (best >= 0) return best;
  double best_cost = 0.0;
  for (const auto& v : lane_table()) {
    if (v.NG < n || v.PM < std::max(P, 1)) continue;
    const double G = v.G();
    const double lane_work = G * v.NG * 4.0 + G * 40.0 + v.PM * 4.0 + (v.L > 1 ? v.NG * 2.0 : 0.0);
    const double waves = std::ceil((double)N * v.L / 64.0);
    const double rounds = std::ceil(waves / 1024.0);
    // a wave alone on its SIMD runs about 4x slower than the issue rate
    const double lat = waves < 2048.0 ? 4.0 : 1.0;
    const double cost = lane_work * rounds * lat;
    if (best < 0 || cost < best_cost) {
      best = v.id;
      best_cost = cost;
    }
  }
  return best;
}

std::string tune_key(int n, int P, int64_t N, int precision) {
  int nb = 0;
  while (((int64_t)1 << (nb + 1)) <= N) ++nb;  // floor(log2 N)
  return std::to_string(n) + "/" + std::to_string(P) + "/" + std::to_string(nb) + "/" +
         std::to_string(precision);
}

int pick_variant(Context* c, int n, int P, int64_t N, int precision) {
  auto it = c->tuned.find(tune_key(n, P, N, precision));
  if (it != c->tuned.end() && it->second >= 0 && it->second < n_variants()) {
    const VariantInfo& v = variant(it->second);
    if (v.NG >= n && v.PM >= P) return it->second;
  }
  return choose_variant(n, P, N);
}

// Tuner cache file: one {"key": ..., "variant": ...} object per line.
static void load_tune_cache(Context* c) {
  const char* path = std::getenv("FMC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char key[256];
    int vid = -1;
    if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"variant\": %d", key, &vid) == 2) c->tuned[key] = vid;
  }
  std::fclose(f);
}

static void save_tune_entry(const std::string& key, int vid) {
  const char* path = std::getenv("FMC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"variant\": %d}\n", key.c_str(), vid);
  std::fclose(f);
}

// ---------------------------------------------------------------------------
// Device memory of a context: named, grow-only buffers within the budget.
// ---------------------------------------------------------------------------
int Context::ensure(const char* name, size_t bytes, void** out) {
  bytes = std::max<size_t>(bytes, 256);
  bytes = (bytes + 255) & ~size_t(255);
  DevBuf& b = bufs[name];
  if (b.cap >= bytes) {
    *out = b.p;
    return FMC_OK;
  }
  const size_t new_held = held - b.cap + bytes;
  if (new_held > budget)
    return fail(FMC_ENOMEM, std::string("HBM budget exceeded allocating ") + name + " (" +
                                std::to_string(bytes) + " bytes, budget " +
                                std::to_string(budget) + ")");
  if (b.p) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
    (void)hipFree(b.p);
    held -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMC_ENOMEM, std::string("hipMalloc failed for ") + name + ": " + hipGetErrorString(e));
  }
  b.p = p;
  b.cap = bytes;
  held += bytes;
  peak = std::max(peak, held);
  ++alloc_gen;
  *out = p;
  return FMC_OK;
}

int Context::host_stage(const char* name, size_t bytes, void** out) {
  bytes = std::max<size_t>(bytes, 256);
  DevBuf& b = pinned[name];
  if (b.cap < bytes) {
    if (b.p) {
      hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
      (void)hipHostFree(b.p);
      b.p = nullptr;
      b.cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FMC_ENOMEM, std::string("hipHostMalloc failed for ") + name);
    }
    b.p = p;
    b.cap = bytes;
  }
  *out = b.p;
  return FMC_OK;
}

void Context::release_all() {
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  bufs.clear();
  for (auto& kv : pinned)
    if (kv.second.p) (void)hipHostFree(kv.second.p);
  pinned.clear();
  held = 0;
}

int Stager::upload(Context* c, const char* name, hipStream_t st) {
  if (bytes.empty()) return FMC_OK;
  if (!st) st = c->stream;
  void *d = nullptr, *h = nullptr;
  int rc = c->ensure(name, bytes.size(), &d);
  if (rc) return rc;
  if ((rc = c->host_stage(name, bytes.size(), &h))) return rc;
  std::memcpy(h, bytes.data(), bytes.size());
  hipError_t e = hipMemcpyAsync(d, h, bytes.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  for (auto& f : fix) *f.second = (unsigned char*)d + f.first;
  return FMC_OK;
}

static int check_network(const fmc_network* net) {
  if (!net) return fail(FMC_EINVAL, "network is NULL");
  if (net->n_bus < 1 || net->n_gen < 1 || net->n_branch < 0)
    return fail(FMC_EINVAL, "network sizes must be n_bus >= 1, n_gen >= 1, n_branch >= 0");
  if ((net->n_branch > 0 && (!net->br_from || !net->br_to || !net->br_r || !net->br_x)) ||
      !net->gen_bus || !net->gen_xdp)
    return fail(FMC_EINVAL, "network arrays missing");
  for (int k = 0; k < net->n_branch; ++k) {
    const int f = net->br_from[k], t = net->br_to[k];
    if (f < 0 || f >= net->n_bus || t < 0 || t >= net->n_bus || f == t)
      return fail(FMC_EINVAL, "branch " + std::to_string(k) + " has invalid end buses");
  }
  for (int g = 0; g < net->n_gen; ++g) {
    if (net->gen_bus[g] < 0 || net->gen_bus[g] >= net->n_bus)
      return fail(FMC_EINVAL, "generator " + std::to_string(g) + " bus out of range");
    if (!(net->gen_xdp[g] > 0.0)) return fail(FMC_EINVAL, "X'd must be positive");
  }
  return FMC_OK;
}

// Reduce a network on the device into Yd (double2 [n_gen^2]); status to *st_dev.
int kron_on_device(Context* c, const fmc_network* net, double2* Yd, int* st_dev, const char* tag) {
  int rc = check_network(net);
  if (rc) return rc;
  Stager sg;
  NetDev nd{};
  nd.n_bus = net->n_bus;
  nd.n_branch = net->n_branch;
  nd.n_gen = net->n_gen;
  sg.add(net->br_from, net->n_branch, &nd.from);
  sg.add(net->br_to, net->n_branch, &nd.to);
  sg.add(net->br_r, net->n_branch, &nd.r);
  sg.add(net->br_x, net->n_branch, &nd.x);
  sg.add(net->br_b, net->n_branch, &nd.b);
  sg.add(net->load_g, net->n_bus, &nd.lg);
  sg.add(net->load_b, net->n_bus, &nd.lb);
  sg.add(net->gen_bus, net->n_gen, &nd.gen_bus);
  sg.add(net->gen_xdp, net->n_gen, &nd.xdp);
  if ((rc = sg.upload(c, tag))) return rc;
  void* work = nullptr;
  const size_t wbytes = kron_work_bytes(net->n_bus, net->n_gen);
  if ((rc = c->ensure("kron_work", wbytes, &work))) return rc;
  hipError_t e = launch_kron(nd, (double2*)work, Yd, st_dev, c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, std::string("kron launch: ") + hipGetErrorString(e));
  return FMC_OK;
}

int validate(const fmc_system* sys, const fmc_disturbance* dist, const fmc_params* par,
             int64_t* S_out) {
  if (!sys || !dist || !par) return fail(FMC_EINVAL, "NULL system, disturbance or params");
  if (!(par->dt > 0.0) || !(par->T > 0.0)) return fail(FMC_EINVAL, "T and dt must be positive");
  const double sd = par->T / par->dt;
  const int64_t S = (int64_t)std::llround(sd);
  if (S < 1 || std::fabs((double)S * par->dt - par->T) > 1e-9 * par->T)
    return fail(FMC_EINVAL, "T/dt must be an integer number of steps");
  if (par->K < 1) return fail(FMC_EINVAL, "K must be >= 1");
  if (par->N < 2) return fail(FMC_EINVAL, "N must be >= 2");
  if (par->ddof < 0 || par->ddof >= par->N) return fail(FMC_EINVAL, "ddof must be in [0, N)");
  if (par->basis != FMC_BASIS_PAPER && par->basis != FMC_BASIS_EIGEN && par->basis != FMC_BASIS_EM)
    return fail(FMC_EINVAL, "unknown basis");
  if (par->basis == FMC_BASIS_EM && par->K != S)
    return fail(FMC_EINVAL, "the EM basis needs K = S (one normal per step and process)");
  if (par->sampler != FMC_LHS && par->sampler != FMC_SRS && par->sampler != FMC_LHS_DECOR)
    return fail(FMC_EINVAL, "unknown sampler");
  if (par->integrator != FMC_RK4 && par->integrator != FMC_TRAP)
    return fail(FMC_EINVAL, "unknown integrator");
  if (par->integrator == FMC_TRAP) {
    if (par->precision != FMC_F64 || sys->model != FMC_CLASSICAL)
      return fail(FMC_EINVAL, "the implicit trapezoid runs in FP64 on classical machines");
    if (sys->n_gen > kTrapMaxGen || dist->n_proc > 8)
      return fail(FMC_EINVAL, "the implicit trapezoid takes at most 16 machines and 8 processes");
  }
  if (par->precision < FMC_F64 || par->precision > FMC_BF16X3)
    return fail(FMC_EINVAL, "unknown precision");
  const int n = sys->n_gen;
  if (n < 1) return fail(FMC_EINVAL, "n_gen must be >= 1");
  if (sys->model != FMC_CLASSICAL && sys->model != FMC_FLUXDECAY_IEEET1)
    return fail(FMC_EINVAL, "unknown generator model");
  if (sys->model == FMC_FLUXDECAY_IEEET1) {
    if (!sys->model_params) return fail(FMC_EINVAL, "the flux-decay model needs model_params");
    if (par->precision == FMC_F64)
      return fail(FMC_EINVAL, "the flux-decay model integrates in FP32 (FMC_F32 or FMC_BF16X3)");
    if (n > kFdMaxGen) return fail(FMC_EINVAL, "the flux-decay model takes at most 256 machines");
    if (par->variant < -1 || par->variant > 1 || (par->variant == 1 && par->precision != FMC_BF16X3))
      return fail(FMC_EINVAL, "flux-decay variant: -1 or 0 (FP32 network product) or 1 (BF16 x3 "
                              "network product, FMC_BF16X3 only)");
    const int nw = ((n + 15) / 16 + 1) / 2;  // waves of the flux-decay integrator
    if (dist->n_proc > std::min(kFdMaxProc, 4 * nw))
      return fail(FMC_EINVAL, "too many disturbance processes for the flux-decay model (at most "
                              "min(32, 4 ceil(ceil(n/16)/2)))");
    const int n_pad = 16 * ((n + 15) / 16), n_padk = 32 * ((n + 31) / 32);
    if (fd_lds_bytes(n_pad, n_padk, fd_bf16_product(par), dist->n_proc) > kFdMaxLds)
      return fail(FMC_EINVAL, "flux-decay system too large for one workgroup's LDS (reduce the "
                              "machines or the processes)");
    for (int i = 0; i < n; ++i) {
      const double* q = sys->model_params + (int64_t)i * kFdParams;
      for (int k = 0; k < kFdParams; ++k)
        if (!std::isfinite(q[k])) return fail(FMC_EINVAL, "flux-decay parameters must be finite");
      if (!(q[kFdXdp] > 0.0) || !(q[kFdTdo] > 0.0) || !(q[kFdTa] > 0.0) || !(q[kFdTe] > 0.0) ||
          !(q[kFdTf] > 0.0) || q[kFdKa] < 0.0)
        return fail(FMC_EINVAL, "flux-decay parameters: X'd, T'do, TA, TE, TF > 0 and KA >= 0");
    }
  }
  if (sys->event) {
    const fmc_event* ev = sys->event;
    if (sys->model != FMC_CLASSICAL)
      return fail(FMC_EINVAL, "network events run with the classical model");
    const int64_t se = (int64_t)std::llround(ev->t / par->dt);
    if (!(ev->t > 0.0) || se < 1 || se >= S || std::fabs((double)se * par->dt - ev->t) > 1e-9 * par->T)
      return fail(FMC_EINVAL, "the event time must be a whole number of steps in (0, T)");
    if (ev->tripped < -1 || ev->tripped >= n) return fail(FMC_EINVAL, "tripped machine out of range");
    if (!ev->Y_re != !ev->Y_im || !ev->Yinf_re != !ev->Yinf_im)
      return fail(FMC_EINVAL, "event admittances need both real and imaginary parts");
    if (ev->Yinf_re && !sys->infinite_bus)
      return fail(FMC_EINVAL, "a post-event infinite-bus coupling needs an infinite-bus system");
    if (!ev->Y_re && (ev->tripped < 0 || sys->Y_re || !sys->net))
      return fail(FMC_EINVAL, "an event needs its admittance, or a tripped machine of a network system");
    if (ev->Y_re && ev->tripped >= 0) {
      const int g = ev->tripped;
      for (int k = 0; k < n; ++k)
        if (ev->Y_re[g * n + k] != 0.0 || ev->Y_im[g * n + k] != 0.0 || ev->Y_re[k * n + g] != 0.0 ||
            ev->Y_im[k * n + g] != 0.0)
          return fail(FMC_EINVAL, "the tripped machine's row and column of the event admittance must be zero");
      if (ev->Yinf_re && (ev->Yinf_re[g] != 0.0 || ev->Yinf_im[g] != 0.0))
        return fail(FMC_EINVAL, "the tripped machine's infinite-bus coupling must be zero");
    }
  }
  if (!sys->H || !sys->D || !sys->E) return fail(FMC_EINVAL, "H, D and E are required");
  for (int i = 0; i < n; ++i) {
    if (!(sys->H[i] > 0.0)) return fail(FMC_EINVAL, "H must be positive");
    if (!std::isfinite(sys->D[i]) || !std::isfinite(sys->E[i])) return fail(FMC_EINVAL, "D, E must be finite");
  }
  if (!sys->delta0 && !(sys->Pm && sys->infinite_bus))
    return fail(FMC_EINVAL, "delta0 is required unless Pm is given on an infinite-bus system");
  if (!sys->Y_re && !sys->net) return fail(FMC_EINVAL, "give Y_re/Y_im or a network");
  if (sys->Y_re && !sys->Y_im) return fail(FMC_EINVAL, "Y_im missing");
  if (sys->net && !sys->Y_re && sys->net->n_gen != n) return fail(FMC_EINVAL, "network n_gen differs from system n_gen");
  if (sys->infinite_bus && (!sys->Yinf_re || !sys->Yinf_im))
    return fail(FMC_EINVAL, "infinite-bus coupling Yinf missing");
  if (dist->n_proc < 1) return fail(FMC_EINVAL, "at least one disturbance process is required");
  if (!dist->gen || !dist->theta || (!dist->sigma && !dist->sigma_mat))
    return fail(FMC_EINVAL, "disturbance arrays missing");
  for (int p = 0; p < dist->n_proc; ++p) {
    if (dist->gen[p] < 0 || dist->gen[p] >= n) return fail(FMC_EINVAL, "disturbance machine index out of range");
    if (!(dist->theta[p] >= 0.0)) return fail(FMC_EINVAL, "theta must be >= 0");
    if (!dist->sigma_mat && !(dist->sigma[p] >= 0.0)) return fail(FMC_EINVAL, "sigma must be >= 0");
  }
  if (dist->sigma_mat)
    for (int q = 0; q < dist->n_proc * dist->n_proc; ++q)
      if (!std::isfinite(dist->sigma_mat[q])) return fail(FMC_EINVAL, "sigma_mat must be finite");
  if (dist->calculus != FMC_ITO && dist->calculus != FMC_STRATONOVICH)
    return fail(FMC_EINVAL, "calculus must be FMC_ITO or FMC_STRATONOVICH");
  if (dist->proc) {
    if (par->integrator != FMC_RK4 || sys->model != FMC_CLASSICAL)
      return fail(FMC_EINVAL, "general Ito processes run with FMC_RK4 on classical machines");
    for (int p = 0; p < dist->n_proc; ++p) {
      const fmc_process& q = dist->proc[p];
      const double v[11] = {q.a, q.b, q.theta, q.mu[0], q.mu[1], q.mu[2],
                            q.sg[0], q.sg[1], q.sg[2], q.gain, q.ref};
      for (double x : v)
        if (!std::isfinite(x)) return fail(FMC_EINVAL, "process parameters must be finite");
      if (q.kind < FMC_PROC_OU || q.kind > FMC_PROC_POLY) return fail(FMC_EINVAL, "unknown process kind");
      if (q.kind >= FMC_PROC_GAUSS && q.kind <= FMC_PROC_LAPLACE && !(q.theta >= 0.0))
        return fail(FMC_EINVAL, "a Table I process needs theta >= 0");
      if ((q.kind == FMC_PROC_BETA || q.kind == FMC_PROC_GAMMA) && !(q.a > 0.0 && q.b > 0.0))
        return fail(FMC_EINVAL, "the Beta and Gamma rows need a, b > 0");
      if ((q.kind == FMC_PROC_GAUSS || q.kind == FMC_PROC_LAPLACE) && !(q.b >= 0.0))
        return fail(FMC_EINVAL, "the Gaussian and Laplace rows need b >= 0");
      if (dist->sigma_mat && q.kind != FMC_PROC_OU)
        return fail(FMC_EINVAL, "a state-dependent diffusion has no column in sigma_mat");
    }
  }
  if (par->sampler == FMC_LHS_DECOR && !par->zeta_in) {
    const int64_t M = (int64_t)dist->n_proc * par->K;
    if (M > kDecorMaxM || par->N <= M || par->N > kDecorMaxN)
      return fail(FMC_EINVAL, "FMC_LHS_DECOR needs n_proc*K <= 1024 and n_proc*K < N < 2^31");
  }
  *S_out = S;
  return FMC_OK;
}

// Stage the machine/disturbance data and run setup -> canonical coefficients.
int stage_scenario(Context* c, const fmc_system* sys, const fmc_disturbance* dist,
                   const char* tag, double** canon_out, int32_t** gen_out, int** status_out) {
  const int n = sys->n_gen, P = dist->n_proc;
  int rc;
  Stager sg;
  SetupDev sd{};
  sd.n = n;
  sd.P = P;
  std::vector<double2> Yh, Yinfh;
  if (sys->Y_re) {
    Yh.resize((size_t)n * n);
    for (size_t q = 0; q < Yh.size(); ++q) Yh[q] = make_double2(sys->Y_re[q], sys->Y_im[q]);
  }
  if (sys->infinite_bus) {
    Yinfh.resize(n);
    for (int i = 0; i < n; ++i) Yinfh[i] = make_double2(sys->Yinf_re[i], sys->Yinf_im[i]);
  }
  const int32_t* gen_d = nullptr;
  sg.add(sys->H, n, &sd.H);
  sg.add(sys->D, n, &sd.D);
  sg.add(sys->E, n, &sd.E);
  sg.add(sys->delta0, n, &sd.delta0);
  sg.add(sys->Pm, n, &sd.Pm);
  sg.add(Yh.empty() ? nullptr : Yh.data(), Yh.size(), &sd.Y);
  sg.add(Yinfh.empty() ? nullptr : Yinfh.data(), Yinfh.size(), &sd.Yinf);
  sg.add(dist->theta, P, &sd.theta);
  sg.add(dist->sigma, P, &sd.sigma);
  sg.add(dist->xi0, P, &sd.xi0);
  sg.add(dist->gen, P, &gen_d);
  std::string nm = std::string("stage_") + tag;
  if ((rc = sg.upload(c, nm.c_str()))) return rc;
  sd.inf_bus = sys->infinite_bus ? 1 : 0;
  sd.V_inf = sys->V_inf;
  void *status = nullptr, *work = nullptr, *canon = nullptr, *ybuf = nullptr;
  if ((rc = c->ensure((std::string("status_") + tag).c_str(), 64, &status))) return rc;
  if ((rc = c->ensure((std::string("setup_work_") + tag).c_str(),
                      (size_t)(3 * n * n + 8 * n + 64) * sizeof(double), &work)))
    return rc;
  CanonLayout L{n, P};
  if ((rc = c->ensure((std::string("canon_") + tag).c_str(), (size_t)L.size() * sizeof(double), &canon)))
    return rc;
  hipError_t e = launch_fill_i64((int64_t*)status, 0, 8, c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  if (!sd.Y) {
    if ((rc = c->ensure((std::string("yred_") + tag).c_str(), (size_t)n * n * sizeof(double2), &ybuf)))
      return rc;
    if ((rc = kron_on_device(c, sys->net, (double2*)ybuf, (int*)status + 1))) return rc;
    sd.Y = (const double2*)ybuf;
  }
  sd.work = (double*)work;
  sd.canon = (double*)canon;
  sd.status = (int*)status;
  e = launch_setup(sd, c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, std::string("setup launch: ") + hipGetErrorString(e));
  *canon_out = (double*)canon;
  *gen_out = (int32_t*)gen_d;
  *status_out = (int*)status;
  return FMC_OK;
}

int64_t auto_chunk(int64_t S, int P, int64_t N, int bytes_per) {
  const double target = 96.0 * 1024 * 1024;  // keep a chunk of paths in the 256 MB last-level cache
  const double col = (double)P * (double)N * bytes_per;
  int64_t cols = (int64_t)(target / col);
  int64_t sc = std::max<int64_t>(8, (cols - 1) / 2);
  return std::min<int64_t>(sc, S);
}

int mix_design(Context* c, const fmc_disturbance* dist, int32_t K, int64_t N, const double** zeta,
               hipStream_t st) {
  const int P = dist->n_proc;
  void *s_d = nullptr, *out = nullptr, *h = nullptr;
  int rc;
  if ((rc = c->ensure("sigma_mat", (size_t)P * P * sizeof(double), &s_d))) return rc;
  if ((rc = c->ensure("zeta_mix", (size_t)P * K * N * sizeof(double), &out))) return rc;
  if ((rc = c->host_stage("sigma_mat", (size_t)P * P * sizeof(double), &h))) return rc;
  std::memcpy(h, dist->sigma_mat, (size_t)P * P * sizeof(double));
  hipError_t e = hipMemcpyAsync(s_d, h, (size_t)P * P * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_mix_design((const double*)s_d, P, K, N, *zeta, (double*)out, st);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  *zeta = (const double*)out;
  return FMC_OK;
}

}  // namespace fmc

using namespace fmc;

extern "C" {

int fmc_abi_version(void) { return FMC_ABI_VERSION; }

const char* fmc_last_error(void) { return g_err.c_str(); }

int fmc_context_create(int device, size_t hbm_budget, void* stream, fmc_context** out) {
  if (!out) return fail(FMC_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(FMC_EDEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(FMC_EDEVICE, "device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  Context* c = new Context();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->budget = hbm_budget ? hbm_budget : (size_t)(0.9 * (double)free_b);
  e = rrf_scratch_init(device);  // the allocation-free entry point's scratch
  if (e != hipSuccess) {
    delete c;
    return fail(FMC_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  }
  for (auto& ev : c->ev) {
    if (hipEventCreate(&ev) != hipSuccess) {
      delete c;
      return fail(FMC_EDEVICE, "hipEventCreate failed");
    }
  }
  load_tune_cache(c);
  *out = reinterpret_cast<fmc_context*>(c);
  return FMC_OK;
}

int fmc_context_destroy(fmc_context* ctx) {
  if (!ctx) return FMC_OK;
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  serve_shutdown(c);
  (void)hipStreamSynchronize(c->stream);
  if (c->bstream) (void)hipStreamSynchronize(c->bstream);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.second);
  c->graphs.clear();
  if (c->bstream) (void)hipStreamDestroy(c->bstream);
  if (c->gstream) {
    (void)hipStreamSynchronize(c->gstream);
    (void)hipStreamDestroy(c->gstream);
  }
  for (auto& e : c->gev)
    if (e) (void)hipEventDestroy(e);
  for (auto& s : c->cstream)
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (auto& e : c->cev)
    if (e) (void)hipEventDestroy(e);
  c->release_all();
  for (auto& ev : c->ev) (void)hipEventDestroy(ev);
  delete c;
  return FMC_OK;
}

int fmc_set_stream(fmc_context* ctx, void* stream) {
  if (!ctx) return fail(FMC_EINVAL, "ctx is NULL");
  reinterpret_cast<Context*>(ctx)->stream = (hipStream_t)stream;
  return FMC_OK;
}

int fmc_kron_reduce(fmc_context* ctx, const fmc_network* net, double* Y_re, double* Y_im) {
  if (!ctx || !Y_re || !Y_im) return fail(FMC_EINVAL, "NULL argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  int rc = check_network(net);
  if (rc) return rc;
  (void)hipSetDevice(c->device);
  void *yd = nullptr, *st = nullptr;
  const int ng = net->n_gen;
  if ((rc = c->ensure("kr_y", (size_t)ng * ng * sizeof(double2), &yd))) return rc;
  if ((rc = c->ensure("kr_status", 64, &st))) return rc;
  if ((rc = kron_on_device(c, net, (double2*)yd, (int*)st))) return rc;
  std::vector<double2> h((size_t)ng * ng);
  int status = 0;
  hipError_t e = hipMemcpyAsync(h.data(), yd, h.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&status, st, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  if (status != 0) return fail(FMC_EINVAL, "network reduction failed (singular Y_BB)");
  for (size_t q = 0; q < h.size(); ++q) {
    Y_re[q] = h[q].x;
    Y_im[q] = h[q].y;
  }
  return FMC_OK;
}

static int decorrelate_and_check(Context* c, int32_t M, int64_t N, double* zeta, int32_t* strata,
                                 const int32_t* lhs_strata);


int fmc_lhs(fmc_context* ctx, uint64_t seed, int32_t M, int64_t N, int32_t sampler,
            int32_t* strata, double* zeta) {
  if (!ctx || !zeta) return fail(FMC_EINVAL, "NULL argument");
  if (M < 1 || N < 1) return fail(FMC_EINVAL, "M and N must be >= 1");
  if (sampler != FMC_LHS && sampler != FMC_SRS && sampler != FMC_LHS_DECOR)
    return fail(FMC_EINVAL, "unknown sampler");
  if (N > (int64_t)1 << 40) return fail(FMC_EINVAL, "N too large");
  if (sampler == FMC_LHS_DECOR && (M > kDecorMaxM || N <= M || N > kDecorMaxN))
    return fail(FMC_EINVAL, "FMC_LHS_DECOR needs M <= 1024 and M < N < 2^31");
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  int32_t* lhs_strata = strata;
  if (sampler == FMC_LHS_DECOR && !lhs_strata) {
    void* p = nullptr;
    int rc = c->ensure("dc_strata", (size_t)M * N * sizeof(int32_t), &p);
    if (rc) return rc;
    lhs_strata = (int32_t*)p;
  }
  hipError_t e = launch_lhs(seed, M, N, sampler == FMC_SRS ? FMC_SRS : FMC_LHS, lhs_strata, zeta,
                            c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  if (sampler != FMC_LHS_DECOR) return FMC_OK;
  return decorrelate_and_check(c, M, N, zeta, strata, lhs_strata);
}

int fmc_rrf_rms(fmc_context* ctx, const double* traj, int64_t n, int64_t S, int32_t V,
                const double* w, double dt, double* rrf) {
  if (!ctx || !w || (n > 0 && (!traj || !rrf))) return fail(FMC_EINVAL, "NULL argument");
  if (n < 0 || n > INT32_MAX || S < 1 || V < 1 || V > 2048 || !(dt > 0.0))
    return fail(FMC_EINVAL, "need 0 <= n < 2^31, S >= 1, 1 <= V <= 2048, dt > 0");
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  void *wd = nullptr, *h = nullptr;
  int rc;
  if ((rc = c->ensure("rrf_w", (size_t)V * sizeof(double), &wd))) return rc;
  if ((rc = c->host_stage("rrf_w", (size_t)V * sizeof(double), &h))) return rc;
  std::memcpy(h, w, (size_t)V * sizeof(double));
  hipError_t e = hipMemcpyAsync(wd, h, (size_t)V * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_rrf_rms(traj, n, S, V, (const double*)wd, dt, rrf, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  return FMC_OK;
}

int fmc_rrf_rms_noalloc(fmc_context* ctx, const double* traj, int64_t n, int64_t S, int32_t V,
                        const double* w, double dt, double* rrf) {
  if (!ctx || !w || (n > 0 && (!traj || !rrf))) return fail(FMC_EINVAL, "NULL argument");
  if (n < 0 || n > INT32_MAX || S < 1 || V < 1 || !(dt > 0.0))
    return fail(FMC_EINVAL, "need 0 <= n < 2^31, S >= 1, V >= 1, dt > 0");
  if (V > kRrfStaticMaxV)
    return fail(FMC_EINVAL, "V = " + std::to_string(V) + " exceeds the static scratch (" +
                                std::to_string(kRrfStaticMaxV) + " weights)");
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  double* wd = rrf_scratch(c->device);
  if (!wd) return fail(FMC_EDEVICE, "no scratch address for this device");
  hipError_t e = hipMemcpyAsync(wd, w, (size_t)V * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_rrf_rms(traj, n, S, V, wd, dt, rrf, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  return FMC_OK;
}

int fmc_lhs_decorrelate(fmc_context* ctx, int32_t M, int64_t N, double* zeta, int32_t* strata) {
  if (!ctx || !zeta) return fail(FMC_EINVAL, "NULL argument");
  if (M < 1 || M > kDecorMaxM || N <= M || N > kDecorMaxN)
    return fail(FMC_EINVAL, "correlation reduction needs M <= 1024 and M < N < 2^31");
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  return decorrelate_and_check(c, M, N, zeta, strata, nullptr);
}

// The reduction on the context's stream, then a wait for its status.
static int decorrelate_and_check(Context* c, int32_t M, int64_t N, double* zeta, int32_t* strata,
                                 const int32_t* lhs_strata) {
  int32_t* st_d = nullptr;
  int rc = decorrelate_design(c, M, N, zeta, strata, lhs_strata, &st_d, c->stream);
  if (rc) return rc;
  void* h = nullptr;
  if ((rc = c->host_stage("dc_status", 64, &h))) return rc;
  hipError_t e = hipMemcpyAsync(h, st_d, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  if (*(int32_t*)h != 0)
    return fail(FMC_EINVAL, "the design's sample covariance is not positive definite (design left unchanged)");
  return FMC_OK;
}

int fmc_basis(fmc_context* ctx, int32_t basis, int32_t K, int64_t S, double T, double* phi) {
  if (!ctx || !phi) return fail(FMC_EINVAL, "NULL argument");
  if (K < 1 || S < 1 || !(T > 0.0)) return fail(FMC_EINVAL, "K >= 1, S >= 1, T > 0 required");
  if (basis != FMC_BASIS_PAPER && basis != FMC_BASIS_EIGEN && basis != FMC_BASIS_EM)
    return fail(FMC_EINVAL, "unknown basis");
  if (basis == FMC_BASIS_EM && K > S) return fail(FMC_EINVAL, "the EM basis has at most S rows");
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  hipError_t e = launch_basis(basis, K, S, T, phi, c->stream);
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  return FMC_OK;
}

int fmc_kle_paths(fmc_context* ctx, int32_t precision, int32_t P, int32_t K, int64_t N, int64_t C,
                  int64_t c0, const double* zeta, const double* phi, int64_t phi_ld, void* w) {
  if (!ctx || !zeta || !phi || !w) return fail(FMC_EINVAL, "NULL argument");
  if (P < 1 || K < 1 || N < 1 || C < 1 || c0 < 0 || phi_ld < c0 + C)
    return fail(FMC_EINVAL, "bad sizes (need P, K, N, C >= 1 and phi_ld >= c0 + C)");
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  hipError_t e;
  if (precision == FMC_F64)
    e = launch_kle_f64(zeta, phi, phi_ld, P, K, N, C, c0, (double*)w, c->stream);
  else if (precision == FMC_F32)
    e = launch_kle_f64_to_f32(zeta, phi, phi_ld, P, K, N, C, c0, (float*)w, c->stream);
  else if (precision == FMC_BF16X3) {
    // split the operands once (the columns c0..c0+C-1 of phi only), then contract
    const int Kp = kle_kp(K);
    void *pp = nullptr, *zz = nullptr;
    int rc;
    if ((rc = c->ensure("kp_phi16", (size_t)2 * C * Kp * 2, &pp))) return rc;
    if ((rc = c->ensure("kp_zeta16", (size_t)2 * P * N * Kp * 2, &zz))) return rc;
    void* pl = (char*)pp + (size_t)C * Kp * 2;
    void* zl = (char*)zz + (size_t)P * N * Kp * 2;
    e = launch_split_bf16(phi + c0, phi_ld, K, C, Kp, 1, 0, 0, pp, pl, c->stream);
    if (e == hipSuccess)
      e = launch_split_bf16(zeta, N, K, N, Kp, P, (int64_t)K * N, N * Kp, zz, zl, c->stream);
    if (e == hipSuccess)
      e = launch_kle_bf16x3_split(pp, pl, Kp, zz, zl, P, N, C, 0, (float*)w, c->stream);
  } else
    return fail(FMC_EINVAL, "unknown precision");
  if (e != hipSuccess) return fail(FMC_EDEVICE, hipGetErrorString(e));
  return FMC_OK;
}

int fmc_autotune(fmc_context* ctx, const fmc_scenario* scen, int32_t* variant_out) {
  if (!ctx || !scen || !scen->sys || !scen->dist || !scen->par || !variant_out)
    return fail(FMC_EINVAL, "NULL argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  int64_t S = 0;
  int rc = validate(scen->sys, scen->dist, scen->par, &S);
  if (rc) return rc;
  if (scen->sys->model != FMC_CLASSICAL)
    return fail(FMC_EINVAL, "the flux-decay model has a single integrator: nothing to tune");
  const int n = scen->sys->n_gen, P = scen->dist->n_proc;
  const int64_t N = scen->par->N;
  const int V = 2 * n + P;
  // Short horizon at the real N, three time chunks long so that the KLE
  // contraction of the next chunk runs beside the integrator as in a full
  // run; the whole run is timed (the merge of a variant's partials counts).
  const int bw = scen->par->precision == FMC_F64 ? 8 : 4;
  const int64_t St = std::min<int64_t>(S, std::max<int64_t>(96, 3 * auto_chunk(S, P, N, bw)));
  fmc_params par = *scen->par;
  par.T = (double)St * par.dt;
  par.time_chunk = 0;
  void *m = nullptr, *v = nullptr;
  if ((rc = c->ensure("tune_mean", (size_t)(St + 1) * V * sizeof(double), &m))) return rc;
  if ((rc = c->ensure("tune_var", (size_t)(St + 1) * V * sizeof(double), &v))) return rc;
  int best = -1;
  double best_t = 0.0;
  // the implicit trapezoid runs on the one-trajectory-per-lane variants only
  // (fmc_run picks among those itself); a choice for it, or for general Ito
  // processes, is returned but not kept for the scenario's shape, whose
  // cached variant serves the OU form
  const bool trap = scen->par->integrator == FMC_TRAP;
  const bool keep = !trap && scen->dist->proc == nullptr;
  for (int id = 0; id < n_variants(); ++id) {
    const VariantInfo& vi = variant(id);
    if (vi.NG < n || vi.PM < P) continue;
    if (trap && (vi.L != 1 || vi.NG > kTrapMaxGen)) continue;
    par.variant = id;
    fmc_report rep;
    fmc_outputs out{};
    out.mean = (double*)m;
    out.var = (double*)v;
    out.mem_kind = FMC_MEM_DEVICE;
    out.report = &rep;
    double t = 0.0;
    for (int rep_i = 0; rep_i < 2; ++rep_i) {  // first run warms caches and allocations
      rc = run_single(c, scen->sys, scen->dist, &par, &out);
      if (rc != FMC_OK && rc != FMC_ENONFINITE) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
      }
      t = rep.t_total_s;
    }
    if (best < 0 || t < best_t) {
      best = id;
      best_t = t;
    }
  }
  if (best < 0) return fail(FMC_EINVAL, "no integrator variant fits the scenario");
  if (keep) {
    const std::string key = tune_key(n, P, N, scen->par->precision);
    c->tuned[key] = best;
    save_tune_entry(key, best);
  }
  *variant_out = best;
  return FMC_OK;
}

int fmc_run(fmc_context* ctx, const fmc_system* sys, const fmc_disturbance* dist,
            const fmc_params* par, fmc_outputs* out) {
  if (!ctx || !out) return fail(FMC_EINVAL, "NULL context or outputs");
  Context* c = reinterpret_cast<Context*>(ctx);
  const int rc = run_single(c, sys, dist, par, out);
  // a failed call may have left copies and kernels in flight that read staging
  // buffers the next call rewrites: drain the streams before returning
  if (rc != FMC_OK && rc != FMC_ENONFINITE) {
    (void)hipStreamSynchronize(c->stream);
    if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  }
  return rc;
}

}  // extern "C"
