// fmc_serve.hip -- served form of the method (continuous batching).
//
// Admission is by HBM footprint: everything a request needs for its whole life
// (its staged inputs, design, basis, one time chunk of KLE paths, integrator
// state, statistics rows, results) is carved from one device arena when it is
// submitted, or the submit is refused (FMC_EBUSY: not now, FMC_ENOMEM: never).
// A server thread advances every admitted request together in ticks: a tick
// rebuilds the next time chunk of KLE paths of each active request and runs
// all their work items in the persistent batched integrator, whose trajectory
// state stays on the device between ticks.  Requests that arrive meanwhile
// join at the next tick; finished ones are merged, copied out and leave, and
// their memory goes back to the arena.
//
// A request's result depends only on the request: its work items and time
// chunks are fixed by its own sizes, so it is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fmc_runtime.hpp"
#include "serve_arena.hpp"

namespace fmc {

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kTickBytes = size_t(16) << 20;  // per-tick upload region (args, items, orders)
constexpr int64_t kMaxItems = 1024;             // work items per request
constexpr int kMaxActive = 256;                 // requests admitted at once
constexpr int64_t kDefaultChunk = 200;          // steps per tick
constexpr int64_t kDefaultChunkFd = 12;         // steps per tick of a flux-decay request
constexpr size_t kAlign = serve::kAlign;

size_t al(size_t x) { return serve::align_up(x); }

struct Request {
  uint64_t ticket = 0;
  fmc_params par{};
  fmc_outputs out{};
  int n = 0, P = 0, K = 0, V = 0;
  int64_t N = 0, S = 0, C = 0, M = 0, Sc = 0;
  int64_t s_prev = 0, s_next = 0;  // steps of the last tick: [s_prev, s_next)
  bool has_Y = false, inf_bus = false;
  int32_t n_bus = 0;
  double f0 = 60.0, V_inf = 0.0;
  // staged inputs (copied at submit; device pointers patched at upload)
  Stager sg;
  SetupDev sd{};
  NetDev nd{};
  const int32_t* gen_d = nullptr;
  // flux-decay request (its own integrator; no batched variant)
  bool fd = false;
  int n_pad = 0, NW = 0;
  const double *E_d = nullptr, *prm_d = nullptr;  // staged E and parameters
  double* fdblk = nullptr;
  float* fdcoef = nullptr;
  float2* fdap = nullptr;
  float* xstate = nullptr;
  // plan
  int vid = -1;
  BatchVariantInfo bv{};
  int64_t tiles = 0, tiles_per_item = 0, n_items = 0;
  double cost_tile = 0.0;
  // arena blocks
  std::vector<std::pair<size_t, size_t>> blocks;
  unsigned char* inbuf = nullptr;
  double *canon = nullptr, *phi = nullptr, *zeta = nullptr, *mean = nullptr, *var = nullptr,
         *work = nullptr;
  double2 *ybuf = nullptr, *kwork = nullptr, *part = nullptr;
  float *coef = nullptr, *w = nullptr, *state = nullptr;
  int* status = nullptr;              // [0] setup, [1] reduction
  unsigned long long* cnt = nullptr;  // non-finite count, smallest bad index
  int64_t footprint = 0;
  // life cycle
  int code = FMC_EAGAIN;  // FMC_EAGAIN while pending, then the final status
  bool cancel = false;
  Clock::time_point t_submit, t_start, t_done;
  size_t pin_status = 0;  // offset of the status readback in the pinned buffer
};

using ReqP = std::shared_ptr<Request>;

// Device sizes of one request, in carve order.
enum { B_IN, B_CANON, B_COEF, B_PHI, B_ZETA, B_W, B_STATE, B_PART, B_MEAN, B_VAR, B_WORK,
       B_YBUF, B_KWORK, B_STATUS, B_FDBLK, B_FDAP, B_XSTATE, B_COUNT };

std::vector<size_t> parts_of(const Request& r) {
  std::vector<size_t> z(B_COUNT, 0);
  z[B_IN] = r.sg.bytes.size();
  z[B_CANON] = (size_t)CanonLayout{r.n, r.P}.size() * 8;
  z[B_PHI] = (size_t)r.K * r.C * 8;
  z[B_ZETA] = (size_t)r.M * r.N * 8;
  z[B_W] = (size_t)(2 * r.Sc + 1) * r.P * r.N * 4;
  if (r.fd) {
    z[B_COEF] = (size_t)FdPack{r.n_pad}.size() * 4;
    z[B_FDBLK] = (size_t)FdLayout{r.n}.size() * 8;
    z[B_FDAP] = fd_bf16_product(&r.par)
                    ? fd_ap16_bytes(r.n_pad, 32 * ((r.n + 31) / 32))
                    : (size_t)(r.n_pad / 16) * (r.n_pad / 4) * 64 * sizeof(float2);
    z[B_STATE] = (size_t)r.tiles * r.NW * 48 * 64 * 4;
    z[B_XSTATE] = (size_t)r.tiles * (kFdMaxProc + kFdOffsetRows) * 16 * 4;
  } else {
    z[B_COEF] = batch_coef_floats(r.bv) * 4;
    z[B_STATE] = batch_state_floats(r.bv, r.tiles) * 4;
  }
  // statistics rows of one chunk: per work item (classical), per tile (flux decay)
  z[B_PART] = (size_t)(r.fd ? r.tiles : r.n_items) * (r.Sc + 1) * r.V * 16;
  z[B_MEAN] = z[B_VAR] = (size_t)(r.S + 1) * r.V * 8;
  z[B_WORK] = (size_t)(3 * r.n * r.n + 8 * r.n + 64) * 8;
  z[B_YBUF] = r.has_Y ? 0 : (size_t)r.n * r.n * 16;
  z[B_KWORK] = r.has_Y ? 0 : kron_work_bytes(r.n_bus, r.n);
  z[B_STATUS] = 64;
  return z;
}

size_t footprint_of(const Request& r) { return serve::footprint(parts_of(r)); }

// Sizes, variant (the smallest batched variant that fits unless one is forced),
// time chunk and work items of a request.
int plan_request(Request& r, const fmc_system* s, const fmc_disturbance* d, const fmc_params* p,
                 int64_t S) {
  r.par = *p;
  r.n = s->n_gen;
  r.P = d->n_proc;
  r.K = p->K;
  r.fd = s->model == FMC_FLUXDECAY_IEEET1;
  r.V = (r.fd ? 6 * r.n : 2 * r.n) + r.P;
  r.N = p->N;
  r.S = S;
  r.C = 2 * S + 1;
  r.M = (int64_t)r.P * r.K;
  r.has_Y = s->Y_re != nullptr;
  r.n_bus = r.has_Y ? 0 : s->net->n_bus;
  r.inf_bus = s->infinite_bus != 0;
  r.V_inf = s->V_inf;
  r.f0 = s->f0_hz > 0.0 ? s->f0_hz : 60.0;
  if (p->precision != FMC_F32 && p->precision != FMC_BF16X3)
    return fail(FMC_EINVAL, "the served form integrates in FP32 (FMC_F32 or FMC_BF16X3)");
  if (p->zeta_in) return fail(FMC_EINVAL, "served requests draw their own design (zeta_in must be NULL)");
  if (r.fd) {
    // the flux-decay integrator: 16-trajectory tiles in contiguous items
    // (kFdItems of them), a short default chunk so
    // that a large request does not stretch every tick
    r.n_pad = 16 * ((r.n + 15) / 16);
    r.NW = (r.n_pad / 16 + 1) / 2;
    r.Sc = std::min<int64_t>(S, p->time_chunk > 0 ? p->time_chunk : kDefaultChunkFd);
    FdPlan pl{};
    fd_plan(r.N, kFdItems, &pl);
    r.tiles = pl.tiles;
    r.tiles_per_item = pl.tiles_per_item;
    r.n_items = pl.n_items;
    return FMC_OK;
  }
  int vid = p->variant;
  if (vid < 0) vid = default_batch_variant(r.n, r.P, p->precision);
  if (vid < 0 || vid >= n_batch_variants()) return fail(FMC_EINVAL, "no batched variant fits the request");
  r.vid = vid;
  r.bv = batch_variant(vid);
  if (!batch_fits(r.bv, r.n, r.P, p->precision))
    return fail(FMC_EINVAL, "variant does not fit the request (size, or a BF16 x3 product for "
                            "an FMC_F32 request)");
  r.Sc = std::min<int64_t>(S, p->time_chunk > 0 ? p->time_chunk : kDefaultChunk);
  r.tiles = (r.N + r.bv.TB - 1) / r.bv.TB;
  r.cost_tile = (double)r.S * r.bv.TB * (8.0 * r.bv.NG * r.bv.NG + 45.0 * r.bv.NG + 4.0 * r.P);
  // fine items (up to kMaxItems): a request alone still spreads over the chip
  r.tiles_per_item = (r.tiles + kMaxItems - 1) / kMaxItems;
  r.n_items = (r.tiles + r.tiles_per_item - 1) / r.tiles_per_item;
  return FMC_OK;
}

// Copy the request's inputs into its staging bytes (device layout of the
// setup kernels).
void stage_inputs(Request& r, const fmc_system* s, const fmc_disturbance* d) {
  const int n = r.n, P = r.P;
  std::vector<double2> Yh, Yinfh;
  if (s->Y_re) {
    Yh.resize((size_t)n * n);
    for (size_t q = 0; q < Yh.size(); ++q) Yh[q] = make_double2(s->Y_re[q], s->Y_im[q]);
  }
  if (s->infinite_bus) {
    Yinfh.resize(n);
    for (int k = 0; k < n; ++k) Yinfh[k] = make_double2(s->Yinf_re[k], s->Yinf_im[k]);
  }
  Stager& sg = r.sg;
  r.sd.n = n;
  r.sd.P = P;
  sg.add(s->H, n, &r.sd.H);
  sg.add(s->D, n, &r.sd.D);
  sg.add(s->E, n, &r.sd.E);
  sg.add(s->delta0, n, &r.sd.delta0);
  sg.add(s->Pm, n, &r.sd.Pm);
  sg.add(Yh.empty() ? nullptr : Yh.data(), Yh.size(), &r.sd.Y);
  sg.add(Yinfh.empty() ? nullptr : Yinfh.data(), Yinfh.size(), &r.sd.Yinf);
  sg.add(d->theta, P, &r.sd.theta);
  sg.add(d->sigma, P, &r.sd.sigma);
  sg.add(d->xi0, P, &r.sd.xi0);
  sg.add(d->gen, P, &r.gen_d);
  if (!s->Y_re) {
    const fmc_network* nt = s->net;
    r.nd.n_bus = nt->n_bus;
    r.nd.n_branch = nt->n_branch;
    r.nd.n_gen = nt->n_gen;
    sg.add(nt->br_from, nt->n_branch, &r.nd.from);
    sg.add(nt->br_to, nt->n_branch, &r.nd.to);
    sg.add(nt->br_r, nt->n_branch, &r.nd.r);
    sg.add(nt->br_x, nt->n_branch, &r.nd.x);
    sg.add(nt->br_b, nt->n_branch, &r.nd.b);
    sg.add(nt->load_g, nt->n_bus, &r.nd.lg);
    sg.add(nt->load_b, nt->n_bus, &r.nd.lb);
    sg.add(nt->gen_bus, nt->n_gen, &r.nd.gen_bus);
    sg.add(nt->gen_xdp, nt->n_gen, &r.nd.xdp);
  }
  if (r.fd) {
    sg.add(s->E, n, &r.E_d);
    sg.add(s->model_params, (size_t)n * kFdParams, &r.prm_d);
  }
  r.sd.inf_bus = r.inf_bus ? 1 : 0;
  r.sd.V_inf = r.V_inf;
}

}  // namespace

struct ServeState {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  serve::Arena arena;
  char* arena_base = nullptr;
  unsigned char* tick_dev = nullptr;  // upload region of a tick (outside the arena)
  hipStream_t st = nullptr;
  // per tick, the size classes and the flux-decay integrators run on their
  // own streams (forked from st after the paths, joined before the merges)
  hipStream_t lst[kBatchClasses + 1] = {};
  hipEvent_t lev[kBatchClasses + 2] = {};  // [k]: lane k done, [kBatchClasses + 1]: fork
  unsigned char* pin = nullptr;  // page-locked staging of a tick
  size_t pin_cap = 0;
  int n_cu = 0, bpc[kBatchClasses] = {};
  uint64_t next_ticket = 1;
  std::deque<ReqP> incoming;
  std::vector<ReqP> active;
  std::map<uint64_t, ReqP> all;
};

namespace {

std::mutex g_create_mu;  // creation of a context's server

// Admission: all of the request's parts from the arena, or none.
int admit(ServeState* ss, Request& r) {
  const std::vector<size_t> z = parts_of(r);
  const int used = (int)(ss->active.size() + ss->incoming.size());
  const serve::Decision d = serve::admit(ss->arena, z, used, kMaxActive, &r.blocks);
  if (d == serve::NEVER) return fail(FMC_ENOMEM, "request footprint exceeds the serving arena");
  if (d == serve::NOT_NOW) return fail(FMC_EBUSY, "no serving slot or not enough free HBM in the arena now");
  void* ptr[B_COUNT] = {};
  size_t q = 0;
  for (int k = 0; k < B_COUNT; ++k)
    if (z[k]) ptr[k] = ss->arena_base + r.blocks[q++].first;
  r.inbuf = (unsigned char*)ptr[B_IN];
  r.canon = (double*)ptr[B_CANON];
  r.coef = (float*)ptr[B_COEF];
  r.phi = (double*)ptr[B_PHI];
  r.zeta = (double*)ptr[B_ZETA];
  r.w = (float*)ptr[B_W];
  r.state = (float*)ptr[B_STATE];
  r.part = (double2*)ptr[B_PART];
  r.mean = (double*)ptr[B_MEAN];
  r.var = (double*)ptr[B_VAR];
  r.work = (double*)ptr[B_WORK];
  r.ybuf = (double2*)ptr[B_YBUF];
  r.kwork = (double2*)ptr[B_KWORK];
  r.status = (int*)ptr[B_STATUS];
  r.cnt = (unsigned long long*)((char*)r.status + 32);
  r.fdblk = (double*)ptr[B_FDBLK];
  r.fdap = (float2*)ptr[B_FDAP];
  r.xstate = (float*)ptr[B_XSTATE];
  r.footprint = (int64_t)serve::footprint(z);
  return FMC_OK;
}

void release(ServeState* ss, Request& r) {
  for (auto& b : r.blocks) ss->arena.release(b.first, b.second);
  r.blocks.clear();
}

#define SCHK(expr)                                                                       \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(FMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

// Page-locked staging for one tick; nothing is in flight at a tick's start.
int ensure_pin(ServeState* ss, size_t bytes) {
  if (ss->pin_cap >= bytes) return FMC_OK;
  if (ss->pin) (void)hipHostFree(ss->pin);
  ss->pin = nullptr;
  ss->pin_cap = 0;
  const size_t cap = std::max(al(bytes) * 2, size_t(1) << 20);
  SCHK(hipHostMalloc((void**)&ss->pin, cap, hipHostMallocDefault));
  ss->pin_cap = cap;
  return FMC_OK;
}

// Upload a newly started request's inputs and enqueue its setup: network
// reduction, operating point, packed coefficients, basis and design.
int start_request(ServeState* ss, Request& r, size_t* pin_off) {
  hipStream_t st = ss->st;
  const size_t nb = r.sg.bytes.size();
  if (nb) {
    std::memcpy(ss->pin + *pin_off, r.sg.bytes.data(), nb);
    SCHK(hipMemcpyAsync(r.inbuf, ss->pin + *pin_off, nb, hipMemcpyHostToDevice, st));
    *pin_off += al(nb);
    for (auto& f : r.sg.fix) *f.second = r.inbuf + f.first;
  }
  SCHK(launch_fill_i64((int64_t*)r.status, 0, 4, st));
  SCHK(launch_fill_i64((int64_t*)r.cnt, 0, 1, st));
  SCHK(launch_fill_i64((int64_t*)r.cnt + 1, LLONG_MAX, 1, st));
  if (!r.has_Y) {
    SCHK(launch_kron(r.nd, r.kwork, r.ybuf, r.status + 1, st));
    r.sd.Y = r.ybuf;
  }
  r.sd.work = r.work;
  r.sd.canon = r.canon;
  r.sd.status = r.status;
  SCHK(launch_setup(r.sd, st));
  if (r.fd) {
    SCHK(launch_setup_fd(r.canon, r.n, r.P, r.E_d, r.prm_d, r.fdblk, st));
    // constants and the FP32 product's Y; the BF16 x3 product's Y (never
    // smaller) then overwrites the Y buffer
    SCHK(launch_pack_fd(r.canon, r.n, r.P, r.prm_d, r.fdblk, r.gen_d, r.n_pad, r.coef, r.fdap, st));
    if (fd_bf16_product(&r.par))
      SCHK(launch_pack_fd_y16(r.canon, r.n, r.n_pad, 32 * ((r.n + 31) / 32), r.fdap, st));
  } else {
    SCHK(launch_pack_batch(r.bv, r.canon, r.n, r.P, r.gen_d, r.coef, st));
  }
  SCHK(launch_basis(r.par.basis, r.K, r.S, r.par.T, r.phi, st));
  SCHK(launch_lhs(r.par.seed, (int32_t)r.M, r.N, r.par.sampler, nullptr, r.zeta, st));
  return FMC_OK;
}

// One tick: start the fresh requests, then the next time chunk of every active
// request; finished requests are merged and copied out.  Ends with the
// serving stream drained.
int run_tick(ServeState* ss, const std::vector<ReqP>& fresh, const std::vector<ReqP>& act,
             std::vector<ReqP>& finishing) {
  hipStream_t st = ss->st;
  const int na = (int)act.size();
  int64_t n_items = 0;  // items of the batched (classical) integrator
  for (auto& r : act)
    if (!r->fd) n_items += r->n_items;
  const size_t up_bytes = al(sizeof(IntegArgs<float>) * na) + al(sizeof(BatchItem) * n_items) +
                          al(sizeof(int32_t) * n_items);
  if (up_bytes + kAlign > kTickBytes) return fail(FMC_EINVAL, "too many work items in one tick");
  size_t pin_need = up_bytes + al(64) * na;
  for (auto& r : fresh) pin_need += al(r->sg.bytes.size());
  int rc = ensure_pin(ss, pin_need);
  if (rc) return rc;
  size_t pin_off = 0;
  for (auto& r : fresh)
    if ((rc = start_request(ss, *r, &pin_off))) return rc;

  std::vector<IntegArgs<float>> args(na);
  std::vector<BatchItem> items;
  items.reserve(n_items);
  std::vector<std::vector<int32_t>> order(kBatchClasses);
  std::vector<double> icost;
  icost.reserve(n_items);
  std::vector<std::pair<FdArgs, int64_t>> fd_launch;
  for (int i = 0; i < na; ++i) {
    Request& r = *act[i];
    const int64_t s0 = r.s_next, s1 = std::min<int64_t>(r.S, s0 + r.Sc);
    const int64_t cols = 2 * (s1 - s0) + 1;
    if (r.par.precision == FMC_F32)
      SCHK(launch_kle_f64_to_f32(r.zeta, r.phi, r.C, r.P, r.K, r.N, cols, 2 * s0, r.w, st));
    else
      SCHK(launch_kle_bf16x3(r.zeta, r.phi, r.C, r.P, r.K, r.N, cols, 2 * s0, r.w, st));
    if (r.fd) {
      FdArgs f{};
      f.coef = r.coef;
      f.ap = r.fdap;
      f.ap16 = fd_bf16_product(&r.par) ? (const void*)r.fdap : nullptr;
      f.n_padk = 32 * ((r.n + 31) / 32);
      f.w = r.w;
      f.state = r.state;
      f.xstate = r.xstate;
      f.off = r.fdblk + FdLayout{r.n}.off();
      f.nonfinite = r.cnt;
      f.first_bad = (long long*)r.cnt + 1;
      f.rows = r.part;
      f.row_stride = (r.Sc + 1) * r.V;
      f.row_base = s0;
      f.n = r.n;
      f.P = r.P;
      f.V = r.V;
      f.n_pad = r.n_pad;
      f.N = r.N;
      f.S = r.S;
      f.s_begin = s0;
      f.s_end = s1;
      f.c_base = 2 * s0;
      f.tiles = r.tiles;
      f.tiles_per_item = r.tiles_per_item;
      f.dt = (float)r.par.dt;
      f.wb = (float)(2.0 * M_PI * r.f0);
      f.recenter = r.inf_bus ? 0 : 1;
      fd_launch.push_back({f, r.n_items});
      r.s_prev = s0;
      r.s_next = s1;
      if (s1 == r.S) finishing.push_back(act[i]);
      continue;
    }
    IntegArgs<float>& a = args[i];
    a.coef = r.coef;
    a.w = r.w;
    a.state = r.state;
    a.partial = nullptr;
    a.delta0 = r.canon + CanonLayout{r.n, r.P}.delta0();
    a.traj_slot = nullptr;
    a.traj = nullptr;
    a.nonfinite = r.cnt;
    a.first_bad = (long long*)r.cnt + 1;
    a.n = r.n;
    a.P = r.P;
    a.V = r.V;
    a.N = r.N;
    a.S = r.S;
    a.s_begin = s0;
    a.s_end = s1;
    a.c_base = 2 * s0;
    a.lanes = r.tiles * 64 * 4;
    a.dt = (float)r.par.dt;
    a.wb = (float)(2.0 * M_PI * r.f0);
    a.recenter = r.inf_bus ? 0 : 1;
    a.n_ref = r.n;
    const double frac = (double)(s1 - s0) / (double)r.S;
    for (int64_t k = 0; k < r.n_items; ++k) {
      BatchItem it;
      it.rows = r.part + k * (r.Sc + 1) * r.V;  // this chunk's rows (steps s0..s1)
      it.tile0 = k * r.tiles_per_item;
      it.tile1 = std::min<int64_t>(r.tiles, it.tile0 + r.tiles_per_item);
      it.scen = i;
      it.variant = r.vid;
      order[r.bv.cls].push_back((int32_t)items.size());
      icost.push_back(r.cost_tile * frac * (double)(it.tile1 - it.tile0));
      items.push_back(it);
    }
    r.s_prev = s0;
    r.s_next = s1;
    if (s1 == r.S) finishing.push_back(act[i]);
  }
  for (auto& o : order)
    std::stable_sort(o.begin(), o.end(), [&](int32_t x, int32_t y) { return icost[x] > icost[y]; });
  std::vector<int32_t> flat;
  flat.reserve(n_items);
  int64_t off[kBatchClasses + 1];
  for (int k = 0; k < kBatchClasses; ++k) {
    off[k] = (int64_t)flat.size();
    flat.insert(flat.end(), order[k].begin(), order[k].end());
  }
  off[kBatchClasses] = (int64_t)flat.size();

  // tick upload: [heads | args | items | order]
  unsigned char* hp = ss->pin + pin_off;
  unsigned char* dp = ss->tick_dev + kAlign;
  size_t o = 0;
  std::memcpy(hp + o, args.data(), sizeof(IntegArgs<float>) * na);
  const IntegArgs<float>* args_d = (const IntegArgs<float>*)(dp + o);
  o += al(sizeof(IntegArgs<float>) * na);
  std::memcpy(hp + o, items.data(), sizeof(BatchItem) * n_items);
  const BatchItem* items_d = (const BatchItem*)(dp + o);
  o += al(sizeof(BatchItem) * n_items);
  std::memcpy(hp + o, flat.data(), sizeof(int32_t) * n_items);
  const int32_t* order_d = (const int32_t*)(dp + o);
  o += al(sizeof(int32_t) * n_items);
  SCHK(hipMemcpyAsync(dp, hp, o, hipMemcpyHostToDevice, st));
  pin_off += o;
  int32_t* heads = (int32_t*)ss->tick_dev;
  SCHK(launch_fill_i64((int64_t*)heads, 0, 8, st));
  // lanes of the tick: the size classes with items, then the flux-decay
  // integrators (one after another on the last lane)
  bool on[kBatchClasses + 1];
  int n_on = 0;
  for (int k = 0; k < kBatchClasses; ++k) n_on += on[k] = off[k + 1] > off[k];
  n_on += on[kBatchClasses] = !fd_launch.empty();
  const bool fork = n_on > 1;
  if (fork) SCHK(hipEventRecord(ss->lev[kBatchClasses + 1], st));
  auto lane = [&](int k) {
    if (!fork) return st;
    (void)hipStreamWaitEvent(ss->lst[k], ss->lev[kBatchClasses + 1], 0);
    return ss->lst[k];
  };
  for (int k = 0; k < kBatchClasses; ++k) {
    if (!on[k]) continue;
    const int64_t nk = off[k + 1] - off[k];
    const int grid = (int)std::min<int64_t>(nk, (int64_t)ss->bpc[k] * ss->n_cu);
    BatchArgs b{args_d, items_d, order_d + off[k], (int32_t)nk, heads + 2 * k};
    SCHK(launch_persistent(k, b, grid, lane(k)));
  }
  if (on[kBatchClasses]) {
    const hipStream_t ls = lane(kBatchClasses);
    for (auto& f : fd_launch) SCHK(launch_rk4_fd(f.first, f.second, ls));
  }
  if (fork)
    for (int k = 0; k <= kBatchClasses; ++k)
      if (on[k]) {
        SCHK(hipEventRecord(ss->lev[k], ss->lst[k]));
        SCHK(hipStreamWaitEvent(st, ss->lev[k], 0));
      }
  // rows completed by this tick: s0+1..s1 (and row 0 in a request's first chunk)
  for (int i = 0; i < na; ++i) {
    Request& r = *act[i];
    const int64_t first = r.s_prev == 0 ? 0 : r.s_prev + 1, rows = r.s_next - first + 1;
    // FP64 offsets added back: delta0 (classical), or the 6n operating-point
    // values of the flux-decay states
    const double* offs = r.fd ? r.fdblk + FdLayout{r.n}.off() : r.canon + CanonLayout{r.n, r.P}.delta0();
    const int n_off = r.fd ? 6 * r.n : r.n;
    const int64_t groups = r.fd ? r.tiles : r.n_items;
    const int group = r.fd ? 16 : (int)(r.tiles_per_item * r.bv.TB);
    SCHK(launch_stats_merge_rows(r.part + (first - r.s_prev) * r.V, (r.Sc + 1) * r.V, groups, group,
                                 r.N, rows, r.V, n_off, r.par.ddof, offs, r.mean + first * r.V,
                                 r.var + first * r.V, st));
  }
  for (auto& rp : finishing) {
    Request& r = *rp;
    const size_t sv = (size_t)(r.S + 1) * r.V * 8;
    const hipMemcpyKind kind =
        r.out.mem_kind == FMC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    SCHK(hipMemcpyAsync(r.out.mean, r.mean, sv, kind, st));
    SCHK(hipMemcpyAsync(r.out.var, r.var, sv, kind, st));
    r.pin_status = pin_off;
    SCHK(hipMemcpyAsync(ss->pin + pin_off, r.status, 48, hipMemcpyDeviceToHost, st));
    pin_off += al(64);
  }
  SCHK(hipStreamSynchronize(st));
  return FMC_OK;
}

void finish(ServeState* ss, Request& r, int code) {
  r.code = code;
  r.t_done = Clock::now();
  release(ss, r);
}

void write_report(ServeState* ss, Request& r) {
  const int* sh = (const int*)(ss->pin + r.pin_status);
  const unsigned long long* cn = (const unsigned long long*)(ss->pin + r.pin_status + 32);
  int code = FMC_OK;
  if (sh[1] != 0) code = FMC_EINVAL;         // singular network reduction
  else if (sh[0] != 0) code = FMC_ENOTCONV;  // operating point not found
  else if (cn[0] != 0) code = FMC_ENONFINITE;
  const int64_t nbad = (int64_t)cn[0], first = cn[0] ? (int64_t)cn[1] : -1;
  finish(ss, r, code);
  if (r.out.report) {
    fmc_report* rep = r.out.report;
    std::memset(rep, 0, sizeof(*rep));
    rep->n_nonfinite = nbad;
    rep->first_nonfinite = first;
    rep->variant_id = r.fd ? (fd_bf16_product(&r.par) ? 1 : 0) : r.vid;
    rep->lanes_per_traj = r.fd ? 1 : r.bv.L;
    rep->tile = (int32_t)(r.tiles_per_item * (r.fd ? 16 : r.bv.TB));
    rep->time_chunk = (int32_t)r.Sc;
    rep->hbm_peak_bytes = r.footprint;
    rep->queue_wait_s = std::chrono::duration<double>(r.t_start - r.t_submit).count();
    rep->latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    rep->t_total_s = std::chrono::duration<double>(r.t_done - r.t_start).count();
  }
}

void server_loop(Context* c, ServeState* ss) {
  (void)hipSetDevice(c->device);
  for (;;) {
    std::vector<ReqP> fresh, act;
    {
      std::unique_lock<std::mutex> lk(ss->mu);
      ss->cv_work.wait(lk, [&] { return ss->stop || !ss->incoming.empty() || !ss->active.empty(); });
      if (ss->stop) return;
      // cancelled requests leave at the tick boundary (nothing of theirs is in flight)
      bool gone = false;
      for (auto it = ss->active.begin(); it != ss->active.end();) {
        if ((*it)->cancel) {
          finish(ss, **it, FMC_ECANCELLED);
          it = ss->active.erase(it);
          gone = true;
        } else {
          ++it;
        }
      }
      const auto now = Clock::now();
      while (!ss->incoming.empty() && (int)ss->active.size() < kMaxActive) {
        ReqP r = ss->incoming.front();
        ss->incoming.pop_front();
        if (r->cancel) {
          finish(ss, *r, FMC_ECANCELLED);
          gone = true;
          continue;
        }
        r->t_start = now;
        fresh.push_back(r);
        ss->active.push_back(r);
      }
      if (gone) ss->cv_done.notify_all();
      act = ss->active;
    }
    if (act.empty()) continue;
    std::vector<ReqP> finishing;
    const int rc = run_tick(ss, fresh, act, finishing);
    if (rc) (void)hipStreamSynchronize(ss->st);
    std::lock_guard<std::mutex> lk(ss->mu);
    if (rc) {
      // a failed tick ends every active request with its status
      for (auto& r : ss->active) finish(ss, *r, rc);
      ss->active.clear();
    } else {
      for (auto& rp : finishing) {
        write_report(ss, *rp);
        ss->active.erase(std::find(ss->active.begin(), ss->active.end(), rp));
      }
    }
    if (rc || !finishing.empty()) ss->cv_done.notify_all();
  }
}

int ensure_server(Context* c) {
  std::lock_guard<std::mutex> g(g_create_mu);
  if (c->serve) return FMC_OK;
  const size_t avail = c->budget > c->held ? c->budget - c->held : 0;
  size_t want = 0;
  if (const char* e = std::getenv("FMC_SERVE_ARENA_BYTES")) want = (size_t)std::strtoull(e, nullptr, 10);
  if (!want) want = std::min<size_t>((size_t)(0.5 * (double)avail), size_t(32) << 30);
  want = std::min(want, avail > kTickBytes ? avail - kTickBytes : 0);
  if (want < (size_t(64) << 20)) return fail(FMC_ENOMEM, "HBM budget too small for a serving arena");
  void *arena = nullptr, *tick = nullptr;
  int rc = c->ensure("serve_arena", want, &arena);
  if (rc) return rc;
  if ((rc = c->ensure("serve_tick", kTickBytes, &tick))) return rc;
  std::unique_ptr<ServeState> ss(new ServeState());
  ss->arena.init(want);
  ss->arena_base = (char*)arena;
  ss->tick_dev = (unsigned char*)tick;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess)
    return fail(FMC_EDEVICE, "hipGetDeviceProperties failed");
  ss->n_cu = prop.multiProcessorCount;
  for (int k = 0; k < kBatchClasses; ++k) ss->bpc[k] = persistent_blocks_per_cu(k);
  if (hipStreamCreateWithFlags(&ss->st, hipStreamNonBlocking) != hipSuccess)
    return fail(FMC_EDEVICE, "cannot create the serving stream");
  for (auto& l : ss->lst)
    if (hipStreamCreateWithFlags(&l, hipStreamNonBlocking) != hipSuccess)
      return fail(FMC_EDEVICE, "cannot create the serving streams");
  for (auto& e : ss->lev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return fail(FMC_EDEVICE, "cannot create the serving events");
  c->serve = ss.release();
  c->serve->th = std::thread(server_loop, c, c->serve);
  return FMC_OK;
}

// Final status of a ticket; the ticket is forgotten once it is reported.
int report_final(ServeState* ss, std::map<uint64_t, ReqP>::iterator it) {
  const int code = it->second->code;
  ss->all.erase(it);
  if (code == FMC_OK) return FMC_OK;
  const char* what = code == FMC_ECANCELLED   ? "request was cancelled"
                     : code == FMC_ENONFINITE ? "some sample paths became non-finite"
                     : code == FMC_ENOTCONV   ? "operating point not found"
                     : code == FMC_EINVAL     ? "singular network reduction"
                                              : "request failed on the device";
  return fail(code, what);
}

}  // namespace

void serve_shutdown(Context* c) {
  ServeState* ss = c->serve;
  if (!ss) return;
  {
    std::lock_guard<std::mutex> lk(ss->mu);
    ss->stop = true;
  }
  ss->cv_work.notify_all();
  if (ss->th.joinable()) ss->th.join();
  if (ss->st) {
    (void)hipStreamSynchronize(ss->st);
    (void)hipStreamDestroy(ss->st);
  }
  for (auto& l : ss->lst)
    if (l) {
      (void)hipStreamSynchronize(l);
      (void)hipStreamDestroy(l);
    }
  for (auto& e : ss->lev)
    if (e) (void)hipEventDestroy(e);
  if (ss->pin) (void)hipHostFree(ss->pin);
  delete ss;
  c->serve = nullptr;
}

}  // namespace fmc

using namespace fmc;

extern "C" {

int fmc_footprint(const fmc_scenario* scen, int64_t* bytes) {
  if (!scen || !bytes || !scen->sys || !scen->dist || !scen->par)
    return fail(FMC_EINVAL, "NULL argument");
  int64_t S = 0;
  int rc = validate(scen->sys, scen->dist, scen->par, &S);
  if (rc) return rc;
  const fmc_params* par = scen->par;
  const bool decor = par->sampler == FMC_LHS_DECOR && !par->zeta_in;
  const bool mixed = scen->dist->sigma_mat != nullptr;
  if (par->precision != FMC_F64 && !par->zeta_in && !decor && !mixed) {
    // reduced precision: the admission footprint of the served form
    Request r;
    if ((rc = plan_request(r, scen->sys, scen->dist, par, S))) return rc;
    stage_inputs(r, scen->sys, scen->dist);
    *bytes = (int64_t)footprint_of(r);
    return FMC_OK;
  }
  // FP64 (single-run form): design, basis, two chunks of paths, state, partials
  const int64_t n = scen->sys->n_gen, P = scen->dist->n_proc, K = par->K, N = par->N;
  const int64_t V = 2 * n + P, C = 2 * S + 1;
  const int64_t bw = par->precision == FMC_F64 ? 8 : 4;
  const int64_t groups = (N + 63) / 64;
  const int64_t Sc = auto_chunk(S, (int)P, N, (int)bw);
  int64_t b = 0;
  b += P * K * N * 8;                        // zeta
  b += K * C * 8;                            // basis
  b += 2 * (2 * Sc + 1) * P * N * bw;        // two chunks of KLE paths (double buffer)
  b += (2 * n + P + 16) * groups * 64 * bw;  // state
  b += groups * (S + 1) * V * 16;            // per-group statistics
  b += 2 * (S + 1) * V * 8;                  // mean, var
  b += 2 * n * n * 16 + 64 * n;              // reduced network, coefficients
  if (decor) b += (int64_t)decorrelate_workspace((int32_t)(P * K), N);
  if (mixed) b += P * K * N * 8 + P * P * 8;  // mixed design, diffusion matrix
  *bytes = b;
  return FMC_OK;
}

int fmc_submit(fmc_context* ctx, const fmc_scenario* scen, fmc_outputs* out, uint64_t* ticket) {
  if (!ctx || !scen || !out || !ticket || !scen->sys || !scen->dist || !scen->par)
    return fail(FMC_EINVAL, "NULL argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  int64_t S = 0;
  int rc = validate(scen->sys, scen->dist, scen->par, &S);
  if (rc) return rc;
  if (scen->par->sampler == FMC_LHS_DECOR)
    return fail(FMC_EINVAL, "FMC_LHS_DECOR runs through fmc_run only");
  if (scen->dist->sigma_mat) return fail(FMC_EINVAL, "a diffusion matrix runs through fmc_run only");
  if (scen->dist->proc) return fail(FMC_EINVAL, "general Ito processes run through fmc_run only");
  if (scen->sys->event) return fail(FMC_EINVAL, "network events run through fmc_run only");
  if (scen->par->integrator != FMC_RK4)
    return fail(FMC_EINVAL, "the implicit trapezoid runs through fmc_run only");
  if (!out->mean || !out->var) return fail(FMC_EINVAL, "mean and var outputs are required");
  if (out->mem_kind != FMC_MEM_HOST && out->mem_kind != FMC_MEM_DEVICE)
    return fail(FMC_EINVAL, "unknown mem_kind");
  if (out->n_traj != 0 || out->strata || out->zeta || out->rrf)
    return fail(FMC_EINVAL, "served requests return mean and var only");
  auto r = std::make_shared<Request>();
  if ((rc = plan_request(*r, scen->sys, scen->dist, scen->par, S))) return rc;
  stage_inputs(*r, scen->sys, scen->dist);
  r->out = *out;
  (void)hipSetDevice(c->device);
  if ((rc = ensure_server(c))) return rc;
  ServeState* ss = c->serve;
  std::lock_guard<std::mutex> lk(ss->mu);
  if ((rc = admit(ss, *r))) return rc;
  r->ticket = ss->next_ticket++;
  r->t_submit = Clock::now();
  ss->incoming.push_back(r);
  ss->all[r->ticket] = r;
  *ticket = r->ticket;
  ss->cv_work.notify_all();
  return FMC_OK;
}

int fmc_poll(fmc_context* ctx, uint64_t ticket) {
  if (!ctx) return fail(FMC_EINVAL, "ctx is NULL");
  Context* c = reinterpret_cast<Context*>(ctx);
  ServeState* ss = c->serve;
  if (!ss) return fail(FMC_EINVAL, "unknown ticket");
  std::lock_guard<std::mutex> lk(ss->mu);
  auto it = ss->all.find(ticket);
  if (it == ss->all.end()) return fail(FMC_EINVAL, "unknown ticket");
  if (it->second->code == FMC_EAGAIN) return FMC_EAGAIN;
  return report_final(ss, it);
}

int fmc_wait(fmc_context* ctx, uint64_t ticket, double timeout_s) {
  if (!ctx) return fail(FMC_EINVAL, "ctx is NULL");
  Context* c = reinterpret_cast<Context*>(ctx);
  ServeState* ss = c->serve;
  if (!ss) return fail(FMC_EINVAL, "unknown ticket");
  std::unique_lock<std::mutex> lk(ss->mu);
  auto it = ss->all.find(ticket);
  if (it == ss->all.end()) return fail(FMC_EINVAL, "unknown ticket");
  ReqP r = it->second;
  const auto done = [&] { return r->code != FMC_EAGAIN; };
  if (timeout_s < 0) {
    ss->cv_done.wait(lk, done);
  } else if (!ss->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return fail(FMC_ETIMEDOUT, "request still running");
  }
  it = ss->all.find(ticket);
  if (it == ss->all.end()) return fail(FMC_EINVAL, "ticket was reported by another call");
  return report_final(ss, it);
}

int fmc_cancel(fmc_context* ctx, uint64_t ticket) {
  if (!ctx) return fail(FMC_EINVAL, "ctx is NULL");
  Context* c = reinterpret_cast<Context*>(ctx);
  ServeState* ss = c->serve;
  if (!ss) return fail(FMC_EINVAL, "unknown ticket");
  std::lock_guard<std::mutex> lk(ss->mu);
  auto it = ss->all.find(ticket);
  if (it == ss->all.end()) return fail(FMC_EINVAL, "unknown ticket");
  if (it->second->code == FMC_EAGAIN) it->second->cancel = true;
  ss->cv_work.notify_all();
  return FMC_OK;
}

}  // extern "C"
