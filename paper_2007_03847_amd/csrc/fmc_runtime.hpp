// fmc_runtime.hpp -- host-side context and helpers shared by the runtime files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fmc.h"
#include "fmc_internal.hpp"

namespace fmc {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct ServeState;  // continuous-batching server (fmc_serve.hip)

struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0, held = 0, peak = 0;
  std::map<std::string, DevBuf> bufs;
  std::map<std::string, DevBuf> pinned;  // page-locked host staging, grow-only
  hipEvent_t ev[8] = {};
  ServeState* serve = nullptr;
  std::map<std::string, int> tuned;  // autotuner cache: key -> variant id
  uint64_t alloc_gen = 0;            // bumped whenever a device buffer moves
  hipStream_t bstream = nullptr;     // capture stream of the batched form
  hipStream_t gstream = nullptr;     // KLE contractions overlapped with the integrator
  hipEvent_t gev[4] = {};            // [b]: paths of buffer b ready, [2+b]: buffer b consumed
  // batched form: one stream per size class so that a tick's class launches
  // share the chip (forked from and joined back into bstream inside the graph)
  hipStream_t cstream[kBatchClasses] = {};
  hipEvent_t cev[kBatchClasses + 1] = {};  // [cl]: class cl done, [kBatchClasses]: fork
  std::map<std::string, std::pair<uint64_t, hipGraphExec_t>> graphs;  // shape -> (gen, graph)

  int ensure(const char* name, size_t bytes, void** out);
  // Page-locked host buffer for asynchronous uploads.  A buffer is rewritten
  // only by a later call on this context, and every call that uploads from it
  // synchronises the stream before it returns, so no copy is in flight then.
  int host_stage(const char* name, size_t bytes, void** out);
  void release_all();
};

// Host staging of small arrays into one device upload (through a pinned
// buffer of the context, no stream synchronisation).
struct Stager {
  std::vector<unsigned char> bytes;
  std::vector<std::pair<size_t, void**>> fix;  // (offset, where to store device ptr)
  template <typename T>
  void add(const T* src, size_t count, const T** dst) {
    if (!src || count == 0) {
      *dst = nullptr;
      return;
    }
    const size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + count * sizeof(T));
    std::memcpy(bytes.data() + off, src, count * sizeof(T));
    fix.push_back({off, (void**)dst});
  }
  int upload(Context* c, const char* name, hipStream_t st = nullptr);
};

int validate(const fmc_system* sys, const fmc_disturbance* dist, const fmc_params* par,
             int64_t* S_out);
int stage_scenario(Context* c, const fmc_system* sys, const fmc_disturbance* dist,
                   const char* tag, double** canon_out, int32_t** gen_out, int** status_out);
// Kron reduction on the context's stream; the network's arrays are staged
// under `tag` (a tag per network that may be in flight at the same time).
int kron_on_device(Context* c, const fmc_network* net, double2* Yd, int* st_dev,
                   const char* tag = "net");
int choose_variant(int n, int P, int64_t N);
std::string tune_key(int n, int P, int64_t N, int precision);
int pick_variant(Context* c, int n, int P, int64_t N, int precision);
// Batched variants: whether one may run (n, P, precision), and the untuned
// choice of the served form.
bool batch_fits(const BatchVariantInfo& b, int n, int P, int precision);
// Flux-decay systems: the network product on BF16 x3 split products (asked
// for with variant 1 under FMC_BF16X3), else in FP32.
inline bool fd_bf16_product(const fmc_params* p) {
  return p->precision == FMC_BF16X3 && p->variant == 1;
}
int default_batch_variant(int n, int P, int precision);
int64_t auto_chunk(int64_t S, int P, int64_t N, int bytes_per);
int ensure_gstream(Context* c);  // the second stream of fmc_run and its events
int run_single(Context* c, const fmc_system* sys, const fmc_disturbance* dist,
               const fmc_params* par, fmc_outputs* out);
void serve_shutdown(Context* c);
// Correlation-reducing permutation of a device design [M][N] in place on
// stream st (FMC_LHS_DECOR).  strata (nullable) receives each entry's rank in
// its row.  lhs_strata (nullable): the strata of an LHS design as k_lhs wrote
// them (a permutation of 0..N-1 per row), which then stand for the ranks of
// its values; never a caller's array.  *status_out points at a device int32
// that is 1 once the stream has run if the design's covariance was not
// positive definite (the design is then left as it was).
int decorrelate_design(Context* c, int32_t M, int64_t N, double* zeta, int32_t* strata,
                       const int32_t* lhs_strata, int32_t** status_out, hipStream_t st);
size_t decorrelate_workspace(int32_t M, int64_t N);
// Correlated disturbances: *zeta (device [P*K][N]) is replaced by the design
// mixed through dist->sigma_mat (a context buffer) on stream st.
int mix_design(Context* c, const fmc_disturbance* dist, int32_t K, int64_t N, const double** zeta,
               hipStream_t st);
// A copy of a disturbance whose diffusion matrix replaces sigma: sigma is
// then 1 for every process (the mixed design carries the matrix).
struct UnitSigma {
  std::vector<double> one;
  fmc_disturbance d;
  const fmc_disturbance* apply(const fmc_disturbance* dist) {
    if (!dist->sigma_mat) return dist;
    one.assign((size_t)dist->n_proc, 1.0);
    d = *dist;
    d.sigma = one.data();
    return &d;
  }
};

// Flux-decay path: tiles of 16 trajectories, contiguous work items of
// tiles_per_item tiles, one workgroup per item.
struct FdPlan {
  int64_t tiles, tiles_per_item, n_items;
};
constexpr int kFdItems = 256;  // work items of a flux-decay run: one per CU of an MI355X
int fd_plan(int64_t N, int n_cu, FdPlan* p);
int run_fd(Context* c, const fmc_system* sys, const fmc_disturbance* dist, const fmc_params* par,
           fmc_outputs* out, int64_t S);

}  // namespace fmc
