// fmc_runtime.hpp -- host-side context and helpers shared by the runtime files.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>

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

  int ensure(const char* name, size_t bytes, void** out);
  // Page-locked host buffer for asynchronous uploads.  A buffer is rewritten
  // only by a later call on this context, and every call that uploads from it
  // synchronises the stream before it returns, so no copy is in flight then.
  int host_stage(const char* name, size_t bytes, void** out);
  void release_all();
};

int validate(const fmc_system* sys, const fmc_disturbance* dist, const fmc_params* par,
             int64_t* S_out);
int stage_scenario(Context* c, const fmc_system* sys, const fmc_disturbance* dist,
                   const char* tag, double** canon_out, int32_t** gen_out, int** status_out);
int kron_on_device(Context* c, const fmc_network* net, double2* Yd, int* st_dev);
int choose_variant(int n, int P, int64_t N);
std::string tune_key(int n, int P, int64_t N, int precision);
int pick_variant(Context* c, int n, int P, int64_t N, int precision);
int64_t auto_chunk(int64_t S, int P, int64_t N, int bytes_per);
int run_single(Context* c, const fmc_system* sys, const fmc_disturbance* dist,
               const fmc_params* par, fmc_outputs* out);
void serve_shutdown(Context* c);

}  // namespace fmc
