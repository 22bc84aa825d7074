// fmc_serve.hip -- batched (persistent launch) and served (continuous
// batching) forms of the method.
#include <hip/hip_runtime.h>

#include <string>

#include "fmc_runtime.hpp"

namespace fmc {

struct ServeState {};

void serve_shutdown(Context* c) {
  delete c->serve;
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
  const int64_t n = scen->sys->n_gen, P = scen->dist->n_proc, K = scen->par->K, N = scen->par->N;
  const int64_t V = 2 * n + P, C = 2 * S + 1;
  const int64_t bw = scen->par->precision == FMC_F64 ? 8 : 4;
  const int64_t groups = (N + 63) / 64;
  const int64_t Sc = auto_chunk(S, (int)P, N, (int)bw);
  int64_t b = 0;
  b += P * K * N * 8;                 // zeta
  b += K * C * 8;                     // basis
  b += (2 * Sc + 1) * P * N * bw;     // one chunk of KLE paths
  b += (2 * n + P + 16) * groups * 64 * bw;  // state
  b += groups * (S + 1) * V * 16;     // per-group statistics
  b += 2 * (S + 1) * V * 8;           // mean, var
  b += 2 * n * n * 16 + 64 * n;       // reduced network, coefficients
  *bytes = b;
  return FMC_OK;
}

int fmc_submit(fmc_context* ctx, const fmc_scenario* scen, fmc_outputs* out, uint64_t* ticket) {
  (void)ctx; (void)scen; (void)out; (void)ticket;
  return fail(FMC_EINVAL, "fmc_submit: not available in this build");
}

int fmc_poll(fmc_context* ctx, uint64_t ticket) {
  (void)ctx; (void)ticket;
  return fail(FMC_EINVAL, "unknown ticket");
}

int fmc_wait(fmc_context* ctx, uint64_t ticket, double timeout_s) {
  (void)ctx; (void)ticket; (void)timeout_s;
  return fail(FMC_EINVAL, "unknown ticket");
}

int fmc_cancel(fmc_context* ctx, uint64_t ticket) {
  (void)ctx; (void)ticket;
  return fail(FMC_EINVAL, "unknown ticket");
}

}  // extern "C"
