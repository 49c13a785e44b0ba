// NSPT Euler-Langevin step of the TEK model (validation only so far).
#include <cmath>

#include "pm_nspt.h"

namespace pm {

namespace {
bool valid_params(int replicas, const nspt_params* p, int prec) {
  if (!p || replicas < 1) return false;
  if (prec != PM_PREC_FP64 && prec != PM_PREC_FP32 && prec != PM_PREC_BF16X3) return false;
  if (p->L < 1 || p->L % 2 == 0 || p->n != p->L * p->L) return false;
  if (p->ntrunc < 0 || p->ntrunc > PM_MAX_NTRUNC) return false;
  if (!std::isfinite(p->eps) || p->eps <= 0.0) return false;
  return true;
}
}  // namespace

size_t nspt_workspace_bytes(int replicas, const nspt_params* p, int prec) {
  if (!valid_params(replicas, p, prec)) return 0;
  const size_t E = static_cast<size_t>(p->n) * p->n;
  return static_cast<size_t>(replicas) * 64 * (p->ntrunc + 1) * E * 16;
}

pm_status nspt_step(void* U, const void* eta, int replicas, const nspt_params* p, int prec,
                    void* workspace, size_t workspace_bytes, hipStream_t) {
  if (!valid_params(replicas, p, prec)) return PM_ERR_INVALID;
  if (!U || !eta || !workspace) return PM_ERR_INVALID;
  if (workspace_bytes < nspt_workspace_bytes(replicas, p, prec)) return PM_ERR_WORKSPACE;
  return PM_ERR_UNSUPPORTED;
}

}  // namespace pm
