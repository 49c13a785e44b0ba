// Internal interface of the NSPT updates (pm_nspt.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "polymat.h"

namespace pm {

size_t nspt_workspace_bytes(int replicas, const nspt_params* params, int precision);
pm_status nspt_step(void* U, const void* eta, int replicas, const nspt_params* params, int precision,
                    void* workspace, size_t workspace_bytes, hipStream_t stream);
pm_status nspt_series_action(const void* U, int replicas, const nspt_params* params, int precision, double* S,
                             void* workspace, size_t workspace_bytes, hipStream_t stream);
pm_status nspt_wilson(const void* U, int replicas, const nspt_params* params, int a, int b, int precision,
                      double* W, void* workspace, size_t workspace_bytes, hipStream_t stream);
pm_status nspt_noise(void* eta, int replicas, int n, unsigned long long seed, unsigned long long step,
                     hipStream_t stream);
pm_status nspt_steps(void* U, int replicas, const nspt_params* params, unsigned long long seed,
                     unsigned long long step0, int nsteps, int precision, void* workspace, size_t workspace_bytes,
                     hipStream_t stream);
pm_status nspt_gauge(void* U, int replicas, const nspt_params* params, double alpha, int precision,
                     void* workspace, size_t workspace_bytes, hipStream_t stream);
pm_status nspt_md(void* U, void* P, const void* eta, int replicas, const nspt_params* params, int nsteps,
                  int precision, void* workspace, size_t workspace_bytes, hipStream_t stream);

}  // namespace pm
