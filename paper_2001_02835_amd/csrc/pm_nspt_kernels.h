// Launch interface of the NSPT-specific kernels (pm_nspt_kernels.hip).
#pragma once

#include "pm_kernels.h"

namespace pm {

constexpr int kMaxAdd = 8;

// Re-truncation of a Fourier-space product (see pm_nspt_kernels.hip).
struct RetruncJob {
  const void* src;         // [L][E] product (FP64/FP32), or null for "no product"
  void* dst;               // [L][E] Fourier output in the product-input format
  double2* tdst;           // optional [nord][E] time-domain output (same scaling)
  const double2* add;      // addend a (a < nadd) at add + a * add_stride: [nord][E]
  size_t add_stride;       // elements between consecutive addends
  int E;
  int n;
  int nord;
  int pad_;
};
constexpr int kMaxRetruncJobs = 48;
struct RetruncArgs {
  RetruncJob jobs[kMaxRetruncJobs];
  double2 coef[kMaxAdd];   // addend weights (shared by the jobs of a launch)
  double2 idcoef;          // weight of the unit series
  int nadd;
  int njobs;
};

// Inverse transform of sum_q coef[q] * src[q], unscaled, orders kmin..nord-1.
// nsrc is 1, 6 or 8 (the instantiated source counts), the same for every job
// of a launch.
constexpr int kMaxCombine = 8;
struct CombineJob {
  const void* src[kMaxCombine];
  double2 coef[kMaxCombine];
  double2* dst;
  const ScaleRec* rec;
  int nsrc;
  int E;
  int nord;
  int kmin;
};
constexpr int kMaxCombineJobs = 12;
struct CombineArgs { CombineJob jobs[kMaxCombineJobs]; int njobs; };

struct TraceJob {
  const double2* src;      // [nord][n][n]
  double2* out;            // [nord]
  int n;
  int nord;
};
struct TraceArgs { TraceJob jobs[kMaxTransformJobs]; int njobs; };

struct ForceJob {
  const double2* M;        // [nord][n][n], unscaled
  const double2* tr;       // [nord] traces of M
  const double2* eta;      // [n][n] noise (Langevin form), or null for none
  double2* P;              // [nord][n][n] momentum series, updated (MD form)
  double2* Y;              // [nord][n][n] output, multiplied by s^k, or null (MD form only)
  const ScaleRec* rec;
  int n;
  int nord;
};
constexpr int kMaxForceJobs = 48;
// md == 0: Y = i (eps F + sqrt(2 eps) eta g).  md == 1: P^(k) += kick F^(k)
// for k >= 1, then Y = i dt P.
struct ForceArgs {
  ForceJob jobs[kMaxForceJobs];
  double eps;
  double noise_amp;
  double kick;
  double dt;
  int md;
  int njobs;
};

// Momentum refresh: P^(1) = eta, every other order zero.
struct RefreshJob {
  double2* P;              // [nord][E]
  const double2* eta;      // [E]
  int E;
  int nord;
};
constexpr int kMaxRefreshJobs = 64;
struct RefreshArgs { RefreshJob jobs[kMaxRefreshJobs]; int njobs; };
constexpr int kMaxMdSteps = 100000;

// S[i] = c0 delta_{k0} + c1 Re tr[i], k = i mod nord (action or Wilson-loop series).
struct ActionArgs { const double2* tr; double* S; double c0; double c1; int nord; int count; };

// x^(k) <- s^k x^(k) in place (order k of a [nord][E] series).
struct SeriesScaleJob {
  double2* x;
  const ScaleRec* rec;
  int E;
  int nord;
};
constexpr int kMaxSeriesScaleJobs = 64;
struct SeriesScaleArgs { SeriesScaleJob jobs[kMaxSeriesScaleJobs]; int njobs; };

// lin: transform length of the products being re-truncated; lout: length of
// the forward transform written (lout == lin, or 2 lin for lin <= 32).
hipError_t launch_retrunc(const RetruncArgs& a, int lin, int lout, int max_entries, FourierType fin,
                          FourierType fout, hipStream_t s);
hipError_t launch_inv_combine(const CombineArgs& a, int L, int max_entries, FourierType fin, hipStream_t s);
hipError_t launch_trace(const TraceArgs& a, int max_nord, hipStream_t s);
hipError_t launch_force(const ForceArgs& a, int n, int max_nord, hipStream_t s);
hipError_t launch_refresh(const RefreshArgs& a, hipStream_t s);

// Counter-based Langevin noise: `count` Hermitian traceless n x n matrices
// (matrix m = 4 r + mu) of step `step` under `seed` (Philox4x64-10 and
// Box-Muller; the mapping is documented with nspt_noise in polymat.h).
struct NoiseArgs {
  double2* eta;            // [count][n][n]
  unsigned long long seed;
  unsigned long long step;
  int n;
  int count;
};
hipError_t launch_noise(const NoiseArgs& a, hipStream_t s);
hipError_t launch_action(const ActionArgs& a, hipStream_t s);
hipError_t launch_series_scale(const SeriesScaleArgs& a, int max_nord, hipStream_t s);

}  // namespace pm
