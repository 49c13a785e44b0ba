// Internal launch interface between the host runtime (polymat.cpp) and the
// HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pm {

struct ScaleRec;

// ---------------------------------------------------------------- transforms

// Forward transform job: At^(p) = sum_k s^k A^(k) w^{kp}, p < L.
struct FwdJob {
  const double2* src;      // [nord][E] complex128
  void* dst;               // [L][E] double2 (FP64) or float2 (FP32); BF16: see below
  const ScaleRec* rec;     // s^k table
  int E;                   // n * n
  int nord;                // ntrunc + 1
  int n;                   // matrix size (row length of the BF16 planes)
  int pad_;
};

// Inverse transform job: C^(k) = s^-k (1/L) sum_p Ct^(p) w^{-kp}, k < nord.
struct InvJob {
  const void* src;         // [L][E] double2 or float2
  double2* dst;            // [nord][E] complex128
  ScaleRec* rec;           // s^-k / L table; out_bad is set on a non-finite store
  int E;
  int nord;
};

constexpr int kMaxTransformJobs = 64;

struct FwdArgs { FwdJob jobs[kMaxTransformJobs]; int njobs; };
struct InvArgs { InvJob jobs[kMaxTransformJobs]; int njobs; };

// Element type of the Fourier coefficients.
enum FourierType { kF64 = 0, kF32 = 1, kBF16Split = 2 };

hipError_t launch_forward(const FwdArgs& a, int L, int max_entries, FourierType t, hipStream_t s);
hipError_t launch_inverse(const InvArgs& a, int L, int max_entries, FourierType t, hipStream_t s);

// ------------------------------------------------------------------ rescale

constexpr int kNormChunks = 16;   // partial sums per (series, order)

struct NormJob {
  const double2* src;      // [nord][E]
  double* partial;         // [nord][kNormChunks]
  int E;
  int nord;
};
struct NormArgs { NormJob jobs[kMaxTransformJobs]; int njobs; };

struct ScaleJob {
  const double* partA;     // [nser][nord][kNormChunks] or null when s is fixed
  const double* partB;     // (norms of nser stacked series are combined)
  ScaleRec* rec;
  int nord;
  int L;
  double fixed_s;          // > 0: use it; 0: choose from the norms
  int nser;                // series stacked in partA (and in partB when nser_b == 0)
  int nser_b;              // > 0: series stacked in partB
};
struct ScaleArgs { ScaleJob jobs[kMaxTransformJobs]; int njobs; };

hipError_t launch_norms(const NormArgs& a, int max_nord, hipStream_t s);
hipError_t launch_scale(const ScaleArgs& a, hipStream_t s);

// --------------------------------------------------------------- products

// One product over all L modes: Ct^(p) = opA(At)^(p) opB(Bt)^(p), where a
// conjugated operand reads mode (L - p) mod L and is conjugate-transposed.
struct GemmJob {
  const void* A;
  const void* B;
  void* C;
  int n;
  int L;
  int opA;
  int opB;
  int tiles_m;
  int tiles_n;
  int tile_begin;          // first logical tile id of this job
  int pad_;
};

constexpr int kMaxGemmJobs = 48;
struct GemmArgs { GemmJob jobs[kMaxGemmJobs]; int njobs; int total_tiles; };

// Product tile configurations: rows x columns of C per work-group.  All jobs
// of one launch share the configuration and the operand forms.
struct GemmShape { int bm, bn; };
int gemm_num_configs(FourierType t);
GemmShape gemm_shape(FourierType t, int cfg);
int gemm_config(FourierType t, int n, int L);   // tuned choice for matrix size n and transform length L
bool gemm_uses_g3();                            // three-product complex form in use
hipError_t launch_gemm(const GemmArgs& a, FourierType t, int cfg, hipStream_t s);
// Direct convolution (eq. (5)) of FP64 time-domain series: job.L = ntrunc + 1
// output orders, 64 x 64 tiles (tiles_m = tiles_n = ceil(n / 64)).
constexpr int kConvTile = 64;
hipError_t launch_conv(const GemmArgs& a, hipStream_t s);
int gemm_tile_bf16();
hipError_t launch_gemm_bf16(const GemmArgs& a, hipStream_t s);

// Phase timing (polymat.cpp): when enabled, each launch is bracketed by two
// HIP events on its stream.
struct PhaseMark {
  int phase;
  hipEvent_t a;
};
PhaseMark phase_begin(int phase, hipStream_t s);
void phase_end(const PhaseMark& m, hipStream_t s);
template <typename F>
hipError_t timed(int phase, hipStream_t s, F&& launch) {
  PhaseMark m = phase_begin(phase, s);
  hipError_t e = launch();
  phase_end(m, s);
  return e;
}

// Leading dimension (elements) of one BF16 plane row for matrix size n.
__host__ __device__ inline int bf16_ld(int n) { return (n + 7) / 8 * 8; }

}  // namespace pm
