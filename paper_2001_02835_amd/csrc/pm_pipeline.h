// Persistent batch pipeline: the interface between the host runtime and the
// one-launch form of a batch of FP64 FFT-CONV products (Section 2, Steps 1-5
// and the batching paragraph).  Not part of the public ABI.
//
// A batch of up to kMaxPipeProblems products is cut into tickets: per-order
// norms (NORM), the choice of s (SCALE), forward-transform blocks (FWD),
// 64 x 64 product tiles of one mode (GEMM) and inverse-transform blocks (INV).
// Work-groups of one persistent launch claim tickets in a fixed order through
// a device counter; a ticket that needs the output of another waits for that
// problem's completion counter of the previous stage.  Every dependency
// precedes its dependent in the ticket order, so a ticket only waits for
// tickets that running work-groups already hold, and the launch cannot
// deadlock whatever the number of resident work-groups.
#pragma once

#include <hip/hip_runtime.h>

#include "pm_common.h"
#include "pm_kernels.h"

namespace pm {

constexpr int kMaxPipeProblems = 64;
constexpr int kMaxPipeSegs = 5 * kMaxPipeProblems;
constexpr int kPipeInitChunk = 24;        // problem descriptors per set-up launch
constexpr int kPipeTile = 64;             // product tile (rows and columns)
constexpr int kPipeRep = 2;               // transform blocks per ticket and half work-group

enum PipeStage { kStNorm = 0, kStScale = 1, kStFwd = 2, kStGemm = 3, kStInv = 4 };

// Device-memory (global address space) pointer.  The descriptors below are
// read from device memory by the pipeline kernel; typed this way, every access
// through them compiles to global instructions instead of flat ones (flat
// accesses share a completion counter with LDS and would serialise the load
// pipelines of the product tiles).
#define PM_GLOBAL __attribute__((address_space(1)))

// One product of the pipeline (device copy written by the set-up kernel).
struct PipeProblem {
  const PM_GLOBAL double2* A;
  const PM_GLOBAL double2* B;
  PM_GLOBAL double2* C;
  PM_GLOBAL double2* At;     // Fourier coefficients of A, B and of the product (FP64 [L][n][n])
  PM_GLOBAL double2* Bt;
  PM_GLOBAL double2* Ct;
  PM_GLOBAL double* partA;   // per-order norms [nord][kNormChunks] (the pipeline fills chunk 0)
  PM_GLOBAL double* partB;
  PM_GLOBAL ScaleRec* rec;
  double scale;       // > 0: fixed s; 0: chosen from the norms
  int n;
  int nord;
  int ops;            // op_a | op_b << 1
  int pad_;
};

// Per-product control block in the product's workspace region.  done[s] counts
// the finished tickets of stage s; next and abort are used in the first
// product's block only (the ticket counter and the abort flag of the launch).
struct PipeSlot {
  PipeProblem prob;
  unsigned int done[4];
  unsigned int next;
  unsigned int abort;
  unsigned int pad_[10];
};

struct PipeSeg {
  unsigned int start;        // first ticket
  unsigned short stage;
  unsigned short prob;       // index into PipeArgs::slot
};

struct PipeArgs {
  PipeSlot* slot[kMaxPipeProblems];
  PipeSeg segs[kMaxPipeSegs];
  int nseg;
  unsigned int total;        // number of tickets
  unsigned int spin_limit;   // bound of every wait (polls); then the launch aborts
};

struct PipeInitArgs {
  PipeProblem probs[kPipeInitChunk];
  PipeSlot* slot[kPipeInitChunk];
  PipeSlot* ctl;             // slot of the launch's ticket counter and abort flag
  int count;
  int reset_ctl;
};

// ---- ticket counts, shared by the host plan and the kernel

__host__ __device__ inline int pipe_tlen(int nord) {
  int L = 4;
  while (L < 2 * nord) L *= 2;
  return L;
}
// lanes per matrix entry in the pipeline's transforms: two from L = 64 on, so
// that a lane's registers fit the 128 of four wavefronts per SIMD
__host__ __device__ constexpr int pipe_split(int L) { return L >= 64 ? 2 : 1; }
// entries of one transform ticket: two half work-groups, kPipeRep blocks each
__host__ __device__ inline int pipe_ent(int L) { return 2 * kPipeRep * (64 / pipe_split(L)); }
__host__ __device__ inline int pipe_blocks(int n, int L) { return (n * n + pipe_ent(L) - 1) / pipe_ent(L); }
__host__ __device__ inline int pipe_tiles(int n) { return (n + kPipeTile - 1) / kPipeTile; }
__host__ __device__ inline unsigned pipe_count(const PipeProblem& p, int stage) {
  const int L = pipe_tlen(p.nord);
  switch (stage) {
    case kStNorm: return p.scale > 0.0 ? 0u : 2u * p.nord;
    case kStScale: return 1u;
    case kStFwd: return 2u * pipe_blocks(p.n, L);
    case kStGemm: return static_cast<unsigned>(L) * pipe_tiles(p.n) * pipe_tiles(p.n);
    default: return static_cast<unsigned>(pipe_blocks(p.n, L));
  }
}

hipError_t launch_pipeline_init(const PipeInitArgs& a, hipStream_t s);
hipError_t launch_pipeline(const PipeArgs& a, int grid, hipStream_t s);
int pipeline_threads();

}  // namespace pm
