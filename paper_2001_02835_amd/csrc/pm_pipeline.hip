// Persistent batch pipeline: every step of FFT-CONV (Section 2, Steps 1-5,
// eqs. (6)-(9)) for a batch of FP64 products in one launch, so that the
// HBM-bound transforms of some products run beside the matrix-core-bound
// mode-wise products of others (the batching paragraph of Section 2: the
// transforms are batched over matrix entries and the products over modes;
// here the problems of a batch may differ in N and ntrunc).
//
// Tickets (pm_pipeline.h) are claimed in a fixed order through an atomic
// counter; per problem the stages are NORM -> SCALE -> FWD -> GEMM -> INV,
// and the host orders the tickets so that the preparation of the next
// problems is interleaved with the products of the current ones:
//   iteration i:  SCALE(i-1), NORM(i), FWD(i-2), GEMM(i-3), INV(i-5)
// over the problems sorted by product work, largest first.
//
// Synchronisation: a finished ticket makes its stores visible to the whole
// device (release at agent scope: the XCD's L2 is written back) and adds one
// to its problem's counter; a waiting work-group polls that counter with
// relaxed loads and takes one acquire fence when it is complete.  Every wait
// is bounded (spin_limit polls); a wait that runs out sets the launch's abort
// flag, and every work-group that sees the flag leaves its loop, so the
// launch always ends.
#include "pm_fft.h"
#include "pm_gemm_impl.h"
#include "pm_pipeline.h"
#include "pm_scale.h"

namespace pm {

namespace {

constexpr int kThreads = 2 * kFftThreads;   // 8 wavefronts; two transform halves
// product tiles of 64 x 64 (8 wavefronts of 2 x 1 blocks of 16 x 16)
constexpr int kWM = 2, kWN = 1, kWGM = 2, kWGN = 4;
static_assert(16 * kWM * kWGM == kPipeTile && 16 * kWN * kWGN == kPipeTile, "pipeline tile shape");
static_assert(kWave * kWGM * kWGN == kThreads, "pipeline work-group size");
constexpr size_t kGemmLds = gemm_detail::Tile2<double, kWM, kWN, kWGM, kWGN>::kLdsBytes;
// one transform half: L/2 x ENT entries of 16 bytes (2048 entries for L = 64 and 128)
constexpr size_t kHalfLds = sizeof(double2) * 2048;
constexpr size_t kLds = kGemmLds > 2 * kHalfLds ? kGemmLds : 2 * kHalfLds;

// generic view of a descriptor pointer (the global-ness propagates from the cast)
template <typename T>
__device__ __forceinline__ T* gen(PM_GLOBAL T* p) {
  return (T*)p;
}

__device__ __forceinline__ int pipe_wait(unsigned int* cnt, unsigned int need, unsigned int* abort,
                                         unsigned int limit) {
  unsigned int spins = 0;
  for (;;) {
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) break;
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return 0;
    if (++spins > limit) {
      __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return 1;
}

// NORM ticket: ||X^(k)||_F^2 of one order of one operand over all entries
// (eight independent loads in flight per thread), stored as chunk 0 of the
// norm record; the other chunks are zeroed.
__device__ __forceinline__ void norm_ticket(const PipeProblem& P, unsigned int local, double* red) {
  const int side = local / P.nord, k = local % P.nord;
  const int E = P.n * P.n;
  const double2* x = gen(side ? P.B : P.A) + static_cast<size_t>(k) * E;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int e0 = threadIdx.x; e0 < E; e0 += 8 * kThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads;
      if (e < E) {
        const double2 v = x[e];
        s[u] = fma(v.x, v.x, fma(v.y, v.y, s[u]));
      }
    }
  }
  double sum = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = sum;
  __syncthreads();
  double* part = gen(side ? P.partB : P.partA) + k * kNormChunks;
  if (threadIdx.x < kNormChunks) {
    double v = 0.0;
    if (threadIdx.x == 0) v = ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7]));
    part[threadIdx.x] = v;
  }
}

// FWD ticket: Steps 1-2 for kPipeRep blocks of ENT entries per half
// work-group (rescale by s^k and zero padding while staging in LDS).
template <int L>
__device__ __forceinline__ void fwd_ticket(const PipeProblem& P, unsigned int local, char* smem) {
  constexpr int S = pipe_split(L);
  constexpr int ENT = kEnt / S;
  constexpr int KSTEP = kFftThreads / ENT;
  typedef double2 Tile[L / 2][ENT];
  static_assert(sizeof(Tile) <= kHalfLds, "transform tile");
  const int nblk = pipe_blocks(P.n, L);
  const int side = local / nblk, blk = local % nblk;
  const int h = threadIdx.x / kFftThreads;
  const int tid = threadIdx.x % kFftThreads;
  Tile& tile = *reinterpret_cast<Tile*>(smem + h * kHalfLds);
  const double2* src = gen(side ? P.B : P.A);
  void* dst = gen(side ? P.Bt : P.At);
  const int E = P.n * P.n;
  const int lane = tid & (kWave - 1), r = tid / kWave, el = tid % ENT;
#pragma unroll 1
  for (int rep = 0; rep < kPipeRep; ++rep) {
    const int e = ((blk * kPipeRep + rep) * 2 + h) * ENT + el;
    const bool valid = e < E;
    for (int k = tid / ENT; k < L / 2; k += KSTEP) {
      double2 v = (valid && k < P.nord) ? src[static_cast<size_t>(k) * E + e] : make_double2(0.0, 0.0);
      tile[k][el] = k < P.nord ? cscale(v, P.rec->spow[k]) : v;
    }
    __syncthreads();
    forward_from_tile<L, kF64, S>(tile, lane, r, dst, E, P.n, e, valid);
    __syncthreads();
  }
}

// INV ticket: Steps 4-5 (inverse transform, 1/L, truncation, unscaling).
template <int L>
__device__ __forceinline__ void inv_ticket(const PipeProblem& P, unsigned int local, char* smem) {
  constexpr int S = pipe_split(L);
  constexpr int ENT = kEnt / S;
  constexpr int KSTEP = kFftThreads / ENT;
  typedef double2 Acc[L / 2][ENT];
  static_assert(sizeof(Acc) <= kHalfLds, "transform tile");
  const int h = threadIdx.x / kFftThreads;
  const int tid = threadIdx.x % kFftThreads;
  Acc& acc = *reinterpret_cast<Acc*>(smem + h * kHalfLds);
  const int E = P.n * P.n;
  const int lane = tid & (kWave - 1), r = tid / kWave, el = tid % ENT;
  bool bad = false;
#pragma unroll 1
  for (int rep = 0; rep < kPipeRep; ++rep) {
    const int e = ((static_cast<int>(local) * kPipeRep + rep) * 2 + h) * ENT + el;
    const bool valid = e < E;
    auto load = [&](int p) { return valid ? load_mode<kF64>(gen(P.Ct), E, p, e) : make_double2(0.0, 0.0); };
    inverse_to_lds<L, S>(load, acc, lane, r);
    if (valid) {
      for (int k = tid / ENT; k < P.nord; k += KSTEP) {
        const double2 v = cscale(acc[k][el], P.rec->sinv[k]);
        bad = bad || !isfinite(v.x) || !isfinite(v.y);
        gen(P.C)[static_cast<size_t>(k) * E + e] = v;
      }
    }
    __syncthreads();
  }
  if (bad) P.rec->out_bad = 1u;
}

// GEMM ticket: one 64 x 64 tile of one mode (Step 3, eq. (8)), three-product
// complex form.
template <bool OA, bool OB>
__device__ __forceinline__ void gemm_ticket(const PipeProblem& P, unsigned int local, char* smem) {
  const int L = pipe_tlen(P.nord);
  const int tiles = pipe_tiles(P.n);
  const int per = tiles * tiles;
  const int p = local / per, rem = local % per;
  GemmJob jb{};
  jb.A = gen(P.At);
  jb.B = gen(P.Bt);
  jb.C = gen(P.Ct);
  jb.n = P.n;
  jb.L = L;
  jb.opA = OA;
  jb.opB = OB;
  jb.tiles_m = tiles;
  jb.tiles_n = tiles;
  gemm_detail::cgemm2_tile<double, kWM, kWN, kWGM, kWGN, OA, OB, true, false, true>(jb, p, rem / tiles, rem % tiles,
                                                                                   smem);
}

template <int L>
__device__ __forceinline__ void transform_ticket(bool fwd, const PipeProblem& P, unsigned int local, char* smem) {
  if (fwd) fwd_ticket<L>(P, local, smem);
  else inv_ticket<L>(P, local, smem);
}

__global__ __launch_bounds__(kThreads, 4) void k_pipeline(PipeArgs args) {
  __shared__ __attribute__((aligned(16))) char smem[kLds];
  __shared__ double red[kThreads / kWave];
  __shared__ unsigned int s_ticket;
  __shared__ int s_go;
  PipeSlot* ctl = args.slot[0];
  for (;;) {
    if (threadIdx.x == 0) {
      const bool stop = __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
      s_ticket = stop ? args.total : atomicAdd(&ctl->next, 1u);
    }
    __syncthreads();
    const unsigned int t = s_ticket;
    if (t >= args.total) break;
    // the segment of ticket t
    int lo = 0, hi = args.nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (args.segs[mid].start <= t) lo = mid;
      else hi = mid - 1;
    }
    const int stage = args.segs[lo].stage;
    const unsigned int local = t - args.segs[lo].start;
    PipeSlot* S = args.slot[args.segs[lo].prob];
    const PipeProblem& P = S->prob;
    // the stage this ticket depends on, if any
    int dep = -1;
    unsigned int need = 0;
    if (stage == kStScale && P.scale <= 0.0) { dep = kStNorm; need = pipe_count(P, kStNorm); }
    else if (stage == kStFwd) { dep = kStScale; need = 1; }
    else if (stage == kStGemm) { dep = kStFwd; need = pipe_count(P, kStFwd); }
    else if (stage == kStInv) { dep = kStGemm; need = pipe_count(P, kStGemm); }
    if (dep >= 0) {
      if (threadIdx.x == 0) s_go = pipe_wait(&S->done[dep], need, &ctl->abort, args.spin_limit);
      __syncthreads();
      if (!s_go) break;
    }
    const int L = pipe_tlen(P.nord);
    if (stage == kStNorm) {
      norm_ticket(P, local, red);
    } else if (stage == kStScale) {
      if (threadIdx.x < kWave) {
        ScaleJob j{};
        j.partA = gen(P.partA);
        j.partB = gen(P.partB);
        j.rec = gen(P.rec);
        j.nord = P.nord;
        j.L = L;
        j.fixed_s = P.scale;
        j.nser = 1;
        j.nser_b = 0;
        scale_wave(j, threadIdx.x);
      }
    } else if (stage == kStGemm) {
      switch (P.ops) {
        case 0: gemm_ticket<false, false>(P, local, smem); break;
        case 1: gemm_ticket<true, false>(P, local, smem); break;
        case 2: gemm_ticket<false, true>(P, local, smem); break;
        default: gemm_ticket<true, true>(P, local, smem); break;
      }
    } else {
      const bool fwd = stage == kStFwd;
      switch (L) {
        case 4: transform_ticket<4>(fwd, P, local, smem); break;
        case 8: transform_ticket<8>(fwd, P, local, smem); break;
        case 16: transform_ticket<16>(fwd, P, local, smem); break;
        case 32: transform_ticket<32>(fwd, P, local, smem); break;
        case 64: transform_ticket<64>(fwd, P, local, smem); break;
        default: transform_ticket<128>(fwd, P, local, smem); break;
      }
    }
    __syncthreads();
    // publish: this work-group's stores, then the problem's stage counter
    if (stage != kStInv && threadIdx.x == 0)
      __hip_atomic_fetch_add(&S->done[stage], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_pipeline_init(PipeInitArgs a) {
  const int i = threadIdx.x;
  if (i < a.count) {
    PipeSlot* S = a.slot[i];
    S->prob = a.probs[i];
#pragma unroll
    for (int s = 0; s < 4; ++s) S->done[s] = 0u;
  }
  if (a.reset_ctl && i == 0) {
    a.ctl->next = 0u;
    a.ctl->abort = 0u;
  }
}

}  // namespace

int pipeline_threads() { return kThreads; }

hipError_t launch_pipeline_init(const PipeInitArgs& a, hipStream_t s) {
  k_pipeline_init<<<1, kWave, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_pipeline(const PipeArgs& a, int grid, hipStream_t s) {
  k_pipeline<<<grid, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pm
