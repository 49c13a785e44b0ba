// Mode-wise complex matrix products (FFT-CONV Step 3, eq. (8)) on MFMA.
//
// For every product job and every mode p < L:
//     Ct^(p) = opA(At)^(p) * opB(Bt)^(p)
// where a plain operand X reads mode p of its transform and a conjugated
// operand (the series X^+) reads mode (L - p) mod L conjugate-transposed:
// the transform of X^+ at mode p is (Xt^(-p))^+, so X^+ costs no extra pass.
//
// Coefficients are interleaved complex (re, im) in FP64 or FP32, unpadded
// N x N row-major per mode.  A complex product is four real MFMA products
// (re*re - im*im, re*im + im*re).  One work-group computes a BM x BN tile of
// one mode with WGM x WGN wavefronts of WM x WN 16x16 blocks each; K is
// staged through double-buffered LDS in chunks of 16.  Ragged edges are
// zero-filled on load; whole 16x16 blocks and whole k-steps of 4 that lie
// outside the matrix are skipped.  Logical tile ids are remapped so that the
// tiles of one mode run on one XCD and share its L2.
#include "pm_common.h"
#include "pm_kernels.h"

#include <cstdlib>

namespace pm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Cx;
template <> struct Cx<double> {
  using T2 = double2;
  using Acc = d4;
  static constexpr int kPad = 1;   // LDS row pad (elements): 65 * 16 B = 4 banks shift
  __device__ static __forceinline__ Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of lane l sits at row 4 v + l / 16, column l % 16
  __device__ static __forceinline__ int out_row(int lane, int v) { return 4 * v + lane / 16; }
};
template <> struct Cx<float> {
  using T2 = float2;
  using Acc = f4;
  static constexpr int kPad = 2;
  __device__ static __forceinline__ Acc mfma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of lane l sits at row 4 (l / 16) + v, column l % 16
  __device__ static __forceinline__ int out_row(int lane, int v) { return 4 * (lane / 16) + v; }
};

template <typename T2> __device__ __forceinline__ T2 zero2() { T2 z; z.x = 0; z.y = 0; return z; }
template <typename T2> __device__ __forceinline__ T2 conj2(T2 v) { v.y = -v.y; return v; }

template <typename T, int WM, int WN, int WGM, int WGN>
struct GemmCfg {
  static constexpr int BM = 16 * WM * WGM;
  static constexpr int BN = 16 * WN * WGN;
  static constexpr int BK = 16;
  static constexpr int NT = kWave * WGM * WGN;
  static constexpr int LA = (BM * BK) / NT;    // A elements loaded per thread per chunk
  static constexpr int LB = (BK * BN) / NT;
  static_assert((BM * BK) % NT == 0 && (BK * BN) % NT == 0, "tile/thread mismatch");
};

// Uniform (SGPR) copy of a wave-uniform predicate, so the compiler branches on
// the scalar unit instead of masking lanes.
__device__ __forceinline__ bool uniform(bool b) { return __builtin_amdgcn_readfirstlane(b ? 1 : 0) != 0; }

// G3 selects the three-product form of the complex multiply-accumulate
// (Gauss): P1 += Xr Yr, P2 += Xi Yi, P3 += (Xr + Xi)(Yr + Yi), then
// Re = P1 - P2, Im = P3 - P1 - P2.  It issues 3 MFMAs per k-step and block
// instead of 4; the sums Xr + Xi and Yr + Yi are formed in registers from the
// staged fragments, so memory traffic is unchanged.
template <typename T, int WM, int WN, int WGM, int WGN, bool OPA, bool OPB, bool G3>
__global__ __launch_bounds__(kWave * WGM * WGN) void k_cgemm(GemmArgs args) {
  using C = Cx<T>;
  using T2 = typename C::T2;
  using Acc = typename C::Acc;
  using G = GemmCfg<T, WM, WN, WGM, WGN>;
  constexpr int BM = G::BM, BN = G::BN, BK = G::BK, NT = G::NT;
  constexpr int PAD = C::kPad;

  __shared__ T2 As[2][BK][BM + PAD];
  __shared__ T2 Bs[2][BK][BN + PAD];

  // ---- which job, mode and tile
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  int jidx = 0;
  for (int j = 1; j < args.njobs; ++j)
    if (id >= args.jobs[j].tile_begin) jidx = j;
  const GemmJob& jb = args.jobs[jidx];
  const int local = id - jb.tile_begin;
  const int per_mode = jb.tiles_m * jb.tiles_n;
  const int p = local / per_mode;
  const int rem = local - p * per_mode;
  const int tm = rem / jb.tiles_n;
  const int tn = rem - tm * jb.tiles_n;
  const int n = jb.n, L = jb.L;
  const size_t E = static_cast<size_t>(n) * n;
  const int pa = OPA ? (L - p) % L : p;
  const int pb = OPB ? (L - p) % L : p;
  const T2* __restrict__ Ag = reinterpret_cast<const T2*>(jb.A) + pa * E;
  const T2* __restrict__ Bg = reinterpret_cast<const T2*>(jb.B) + pb * E;
  T2* __restrict__ Cg = reinterpret_cast<T2*>(jb.C) + static_cast<size_t>(p) * E;
  const int row0 = tm * BM, col0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int wr = wave / WGN, wc = wave - (wave / WGN) * WGN;
  const int wrow0 = wr * 16 * WM, wcol0 = wc * 16 * WN;
  const int li = lane & 15, lk = lane >> 4;

  // ---- per-thread staging coordinates (fixed over the K loop)
  // A element (i, k): plain -> Ag[i][k] (coalesced along k); conjugated ->
  // conj(Ag[k][i]) (coalesced along i).  Same idea for B with (k, j).
  int a_i[G::LA], a_k[G::LA], b_j[G::LB], b_k[G::LB];
#pragma unroll
  for (int u = 0; u < G::LA; ++u) {
    const int q = tid + NT * u;
    if (!OPA) { a_k[u] = q % BK; a_i[u] = q / BK; } else { a_i[u] = q % BM; a_k[u] = q / BM; }
  }
#pragma unroll
  for (int u = 0; u < G::LB; ++u) {
    const int q = tid + NT * u;
    if (!OPB) { b_j[u] = q % BN; b_k[u] = q / BN; } else { b_k[u] = q % BK; b_j[u] = q / BK; }
  }

  T2 ra[G::LA], rb[G::LB];
  bool oka[G::LA], okb[G::LB];
  // Branch-free loads: out-of-range elements read a clamped in-range address;
  // they are replaced by zero only when written to LDS, so that the loads of
  // the next chunk stay in flight while the current chunk is multiplied.
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < G::LA; ++u) {
      const int gi = row0 + a_i[u], gk = k0 + a_k[u];
      const bool ok = gi < n && gk < n;
      const int ci = ok ? gi : 0, ck = ok ? gk : 0;
      ra[u] = OPA ? Ag[static_cast<size_t>(ck) * n + ci] : Ag[static_cast<size_t>(ci) * n + ck];
      oka[u] = ok;
    }
#pragma unroll
    for (int u = 0; u < G::LB; ++u) {
      const int gj = col0 + b_j[u], gk = k0 + b_k[u];
      const bool ok = gj < n && gk < n;
      const int cj = ok ? gj : 0, ck = ok ? gk : 0;
      rb[u] = OPB ? Bg[static_cast<size_t>(cj) * n + ck] : Bg[static_cast<size_t>(ck) * n + cj];
      okb[u] = ok;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int u = 0; u < G::LA; ++u) {
      T2 v;
      v.x = oka[u] ? ra[u].x : T(0);
      v.y = oka[u] ? (OPA ? -ra[u].y : ra[u].y) : T(0);
      As[buf][a_k[u]][a_i[u]] = v;
    }
#pragma unroll
    for (int u = 0; u < G::LB; ++u) {
      T2 v;
      v.x = okb[u] ? rb[u].x : T(0);
      v.y = okb[u] ? (OPB ? -rb[u].y : rb[u].y) : T(0);
      Bs[buf][b_k[u]][b_j[u]] = v;
    }
  };

  // 4-product form: cr, ci.  3-product form: cr = P1, ci = P2, c3 = P3.
  Acc cr[WM][WN], ci[WM][WN], c3[G3 ? WM : 1][G3 ? WN : 1];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) { cr[a][b] = Acc{0, 0, 0, 0}; ci[a][b] = Acc{0, 0, 0, 0}; }
  if constexpr (G3) {
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
      for (int b = 0; b < WN; ++b) c3[a][b] = Acc{0, 0, 0, 0};
  }

  // wave-uniform activity of each 16x16 block (blocks fully outside the matrix are skipped)
  bool act[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b)
      act[a][b] = uniform(row0 + wrow0 + 16 * a < n && col0 + wcol0 + 16 * b < n);

  auto mma_step = [&](int buf, int s) {
    const int kk = 4 * s + lk;
    T2 fa[WM], fb[WN];
#pragma unroll
    for (int a = 0; a < WM; ++a) fa[a] = As[buf][kk][wrow0 + 16 * a + li];
#pragma unroll
    for (int b = 0; b < WN; ++b) fb[b] = Bs[buf][kk][wcol0 + 16 * b + li];
    if constexpr (G3) {
      T sa[WM], sb[WN];
#pragma unroll
      for (int a = 0; a < WM; ++a) sa[a] = fa[a].x + fa[a].y;
#pragma unroll
      for (int b = 0; b < WN; ++b) sb[b] = fb[b].x + fb[b].y;
#pragma unroll
      for (int a = 0; a < WM; ++a) {
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          if (act[a][b]) {
            cr[a][b] = C::mfma(fa[a].x, fb[b].x, cr[a][b]);
            ci[a][b] = C::mfma(fa[a].y, fb[b].y, ci[a][b]);
            c3[a][b] = C::mfma(sa[a], sb[b], c3[a][b]);
          }
        }
      }
    } else {
#pragma unroll
      for (int a = 0; a < WM; ++a) {
        const T nai = -fa[a].y;
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          if (act[a][b]) {
            cr[a][b] = C::mfma(fa[a].x, fb[b].x, cr[a][b]);
            ci[a][b] = C::mfma(fa[a].x, fb[b].y, ci[a][b]);
          }
        }
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          if (act[a][b]) {
            cr[a][b] = C::mfma(nai, fb[b].y, cr[a][b]);
            ci[a][b] = C::mfma(fa[a].y, fb[b].x, ci[a][b]);
          }
        }
      }
    }
  };

  const int nchunks = (n + BK - 1) / BK;
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    const int k0 = c * BK;
    if (c + 1 < nchunks) load_chunk(k0 + BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s)
      if (k0 + 4 * s < n) mma_step(buf, s);
    if (c + 1 < nchunks) store_chunk(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: interleave re/im and store the tile
#pragma unroll
  for (int a = 0; a < WM; ++a) {
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      const int gj = col0 + wcol0 + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + wrow0 + 16 * a + C::out_row(lane, v);
        if (gi < n && gj < n) {
          T2 o;
          if constexpr (G3) {
            o.x = cr[a][b][v] - ci[a][b][v];
            o.y = c3[a][b][v] - cr[a][b][v] - ci[a][b][v];
          } else {
            o.x = cr[a][b][v];
            o.y = ci[a][b][v];
          }
          Cg[static_cast<size_t>(gi) * n + gj] = o;
        }
      }
    }
  }
}

// Tile shapes: 64 x 64 tiles with four wavefronts of 2 x 2 blocks.
// Three-product complex form on by default; POLYMAT_GEMM_4M=1 in the
// environment selects the four-product form (read once per process).
const bool g_gemm_g3 = [] {
  const char* e = getenv("POLYMAT_GEMM_4M");
  return !(e && e[0] == '1');
}();
constexpr int kWM = 2, kWN = 2, kWGM = 2, kWGN = 2;

}  // namespace

int gemm_tile(FourierType t) {
  return t == kBF16Split ? gemm_tile_bf16() : 16 * kWM * kWGM;
}

template <typename T, bool G3>
hipError_t launch_typed(const GemmArgs& a, hipStream_t s) {
  // all jobs of one launch share their operand forms (the host groups them)
  const int oa = a.jobs[0].opA, ob = a.jobs[0].opB;
  constexpr int nt = kWave * kWGM * kWGN;
  if (!oa && !ob) k_cgemm<T, kWM, kWN, kWGM, kWGN, false, false, G3><<<a.total_tiles, nt, 0, s>>>(a);
  else if (!oa && ob) k_cgemm<T, kWM, kWN, kWGM, kWGN, false, true, G3><<<a.total_tiles, nt, 0, s>>>(a);
  else if (oa && !ob) k_cgemm<T, kWM, kWN, kWGM, kWGN, true, false, G3><<<a.total_tiles, nt, 0, s>>>(a);
  else k_cgemm<T, kWM, kWN, kWGM, kWGN, true, true, G3><<<a.total_tiles, nt, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& a, FourierType t, hipStream_t s) {
  if (a.njobs <= 0 || a.total_tiles <= 0) return hipSuccess;
  if (t == kF64) return g_gemm_g3 ? launch_typed<double, true>(a, s) : launch_typed<double, false>(a, s);
  if (t == kF32) return g_gemm_g3 ? launch_typed<float, true>(a, s) : launch_typed<float, false>(a, s);
  return launch_gemm_bf16(a, s);
}

}  // namespace pm
