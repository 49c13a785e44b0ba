#pragma once
// Mode-wise complex matrix products (FFT-CONV Step 3, eq. (8)) on MFMA:
// the kernel template shared by the FP64 and FP32 instantiations.
//
// For every product job and every mode p < L:
//     Ct^(p) = opA(At)^(p) * opB(Bt)^(p)
// where a plain operand X reads mode p of its transform and a conjugated
// operand (the series X^+) reads mode (L - p) mod L conjugate-transposed:
// the transform of X^+ at mode p is (Xt^(-p))^+, so X^+ costs no extra pass.
//
// Coefficients are interleaved complex (re, im) in FP64 or FP32, unpadded
// N x N row-major per mode.  A complex product is three real MFMA products
// in the Gauss form (four, re*re - im*im and re*im + im*re, when selected;
// see G3 below).  One work-group computes a BM x BN tile of
// one mode with WGM x WGN wavefronts of WM x WN 16x16 blocks each; K is
// staged through double-buffered LDS in chunks of 16.  Ragged edges are
// zero-filled on load; whole 16x16 blocks and whole k-steps of 4 that lie
// outside the matrix are skipped.  Logical tile ids are remapped so that the
// tiles of one mode run on one XCD and share its L2.
#include "pm_common.h"
#include "pm_kernels.h"

#include <cstdlib>

namespace pm {

namespace gemm_detail {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Cx;
template <> struct Cx<double> {
  using T2 = double2;
  using Acc = d4;
  // LDS tile of BK = 16 rows of W elements (see the layout note at Tile2):
  // rows of W elements, every fourth row start moved on by 4 elements, and
  // the two low bits of the column XOR-ed with k & 3
  static constexpr bool kSwizzle = true;
  __host__ __device__ static constexpr int tile_elems(int W) { return 16 * W + 16; }
  __device__ static __forceinline__ int lds(int W, int k, int x) { return k * W + (k >> 2) * 4 + (x ^ (k & 3)); }
  __device__ static __forceinline__ Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of lane l sits at row 4 v + l / 16, column l % 16
  __device__ static __forceinline__ int out_row(int lane, int v) { return 4 * v + lane / 16; }
};
template <> struct Cx<float> {
  using T2 = float2;
  using Acc = f4;
  // LDS tile: rows of W + 1 elements
  static constexpr bool kSwizzle = false;
  __host__ __device__ static constexpr int tile_elems(int W) { return 16 * (W + 1); }
  __device__ static __forceinline__ int lds(int W, int k, int x) { return k * (W + 1) + x; }
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

// The kernel: both operand tiles are staged k-major in LDS (A as [k][i], B
// as [k][j]), so that every fragment read is a run of 16 elements across the
// 16 lanes of a lane group, and the k index is permuted across the lane
// groups of the MFMA (the MFMA only needs A and B to agree on it).  The
// fragments of the next k-step are read from LDS while the current MFMAs
// issue.
//
// Layout of the 16-byte (FP64 complex) elements.  A 128-bit LDS read of a
// wavefront runs at full rate on gfx950 (measured) when the four lane groups
// see the same arrangement of 16-byte slots within 256 bytes, up to a common
// shift and an XOR of the slot index by 0..3 that may differ per group; rows
// of 65 elements read by different groups (a different rotation per group)
// cost four times the cycles.  The FP64 tiles therefore use rows of W = 64
// elements (1 KB, so that rows start on the same slot), every block of four
// rows moved on by 4 elements (64 bytes), and the two low bits of the column
// XOR-ed with k & 3; in k-step s lane group g contracts k = g + 4 s.  A
// fragment read of k-step s then sees slot (li ^ g) + 4 s in lane li of group
// g (a common shift and a per-group XOR), with the k-step in the address
// offset only; the transposed stores of A (16 lanes writing one column of 16
// rows) land in 16 distinct slots.  The FP32 tiles (8-byte elements, 64-bit
// reads) keep rows of 65 elements and k = 4 g + s.
template <typename T, int WM, int WN, int WGM, int WGN>
struct Tile2 {
  using T2 = typename Cx<T>::T2;
  using G = GemmCfg<T, WM, WN, WGM, WGN>;
  static constexpr int BM = G::BM, BN = G::BN, BK = G::BK;
  static constexpr int kAElems = 2 * Cx<T>::tile_elems(BM);
  static constexpr int kBElems = 2 * Cx<T>::tile_elems(BN);
  static constexpr size_t kLdsBytes = sizeof(T2) * (kAElems + kBElems);
};

// Eight wavefronts of 2 blocks each: built for four wavefronts per SIMD, so
// that two work-groups share a CU (their LDS fits twice).
template <int WM, int WN, int WGM, int WGN>
constexpr int cgemm2_min_waves() { return (WM * WN <= 2 && WGM * WGN == 8) ? 4 : 1; }

// CONV selects the direct form of eq. (5) instead of a Fourier mode: p is an
// output order k, A and B are time-domain series [L = ntrunc+1][n][n], and
// the contraction runs over (l, kk) for l = 0..k: C^(k) = sum_l opA(A)^(l)
// opB(B)^(k-l), one K block of n per term (each block zero-padded to whole
// chunks).
template <typename T, int WM, int WN, int WGM, int WGN, bool OPA, bool OPB, bool G3, bool CONV = false,
          bool ONE_STAGE = false>
__device__ __forceinline__ void cgemm2_tile(const GemmJob& jb, int p, int tm, int tn, char* smem) {
  using C = Cx<T>;
  using T2 = typename C::T2;
  using Acc = typename C::Acc;
  using G = GemmCfg<T, WM, WN, WGM, WGN>;
  constexpr int BM = G::BM, BN = G::BN, BK = G::BK, NT = G::NT;
  constexpr int TA = C::tile_elems(BM), TB = C::tile_elems(BN);
  // the k of lane group g in k-step s
  auto kidx = [](int g, int s) { return C::kSwizzle ? g + 4 * s : 4 * g + s; };
  T2* As = reinterpret_cast<T2*>(smem);                                   // [2][TA]
  T2* Bs = reinterpret_cast<T2*>(smem + sizeof(T2) * Tile2<T, WM, WN, WGM, WGN>::kAElems);   // [2][TB]

  const int n = jb.n, L = jb.L;
  const size_t E = static_cast<size_t>(n) * n;
  const int pa = CONV ? 0 : (OPA ? (L - p) % L : p);
  const int pb = CONV ? 0 : (OPB ? (L - p) % L : p);
  const T2* __restrict__ Ag = reinterpret_cast<const T2*>(jb.A) + pa * E;
  const T2* __restrict__ Bg = reinterpret_cast<const T2*>(jb.B) + pb * E;
  T2* __restrict__ Cg = reinterpret_cast<T2*>(jb.C) + static_cast<size_t>(p) * E;
  const int cpl = (n + BK - 1) / BK;   // chunks per term (CONV)
  const int row0 = tm * BM, col0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  // wavefront (wr, wc) owns the 16 x 16 blocks (wr + WGM a, wc + WGN b) of the
  // tile.  Interleaved this way, the blocks of a ragged edge tile that lie
  // inside the matrix are spread over all wavefronts instead of leaving whole
  // wavefronts idle; wr varies fastest with the wavefront index, so that the
  // wavefronts of one SIMD (w, w + 4, ...) take different tile columns.
  const int wr = wave % WGM, wc = wave / WGM;
  auto brow = [&](int a) { return 16 * (wr + WGM * a); };
  auto bcol = [&](int b) { return 16 * (wc + WGN * b); };
  const int li = lane & 15, lg = lane >> 4;

  // staging coordinates: tile element (i, kk) of A and (kk, j) of B
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

  // register stages of the global loads.  With two (the 2-block, 8-wavefront
  // shapes, which fit in 128 registers) the loads of chunk c + 2 are in
  // flight while chunk c is multiplied and chunk c + 1 goes to LDS; with one
  // the loads run one chunk ahead.
  constexpr bool PF2 = cgemm2_min_waves<WM, WN, WGM, WGN>() == 4 && !ONE_STAGE;
  constexpr int D = PF2 ? 2 : 1;
  struct Stage {
    T2 ra[G::LA], rb[G::LB];
    bool oka[G::LA], okb[G::LB];
  };
  Stage st0, st1;
  // chunk c: its k offset within the current term, and (CONV) the term's
  // operand orders l and p - l
  auto chunk_k0 = [&](int c) { return CONV ? (c - (c / cpl) * cpl) * BK : c * BK; };
  auto load_chunk = [&](int c, Stage& S) {
    const int k0 = chunk_k0(c);
    const T2* __restrict__ Ac = Ag;
    const T2* __restrict__ Bc = Bg;
    if constexpr (CONV) {
      const int l = c / cpl;
      Ac = Ag + static_cast<size_t>(l) * E;
      Bc = Bg + static_cast<size_t>(p - l) * E;
    }
#pragma unroll
    for (int u = 0; u < G::LA; ++u) {
      const int gi = row0 + a_i[u], gk = k0 + a_k[u];
      const bool ok = gi < n && gk < n;
      const int off = ok ? (OPA ? gk * n + gi : gi * n + gk) : 0;
      S.ra[u] = Ac[off];
      S.oka[u] = ok;
    }
#pragma unroll
    for (int u = 0; u < G::LB; ++u) {
      const int gj = col0 + b_j[u], gk = k0 + b_k[u];
      const bool ok = gj < n && gk < n;
      const int off = ok ? (OPB ? gj * n + gk : gk * n + gj) : 0;
      S.rb[u] = Bc[off];
      S.okb[u] = ok;
    }
  };
  auto store_chunk = [&](int buf, const Stage& S) {
#pragma unroll
    for (int u = 0; u < G::LA; ++u) {
      T2 v;
      v.x = S.oka[u] ? S.ra[u].x : T(0);
      v.y = S.oka[u] ? (OPA ? -S.ra[u].y : S.ra[u].y) : T(0);
      As[buf * TA + C::lds(BM, a_k[u], a_i[u])] = v;
    }
#pragma unroll
    for (int u = 0; u < G::LB; ++u) {
      T2 v;
      v.x = S.okb[u] ? S.rb[u].x : T(0);
      v.y = S.okb[u] ? (OPB ? -S.rb[u].y : S.rb[u].y) : T(0);
      Bs[buf * TB + C::lds(BN, b_k[u], b_j[u])] = v;
    }
  };

  Acc c1[WM][WN], c2[WM][WN], c3[G3 ? WM : 1][G3 ? WN : 1];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      c1[a][b] = Acc{0, 0, 0, 0};
      c2[a][b] = Acc{0, 0, 0, 0};
      if constexpr (G3) c3[a][b] = Acc{0, 0, 0, 0};
    }
  // Thin edge: when n = 16 m + 1 the last block row and block column hold a
  // single row / column of C.  Instead of a whole 16x16 MFMA block, such a
  // block is accumulated on the vector unit (about 1/16 of the work): its
  // fragment of the thin side is the broadcast of the one row (column) of the
  // operand, every lane sums its own k subset (its k of every k-step) of the complex
  // product into components 0 (re) and 1 (im) of the block's unused MFMA
  // accumulator, and the four lane groups are summed at the end.  This removes
  // 2/(m+1) of the MFMA work.
  const bool thin = uniform((n & 15) == 1 && n > 16);
  const int edge = n - 1;                              // the thin row / column
  bool rin[WM], cin[WN], trow[WM], tcol[WN];
#pragma unroll
  for (int a = 0; a < WM; ++a) {
    rin[a] = uniform(row0 + brow(a) < n);
    trow[a] = uniform(thin && row0 + brow(a) == edge);
  }
#pragma unroll
  for (int b = 0; b < WN; ++b) {
    cin[b] = uniform(col0 + bcol(b) < n);
    tcol[b] = uniform(thin && col0 + bcol(b) == edge);
  }
  bool act[WM][WN], thn[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      act[a][b] = rin[a] && cin[b] && !trow[a] && !tcol[b];
      thn[a][b] = rin[a] && cin[b] && (trow[a] || tcol[b]);
    }
  bool wave_thin = false;   // this wave owns a thin block
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) wave_thin = wave_thin || thn[a][b];
  // fragment row / column of each lane: a thin block reads the single row
  // (column) in every lane
  int frow[WM], fcol[WN];
#pragma unroll
  for (int a = 0; a < WM; ++a) frow[a] = brow(a) + (trow[a] ? 0 : li);
#pragma unroll
  for (int b = 0; b < WN; ++b) fcol[b] = bcol(b) + (tcol[b] ? 0 : li);

  // fragments of one k-step; the next k-step's fragments are read from LDS
  // while the current MFMAs issue
  auto read_frags = [&](int buf, int s, T2 (&fa)[WM], T2 (&fb)[WN]) {
    const int kk = kidx(lg, s);
#pragma unroll
    for (int a = 0; a < WM; ++a) fa[a] = As[buf * TA + C::lds(BM, kk, frow[a])];
#pragma unroll
    for (int b = 0; b < WN; ++b) fb[b] = Bs[buf * TB + C::lds(BN, kk, fcol[b])];
  };
  // The sums Xr + Xi and Yr + Yi of the three-product form.  FP64 forms them
  // for the next k-step right after the current k-step's products are
  // issued, so that no MFMA waits on the vector adds that feed it (measured
  // about 1 % faster; FP32 forms them at the products, where that measured
  // slightly faster; so do the direct-convolution and one-stage forms, whose
  // registers would not hold the extra sums).
  constexpr bool EARLY = G3 && std::is_same<T, double>::value && !CONV && !ONE_STAGE;
  T sa0[WM], sb0[WN], sa1[WM], sb1[WN];
  auto sums = [&](const T2 (&fa)[WM], const T2 (&fb)[WN], T (&sa)[WM], T (&sb)[WN]) {
    if constexpr (G3) {
#pragma unroll
      for (int a = 0; a < WM; ++a) sa[a] = fa[a].x + fa[a].y;
#pragma unroll
      for (int b = 0; b < WN; ++b) sb[b] = fb[b].x + fb[b].y;
    }
  };
  auto early_sums = [&](const T2 (&fa)[WM], const T2 (&fb)[WN], T (&sa)[WM], T (&sb)[WN]) {
    if constexpr (EARLY) sums(fa, fb, sa, sb);
  };
  auto mma = [&](const T2 (&fa)[WM], const T2 (&fb)[WN], T (&sa)[WM], T (&sb)[WN]) {
    if constexpr (G3) {
      if constexpr (!EARLY) sums(fa, fb, sa, sb);
#pragma unroll
      for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
          if (act[a][b]) {
            c1[a][b] = C::mfma(fa[a].x, fb[b].x, c1[a][b]);
            c2[a][b] = C::mfma(fa[a].y, fb[b].y, c2[a][b]);
            c3[a][b] = C::mfma(sa[a], sb[b], c3[a][b]);
          }
    } else {
#pragma unroll
      for (int a = 0; a < WM; ++a) {
        const T nai = -fa[a].y;
#pragma unroll
        for (int b = 0; b < WN; ++b)
          if (act[a][b]) {
            c1[a][b] = C::mfma(fa[a].x, fb[b].x, c1[a][b]);
            c2[a][b] = C::mfma(fa[a].x, fb[b].y, c2[a][b]);
            c1[a][b] = C::mfma(nai, fb[b].y, c1[a][b]);
            c2[a][b] = C::mfma(fa[a].y, fb[b].x, c2[a][b]);
          }
      }
    }
    // marked unlikely so that the compiler keeps a branch here: turned into
    // selects, this code would run in every wavefront and read the MFMA
    // accumulators right after the MFMAs that write them
    if (__builtin_expect(wave_thin, 0)) {
      asm volatile("");
#pragma unroll
      for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
          if (__builtin_expect(thn[a][b], 0)) {   // components 0 / 1 of the block's unused accumulator
            c1[a][b][0] = fma(fa[a].x, fb[b].x, fma(-fa[a].y, fb[b].y, c1[a][b][0]));
            c1[a][b][1] = fma(fa[a].x, fb[b].y, fma(fa[a].y, fb[b].x, c1[a][b][1]));
          }
    }
  };

  const int nchunks = CONV ? (p + 1) * cpl : cpl;
  // One chunk.  cur holds chunk c + 1 (stored to the other LDS buffer), nxt
  // receives the loads of chunk c + D (with one stage both are the same
  // registers); on entry fa0 / fb0 hold the fragments of k-step 0.  The
  // store of chunk c + 1 and the barrier come after the third k-step's
  // products: the other buffer was last read before the previous barrier,
  // and every read of this chunk is issued by then.  The fragments of the
  // next chunk's k-step 0 are read right after the barrier, while the last
  // k-step's products run, so that the matrix cores have work across the
  // barrier.
  //
  // Every global load, LDS read and LDS store of a chunk is issued whatever
  // the chunk's position, and only the MFMAs are conditional, so that the
  // compiler counts the loads in flight exactly and waits only for the ones a
  // store or a product needs (a load issued under a branch makes it wait for
  // every load).  Past the end the last chunk is loaded again, a k-step
  // beyond n reads LDS rows that are never multiplied, and the store and the
  // reads after the last chunk touch the idle LDS buffer: all in bounds and
  // without effect.
  T2 fa0[WM], fb0[WN], fa1[WM], fb1[WN];
  auto chunk = [&](int c, const Stage& cur, Stage& nxt) {
    const int buf = c & 1;
    const int k0 = chunk_k0(c);
    load_chunk(c + D < nchunks ? c + D : nchunks - 1, nxt);
    // k-step s of the chunk contracts k = k0 + kidx(g, s); it is needed when its
    // smallest k, k0 + kidx(0, s), is below n
    read_frags(buf, 1, fa1, fb1);
    mma(fa0, fb0, sa0, sb0);
    early_sums(fa1, fb1, sa1, sb1);
    read_frags(buf, 2, fa0, fb0);
    if (k0 + kidx(0, 1) < n) mma(fa1, fb1, sa1, sb1);
    early_sums(fa0, fb0, sa0, sb0);
    read_frags(buf, 3, fa1, fb1);
    if (k0 + kidx(0, 2) < n) mma(fa0, fb0, sa0, sb0);
    early_sums(fa1, fb1, sa1, sb1);
    store_chunk(buf ^ 1, cur);
    __syncthreads();
    read_frags(buf ^ 1, 0, fa0, fb0);
    if (k0 + kidx(0, 3) < n) mma(fa1, fb1, sa1, sb1);
    early_sums(fa0, fb0, sa0, sb0);
  };
  load_chunk(0, st0);
  store_chunk(0, st0);
  if constexpr (PF2) {
    load_chunk(nchunks > 1 ? 1 : 0, st1);
  }
  __syncthreads();
  read_frags(0, 0, fa0, fb0);
  early_sums(fa0, fb0, sa0, sb0);
  if constexpr (PF2) {
    // pairs of chunks, so that the two stages keep fixed registers (an odd
    // last chunk after the loop keeps the loop body free of branches around
    // memory instructions)
    int c = 0;
    for (; c + 1 < nchunks; c += 2) {
      chunk(c, st1, st0);
      chunk(c + 1, st0, st1);
    }
    if (c < nchunks) chunk(c, st1, st0);
  } else {
    for (int c = 0; c < nchunks; ++c) chunk(c, st0, st0);
  }

#pragma unroll
  for (int a = 0; a < WM; ++a) {
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      if (!act[a][b]) continue;
      const int gj = col0 + bcol(b) + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + brow(a) + C::out_row(lane, v);
        if (gi < n && gj < n) {
          T2 o;
          if constexpr (G3) {
            o.x = c1[a][b][v] - c2[a][b][v];
            o.y = c3[a][b][v] - c1[a][b][v] - c2[a][b][v];
          } else {
            o.x = c1[a][b][v];
            o.y = c2[a][b][v];
          }
          Cg[static_cast<size_t>(gi) * n + gj] = o;
        }
      }
    }
  }
  // thin blocks: sum the four lane groups' k subsets (fixed order); lane
  // group 0 stores the thin row / column, lane 0 the corner
#pragma unroll
  for (int a = 0; a < WM; ++a) {
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      if (!thn[a][b]) continue;
      T re = c1[a][b][0], im = c1[a][b][1];
      re += __shfl_xor(re, 16);
      im += __shfl_xor(im, 16);
      re += __shfl_xor(re, 32);
      im += __shfl_xor(im, 32);
      T2 o;
      o.x = re;
      o.y = im;
      const int gi = trow[a] ? edge : row0 + brow(a) + li;
      const int gj = tcol[b] ? edge : col0 + bcol(b) + li;
      const bool mine = (trow[a] && tcol[b]) ? lane == 0 : lg == 0;
      if (mine && gi < n && gj < n) Cg[static_cast<size_t>(gi) * n + gj] = o;
    }
  }
}

// Decode a logical GEMM task id into (job, mode, tile row, tile column) for
// BM x BN tiles, the shorter tiles of a mode last (tile_in_mode; about 1 %
// faster at N = 225).
__device__ __forceinline__ void gemm_task(const GemmJob* jobs, int njobs, int id, int bm, int bn, int& jidx, int& p,
                                          int& tm, int& tn) {
  jidx = 0;
  for (int j = 1; j < njobs; ++j)
    if (id >= jobs[j].tile_begin) jidx = j;
  const GemmJob& jb = jobs[jidx];
  const int local = id - jb.tile_begin;
  const int per_mode = jb.tiles_m * jb.tiles_n;
  p = local / per_mode;
  const int rem = local - p * per_mode;
  tile_in_mode(rem, jb.n, jb.tiles_m, jb.tiles_n, bm, bn, tm, tn);
}

template <typename T, int WM, int WN, int WGM, int WGN, bool OPA, bool OPB, bool G3, bool CONV = false>
__global__ __launch_bounds__(kWave * WGM * WGN, (cgemm2_min_waves<WM, WN, WGM, WGN>())) void k_cgemm2(GemmArgs args) {
  __shared__ __attribute__((aligned(16))) char smem[Tile2<T, WM, WN, WGM, WGN>::kLdsBytes];
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  int jidx, p, tm, tn;
  gemm_task(args.jobs, args.njobs, id, 16 * WM * WGM, 16 * WN * WGN, jidx, p, tm, tn);
  if constexpr (CONV) p = args.jobs[jidx].L - 1 - p;   // highest orders (most terms) first
  cgemm2_tile<T, WM, WN, WGM, WGN, OPA, OPB, G3, CONV>(args.jobs[jidx], p, tm, tn, smem);
}

}  // namespace gemm_detail

// Launch the interleaved-complex product kernel with one tile configuration.
template <typename T, int WM, int WN, int WGM, int WGN>
hipError_t launch_cgemm_cfg(const GemmArgs& a, bool g3, hipStream_t s) {
  using namespace gemm_detail;
  const int oa = a.jobs[0].opA, ob = a.jobs[0].opB;   // shared by all jobs of a launch
  constexpr int nt = kWave * WGM * WGN;
  const int g = a.total_tiles;
#define PM_K(OA, OB, G3) k_cgemm2<T, WM, WN, WGM, WGN, OA, OB, G3><<<g, nt, 0, s>>>(a)
  if (g3) {
    if (!oa && !ob) PM_K(false, false, true);
    else if (!oa && ob) PM_K(false, true, true);
    else if (oa && !ob) PM_K(true, false, true);
    else PM_K(true, true, true);
  } else {
    if (!oa && !ob) PM_K(false, false, false);
    else if (!oa && ob) PM_K(false, true, false);
    else if (oa && !ob) PM_K(true, false, false);
    else PM_K(true, true, false);
  }
#undef PM_K
  return hipGetLastError();
}

// Direct (naive) convolution form: jobs hold time-domain series and L is the
// number of orders; one 64 x 64 tile shape (the FP64 default).
template <typename T>
hipError_t launch_cgemm_conv(const GemmArgs& a, bool g3, hipStream_t s) {
  using namespace gemm_detail;
  const int oa = a.jobs[0].opA, ob = a.jobs[0].opB;   // shared by all jobs of a launch
  const int g = a.total_tiles;
#define PM_KC(OA, OB, G3) k_cgemm2<T, 2, 1, 2, 4, OA, OB, G3, true><<<g, kWave * 8, 0, s>>>(a)
  if (g3) {
    if (!oa && !ob) PM_KC(false, false, true);
    else if (!oa && ob) PM_KC(false, true, true);
    else if (oa && !ob) PM_KC(true, false, true);
    else PM_KC(true, true, true);
  } else {
    if (!oa && !ob) PM_KC(false, false, false);
    else if (!oa && ob) PM_KC(false, true, false);
    else if (oa && !ob) PM_KC(true, false, false);
    else PM_KC(true, true, false);
  }
#undef PM_KC
  return hipGetLastError();
}

// Tile configurations (blocks of 16 x 16 per wavefront WM x WN, wavefronts per
// work-group WGM x WGN).  Index order is part of the tuning table.
#define PM_GEMM_CONFIGS(X)  \
  X(0, 2, 2, 2, 2)          \
  X(1, 2, 2, 4, 2)          \
  X(2, 2, 1, 2, 4)          \
  X(3, 1, 4, 4, 1)          \
  X(4, 2, 4, 2, 1)          \
  X(5, 4, 2, 1, 2)

}  // namespace pm
