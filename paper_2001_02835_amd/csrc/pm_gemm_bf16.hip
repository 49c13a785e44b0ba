// Mode-wise complex products in split-BF16 form (FFT-CONV Step 3, eq. (8)).
//
// Each Fourier coefficient x (an FP64 value from the forward transform) was
// stored as x = hi + lo with hi = RNE_bf16(x) and lo = RNE_bf16(x - hi), as
// one 8-byte entry (re_hi, re_lo, im_hi, im_lo) of a row-major [N][ld] array
// per mode, ld = N rounded up to 8.  A real product X Y is then
// approximated by hi_X hi_Y + hi_X lo_Y + lo_X hi_Y (the lo*lo term is below
// the FP32 accumulation error), and a complex product by four real ones:
//   Re = Xr Yr - Xi Yi,  Im = Xr Yi + Xi Yr   -> 12 BF16 MFMAs per block.
// Accumulation is FP32 (v_mfma_f32_16x16x32_bf16); the result is stored as
// interleaved FP32 complex and transformed back in FP64.
//
// The MFMA wants 8 consecutive k of one row per lane.  A thread fetches 8
// consecutive entries (64 bytes) and separates them into four planes of 8
// BF16 values, which go to LDS with 16-byte stores in the orientation the
// operand has in memory:
//  * contracted index contiguous (left factor as is, right factor
//    conjugated): LDS [rows][k], one 16-byte read per fragment;
//  * the other orientation: LDS [k][rows], read with the CDNA4 transposing
//    LDS load (ds_read_b64_tr_b16), two per fragment.  Its rows are XOR-
//    swizzled in 32-byte segments so that both the 16-byte stores and the
//    transposing reads are free of bank conflicts.
// A work-group computes a 64 x 64 tile of one mode with four wavefronts of
// 2 x 2 blocks of 16 x 16; K is staged in chunks of 32.  The kernel is built
// for three wavefronts per SIMD (the A fragments are read per block row to
// stay within that register budget).
#include "pm_common.h"
#include "pm_kernels.h"

namespace pm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBK = 32;
constexpr int kWaves = 4;
constexpr int kThreadsB = kWave * kWaves;    // 2 x 2 wavefronts, each 2 x 2 blocks of 16 x 16
constexpr int kPitchK = kBK + 8;             // [rows][k] tiles: 80-B rows, conflict-free 16-B reads
constexpr int kPlaneElems = kBM * kPitchK;   // LDS region of one plane (>= kBK * kBM for [k][rows])
constexpr int kTileElems = 4 * kPlaneElems;  // one operand tile, four planes
constexpr int kVecs = 4 * (4 * kBM) / kThreadsB;   // 16-byte vectors staged per thread and operand
static_assert(kVecs == 4, "one vector per plane and thread");
static_assert(kBK * kBM <= kPlaneElems, "transposed tile must fit the plane region");

__device__ __forceinline__ f4 mfma_bf16(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                  c, 0, 0, 0);
}

// zero the bf16 elements e >= valid of an 8-element vector
__device__ __forceinline__ uint4 mask_tail(uint4 v, int valid) {
  if (valid >= 8) return v;
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const uint32_t keep = (2 * d < valid ? 0x0000ffffu : 0u) | (2 * d + 1 < valid ? 0xffff0000u : 0u);
    w[d] &= keep;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint4 flip_sign(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

// Segment swizzle of row k of a [k][64] tile: 16-element (32-byte) segment s
// of row k is stored at segment s ^ seg_swizzle(k).  A transposing read
// touches rows k = 8g + 4h + e (e = 0..3) of one segment; with 128-byte rows
// the swizzle spreads the rows of one read over all 64 banks.
__device__ __forceinline__ int seg_swizzle(int k) { return (k & 3) ^ ((k >> 3) & 1); }

// Split 8 consecutive entries q (two per 16-byte vector) into the four
// planes: dword t of plane P holds component P of entries 2t and 2t + 1.
__device__ __forceinline__ void split_planes(const uint4 (&q)[4], uint4 (&pl)[4]) {
  uint32_t w[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    w[0][t] = (q[t].x & 0xffffu) | (q[t].z << 16);
    w[1][t] = (q[t].x >> 16) | (q[t].z & 0xffff0000u);
    w[2][t] = (q[t].y & 0xffffu) | (q[t].w << 16);
    w[3][t] = (q[t].y >> 16) | (q[t].w & 0xffff0000u);
  }
#pragma unroll
  for (int P = 0; P < 4; ++P) pl[P] = make_uint4(w[P][0], w[P][1], w[P][2], w[P][3]);
}

// One operand tile of 64 rows x 32 k.  KC: element (row, k) of the operand
// is entry base[row * ld + k] (contracted index contiguous), else entry
// base[k * ld + row].  Rows and k beyond n read as zero (the padding columns
// are never written, so k >= n is masked inside a vector too).
template <bool KC>
struct TileOp {
  // Staging registers of one operand tile: the thread's 8 entries as loaded
  // (the planes are separated only when they are stored to LDS, so that the
  // loads of the next chunk stay in flight during this chunk's products).
  struct Raw {
    uint4 q[4];
    int valid;      // entries of the run inside the matrix (<= 0: none)
  };

  __device__ static __forceinline__ void load(const uint2* base, int ld, int n, int row0, int k0, int tid,
                                              Raw& r) {
    int gr, gk;
    if constexpr (KC) {
      const int row = tid >> 2, kc = tid & 3;     // 64 rows x 4 runs of 8 k
      gr = row0 + row;
      gk = k0 + 8 * kc;
      r.valid = n - gk;
    } else {
      const int kk = tid >> 3, rc = tid & 7;      // 32 k x 8 runs of 8 rows
      gk = k0 + kk;
      gr = row0 + 8 * rc;
      r.valid = n - gr;
    }
    const bool ok = gr < n && gk < n;
    if (!ok) r.valid = 0;
    // a run outside the matrix reads entry 0 (always present) and is zeroed
    // at the store; the loads carry no branch
    const size_t off = ok ? (KC ? static_cast<size_t>(gr) * ld + gk : static_cast<size_t>(gk) * ld + gr) : 0;
    const uint4* src = reinterpret_cast<const uint4*>(base + off);
#pragma unroll
    for (int t = 0; t < 4; ++t) r.q[t] = src[t];
  }

  __device__ static __forceinline__ void store(uint16_t* tile, int tid, const Raw& raw, bool conj) {
    uint4 r[kVecs];
    split_planes(raw.q, r);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) r[pl] = raw.valid > 0 ? mask_tail(r[pl], raw.valid) : make_uint4(0, 0, 0, 0);
    if (conj) {
      r[2] = flip_sign(r[2]);
      r[3] = flip_sign(r[3]);
    }
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      uint16_t* p = tile + pl * kPlaneElems;
      if constexpr (KC) {
        const int row = tid >> 2, kc = tid & 3;
        *reinterpret_cast<uint4*>(p + row * kPitchK + 8 * kc) = r[pl];
      } else {
        const int kk = tid >> 3, rc = tid & 7;
        *reinterpret_cast<uint4*>(p + kk * kBM + (((rc >> 1) ^ seg_swizzle(kk)) << 4) + 8 * (rc & 1)) = r[pl];
      }
    }
  }

  // MFMA fragment of rows w0..w0+15 (w0 a multiple of 16): lane l receives
  // row w0 + l % 16 and k = 8 (l / 16) .. 8 (l / 16) + 7.
  __device__ static __forceinline__ uint4 frag(const uint16_t* p, int w0, int lane) {
    if constexpr (KC) {
      return *reinterpret_cast<const uint4*>(p + (w0 + (lane & 15)) * kPitchK + 8 * (lane >> 4));
    } else {
      // The transposing read hands lane 16g + j element j % 4 of the 8-byte
      // words addressed by lanes 16g + j / 4 + 4t, t = 0..3, as its element
      // t.  Lane 16g + 4e + c therefore addresses row k = 8g + 4h + e,
      // columns w0 + 4c .. w0 + 4c + 3, and lane 16g + j receives column
      // w0 + j at rows 8g + 4h + t.
      const int g = lane >> 4, e = (lane >> 2) & 3, c = lane & 3;
      uint2 half[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 8 * g + 4 * h + e;
        const uint16_t* a = p + k * kBM + (((w0 >> 4) ^ seg_swizzle(k)) << 4) + 4 * c;
        const s4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s4*)(a));
        half[h] = __builtin_bit_cast(uint2, v);
      }
      return make_uint4(half[0].x, half[0].y, half[1].x, half[1].y);
    }
  }
};

template <bool OPA, bool OPB>
__global__ __launch_bounds__(kThreadsB, 3) void k_cgemm_bf16x3(GemmArgs args) {
  constexpr bool AKC = !OPA;   // left factor as is: rows contiguous in k
  constexpr bool BKC = OPB;    // right factor conjugated: (Y^+)[k][j] = conj(Y[j][k])
  using TA = TileOp<AKC>;
  using TB = TileOp<BKC>;
  __shared__ __align__(16) uint16_t As[kTileElems];
  __shared__ __align__(16) uint16_t Bs[kTileElems];

  const int id = xcd_remap(blockIdx.x, gridDim.x);
  int jidx = 0;
  for (int j = 1; j < args.njobs; ++j)
    if (id >= args.jobs[j].tile_begin) jidx = j;
  const GemmJob& jb = args.jobs[jidx];
  const int local = id - jb.tile_begin;
  const int per_mode = jb.tiles_m * jb.tiles_n;
  const int p = local / per_mode;
  const int rem = local - p * per_mode;
  int tm, tn;
  tile_in_mode(rem, jb.n, jb.tiles_m, jb.tiles_n, kBM, kBM, tm, tn);
  const int n = jb.n, L = jb.L;
  const int ld = bf16_ld(n);
  const size_t mode = static_cast<size_t>(n) * ld;
  const int pa = OPA ? (L - p) % L : p;
  const int pb = OPB ? (L - p) % L : p;
  const uint2* Ab = reinterpret_cast<const uint2*>(jb.A) + static_cast<size_t>(pa) * mode;
  const uint2* Bb = reinterpret_cast<const uint2*>(jb.B) + static_cast<size_t>(pb) * mode;
  float2* __restrict__ Cg = reinterpret_cast<float2*>(jb.C) + static_cast<size_t>(p) * n * n;

  const int row0 = tm * kBM, col0 = tn * kBM;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int wrow0 = (wave >> 1) * 32, wcol0 = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;

  f4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) { cr[a][b] = f4{0, 0, 0, 0}; ci[a][b] = f4{0, 0, 0, 0}; }
  bool mact[2], nact[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) mact[a] = row0 + wrow0 + 16 * a < n;
#pragma unroll
  for (int b = 0; b < 2; ++b) nact[b] = col0 + wcol0 + 16 * b < n;

  typename TA::Raw ra;
  typename TB::Raw rb;
  const int nk = (n + kBK - 1) / kBK;
  TA::load(Ab, ld, n, row0, 0, tid, ra);
  TB::load(Bb, ld, n, col0, 0, tid, rb);
  for (int c = 0; c < nk; ++c) {
    TA::store(As, tid, ra, OPA);
    TB::store(Bs, tid, rb, OPB);
    __syncthreads();
    // the next chunk's loads (past the end: a chunk of zeros, still in bounds)
    TA::load(Ab, ld, n, row0, (c + 1) * kBK, tid, ra);
    TB::load(Bb, ld, n, col0, (c + 1) * kBK, tid, rb);
    uint4 fb[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) fb[b][pl] = TB::frag(Bs + pl * kPlaneElems, wcol0 + 16 * b, lane);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      uint4 fa[4];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) fa[pl] = TA::frag(As + pl * kPlaneElems, wrow0 + 16 * a, lane);
      const uint4 nih = flip_sign(fa[2]), nil = flip_sign(fa[3]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (mact[a] && nact[b]) {
          // Re: Xr Yr - Xi Yi
          cr[a][b] = mfma_bf16(fa[0], fb[b][0], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[0], fb[b][2], ci[a][b]);
          cr[a][b] = mfma_bf16(fa[0], fb[b][1], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[0], fb[b][3], ci[a][b]);
          cr[a][b] = mfma_bf16(fa[1], fb[b][0], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[1], fb[b][2], ci[a][b]);
          cr[a][b] = mfma_bf16(nih, fb[b][2], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[2], fb[b][0], ci[a][b]);
          cr[a][b] = mfma_bf16(nih, fb[b][3], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[2], fb[b][1], ci[a][b]);
          cr[a][b] = mfma_bf16(nil, fb[b][2], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[3], fb[b][0], ci[a][b]);
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int gj = col0 + wcol0 + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + wrow0 + 16 * a + 4 * lk + v;
        if (gi < n && gj < n) Cg[static_cast<size_t>(gi) * n + gj] = make_float2(cr[a][b][v], ci[a][b][v]);
      }
    }
  }
}

}  // namespace

int gemm_tile_bf16() { return kBM; }

hipError_t launch_gemm_bf16(const GemmArgs& a, hipStream_t s) {
  if (a.njobs <= 0 || a.total_tiles <= 0) return hipSuccess;
  const int oa = a.jobs[0].opA, ob = a.jobs[0].opB;   // shared by all jobs of a launch
  const int g = a.total_tiles;
  if (!oa && !ob) k_cgemm_bf16x3<false, false><<<g, kThreadsB, 0, s>>>(a);
  else if (!oa && ob) k_cgemm_bf16x3<false, true><<<g, kThreadsB, 0, s>>>(a);
  else if (oa && !ob) k_cgemm_bf16x3<true, false><<<g, kThreadsB, 0, s>>>(a);
  else k_cgemm_bf16x3<true, true><<<g, kThreadsB, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pm
