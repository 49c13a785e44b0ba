// Mode-wise complex products in split-BF16 form (FFT-CONV Step 3, eq. (8)).
//
// Each Fourier coefficient x (an FP64 value from the forward transform) was
// stored as x = hi + lo with hi = RNE_bf16(x) and lo = RNE_bf16(x - hi), in
// four BF16 planes per mode: re_hi, re_lo, im_hi, im_lo, each row-major
// [N][ld] with ld = N rounded up to 8.  A real product X Y is then
// approximated by hi_X hi_Y + hi_X lo_Y + lo_X hi_Y (the lo*lo term is below
// the FP32 accumulation error), and a complex product by four real ones:
//   Re = Xr Yr - Xi Yi,  Im = Xr Yi + Xi Yr   -> 12 BF16 MFMAs per block.
// Accumulation is FP32 (v_mfma_f32_16x16x32_bf16); the result is stored as
// interleaved FP32 complex and transformed back in FP64.
//
// The MFMA wants 8 consecutive k of one row per lane.  An operand whose
// contracted index is contiguous in memory (left factor as is, right factor
// conjugated) is copied to LDS with 16-byte moves; the other orientation is
// transposed while staging (8 rows of one k per 16-byte load, scattered).
#include "pm_common.h"
#include "pm_kernels.h"

namespace pm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kPadK = 8;                     // row pitch 40 elements = 80 B: conflict-free 16-B reads
constexpr int kPitch = kBK + kPadK;
constexpr int kThreadsB = 256;               // 4 wavefronts, 2 x 2, each 2 x 2 blocks of 16 x 16

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f4 mfma_bf16(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

// zero the bf16 elements e >= valid of an 8-element vector
__device__ __forceinline__ uint4 mask_tail(uint4 v, int valid) {
  if (valid >= 8) return v;
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int lo = 2 * d, hi = 2 * d + 1;
    uint32_t keep = (lo < valid ? 0x0000ffffu : 0u) | (hi < valid ? 0xffff0000u : 0u);
    w[d] &= keep;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint4 flip_sign(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

struct Operand {
  const uint16_t* base;   // mode base: 4 planes of n * ld elements
  size_t plane;           // n * ld
  int ld;
  bool kcontig;           // contracted index contiguous in memory
  bool conj;              // negate the imaginary planes
};

// Stage one 64 x 32 (rows x k) tile of an operand into registers.
//   kcontig: element (row, k) at base[row * ld + k]  -> 16-B vector = 8 k of one row
//   else   : element (row, k) at base[k * ld + row]  -> 16-B vector = 8 rows of one k
__device__ __forceinline__ void load_tile(const Operand& op, int n, int row0, int k0, int tid, uint4 (&r)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = tid + kThreadsB * u;           // 0..1023
    const int plane = q >> 8;                    // 4 planes x 256 vectors
    const int w = q & 255;
    uint4 v = make_uint4(0, 0, 0, 0);
    const uint16_t* pb = op.base + static_cast<size_t>(plane) * op.plane;
    if (op.kcontig) {
      const int row = w >> 2, kc = w & 3;        // 64 rows x 4 vectors of 8 k
      const int gr = row0 + row, gk = k0 + 8 * kc;
      if (gr < n && gk < n) {
        v = *reinterpret_cast<const uint4*>(pb + static_cast<size_t>(gr) * op.ld + gk);
        v = mask_tail(v, n - gk);
      }
    } else {
      const int kk = w >> 3, rc = w & 7;         // 32 k x 8 vectors of 8 rows
      const int gk = k0 + kk, gr = row0 + 8 * rc;
      if (gk < n && gr < n) {
        v = *reinterpret_cast<const uint4*>(pb + static_cast<size_t>(gk) * op.ld + gr);
        v = mask_tail(v, n - gr);
      }
    }
    if (op.conj && plane >= 2) v = flip_sign(v);
    r[u] = v;
  }
}

__device__ __forceinline__ void store_tile(const Operand& op, uint16_t (*lds)[kBM][kPitch], int tid,
                                           const uint4 (&r)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = tid + kThreadsB * u;
    const int plane = q >> 8;
    const int w = q & 255;
    if (op.kcontig) {
      const int row = w >> 2, kc = w & 3;
      *reinterpret_cast<uint4*>(&lds[plane][row][8 * kc]) = r[u];
    } else {
      const int kk = w >> 3, rc = w & 7;
      const uint32_t d[4] = {r[u].x, r[u].y, r[u].z, r[u].w};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint16_t h = static_cast<uint16_t>((e & 1) ? (d[e >> 1] >> 16) : (d[e >> 1] & 0xffffu));
        lds[plane][8 * rc + e][kk] = h;
      }
    }
  }
}

__global__ __launch_bounds__(kThreadsB) void k_cgemm_bf16x3(GemmArgs args) {
  __shared__ uint16_t As[4][kBM][kPitch];
  __shared__ uint16_t Bs[4][kBN][kPitch];

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
  const int ld = bf16_ld(n);
  const size_t plane = static_cast<size_t>(n) * ld;
  const int pa = jb.opA ? (L - p) % L : p;
  const int pb = jb.opB ? (L - p) % L : p;

  Operand oa, ob;
  oa.base = reinterpret_cast<const uint16_t*>(jb.A) + static_cast<size_t>(pa) * 4 * plane;
  oa.plane = plane;
  oa.ld = ld;
  oa.kcontig = jb.opA == 0;      // left factor as is: [i][k] rows contiguous in k
  oa.conj = jb.opA != 0;
  ob.base = reinterpret_cast<const uint16_t*>(jb.B) + static_cast<size_t>(pb) * 4 * plane;
  ob.plane = plane;
  ob.ld = ld;
  ob.kcontig = jb.opB != 0;      // right factor conjugated: (Y^+)[k][j] = conj(Y[j][k])
  ob.conj = jb.opB != 0;
  float2* __restrict__ Cg = reinterpret_cast<float2*>(jb.C) + static_cast<size_t>(p) * n * n;

  const int row0 = tm * kBM, col0 = tn * kBN;
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

  uint4 ra[4], rb[4];
  const int nk = (n + kBK - 1) / kBK;
  load_tile(oa, n, row0, 0, tid, ra);
  load_tile(ob, n, col0, 0, tid, rb);
  for (int c = 0; c < nk; ++c) {
    store_tile(oa, As, tid, ra);
    store_tile(ob, Bs, tid, rb);
    __syncthreads();
    if (c + 1 < nk) {
      load_tile(oa, n, row0, (c + 1) * kBK, tid, ra);
      load_tile(ob, n, col0, (c + 1) * kBK, tid, rb);
    }
    uint4 fa[2][4], fb[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        fa[a][pl] = *reinterpret_cast<const uint4*>(&As[pl][wrow0 + 16 * a + li][8 * lk]);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        fb[b][pl] = *reinterpret_cast<const uint4*>(&Bs[pl][wcol0 + 16 * b + li][8 * lk]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const uint4 nih = flip_sign(fa[a][2]), nil = flip_sign(fa[a][3]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (mact[a] && nact[b]) {
          // Re: Xr Yr - Xi Yi
          cr[a][b] = mfma_bf16(fa[a][0], fb[b][0], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[a][0], fb[b][2], ci[a][b]);
          cr[a][b] = mfma_bf16(fa[a][0], fb[b][1], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[a][0], fb[b][3], ci[a][b]);
          cr[a][b] = mfma_bf16(fa[a][1], fb[b][0], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[a][1], fb[b][2], ci[a][b]);
          cr[a][b] = mfma_bf16(nih, fb[b][2], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[a][2], fb[b][0], ci[a][b]);
          cr[a][b] = mfma_bf16(nih, fb[b][3], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[a][2], fb[b][1], ci[a][b]);
          cr[a][b] = mfma_bf16(nil, fb[b][2], cr[a][b]);
          ci[a][b] = mfma_bf16(fa[a][3], fb[b][0], ci[a][b]);
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
  k_cgemm_bf16x3<<<a.total_tiles, kThreadsB, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pm
