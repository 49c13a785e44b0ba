// Device building blocks of the order-axis transforms (FFT-CONV Steps 2 and
// 4, eqs. (7) and (9)), shared by the product pipeline and the NSPT step.
//
// One work-group of four wavefronts handles 64 consecutive matrix entries
// (lanes run over entries, so every global access of a wavefront is a
// contiguous run).  With L = 4M and at most 2M nonzero orders:
//   forward  At[4q + r] = sum_{m<M} w_M^{mq} c_r[m],  c_r[m] = w_L^{mr} (a[m] + i^r a[m+M])
//            (one pruned radix-4 step, then a length-M DFT per residue r),
//   inverse  sum_p Ct[p] w_L^{-kp} = sum_r w_L^{-kr} d_r[k mod M],
//            d_r = length-M inverse DFT of the modes p = 4q + r,
// with wavefront r handling residue r and the residues combined in LDS in a
// fixed order (bitwise reproducible).
#pragma once

#include "pm_common.h"
#include "pm_kernels.h"

namespace pm {

constexpr int kEnt = 64;        // entries per work-group
constexpr int kFftThreads = 256;

// ------------------------------------------------------------ BF16 split

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ double bf16_to_double(uint16_t h) {
  return static_cast<double>(__uint_as_float(static_cast<uint32_t>(h) << 16));
}
// hi = RNE_bf16(x), lo = RNE_bf16(x - hi) with x - hi exact in FP64.
__device__ __forceinline__ void split_bf16(double x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne(static_cast<float>(x));
  double r = x - bf16_to_double(hi);
  lo = bf16_rne(static_cast<float>(r));
}

// BF16 split layout of one mode: four planes (re_hi, re_lo, im_hi, im_lo),
// each row-major [n][ld] with ld = n rounded up to a multiple of 8, so that a
// lane of the product kernel can fetch 8 consecutive entries of a row with a
// single 16-byte load.  The padding columns are never written (the product
// kernel masks them).
__device__ __forceinline__ size_t bf16_plane_elems(int n) { return static_cast<size_t>(bf16_ld(n)) * n; }

// Store mode p of entry e (matrix size n, E = n*n entries per mode).
template <FourierType FT>
__device__ __forceinline__ void store_mode(void* dst, int E, int n, int p, int e, double2 v) {
  if constexpr (FT == kF64) {
    reinterpret_cast<double2*>(dst)[static_cast<size_t>(p) * E + e] = v;
  } else if constexpr (FT == kF32) {
    reinterpret_cast<float2*>(dst)[static_cast<size_t>(p) * E + e] =
        make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
  } else {
    const int i = e / n, j = e - (e / n) * n;
    const size_t plane = bf16_plane_elems(n);
    uint16_t* base = reinterpret_cast<uint16_t*>(dst) + static_cast<size_t>(p) * 4 * plane;
    const size_t off = static_cast<size_t>(i) * bf16_ld(n) + j;
    uint16_t rh, rl, ih, il;
    split_bf16(v.x, rh, rl);
    split_bf16(v.y, ih, il);
    base[off] = rh;
    base[plane + off] = rl;
    base[2 * plane + off] = ih;
    base[3 * plane + off] = il;
  }
}

// Load mode p of entry e of a product result (FP64 or FP32 complex).
template <FourierType FT>
__device__ __forceinline__ double2 load_mode(const void* src, int E, int p, int e) {
  if constexpr (FT == kF64) {
    return reinterpret_cast<const double2*>(src)[static_cast<size_t>(p) * E + e];
  } else {
    float2 f = reinterpret_cast<const float2*>(src)[static_cast<size_t>(p) * E + e];
    return make_double2(f.x, f.y);
  }
}

// ------------------------------------------------------------ forward

// Residue R of the forward transform of the orders staged in tile[k][lane]
// (k < nord, already rescaled), stored as modes 4q + R.
template <int L, int R, FourierType FT>
__device__ __forceinline__ void forward_residue(const double2 (*tile)[kEnt], int nord, int lane, void* dst,
                                                int E, int n, int e, bool valid) {
  constexpr int M = L / 4;
  double2 c[M];
  static_for<0, M>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    double2 a0 = (m < nord) ? tile[m][lane] : make_double2(0.0, 0.0);
    double2 a1 = (m + M < nord) ? tile[m + M][lane] : make_double2(0.0, 0.0);
    double2 t = cadd(a0, cmul_ipow<R>(a1));
    c[m] = ctwiddle<m * R, L, +1>(t);
  });
  dft_inplace<M, +1>(c);
  if (valid) {
    static_for<0, M>([&](auto qi) {
      constexpr int q = decltype(qi)::value;
      store_mode<FT>(dst, E, n, 4 * q + R, e, c[q]);
    });
  }
}

template <int L, FourierType FT>
__device__ __forceinline__ void forward_from_tile(const double2 (*tile)[kEnt], int nord, int lane, int r,
                                                  void* dst, int E, int n, int e, bool valid) {
  switch (r) {
    case 0: forward_residue<L, 0, FT>(tile, nord, lane, dst, E, n, e, valid); break;
    case 1: forward_residue<L, 1, FT>(tile, nord, lane, dst, E, n, e, valid); break;
    case 2: forward_residue<L, 2, FT>(tile, nord, lane, dst, E, n, e, valid); break;
    default: forward_residue<L, 3, FT>(tile, nord, lane, dst, E, n, e, valid); break;
  }
}

// ------------------------------------------------------------ inverse

// acc[k][lane] <- sum_p Ct[p] w^{-kp} for k < nord (no 1/L), from the modes
// d[q] = Ct[4q + R] of this thread's entry (d is overwritten).  Ends with a
// barrier, after which every wavefront may read acc.
template <int L, int R>
__device__ __forceinline__ void inverse_from_modes(double2* d, double2 (*acc)[kEnt], int nord, int lane) {
  constexpr int M = L / 4;
  dft_inplace<M, -1>(d);
  auto term = [&](auto ki) {
    constexpr int k = decltype(ki)::value;
    return ctwiddle<k * R, L, -1>(d[k % M]);
  };
  // fixed order: r = 0 writes, r = 1, 2, 3 add
  if constexpr (R == 0) {
    static_for<0, 2 * M>([&](auto ki) {
      constexpr int k = decltype(ki)::value;
      if (k < nord) acc[k][lane] = term(ki);
    });
  }
  __syncthreads();
  if constexpr (R == 1) {
    static_for<0, 2 * M>([&](auto ki) {
      constexpr int k = decltype(ki)::value;
      if (k < nord) acc[k][lane] = cadd(acc[k][lane], term(ki));
    });
  }
  __syncthreads();
  if constexpr (R == 2) {
    static_for<0, 2 * M>([&](auto ki) {
      constexpr int k = decltype(ki)::value;
      if (k < nord) acc[k][lane] = cadd(acc[k][lane], term(ki));
    });
  }
  __syncthreads();
  if constexpr (R == 3) {
    static_for<0, 2 * M>([&](auto ki) {
      constexpr int k = decltype(ki)::value;
      if (k < nord) acc[k][lane] = cadd(acc[k][lane], term(ki));
    });
  }
  __syncthreads();
}

// Same, where load(p) returns mode p of this thread's entry.
template <int L, int R, typename Load>
__device__ __forceinline__ void inverse_residue(Load&& load, double2 (*acc)[kEnt], int nord, int lane) {
  constexpr int M = L / 4;
  double2 d[M];
  static_for<0, M>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    d[q] = load(4 * q + R);
  });
  inverse_from_modes<L, R>(d, acc, nord, lane);
}

template <int L, typename Load>
__device__ __forceinline__ void inverse_to_lds(Load&& load, double2 (*acc)[kEnt], int nord, int lane, int r) {
  switch (r) {
    case 0: inverse_residue<L, 0>(load, acc, nord, lane); break;
    case 1: inverse_residue<L, 1>(load, acc, nord, lane); break;
    case 2: inverse_residue<L, 2>(load, acc, nord, lane); break;
    default: inverse_residue<L, 3>(load, acc, nord, lane); break;
  }
}

}  // namespace pm
