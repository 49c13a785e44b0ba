// Device building blocks of the order-axis transforms (FFT-CONV Steps 2 and
// 4, eqs. (7) and (9)), shared by the product pipeline and the NSPT step.
//
// One work-group of four wavefronts handles ENT consecutive matrix entries
// (lanes run over entries, so every global access of a wavefront is a
// contiguous run).  With L = 4M and at most 2M nonzero orders:
//   forward  At[4q + r] = sum_{m<M} w_M^{mq} c_r[m],  c_r[m] = w_L^{mr} (a[m] + i^r a[m+M])
//            (one pruned radix-4 step, then a length-M DFT per residue r),
//   inverse  sum_p Ct[p] w_L^{-kp} = sum_r w_L^{-kr} d_r[k mod M],
//            d_r = length-M inverse DFT of the modes p = 4q + r,
// with wavefront r handling residue r and the residues combined in LDS in a
// fixed order (bitwise reproducible).  For L <= 64 one lane holds one entry
// (ENT = 64).  For L = 128 two lanes share an entry (ENT = 32): the
// length-M DFT of a residue is split into its even and odd outputs (forward)
// or inputs (inverse), one per half-wavefront, which halves both the LDS tile
// of a work-group and the registers of a lane.
#pragma once

#include "pm_common.h"
#include "pm_kernels.h"

namespace pm {

constexpr int kEnt = 64;        // entries per work-group for L <= 64
constexpr int kFftThreads = 256;

// lanes per matrix entry and entries per work-group for transform length L
template <int L> constexpr int fft_split() { return L >= 128 ? 2 : 1; }
template <int L> constexpr int fft_ent() { return kEnt / fft_split<L>(); }
// occupancy floor (waves per SIMD) given to the compiler: the split form
// keeps few values live, so keep the register allocation within 3 waves
template <int L> constexpr int fft_min_waves() { return L >= 128 ? 3 : 1; }
// the same for a run-time L (grid sizes)
inline int fft_entries_per_group(int L) { return L >= 128 ? kEnt / 2 : kEnt; }

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

// BF16 split layout: per mode a row-major [n][ld] array of 8-byte entries
// (re_hi, re_lo, im_hi, im_lo as four BF16), ld = n rounded up to a multiple
// of 8, so that 8 consecutive entries of a row start on a 64-byte boundary
// and one lane of the transforms stores one entry with one 8-byte write.  The
// padding columns are never written (the product kernel masks them).
__device__ __forceinline__ size_t bf16_mode_entries(int n) { return static_cast<size_t>(bf16_ld(n)) * n; }

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
    uint16_t rh, rl, ih, il;
    split_bf16(v.x, rh, rl);
    split_bf16(v.y, ih, il);
    const size_t off = static_cast<size_t>(p) * bf16_mode_entries(n) + static_cast<size_t>(i) * bf16_ld(n) + j;
    reinterpret_cast<uint2*>(dst)[off] =
        make_uint2(rh | (static_cast<uint32_t>(rl) << 16), ih | (static_cast<uint32_t>(il) << 16));
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

// Residue R of the forward transform of the orders staged in tile[k][el]
// (already rescaled), stored as modes 4q + R.  Every row k < L/2 of the tile
// is read: the caller zero-fills the rows from nord on (branch-free loads let
// the compiler interleave them with the arithmetic).
// S: lanes per matrix entry (1 or 2; the default is the stand-alone kernels' choice).
template <int L, int R, FourierType FT, int S = fft_split<L>()>
__device__ __forceinline__ void forward_residue(const double2 (*tile)[kEnt / S], int lane,
                                                void* dst, int E, int n, int e, bool valid) {
  constexpr int M = L / 4;
  constexpr int ENT = kEnt / S;
  static_assert(S == 1 || S == 2, "one or two lanes per entry");
  if constexpr (S == 1) {
    double2 c[M];
    static_for<0, M>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const double2 a0 = tile[m][lane];
      const double2 a1 = tile[m + M][lane];
      c[m] = ctwiddle<m * R, L, +1>(cadd(a0, cmul_ipow<R>(a1)));
    });
    dft_inplace<M, +1>(c);
    if (valid) {
      static_for<0, M>([&](auto qi) {
        constexpr int q = decltype(qi)::value;
        store_mode<FT>(dst, E, n, 4 * q + R, e, c[q]);
      });
    }
  } else {
    // half h of the wavefront forms the outputs q = 2 q' + h:
    //   X[2q' + h] = sum_{m < M/2} (c[m] + (-1)^h c[m + M/2]) w_M^{m h} w_{M/2}^{m q'}
    constexpr int M2 = M / 2;
    const int el = lane % ENT;
    const bool odd = lane >= ENT;
    const double sg = odd ? -1.0 : 1.0;
    auto cval = [&](auto ci) {
      constexpr int mm = decltype(ci)::value;
      const double2 a0 = tile[mm][el];
      const double2 a1 = tile[mm + M][el];
      return ctwiddle<mm * R, L, +1>(cadd(a0, cmul_ipow<R>(a1)));
    };
    double2 t[M2];
    static_for<0, M2>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const double2 lo = cval(std::integral_constant<int, m>{});
      const double2 hi = cval(std::integral_constant<int, m + M2>{});
      const double2 v = make_double2(lo.x + sg * hi.x, lo.y + sg * hi.y);
      t[m] = odd ? ctwiddle<m, M, +1>(v) : v;
    });
    dft_inplace<M2, +1>(t);
    if (valid) {
      static_for<0, M2>([&](auto qi) {
        constexpr int q = decltype(qi)::value;
        store_mode<FT>(dst, E, n, 4 * (2 * q + (odd ? 1 : 0)) + R, e, t[q]);
      });
    }
  }
}

template <int L, FourierType FT, int S = fft_split<L>()>
__device__ __forceinline__ void forward_from_tile(const double2 (*tile)[kEnt / S], int lane, int r,
                                                  void* dst, int E, int n, int e, bool valid) {
  switch (r) {
    case 0: forward_residue<L, 0, FT, S>(tile, lane, dst, E, n, e, valid); break;
    case 1: forward_residue<L, 1, FT, S>(tile, lane, dst, E, n, e, valid); break;
    case 2: forward_residue<L, 2, FT, S>(tile, lane, dst, E, n, e, valid); break;
    default: forward_residue<L, 3, FT, S>(tile, lane, dst, E, n, e, valid); break;
  }
}

// ------------------------------------------------------------ inverse

// Number of modes a lane loads for residue R, and the mode of its q-th one.
template <int L, int S = fft_split<L>()> constexpr int lane_nmodes() { return L / 4 / S; }
template <int L, int R, int S = fft_split<L>()>
__device__ __forceinline__ int lane_mode(int q, int lane) {
  if constexpr (S == 1) return 4 * q + R;
  else return 4 * (2 * q + (lane >= kEnt / S ? 1 : 0)) + R;
}

// acc[k][el] <- sum_p Ct[p] w^{-kp} for all k < L/2 (no 1/L), from the modes
// d[q] = Ct[lane_mode<L,R>(q)] of this lane (d is overwritten).  Ends with a
// barrier, after which every wavefront may read acc.
//
// One lane per entry: the four residues are summed into acc in four phases
// separated by barriers.  Chained (ROT = false), wavefront r writes or adds
// all rows in phase r while the other three wait.  Rotated (ROT = true, L >= 8),
// every wavefront works in every phase: in phase p wavefront r adds its terms
// to row block (r + p) mod 4 (a quarter of the rows), so block b receives
// the residues b, b-1, b-2, b-3 in that order.  Both orders are fixed, so the
// results are bitwise reproducible.  The rotated form is faster for the
// stand-alone inverse and the re-truncation of FP32 products, slower for the
// weighted-sum inverse and the re-truncation of FP64 products (measured).
template <int L, int R, int S = fft_split<L>(), bool ROT = false>
__device__ __forceinline__ void inverse_from_modes(double2* d, double2 (*acc)[kEnt / S], int lane) {
  constexpr int M = L / 4;
  constexpr int ENT = kEnt / S;
  static_assert(S == 1 || S == 2, "one or two lanes per entry");
  if constexpr (S == 1) {
    dft_inplace<M, -1>(d);
    auto term = [&](auto ki) {
      constexpr int k = decltype(ki)::value;
      return ctwiddle<k * R, L, -1>(d[k % M]);
    };
    if constexpr (ROT && (2 * M) % 4 == 0) {
      constexpr int QB = 2 * M / 4;   // rows per block
      static_for<0, 4>([&](auto pi) {
        constexpr int p = decltype(pi)::value;
        constexpr int b = (R + p) & 3;
        static_for<b * QB, (b + 1) * QB>([&](auto ki) {
          constexpr int k = decltype(ki)::value;
          acc[k][lane] = (p == 0) ? term(ki) : cadd(acc[k][lane], term(ki));
        });
        __syncthreads();
      });
    } else {
      // fixed order: r = 0 writes, r = 1, 2, 3 add
      for (int w = 0; w < 4; ++w) {
        if (w == R) {
          static_for<0, 2 * M>([&](auto ki) {
            constexpr int k = decltype(ki)::value;
            acc[k][lane] = (R == 0) ? term(ki) : cadd(acc[k][lane], term(ki));
          });
        }
        __syncthreads();
      }
    }
  } else {
    // half h holds the length-M/2 inverse DFT of the even (h = 0) or odd
    // (h = 1) modes of residue R; with the partner half's values,
    //   Y[j] = E[j] + w_M^-j O[j],  Y[j + M/2] = E[j] - w_M^-j O[j],
    // and half h keeps Y[j + h M/2], j < M/2.
    constexpr int M2 = M / 2;
    const int el = lane % ENT;
    const bool odd = lane >= ENT;
    dft_inplace<M2, -1>(d);
    // orders k = j + h M/2 and k = j + h M/2 + M; term w_L^{-kR} Y[j + h M/2].
    // The exchange sits inside the residue's turn of the chain so that only
    // d stays live (the whole wavefront takes the same turn).
    for (int w = 0; w < 4; ++w) {
      if (w == R) {
        static_for<0, M2>([&](auto ji) {
          constexpr int j = decltype(ji)::value;
          double2 other;
          other.x = __shfl_xor(d[j].x, ENT);
          other.y = __shfl_xor(d[j].y, ENT);
          const double2 ev = odd ? other : d[j];
          const double2 od = ctwiddle<-j, M, +1>(odd ? d[j] : other);
          const double2 y = odd ? csub(ev, od) : cadd(ev, od);
          static_for<0, 2>([&](auto ti) {
            constexpr int t = decltype(ti)::value;
            constexpr int k_even = j + t * M, k_odd = j + M2 + t * M;
            const double2 te = ctwiddle<k_even * R, L, -1>(y);
            const double2 to = ctwiddle<k_odd * R, L, -1>(y);
            const int k = odd ? k_odd : k_even;
            const double2 v = odd ? to : te;
            acc[k][el] = (R == 0) ? v : cadd(acc[k][el], v);
          });
        });
      }
      __syncthreads();
    }
  }
}

// Same, where load(p) returns mode p of this thread's entry.
template <int L, int R, int S, bool ROT, typename Load>
__device__ __forceinline__ void inverse_residue(Load&& load, double2 (*acc)[kEnt / S], int lane) {
  constexpr int NQ = lane_nmodes<L, S>();
  double2 d[NQ];
  static_for<0, NQ>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    d[q] = load(lane_mode<L, R, S>(q, lane));
  });
  inverse_from_modes<L, R, S, ROT>(d, acc, lane);
}

template <int L, int S = fft_split<L>(), bool ROT = false, typename Load>
__device__ __forceinline__ void inverse_to_lds(Load&& load, double2 (*acc)[kEnt / S], int lane, int r) {
  switch (r) {
    case 0: inverse_residue<L, 0, S, ROT>(load, acc, lane); break;
    case 1: inverse_residue<L, 1, S, ROT>(load, acc, lane); break;
    case 2: inverse_residue<L, 2, S, ROT>(load, acc, lane); break;
    default: inverse_residue<L, 3, S, ROT>(load, acc, lane); break;
  }
}

}  // namespace pm
