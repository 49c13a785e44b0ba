// Internal helpers shared by the HIP sources of the polymat library.
// Device code targets gfx950 (CDNA4, 64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace pm {

// ---------------------------------------------------------------- constants

constexpr int kWave = 64;
constexpr int kMaxL = 128;            // longest order-axis transform built
constexpr int kXcds = 8;              // MI355X: 8 accelerator complex dies

// ----------------------------------------------- compile-time twiddle factors
//
// cos(2 pi j / n) and sin(2 pi j / n) evaluated by the compiler: the angle is
// reduced with integer arithmetic to x = (pi/2) m / n with 0 <= m <= n/2, so
// 0 <= x <= pi/4, where a 12-term Taylor series is accurate to the last bit.

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double x2 = x * x, t = x, s = x;
  for (int i = 1; i <= 12; ++i) {
    t *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int i = 1; i <= 12; ++i) {
    t *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}

struct CS { double c, s; };

constexpr CS cos_sin_2pi(long j, long n) {
  long r = ((j % n) + n) % n;         // angle 2 pi r / n, r in [0, n)
  long q = (4 * r) / n;               // quadrant
  long m = 4 * r - q * n;             // angle within quadrant: (pi/2) m / n
  bool swap = 2 * m > n;
  long mm = swap ? n - m : m;
  double x = (kPi / 2.0) * static_cast<double>(mm) / static_cast<double>(n);
  double c = taylor_cos(x), s = taylor_sin(x);
  if (swap) { double t = c; c = s; s = t; }
  // rotate by q quarter turns: multiply by i^q
  for (long t = 0; t < q; ++t) { double c2 = -s, s2 = c; c = c2; s = s2; }
  return CS{c, s};
}

// Compile-time integer loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// --------------------------------------------------------- complex helpers

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by i^q for a compile-time q
template <int Q>
__device__ __forceinline__ double2 cmul_ipow(double2 a) {
  constexpr int q = ((Q % 4) + 4) % 4;
  if constexpr (q == 0) return a;
  else if constexpr (q == 1) return make_double2(-a.y, a.x);
  else if constexpr (q == 2) return make_double2(-a.x, -a.y);
  else return make_double2(a.y, -a.x);
}
// multiply by w^J, w = exp(SIGN 2 pi i / N), with J and N compile-time
template <int J, int N, int SIGN>
__device__ __forceinline__ double2 ctwiddle(double2 a) {
  constexpr long jj = ((static_cast<long>(J) % N) + N) % N;
  if constexpr (jj == 0) {
    return a;
  } else if constexpr ((4 * jj) % N == 0) {
    return cmul_ipow<SIGN * static_cast<int>((4 * jj) / N)>(a);
  } else {
    constexpr CS w = cos_sin_2pi(SIGN * jj, N);
    return make_double2(a.x * w.c - a.y * w.s, a.x * w.s + a.y * w.c);
  }
}

// In-register DFT of length M (power of two, compile-time):
//   X[q] = sum_m x[m] exp(SIGN 2 pi i m q / M),  result in natural order.
// Radix-2 decimation in time on a bit-reversed copy.
template <int M>
constexpr int bitrev(int v) {
  int r = 0;
  for (int b = 1; b < M; b <<= 1) { r = (r << 1) | (v & 1); v >>= 1; }
  return r;
}

template <int M, int SIGN>
__device__ __forceinline__ void dft_inplace(double2* x) {
  if constexpr (M == 1) {
    return;
  } else {
    double2 y[M];
    static_for<0, M>([&](auto i) { y[bitrev<M>(decltype(i)::value)] = x[decltype(i)::value]; });
    static_for<1, 20>([&](auto st) {
      constexpr int half = 1 << (decltype(st)::value - 1);
      constexpr int span = half * 2;
      if constexpr (span <= M) {
        static_for<0, M / span>([&](auto blk) {
          static_for<0, half>([&](auto t) {
            constexpr int i0 = decltype(blk)::value * span + decltype(t)::value;
            double2 a = y[i0];
            double2 b = ctwiddle<decltype(t)::value, span, SIGN>(y[i0 + half]);
            y[i0] = cadd(a, b);
            y[i0 + half] = csub(a, b);
          });
        });
      }
    });
    static_for<0, M>([&](auto i) { x[decltype(i)::value] = y[decltype(i)::value]; });
  }
}

// --------------------------------------------------------- XCD-aware ids
//
// Work-groups are dealt round-robin to the 8 XCDs (hardware id b runs on XCD
// b % 8).  This maps b to a logical id such that each XCD receives one
// contiguous range of logical ids, so neighbouring tiles (same product, same
// mode) share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  int x = b % kXcds, local = b / kXcds;
  int q = nb / kXcds, r = nb % kXcds;
  int base = (x < r) ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return base + local;
}

// Tile (tm, tn) of the rem-th work-group of one mode of an n x n product
// cut into tiles_m x tiles_n tiles of bm x bn: the full tiles first (row by
// row), then the right edge, the bottom edge and the corner, so that the
// shorter tiles of a launch are dispatched after the longer ones.
__host__ __device__ __forceinline__ void tile_in_mode(int rem, int n, int tiles_m, int tiles_n, int bm, int bn, int& tm,
                                             int& tn) {
  const int fm = (n % bm == 0) ? tiles_m : tiles_m - 1;   // full tile rows
  const int fn = (n % bn == 0) ? tiles_n : tiles_n - 1;   // full tile columns
  if (rem < fm * fn) {
    tm = rem / fn;
    tn = rem - tm * fn;
    return;
  }
  int r2 = rem - fm * fn;
  if (fn < tiles_n) {
    if (r2 < fm) { tm = r2; tn = tiles_n - 1; return; }
    r2 -= fm;
  }
  if (fm < tiles_m && r2 < fn) { tm = tiles_m - 1; tn = r2; return; }
  tm = tiles_m - 1;
  tn = tiles_n - 1;
}

// ------------------------------------------------------------- job tables

// Scale record of one product (device memory, written by the scale kernel):
//   s, two status words, then spow[k] = s^k (k < kMaxL/2), then
//   sinv[k] = s^-k / L.  in_bad is set by the scale kernel when a per-order
//   norm of an operand is not finite (a NaN or Inf input, or |x|^2 beyond the
//   FP64 range); out_bad is cleared by the scale kernel and set by the
//   inverse transform when it stores a non-finite coefficient.
struct ScaleRec {
  double s;
  unsigned int in_bad;
  unsigned int out_bad;
  double spow[kMaxL / 2];
  double sinv[kMaxL / 2];
};

}  // namespace pm
