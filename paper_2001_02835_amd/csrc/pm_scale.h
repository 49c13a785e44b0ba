// Choice of the rescaling factor s of one product (FFT-CONV Step 1 with the
// per-order rescaling g -> s g), computed by one wavefront.  Shared by the
// stand-alone scale kernel and the persistent batch pipeline.
#pragma once

#include "pm_common.h"
#include "pm_kernels.h"

namespace pm {

// Choice of s (log s = t): with a_j = ||A^(j)||, b_j = ||B^(j)|| and
// c_m = sum_j a_j b_{m-j} (m <= 2 ntrunc, the orders of the full product,
// including those the truncation discards), minimise the spread
//   f(t) = max_m (log c_m + m t) - min_{k <= ntrunc} (log c_k + k t)
// over the nonzero c (per-order norms below 1e-15 of the operand's largest
// are treated as zero).  f is convex and piecewise linear.  One wavefront
// evaluates it on a 64-point grid; three refinement rounds shrink the grid
// spacing by 32 each.  Values move between lanes by cross-lane reads only
// (no LDS, no barrier), so any single wavefront of a work-group can run it.
constexpr double kAbsent = 1e300;
constexpr double kNoiseFloor = 1e-15;

// value of v in lane `lane` (a wave-uniform index)
__device__ __forceinline__ double wave_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// tid: lane 0..63 of the calling wavefront.  Writes jb.rec (s, the status
// words, s^k and s^-k / L for k < 64).
__device__ __forceinline__ void scale_wave(const ScaleJob& jb, int tid) {
  const int nord = jb.nord;
  double t = 0.0;
  bool in_bad = false;
  if (jb.fixed_s > 0.0) {
    t = log(jb.fixed_s);
  } else if (nord > 1) {
    // per-order norms: lane k holds a_k, b_k (k < nord <= 64)
    double na = 0.0, nb = 0.0;
    if (tid < nord) {
      double sa[4] = {0.0, 0.0, 0.0, 0.0}, sb[4] = {0.0, 0.0, 0.0, 0.0};
      const int nsb = jb.nser_b > 0 ? jb.nser_b : jb.nser;
      for (int q = 0; q < jb.nser; ++q) {
        const double* pa = jb.partA + (q * nord + tid) * kNormChunks;
#pragma unroll
        for (int c = 0; c < kNormChunks; ++c) sa[c & 3] += pa[c];
      }
      for (int q = 0; q < nsb; ++q) {
        const double* pb = jb.partB + (q * nord + tid) * kNormChunks;
#pragma unroll
        for (int c = 0; c < kNormChunks; ++c) sb[c & 3] += pb[c];
      }
      na = sqrt((sa[0] + sa[1]) + (sa[2] + sa[3]));
      nb = sqrt((sb[0] + sb[1]) + (sb[2] + sb[3]));
    }
    in_bad = __any(!isfinite(na) || !isfinite(nb));
    // orders below 1e-15 of an operand's largest one carry no information in
    // FP64 (e.g. the rounding residue of a product at orders that vanish
    // exactly); they are left out so that s is not chosen to lift them
    double ma = na, mb = nb;
    for (int off = 32; off > 0; off >>= 1) {
      ma = fmax(ma, __shfl_xor(ma, off));
      mb = fmax(mb, __shfl_xor(mb, off));
    }
    if (na < kNoiseFloor * ma) na = 0.0;
    if (nb < kNoiseFloor * mb) nb = 0.0;
    // c_m = sum_j a_j b_{m-j}: lane m holds c_m (m < 64) and c_{m+64}
    double c0 = 0.0, c1 = 0.0;
    const int nm = 2 * nord - 1;
    for (int j = 0; j < nord; ++j) {
      const double aj = wave_bcast(na, j);
      const int m0 = tid - j, m1 = tid + 64 - j;
      const double b0 = __shfl(nb, m0 >= 0 && m0 < nord ? m0 : 0);
      const double b1 = __shfl(nb, m1 >= 0 && m1 < nord ? m1 : 0);
      if (m0 >= 0 && m0 < nord) c0 = fma(aj, b0, c0);
      if (m1 >= 0 && m1 < nord && tid + 64 < nm) c1 = fma(aj, b1, c1);
    }
    const bool ok0 = tid < nm && c0 > 0.0 && isfinite(c0);
    const bool ok1 = tid + 64 < nm && c1 > 0.0 && isfinite(c1);
    const double lc0 = ok0 ? log(c0) : 0.0, lc1 = ok1 ? log(c1) : 0.0;
    // log c_m, or the absent marker, of m = tid (lmax0, lmin0) and tid + 64 (lmax1)
    const double lmax0 = ok0 ? lc0 : -kAbsent, lmax1 = ok1 ? lc1 : -kAbsent;
    const double lmin0 = (ok0 && tid < nord) ? lc0 : kAbsent;
    const bool any = __any(ok0 && tid < nord);
    if (any) {
      double lo = -300.0 / (2.0 * (nord - 1)), hi = -lo;
      for (int round = 0; round < 3; ++round) {
        const double step = (hi - lo) / 63.0;
        const double tt = lo + step * tid;
        // four independent max / min chains over m
        double mx[4] = {-kAbsent, -kAbsent, -kAbsent, -kAbsent}, mn[4] = {kAbsent, kAbsent, kAbsent, kAbsent};
#pragma unroll 2
        for (int m = 0; m < 64; m += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            mx[u] = fmax(mx[u], fma(static_cast<double>(m + u), tt, wave_bcast(lmax0, m + u)));
            mn[u] = fmin(mn[u], fma(static_cast<double>(m + u), tt, wave_bcast(lmin0, m + u)));
          }
        }
        // orders 64..nm-1 (present only when nord > 32; the absent ones read -kAbsent)
        if (nm > 64) {
#pragma unroll 2
          for (int m = 64; m < 128; m += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              mx[u] = fmax(mx[u], fma(static_cast<double>(m + u), tt, wave_bcast(lmax1, m + u - 64)));
          }
        }
        // arg-min over lanes; near-ties (a flat objective, e.g. only one
        // nonzero order) go to the candidate closest to t = 0 (s = 1)
        double f = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3])) - fmin(fmin(mn[0], mn[1]), fmin(mn[2], mn[3]));
        int idx = tid;
        for (int off = 32; off > 0; off >>= 1) {
          const double f2 = __shfl_xor(f, off);
          const int i2 = __shfl_xor(idx, off);
          const double tol = 1e-9 * fmax(1.0, fabs(f));
          const double t1 = fabs(lo + step * idx), t2 = fabs(lo + step * i2);
          const bool better = (f2 < f - tol) || (fabs(f2 - f) <= tol && (t2 < t1 || (t2 == t1 && i2 < idx)));
          if (better) { f = f2; idx = i2; }
        }
        const double tb = lo + step * idx;
        lo = tb - step;
        hi = tb + step;
        t = tb;
      }
    }
  }
  ScaleRec* rec = jb.rec;
  if (tid == 0) {
    rec->s = exp(t);
    rec->in_bad = in_bad ? 1u : 0u;
    rec->out_bad = 0u;
  }
  rec->spow[tid] = exp(t * tid);
  rec->sinv[tid] = exp(-t * tid) / jb.L;
}

}  // namespace pm
