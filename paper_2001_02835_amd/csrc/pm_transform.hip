// Order-axis transforms (FFT-CONV Steps 1-2 and 4-5, eqs. (6)-(9)) and the
// per-order rescaling.
//
// The series layout [k][i][j] keeps the N*N entries of one order contiguous,
// so a transform along the order axis is a batch of N*N strided length-L
// transforms whose batch index is contiguous: consecutive lanes take
// consecutive entries and every global access of a wavefront is one
// contiguous 1 KB run (no transpose pass is needed).
//
// Forward (L = 4M, input orders 0..nord-1 with nord <= 2M, rest zero):
//   At[4q + r] = sum_{m<M} w_M^{mq} c_r[m],   c_r[m] = w_L^{mr} (a[m] + i^r a[m+M])
// i.e. one pruned radix-4 step (the upper half of the padded input is zero)
// followed by a length-M DFT per residue r.  A work-group of four wavefronts
// covers 64 entries; wavefront r computes residue r from the input tile
// staged in LDS.
//
// Inverse: wavefront r loads the modes p = 4q + r, runs a length-M inverse
// DFT d_r, and the four residues are combined as
//   C[k] = (1/L) sum_r w_L^{-kr} d_r[k mod M]   (k < nord)
// through LDS in a fixed order, so results are bitwise reproducible.
#include "pm_common.h"
#include "pm_kernels.h"

#include <hip/hip_bfloat16.h>

namespace pm {

namespace {

constexpr int kEnt = 64;        // entries per work-group
constexpr int kThreads = 256;   // four wavefronts

// --------------------------------------------------------------- stores

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

template <FourierType FT>
__device__ __forceinline__ void store_mode(const FwdJob& jb, int p, int e, double2 v) {
  if constexpr (FT == kF64) {
    reinterpret_cast<double2*>(jb.dst)[static_cast<size_t>(p) * jb.E + e] = v;
  } else if constexpr (FT == kF32) {
    reinterpret_cast<float2*>(jb.dst)[static_cast<size_t>(p) * jb.E + e] =
        make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
  } else {
    const int n = jb.n;
    const int i = e / n, j = e - (e / n) * n;
    const size_t plane = bf16_plane_elems(n);
    uint16_t* base = reinterpret_cast<uint16_t*>(jb.dst) + static_cast<size_t>(p) * 4 * plane;
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

template <FourierType FT>
__device__ __forceinline__ double2 load_mode(const InvJob& jb, int p, int e) {
  if constexpr (FT == kF64) {
    return reinterpret_cast<const double2*>(jb.src)[static_cast<size_t>(p) * jb.E + e];
  } else {
    float2 f = reinterpret_cast<const float2*>(jb.src)[static_cast<size_t>(p) * jb.E + e];
    return make_double2(f.x, f.y);
  }
}

// ------------------------------------------------------------ forward

template <int L, int R, FourierType FT>
__device__ __forceinline__ void forward_residue(const FwdJob& jb, const double2 (*tile)[kEnt],
                                                int lane, int e, bool valid) {
  constexpr int M = L / 4;
  const int nord = jb.nord;
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
      store_mode<FT>(jb, 4 * q + R, e, c[q]);
    });
  }
}

template <int L, FourierType FT>
__global__ __launch_bounds__(kThreads) void k_forward(FwdArgs args) {
  __shared__ double2 tile[L / 2][kEnt];
  const FwdJob& jb = args.jobs[blockIdx.y];
  const int e0 = blockIdx.x * kEnt;
  if (e0 >= jb.E) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = threadIdx.x / kWave;
  const int e = e0 + lane;
  const bool valid = e < jb.E;
  // Step 1 fused: rescale by s^k while staging orders k = r, r+4, ...; the
  // zero padding is never stored (orders >= nord read as zero below).
  for (int k = r; k < jb.nord; k += 4) {
    double2 v = valid ? jb.src[static_cast<size_t>(k) * jb.E + e] : make_double2(0.0, 0.0);
    tile[k][lane] = cscale(v, jb.rec->spow[k]);
  }
  __syncthreads();
  switch (r) {
    case 0: forward_residue<L, 0, FT>(jb, tile, lane, e, valid); break;
    case 1: forward_residue<L, 1, FT>(jb, tile, lane, e, valid); break;
    case 2: forward_residue<L, 2, FT>(jb, tile, lane, e, valid); break;
    default: forward_residue<L, 3, FT>(jb, tile, lane, e, valid); break;
  }
}

// ------------------------------------------------------------ inverse

template <int L, int R, FourierType FT>
__device__ __forceinline__ void inverse_residue(const InvJob& jb, double2 (*acc)[kEnt], int lane, int e,
                                                bool valid) {
  constexpr int M = L / 4;
  const int nord = jb.nord;
  double2 d[M];
  static_for<0, M>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    d[q] = valid ? load_mode<FT>(jb, 4 * q + R, e) : make_double2(0.0, 0.0);
  });
  dft_inplace<M, -1>(d);
  // t_r[k] = w^{-kr} d_r[k mod M]; for k = j + M the extra factor is (-i)^r.
  auto term = [&](auto ki) {
    constexpr int k = decltype(ki)::value;
    return ctwiddle<k * R, L, -1>(d[k % M]);
  };
  // Fixed-order accumulation: r = 0 writes, r = 1, 2 add, r = 3 finishes.
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
      if (k < nord && valid) {
        double2 v = cadd(acc[k][lane], term(ki));
        jb.dst[static_cast<size_t>(k) * jb.E + e] = cscale(v, jb.rec->sinv[k]);
      }
    });
  }
}

template <int L, FourierType FT>
__global__ __launch_bounds__(kThreads) void k_inverse(InvArgs args) {
  __shared__ double2 acc[L / 2][kEnt];
  const InvJob& jb = args.jobs[blockIdx.y];
  const int e0 = blockIdx.x * kEnt;
  if (e0 >= jb.E) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = threadIdx.x / kWave;
  const int e = e0 + lane;
  const bool valid = e < jb.E;
  switch (r) {
    case 0: inverse_residue<L, 0, FT>(jb, acc, lane, e, valid); break;
    case 1: inverse_residue<L, 1, FT>(jb, acc, lane, e, valid); break;
    case 2: inverse_residue<L, 2, FT>(jb, acc, lane, e, valid); break;
    default: inverse_residue<L, 3, FT>(jb, acc, lane, e, valid); break;
  }
}

// ------------------------------------------------------------ norms / scale

// partial[k][chunk] = sum of |x|^2 over the chunk of entries of order k.
__global__ __launch_bounds__(256) void k_norms(NormArgs args) {
  __shared__ double red[256];
  const NormJob& jb = args.jobs[blockIdx.z];
  const int k = blockIdx.y;
  if (k >= jb.nord) return;
  const int chunk = blockIdx.x;
  const int per = (jb.E + kNormChunks - 1) / kNormChunks;
  const int b = chunk * per;
  const int e_end = min(jb.E, b + per);
  const double2* x = jb.src + static_cast<size_t>(k) * jb.E;
  double s = 0.0;
  for (int e = b + threadIdx.x; e < e_end; e += 256) {
    double2 v = x[e];
    s = fma(v.x, v.x, fma(v.y, v.y, s));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) jb.partial[k * kNormChunks + chunk] = red[0];
}

// Choice of s (log s = t): with a_j = ||A^(j)||, b_j = ||B^(j)|| and
// c_m = sum_j a_j b_{m-j} (m <= 2 ntrunc, the orders of the full product,
// including those the truncation discards), minimise the spread
//   f(t) = max_m (log c_m + m t) - min_{k <= ntrunc} (log c_k + k t)
// over the nonzero c.  f is convex and piecewise linear.  One wavefront
// evaluates it on a 64-point grid; three refinement rounds shrink the grid
// spacing by 32 each.
constexpr double kAbsent = 1e300;

__global__ __launch_bounds__(64) void k_scale(ScaleArgs args) {
  __shared__ double na[kMaxL / 2], nb[kMaxL / 2];
  __shared__ double lmax[kMaxL], lmin[kMaxL / 2];
  __shared__ double fval[64];
  const ScaleJob& jb = args.jobs[blockIdx.x];
  const int nord = jb.nord;
  const int tid = threadIdx.x;
  double t = 0.0;
  if (jb.fixed_s > 0.0) {
    t = log(jb.fixed_s);
  } else if (nord > 1) {
    if (tid < nord) {
      double sa = 0.0, sb = 0.0;
      for (int c = 0; c < kNormChunks; ++c) {
        sa += jb.partA[tid * kNormChunks + c];
        sb += jb.partB[tid * kNormChunks + c];
      }
      na[tid] = sqrt(sa);
      nb[tid] = sqrt(sb);
    }
    __syncthreads();
    const int nm = 2 * nord - 1;
    for (int m = tid; m < nm; m += 64) {
      double c = 0.0;
      const int j0 = max(0, m - (nord - 1)), j1 = min(m, nord - 1);
      for (int j = j0; j <= j1; ++j) c = fma(na[j], nb[m - j], c);
      const bool ok = c > 0.0 && isfinite(c);
      const double lc = ok ? log(c) : 0.0;
      lmax[m] = ok ? lc : -kAbsent;
      if (m < nord) lmin[m] = ok ? lc : kAbsent;
    }
    __syncthreads();
    bool any = false;
    for (int k = 0; k < nord; ++k) any |= lmin[k] < kAbsent;
    if (any) {
      double lo = -300.0 / (2.0 * (nord - 1)), hi = -lo;
      for (int round = 0; round < 3; ++round) {
        const double step = (hi - lo) / 63.0;
        const double tt = lo + step * tid;
        double mx = -kAbsent, mn = kAbsent;
        for (int m = 0; m < nord; ++m) {
          mx = fmax(mx, fma(static_cast<double>(m), tt, lmax[m]));
          mn = fmin(mn, fma(static_cast<double>(m), tt, lmin[m]));
        }
        for (int m = nord; m < nm; ++m) mx = fmax(mx, fma(static_cast<double>(m), tt, lmax[m]));
        fval[tid] = mx - mn;
        __syncthreads();
        int best = 0;
        double fb = fval[0];
        for (int i = 1; i < 64; ++i)
          if (fval[i] < fb) { fb = fval[i]; best = i; }
        __syncthreads();
        const double tb = lo + step * best;
        lo = tb - step;
        hi = tb + step;
        t = tb;
      }
    }
  }
  ScaleRec* rec = jb.rec;
  if (tid == 0) rec->s = exp(t);
  rec->spow[tid] = exp(t * tid);
  rec->sinv[tid] = exp(-t * tid) / jb.L;
}

template <FourierType FT>
hipError_t fwd_dispatch(const FwdArgs& a, int L, dim3 grid, hipStream_t s) {
  switch (L) {
    case 4: k_forward<4, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 8: k_forward<8, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 16: k_forward<16, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 32: k_forward<32, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 64: k_forward<64, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 128: k_forward<128, FT><<<grid, kThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <FourierType FT>
hipError_t inv_dispatch(const InvArgs& a, int L, dim3 grid, hipStream_t s) {
  switch (L) {
    case 4: k_inverse<4, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 8: k_inverse<8, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 16: k_inverse<16, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 32: k_inverse<32, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 64: k_inverse<64, FT><<<grid, kThreads, 0, s>>>(a); break;
    case 128: k_inverse<128, FT><<<grid, kThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(const FwdArgs& a, int L, int max_entries, FourierType t, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  dim3 grid((max_entries + kEnt - 1) / kEnt, a.njobs);
  switch (t) {
    case kF64: return fwd_dispatch<kF64>(a, L, grid, s);
    case kF32: return fwd_dispatch<kF32>(a, L, grid, s);
    default: return fwd_dispatch<kBF16Split>(a, L, grid, s);
  }
}

hipError_t launch_inverse(const InvArgs& a, int L, int max_entries, FourierType t, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  dim3 grid((max_entries + kEnt - 1) / kEnt, a.njobs);
  switch (t) {
    case kF64: return inv_dispatch<kF64>(a, L, grid, s);
    default: return inv_dispatch<kF32>(a, L, grid, s);
  }
}

hipError_t launch_norms(const NormArgs& a, int max_nord, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  dim3 grid(kNormChunks, max_nord, a.njobs);
  k_norms<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_scale(const ScaleArgs& a, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  k_scale<<<a.njobs, 64, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pm
