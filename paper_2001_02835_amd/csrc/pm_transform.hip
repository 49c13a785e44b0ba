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
// covers 64 entries (32 at L = 128, where two lanes share an entry);
// wavefront r computes residue r from the input tile staged in LDS.
//
// Inverse: wavefront r loads the modes p = 4q + r, runs a length-M inverse
// DFT d_r, and the four residues are combined as
//   C[k] = (1/L) sum_r w_L^{-kr} d_r[k mod M]   (k < nord)
// through LDS in a fixed order, so results are bitwise reproducible.
#include "pm_fft.h"
#include "pm_scale.h"

namespace pm {

namespace {

template <int L, FourierType FT>
__global__ __launch_bounds__(kFftThreads, fft_min_waves<L>()) void k_forward(FwdArgs args) {
  constexpr int ENT = fft_ent<L>();
  constexpr int KSTEP = kFftThreads / ENT;   // orders staged per pass
  __shared__ double2 tile[L / 2][ENT];
  const FwdJob& jb = args.jobs[blockIdx.y];
  const int e0 = blockIdx.x * ENT;
  if (e0 >= jb.E) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = threadIdx.x / kWave;
  const int el = threadIdx.x % ENT;
  const int e = e0 + el;
  const bool valid = e < jb.E;
  // Step 1 fused: rescale by s^k while staging; the zero padding of Step 2
  // only exists in LDS (rows nord .. L/2-1).
  for (int k = threadIdx.x / ENT; k < L / 2; k += KSTEP) {
    double2 v = (valid && k < jb.nord) ? jb.src[static_cast<size_t>(k) * jb.E + e] : make_double2(0.0, 0.0);
    tile[k][el] = k < jb.nord ? cscale(v, jb.rec->spow[k]) : v;
  }
  __syncthreads();
  forward_from_tile<L, FT>(tile, lane, r, jb.dst, jb.E, jb.n, e, valid);
}

// The length-128 inverse of FP32 products is built for four wavefronts per
// SIMD (a few registers spill): one product's inverse is then two rounds of
// work-groups instead of three, 14 % faster at N = 225.  With FP64 products
// the spills cost more than the extra round saves.
template <int L, FourierType FT>
constexpr int inverse_min_waves() { return (L >= 128 && FT == kF32) ? 4 : fft_min_waves<L>(); }

template <int L, FourierType FT>
__global__ __launch_bounds__(kFftThreads, (inverse_min_waves<L, FT>())) void k_inverse(InvArgs args) {
  constexpr int ENT = fft_ent<L>();
  constexpr int KSTEP = kFftThreads / ENT;
  __shared__ double2 acc[L / 2][ENT];
  const InvJob& jb = args.jobs[blockIdx.y];
  const int e0 = blockIdx.x * ENT;
  if (e0 >= jb.E) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = threadIdx.x / kWave;
  const int el = threadIdx.x % ENT;
  const int e = e0 + el;
  const bool valid = e < jb.E;
  auto load = [&](int p) { return valid ? load_mode<FT>(jb.src, jb.E, p, e) : make_double2(0.0, 0.0); };
  inverse_to_lds<L, fft_split<L>(), true>(load, acc, lane, r);
  // Steps 4-5: 1/L, unscale by s^-k (one table), keep orders < nord
  if (valid) {
    bool bad = false;
    for (int k = threadIdx.x / ENT; k < jb.nord; k += KSTEP) {
      const double2 v = cscale(acc[k][el], jb.rec->sinv[k]);
      bad = bad || !isfinite(v.x) || !isfinite(v.y);
      jb.dst[static_cast<size_t>(k) * jb.E + e] = v;
    }
    // every writer stores the same value; the scale kernel cleared it
    if (bad) jb.rec->out_bad = 1u;
  }
}

// ------------------------------------------------------------ norms / scale

// partial[k][chunk] = sum of |x|^2 over the chunk of entries of order k.
// Four independent loads per thread and pass keep enough reads in flight;
// the sum is reduced within each wavefront, then over the four wavefronts.
__global__ __launch_bounds__(256) void k_norms(NormArgs args) {
  __shared__ double red[4];
  const NormJob& jb = args.jobs[blockIdx.z];
  const int k = blockIdx.y;
  if (k >= jb.nord) return;
  const int chunk = blockIdx.x;
  const int per = (jb.E + kNormChunks - 1) / kNormChunks;
  const int b = chunk * per;
  const int e_end = min(jb.E, b + per);
  const double2* x = jb.src + static_cast<size_t>(k) * jb.E;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int e = b + threadIdx.x;
  for (; e + 768 < e_end; e += 1024) {
    const double2 v0 = x[e], v1 = x[e + 256], v2 = x[e + 512], v3 = x[e + 768];
    s0 = fma(v0.x, v0.x, fma(v0.y, v0.y, s0));
    s1 = fma(v1.x, v1.x, fma(v1.y, v1.y, s1));
    s2 = fma(v2.x, v2.x, fma(v2.y, v2.y, s2));
    s3 = fma(v3.x, v3.x, fma(v3.y, v3.y, s3));
  }
  for (; e < e_end; e += 256) {
    const double2 v = x[e];
    s0 = fma(v.x, v.x, fma(v.y, v.y, s0));
  }
  double sum = (s0 + s1) + (s2 + s3);
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) jb.partial[k * kNormChunks + chunk] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The stand-alone form of the choice of s (the computation of scale_wave in
// pm_scale.h, with the per-order values broadcast through LDS, which is
// faster than the cross-lane reads of the single-wavefront form).
__global__ __launch_bounds__(64) void k_scale(ScaleArgs args) {
  const ScaleJob& jb = args.jobs[blockIdx.x];
  const int nord = jb.nord;
  const int tid = threadIdx.x;
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
    // c_m = sum_j a_j b_{m-j}: lane m holds c_m (m < 64) and c_{m+64}; the
    // norms go through LDS so that the iterations do not wait on each other
    __shared__ double a_s[64], b_s[64];
    a_s[tid] = na;
    b_s[tid] = nb;
    __syncthreads();
    double c0 = 0.0, c1 = 0.0;
    const int nm = 2 * nord - 1;
    for (int j = 0; j < nord; ++j) {
      const double aj = a_s[j];
      const int m0 = tid - j, m1 = tid + 64 - j;
      const double b0 = b_s[m0 >= 0 && m0 < nord ? m0 : 0];
      const double b1 = b_s[m1 >= 0 && m1 < nord ? m1 : 0];
      if (m0 >= 0 && m0 < nord) c0 = fma(aj, b0, c0);
      if (m1 >= 0 && m1 < nord && tid + 64 < nm) c1 = fma(aj, b1, c1);
    }
    const bool ok0 = tid < nm && c0 > 0.0 && isfinite(c0);
    const bool ok1 = tid + 64 < nm && c1 > 0.0 && isfinite(c1);
    const double lc0 = ok0 ? log(c0) : 0.0, lc1 = ok1 ? log(c1) : 0.0;
    const double lmax0 = ok0 ? lc0 : -kAbsent, lmax1 = ok1 ? lc1 : -kAbsent;
    const double lmin0 = (ok0 && tid < nord) ? lc0 : kAbsent;
    const bool any = __any(ok0 && tid < nord);
    if (any) {
      // log c_m (or the absent marker) of every m, for broadcast reads
      __shared__ double lmax_s[128], lmin_s[64];
      lmax_s[tid] = lmax0;
      lmax_s[tid + 64] = lmax1;
      lmin_s[tid] = lmin0;
      __syncthreads();
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
            mx[u] = fmax(mx[u], fma(static_cast<double>(m + u), tt, lmax_s[m + u]));
            mn[u] = fmin(mn[u], fma(static_cast<double>(m + u), tt, lmin_s[m + u]));
          }
        }
        // orders 64..nm-1 (present only when nord > 32; the absent ones read -kAbsent)
        if (nm > 64) {
#pragma unroll 2
          for (int m = 64; m < 128; m += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) mx[u] = fmax(mx[u], fma(static_cast<double>(m + u), tt, lmax_s[m + u]));
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

template <FourierType FT>
hipError_t fwd_dispatch(const FwdArgs& a, int L, dim3 grid, hipStream_t s) {
  switch (L) {
    case 4: k_forward<4, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 8: k_forward<8, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 16: k_forward<16, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 32: k_forward<32, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 64: k_forward<64, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 128: k_forward<128, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <FourierType FT>
hipError_t inv_dispatch(const InvArgs& a, int L, dim3 grid, hipStream_t s) {
  switch (L) {
    case 4: k_inverse<4, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 8: k_inverse<8, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 16: k_inverse<16, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 32: k_inverse<32, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 64: k_inverse<64, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    case 128: k_inverse<128, FT><<<grid, kFftThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(const FwdArgs& a, int L, int max_entries, FourierType t, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  const int ent = fft_entries_per_group(L);
  dim3 grid((max_entries + ent - 1) / ent, a.njobs);
  switch (t) {
    case kF64: return fwd_dispatch<kF64>(a, L, grid, s);
    case kF32: return fwd_dispatch<kF32>(a, L, grid, s);
    default: return fwd_dispatch<kBF16Split>(a, L, grid, s);
  }
}

hipError_t launch_inverse(const InvArgs& a, int L, int max_entries, FourierType t, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  const int ent = fft_entries_per_group(L);
  dim3 grid((max_entries + ent - 1) / ent, a.njobs);
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
