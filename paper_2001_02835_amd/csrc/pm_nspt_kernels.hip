// Kernels of the NSPT Euler-Langevin step (TEK model, eqs. (2)-(3)) that are
// not plain series products:
//
//  * k_retrunc      - re-truncation of a product kept in Fourier space:
//                     inverse transform, drop the orders above ntrunc, add a
//                     linear combination of truncated series (and of the
//                     unit series), forward transform again.  A chain of
//                     star products stays in Fourier space this way, one
//                     HBM read and write per link of the chain.
//  * k_inv_combine  - inverse transform of a weighted sum of products
//                     (the staple combination), with 1/L and unscaling.
//  * k_trace        - Tr M^(k) for every order.
//  * k_force        - D = M - M^+, F = i (D - Tr D / N), and either the
//                     drift-plus-noise exponent Y = i X = i (eps F + sqrt(2 eps) eta g)
//                     (Langevin) or the momentum kick P += c F with the
//                     exponent Y = i dt P (molecular dynamics), rescaled by
//                     s^k for the following products.
//  * k_refresh      - momentum refresh, P^(1) = eta and all other orders zero.
//  * k_series_scale - x^(k) <- s^k x^(k) in place.
//  * k_action       - action or Wilson-loop series from the traces of a loop sum.
//
// All series here are FP64 complex [nord][n][n]; Fourier coefficients use the
// formats of the product kernels (FP64, FP32 or split BF16).
#include "pm_fft.h"
#include "pm_nspt_kernels.h"

namespace pm {

namespace {

// ----------------------------------------------------------- re-truncation

// LIN: length of the product's transform; LOUT: length of the forward
// transform of the result (LOUT >= LIN, both with the same lanes per entry).
template <int LIN, int LOUT, FourierType FIN, FourierType FOUT>
__global__ __launch_bounds__(kFftThreads, fft_min_waves<LOUT>()) void k_retrunc(RetruncArgs args) {
  static_assert(LOUT >= LIN && fft_ent<LIN>() == fft_ent<LOUT>(), "unsupported length pair");
  constexpr int L = LOUT;
  constexpr int ENT = fft_ent<L>();
  constexpr int KSTEP = kFftThreads / ENT;
  __shared__ double2 acc[L / 2][ENT];
  const RetruncJob& jb = args.jobs[blockIdx.y];
  const int E = jb.E;
  const int e0 = blockIdx.x * ENT;
  if (e0 >= E) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = threadIdx.x / kWave;
  const int el = threadIdx.x % ENT;
  const int e = e0 + el;
  const bool valid = e < E;
  const int nord = jb.nord;
  if (jb.src) {
    auto load = [&](int p) { return valid ? load_mode<FIN>(jb.src, E, p, e) : make_double2(0.0, 0.0); };
    inverse_to_lds<LIN, fft_split<LIN>(), FIN == kF32>(load, acc, lane, r);
  }
  // time-domain value of order k: (1/L) inverse + addends (+ identity at order 0)
  const int n = jb.n;
  const bool diag = valid && (e / n) == (e - (e / n) * n);
  for (int k = threadIdx.x / ENT; k < L / 2; k += KSTEP) {
    if (k >= nord) {            // zero padding of the forward transform
      acc[k][el] = make_double2(0.0, 0.0);
      continue;
    }
    double2 x = jb.src ? cscale(acc[k][el], 1.0 / LIN) : make_double2(0.0, 0.0);
    if (valid) {
      for (int a = 0; a < args.nadd; ++a) {
        const double2 y = jb.add[static_cast<size_t>(a) * jb.add_stride + static_cast<size_t>(k) * E + e];
        x = cadd(x, cmul(args.coef[a], y));
      }
      if (k == 0 && diag) x = cadd(x, args.idcoef);
      if (jb.tdst) jb.tdst[static_cast<size_t>(k) * E + e] = x;
    }
    acc[k][el] = x;
  }
  __syncthreads();
  forward_from_tile<L, FOUT>(acc, lane, r, jb.dst, E, n, e, valid);
}

// --------------------------------------------- inverse of a weighted sum

template <int L, FourierType FIN, int NSRC>
__global__ __launch_bounds__(kFftThreads, fft_min_waves<L>()) void k_inv_combine(CombineArgs args) {
  constexpr int ENT = fft_ent<L>();
  constexpr int KSTEP = kFftThreads / ENT;
  __shared__ double2 acc[L / 2][ENT];
  const CombineJob& jb = args.jobs[blockIdx.y];
  const int E = jb.E;
  const int e0 = blockIdx.x * ENT;
  if (e0 >= E) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = threadIdx.x / kWave;
  const int el = threadIdx.x % ENT;
  const int e = e0 + el;
  const bool valid = e < E;
  const int ec = valid ? e : 0;        // clamped entry: loads stay in bounds, the result is not stored
  constexpr int NQ = lane_nmodes<L>();
  // this lane's modes of sum_src coef * src, one source at a time (bounded registers)
  auto build = [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    double2 d[NQ];
    static_for<0, NQ>([&](auto qi) { d[decltype(qi)::value] = make_double2(0.0, 0.0); });
#pragma unroll 1
    for (int q = 0; q < NSRC; ++q) {
      const void* src = jb.src[q];
      const double2 c = jb.coef[q];
      static_for<0, NQ>([&](auto qi) {
        constexpr int m = decltype(qi)::value;
        d[m] = cadd(d[m], cmul(c, load_mode<FIN>(src, E, lane_mode<L, R>(m, lane), ec)));
      });
    }
    inverse_from_modes<L, R>(d, acc, lane);
  };
  switch (r) {
    case 0: build(std::integral_constant<int, 0>{}); break;
    case 1: build(std::integral_constant<int, 1>{}); break;
    case 2: build(std::integral_constant<int, 2>{}); break;
    default: build(std::integral_constant<int, 3>{}); break;
  }
  if (valid)
    for (int k = threadIdx.x / ENT; k < jb.nord; k += KSTEP)
      if (k >= jb.kmin) jb.dst[static_cast<size_t>(k) * E + e] = cscale(acc[k][el], jb.rec->sinv[k]);
}

// ------------------------------------------------------------------ noise

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) on the counter c under
// the key (k0, k1): ten rounds of two 64 x 64 -> 128-bit products and a Weyl
// key schedule.
__device__ __forceinline__ void philox4x64_10(unsigned long long (&c)[4], unsigned long long k0,
                                              unsigned long long k1) {
  constexpr unsigned long long kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr unsigned long long kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
    const unsigned long long hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
    const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += kW0;
    k1 += kW1;
  }
}

// Entry pairs i <= j of matrix blockIdx.y: counter (i n + j, m, step, 0),
// key (seed, 0); u_a = ((x0 >> 11) + 1) 2^-53, u_b = (x1 >> 11) 2^-53,
// Box-Muller z0 = rho cos(2 pi u_b), z1 = rho sin(2 pi u_b), rho = sqrt(-2 ln u_a);
// eta_ij = (z0 + i z1) / sqrt 2 = conj(eta_ji) for i < j, eta_ii = z0.
__global__ __launch_bounds__(256) void k_noise(NoiseArgs a) {
  const int m = blockIdx.y;
  const int n = a.n;
  const size_t E = static_cast<size_t>(n) * n;
  double2* eta = a.eta + static_cast<size_t>(m) * E;
  const double r2 = sqrt(2.0);
  for (size_t e = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; e < E;
       e += static_cast<size_t>(gridDim.x) * 256) {
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<size_t>(i) * n);
    if (i > j) continue;
    unsigned long long c[4] = {static_cast<unsigned long long>(e), static_cast<unsigned long long>(m), a.step, 0ull};
    philox4x64_10(c, a.seed, 0ull);
    const double ua = static_cast<double>((c[0] >> 11) + 1ull) * 0x1.0p-53;
    const double ub = static_cast<double>(c[1] >> 11) * 0x1.0p-53;
    const double rho = sqrt(-2.0 * log(ua));
    const double ang = 2.0 * M_PI * ub;
    const double z0 = rho * cos(ang), z1 = rho * sin(ang);
    if (i == j) {
      eta[e] = make_double2(z0, 0.0);
    } else {
      const double re = z0 / r2, im = z1 / r2;
      eta[e] = make_double2(re, im);
      eta[static_cast<size_t>(j) * n + i] = make_double2(re, -im);
    }
  }
}

// eta_ii -= Tr(eta) / n for matrix blockIdx.x (the diagonal is real); the
// trace is summed in a fixed order (strided partial sums, then a tree).
__global__ __launch_bounds__(256) void k_noise_trace(NoiseArgs a) {
  __shared__ double part[256];
  const int n = a.n;
  const size_t E = static_cast<size_t>(n) * n;
  double2* eta = a.eta + static_cast<size_t>(blockIdx.x) * E;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += eta[static_cast<size_t>(i) * (n + 1)].x;
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  const double tr = part[0] / n;
  for (int i = threadIdx.x; i < n; i += 256) eta[static_cast<size_t>(i) * (n + 1)].x -= tr;
}

// ---------------------------------------------------------------- refresh

// P^(1) = eta, every other order zero (grid-stride over the series).
__global__ __launch_bounds__(256) void k_refresh(RefreshArgs args) {
  const RefreshJob& jb = args.jobs[blockIdx.y];
  const size_t total = static_cast<size_t>(jb.nord) * jb.E;
  for (size_t t = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * 256) {
    const size_t k = t / jb.E;
    jb.P[t] = (k == 1) ? jb.eta[t - jb.E] : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------------ series scale

// x^(k) <- s^k x^(k); grid (entry blocks, order, job).
__global__ __launch_bounds__(256) void k_series_scale(SeriesScaleArgs args) {
  const SeriesScaleJob& jb = args.jobs[blockIdx.z];
  const int k = blockIdx.y;
  if (k >= jb.nord) return;
  const double f = jb.rec->spow[k];
  double2* x = jb.x + static_cast<size_t>(k) * jb.E;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < jb.E; e += gridDim.x * 256) x[e] = cscale(x[e], f);
}

// ----------------------------------------------------------------- action

__global__ __launch_bounds__(256) void k_action(ActionArgs args) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= args.count) return;
  const int k = i % args.nord;
  args.S[i] = (k == 0 ? args.c0 : 0.0) + args.c1 * args.tr[i].x;
}

// ------------------------------------------------------------------ trace

__global__ __launch_bounds__(64) void k_trace(TraceArgs args) {
  const TraceJob& jb = args.jobs[blockIdx.y];
  const int k = blockIdx.x;
  if (k >= jb.nord) return;
  const int n = jb.n;
  const double2* m = jb.src + static_cast<size_t>(k) * n * n;
  double2 s = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < n; i += 64) s = cadd(s, m[static_cast<size_t>(i) * n + i]);
  // fixed-order wave reduction
  for (int off = 32; off > 0; off >>= 1) {
    s.x += __shfl_down(s.x, off);
    s.y += __shfl_down(s.y, off);
  }
  if (threadIdx.x == 0) jb.out[k] = s;
}

// ------------------------------------------------------------------ force

// One 32 x 32 tile (I, J) of one order k: the mirrored tile (J, I) is staged
// through LDS so that both M and M^+ are read with coalesced loads.
constexpr int kTile = 32;

__global__ __launch_bounds__(256) void k_force(ForceArgs args) {
  __shared__ double2 mir[kTile][kTile + 1];
  const ForceJob& jb = args.jobs[blockIdx.z];
  const int k = blockIdx.y;
  const int n = jb.n;
  const int nt = (n + kTile - 1) / kTile;
  if (k >= jb.nord || static_cast<int>(blockIdx.x) >= nt * nt) return;
  const int ti = blockIdx.x / nt, tj = blockIdx.x - (blockIdx.x / nt) * nt;
  const int I0 = ti * kTile, J0 = tj * kTile;
  const size_t E = static_cast<size_t>(n) * n;
  const double2* Mk = jb.M + static_cast<size_t>(k) * E;
  double2* Yk = jb.Y ? jb.Y + static_cast<size_t>(k) * E : nullptr;
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;   // 32 x 8
  // stage M[J0 + a][I0 + b] at mir[a][b]
  for (int a = ty; a < kTile; a += 8) {
    const int gi = J0 + a, gj = I0 + tx;
    mir[a][tx] = (gi < n && gj < n) ? Mk[static_cast<size_t>(gi) * n + gj] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double scale = jb.rec->spow[k];
  const double eps = args.eps;
  const double2 tr = jb.tr[k];
  const double noise = args.noise_amp;   // sqrt(2 eps)
  for (int a = ty; a < kTile; a += 8) {
    const int i = I0 + a, j = J0 + tx;
    if (i >= n || j >= n) continue;
    double2 y = make_double2(0.0, 0.0);
    if (k >= 1) {
      const double2 mij = Mk[static_cast<size_t>(i) * n + j];
      const double2 mji = mir[tx][a];                 // M[j][i]
      // D = M - M^+; Tr D = 2 i Im Tr M
      double2 d = make_double2(mij.x - mji.x, mij.y + mji.y);
      if (i == j) d.y -= 2.0 * tr.y / n;
      if (args.md) {
        // F = i (D - Tr D / N); P += kick F; Y = i dt P
        const size_t at = static_cast<size_t>(k) * E + static_cast<size_t>(i) * n + j;
        double2 pv = jb.P[at];
        pv = make_double2(pv.x - args.kick * d.y, pv.y + args.kick * d.x);
        jb.P[at] = pv;
        y = make_double2(-args.dt * pv.y, args.dt * pv.x);
      } else {
        y = make_double2(-eps * d.x, -eps * d.y);     // i X = -eps (D - Tr D / N)
        if (k == 1 && jb.eta) {
          const double2 et = jb.eta[static_cast<size_t>(i) * n + j];
          y = make_double2(y.x - noise * et.y, y.y + noise * et.x);   // + i sqrt(2 eps) eta
        }
      }
      y = cscale(y, scale);
    }
    if (Yk) Yk[static_cast<size_t>(i) * n + j] = y;
  }
}

template <FourierType FIN, FourierType FOUT>
hipError_t retrunc_dispatch(const RetruncArgs& a, int lin, int lout, dim3 g, hipStream_t s) {
#define PM_RT(A, B)                                                     \
  if (lin == A && lout == B) {                                          \
    k_retrunc<A, B, FIN, FOUT><<<g, kFftThreads, 0, s>>>(a);            \
    return hipGetLastError();                                           \
  }
  PM_RT(4, 4) PM_RT(8, 8) PM_RT(16, 16) PM_RT(32, 32) PM_RT(64, 64) PM_RT(128, 128)
  PM_RT(4, 8) PM_RT(8, 16) PM_RT(16, 32) PM_RT(32, 64)
#undef PM_RT
  return hipErrorInvalidValue;
}

template <FourierType FIN, int NSRC>
hipError_t combine_dispatch(const CombineArgs& a, int L, dim3 g, hipStream_t s) {
  switch (L) {
    case 4: k_inv_combine<4, FIN, NSRC><<<g, kFftThreads, 0, s>>>(a); break;
    case 8: k_inv_combine<8, FIN, NSRC><<<g, kFftThreads, 0, s>>>(a); break;
    case 16: k_inv_combine<16, FIN, NSRC><<<g, kFftThreads, 0, s>>>(a); break;
    case 32: k_inv_combine<32, FIN, NSRC><<<g, kFftThreads, 0, s>>>(a); break;
    case 64: k_inv_combine<64, FIN, NSRC><<<g, kFftThreads, 0, s>>>(a); break;
    case 128: k_inv_combine<128, FIN, NSRC><<<g, kFftThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_retrunc(const RetruncArgs& a, int lin, int lout, int max_entries, FourierType fin,
                          FourierType fout, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  const int ent = fft_entries_per_group(lout);
  dim3 g((max_entries + ent - 1) / ent, a.njobs);
  if (fin == kF64) return retrunc_dispatch<kF64, kF64>(a, lin, lout, g, s);
  if (fout == kF32) return retrunc_dispatch<kF32, kF32>(a, lin, lout, g, s);
  return retrunc_dispatch<kF32, kBF16Split>(a, lin, lout, g, s);
}

hipError_t launch_inv_combine(const CombineArgs& a, int L, int max_entries, FourierType fin, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  const int ent = fft_entries_per_group(L);
  dim3 g((max_entries + ent - 1) / ent, a.njobs);
  // every job of one launch has the same number of sources (1, 6 or 8)
  const int ns = a.jobs[0].nsrc;
  for (int j = 1; j < a.njobs; ++j)
    if (a.jobs[j].nsrc != ns) return hipErrorInvalidValue;
  static_assert(kMaxCombine == 8, "source counts instantiated below");
  if (ns == 1) return fin == kF64 ? combine_dispatch<kF64, 1>(a, L, g, s) : combine_dispatch<kF32, 1>(a, L, g, s);
  if (ns == 6) return fin == kF64 ? combine_dispatch<kF64, 6>(a, L, g, s) : combine_dispatch<kF32, 6>(a, L, g, s);
  if (ns == 8) return fin == kF64 ? combine_dispatch<kF64, 8>(a, L, g, s) : combine_dispatch<kF32, 8>(a, L, g, s);
  return hipErrorInvalidValue;
}

hipError_t launch_noise(const NoiseArgs& a, hipStream_t s) {
  if (a.count <= 0 || a.n <= 0) return hipSuccess;
  const size_t E = static_cast<size_t>(a.n) * a.n;
  const unsigned gx = static_cast<unsigned>(std::min<size_t>((E + 255) / 256, 1024));
  k_noise<<<dim3(gx, a.count), 256, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_noise_trace<<<a.count, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_refresh(const RefreshArgs& a, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  k_refresh<<<dim3(256, a.njobs), 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_series_scale(const SeriesScaleArgs& a, int max_nord, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  k_series_scale<<<dim3(64, max_nord, a.njobs), 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_action(const ActionArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  k_action<<<(a.count + 255) / 256, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs& a, int max_nord, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  k_trace<<<dim3(max_nord, a.njobs), 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_force(const ForceArgs& a, int n, int max_nord, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  const int nt = (n + kTile - 1) / kTile;
  k_force<<<dim3(nt * nt, max_nord, a.njobs), 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pm
