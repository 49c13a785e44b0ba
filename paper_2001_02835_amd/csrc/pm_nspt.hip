// Host orchestration of the NSPT updates of the TEK model (eqs. (1)-(3)) for
// R replicas at once, on the FFT-CONV building blocks: one Euler-Langevin
// step, and one leapfrog trajectory of the molecular-dynamics form of the
// tower (the integrator the paper names below eq. (3)).
//
// Two rescale factors are chosen on the device per update: s from the
// per-order norms of all link series for the staple products, and s' from the
// norms of the exponent Y and of the links for the exponential and the link
// update (Y can grow much faster with the order than U).  Within each group
// every series lives in the rescaled variable (order k multiplied by s^k),
// which keeps its Fourier-space products consistent with each other.  With
// U~ the transforms of the links:
//
//  staples (42 products per replica, 24 re-truncations)
//    Q_mn = U_m * U_n           (m != n)      R_mn = U_m * U_n^+   (m < n)
//    W_mn = U_m^+ * U_n         (m < n)
//    P_mn = Q_mn * Q_nm^+       (m < n)       T_mn = R_mn * W_mn   (all m != n;
//                                              R_mn = R_nm^+, W_mn = W_nm^+ for m > n)
//    The force needs D_m = S_m - S_m^+ only, and the plaquette terms of S_m and
//    S_n are conjugate to each other, so D_m = M_m - M_m^+ with
//    M_m = sum_{n>m} z_mn P_mn - sum_{n<m} z_nm P_nm + sum_{n!=m} z_mn^* T_mn,
//    formed in Fourier space and transformed back once per direction.
//  exponent Y (then rescaled by s'^k)
//    Langevin:  Y_m = i X_m = -eps (D - Tr D / N) + i sqrt(2 eps) eta_m g,  Y^(0) = 0
//    MD:        P^(k) += c F^(k) (k >= 1, F = i (D - Tr D / N)), then Y = i dt P
//  exponential, Paterson-Stockmeyer with block b ~ sqrt(ntrunc + 1)
//    Y^2..Y^b by products; E = sum_q (Y^b)^q B_q(Y), B_q = sum_{i<b} Y^i / (qb + i)!
//    by Horner in Y^b; B_q is added inside the re-truncation of each link.
//  link update
//    U_m <- E_m * U_m, order 0 left as it is (E^(0) = 1 exactly).
#include <algorithm>
#include <cmath>
#include <vector>

#include "pm_common.h"
#include "pm_kernels.h"
#include "pm_nspt.h"
#include "pm_nspt_kernels.h"

namespace pm {

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxNtruncPlus1 = PM_MAX_NTRUNC + 1;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool valid_params(int replicas, const nspt_params* p, int prec) {
  if (!p || replicas < 1 || replicas > 1024) return false;
  if (prec != PM_PREC_FP64 && prec != PM_PREC_FP32 && prec != PM_PREC_BF16X3) return false;
  if (p->L < 1 || p->L % 2 == 0 || p->L > 64 || p->n != p->L * p->L) return false;
  if (p->ntrunc < 0 || p->ntrunc > PM_MAX_NTRUNC) return false;
  if (!std::isfinite(p->eps) || p->eps <= 0.0) return false;
  return true;
}

int tlength(int ntrunc) {
  int L = 4;
  while (L < 2 * (ntrunc + 1)) L *= 2;
  return L;
}

// Paterson-Stockmeyer plan of exp(Y) for Y = O(g): powers Y^2..Y^b at the
// full length L, then Horner in Y^b, Z_Q = B_Q, Z_q = Y^b * Z_{q+1} + B_q
// (Q = ntrunc / b).  Z_q is needed only to order K_q = ntrunc - q b (it is
// multiplied by (Y^b)^q = O(g^{q b}) afterwards), so the product of step q
// runs at the length of order K_q, made at most half the next step's
// length (the re-truncation between two steps at most doubles the length).
// L of 128 keeps one length throughout.
struct ExpPlan {
  int b, Q;
  int len[kMaxNtruncPlus1];   // len[q]: transform length of the product of Horner step q (q < Q)
};

int tlength(int ntrunc);

ExpPlan exp_plan(int ntrunc) {
  const int L = tlength(ntrunc);
  ExpPlan best{};
  long best_cost = -1;
  for (int b = 1; b <= 12; ++b) {
    ExpPlan pl{};
    pl.b = b;
    pl.Q = ntrunc / b;
    long cost = static_cast<long>(b - 1) * L;
    for (int q = 0; q < pl.Q; ++q) {
      int lq = L;
      if (L <= 64 && q > 0) {
        lq = tlength(ntrunc - q * b);
        if (lq < pl.len[q - 1] / 2) lq = pl.len[q - 1] / 2;
      }
      pl.len[q] = lq;
      cost += lq;
    }
    if (best_cost < 0 || cost < best_cost) { best = pl; best_cost = cost; }
  }
  return best;
}

int ps_block(int ntrunc) { return exp_plan(ntrunc).b; }

FourierType in_type(int prec) { return prec == PM_PREC_FP64 ? kF64 : (prec == PM_PREC_FP32 ? kF32 : kBF16Split); }
FourierType out_type(int prec) { return prec == PM_PREC_FP64 ? kF64 : kF32; }

// Workspace layout (per call, all replicas).
struct Layout {
  int n, E, nord, L, R, b;
  size_t fin, fout, tser;        // bytes: Fourier (product input), Fourier (product output), time series
  size_t rec, rec2, unit, part, partY, trc;   // small tables
  size_t Ut, G, Xt, M, Ypt, Ypf, Z, eta;
  size_t total;
};

Layout layout(int R, const nspt_params* p, int prec) {
  Layout l{};
  l.n = p->n;
  l.E = p->n * p->n;
  l.nord = p->ntrunc + 1;
  l.L = tlength(p->ntrunc);
  l.R = R;
  l.b = ps_block(p->ntrunc);
  const size_t E = static_cast<size_t>(l.E);
  l.fin = align_up(prec == PM_PREC_FP64 ? E * l.L * 16
                   : prec == PM_PREC_FP32 ? E * l.L * 8
                                          : static_cast<size_t>(bf16_ld(l.n)) * l.n * 8 * l.L);
  // a G slot holds a product result (output format, length L) or, in the
  // series exponential, a copy of Y^b in the input format at a length <= L/2;
  // the split-BF16 rows are padded to 8 entries, which for n = 1 makes that
  // copy larger than a result
  l.fout = std::max(align_up(E * l.L * (prec == PM_PREC_FP64 ? 16 : 8)), l.fin);
  l.tser = align_up(E * l.nord * 16);
  size_t off = 0;
  l.rec = off;  off += align_up(sizeof(ScaleRec));
  l.rec2 = off; off += align_up(sizeof(ScaleRec));
  l.unit = off; off += align_up(sizeof(ScaleRec));
  l.part = off; off += align_up(static_cast<size_t>(4) * R * l.nord * kNormChunks * sizeof(double));
  l.partY = off; off += align_up(static_cast<size_t>(4) * R * l.nord * kNormChunks * sizeof(double));
  l.trc = off;  off += align_up(static_cast<size_t>(4) * R * l.nord * 16);
  l.Ut = off;   off += static_cast<size_t>(4) * R * l.fin;
  l.G = off;    off += static_cast<size_t>(24) * R * l.fout;
  l.Xt = off;   off += static_cast<size_t>(24) * R * l.fin;
  l.M = off;    off += static_cast<size_t>(4) * R * l.tser;
  l.Ypt = off;  off += static_cast<size_t>(4) * R * l.b * l.tser;
  l.Ypf = off;  off += static_cast<size_t>(4) * R * l.b * l.fin;
  l.Z = off;    off += static_cast<size_t>(4) * R * l.fin;
  l.eta = off;  off += align_up(static_cast<size_t>(4) * R * E * 16);   // noise of nspt_steps
  l.total = off;
  return l;
}

pm_status st(hipError_t e) { return e == hipSuccess ? PM_OK : PM_ERR_DEVICE; }

// twist phases z_{mu nu}
double2 twist(const nspt_params* p, int mu, int nu) {
  const double ang = 2.0 * M_PI * p->k / p->L;
  if (mu < nu) return make_double2(std::cos(ang), std::sin(ang));
  return make_double2(std::cos(ang), -std::sin(ang));
}

// Accumulates GEMM jobs of one operand form and launches them in chunks.
struct GemmBatch {
  FourierType ft;
  hipStream_t s;
  int form;     // opA * 2 + opB
  GemmArgs a{};
  pm_status status = PM_OK;
  int cfg = 0;
  void add(const void* A, const void* B, void* C, int n, int L) {
    if (status) return;
    const int c = gemm_config(ft, n, L);   // one matrix size per NSPT call; L per chain step
    if (a.njobs == kMaxGemmJobs || (a.njobs > 0 && c != cfg)) flush();
    cfg = c;
    const GemmShape sh = gemm_shape(ft, cfg);
    GemmJob& j = a.jobs[a.njobs++];
    j.A = A;
    j.B = B;
    j.C = C;
    j.n = n;
    j.L = L;
    j.opA = form >> 1;
    j.opB = form & 1;
    j.tiles_m = (n + sh.bm - 1) / sh.bm;
    j.tiles_n = (n + sh.bn - 1) / sh.bn;
    j.tile_begin = a.total_tiles;
    a.total_tiles += j.tiles_m * j.tiles_n * L;
  }
  void flush() {
    if (status || a.njobs == 0) return;
    status = st(timed(PM_PHASE_PRODUCT, s, [&] { return launch_gemm(a, ft, cfg, s); }));
    a.njobs = 0;
    a.total_tiles = 0;
  }
};

struct RetruncBatch {
  const Layout* l;
  FourierType fin, fout;
  hipStream_t s;
  int lin = 0, lout = 0, nord = 0;   // 0: the call's L and order count
  RetruncArgs a{};
  pm_status status = PM_OK;
  void add(const void* src, void* dst, double2* tdst, const double2* addbase, size_t add_stride) {
    if (status) return;
    if (a.njobs == kMaxRetruncJobs) flush();
    RetruncJob& j = a.jobs[a.njobs++];
    j.src = src;
    j.dst = dst;
    j.tdst = tdst;
    j.add = addbase;
    j.add_stride = add_stride;
    j.E = l->E;
    j.n = l->n;
    j.nord = nord ? nord : l->nord;
  }
  void flush() {
    if (status || a.njobs == 0) return;
    const int li = lin ? lin : l->L, lo = lout ? lout : l->L;
    status = st(timed(PM_PHASE_RETRUNC, s, [&] { return launch_retrunc(a, li, lo, l->E, fin, fout, s); }));
    a.njobs = 0;
  }
};

}  // namespace

namespace {

// One call's view of the workspace and the stages of a force evaluation and
// link update.  Every stage enqueues on `s` and returns the first error.
struct Run {
  Layout l;
  const nspt_params* p;
  int R, prec;
  FourierType fin, fout;
  hipStream_t s;
  char* ws;
  double2* Ug;
  ScaleRec* rec;
  ScaleRec* rec2;
  ScaleRec* unit;
  double* part;
  double* partY;
  double2* trc;
  size_t series_elems;
  int qslot[4][4], pair[4][4];
  // exponent series per replica: 4 (one per direction, Langevin and MD) or 1
  // (gauge fixing: one Omega for all directions); with conj_update the update
  // is U_m <- E U_m E^+ instead of U_m <- E_m U_m
  int nexp = 4;
  bool conj_update = false;

  Run(void* U, int R_, const nspt_params* p_, int prec_, void* workspace, hipStream_t s_)
      : l(layout(R_, p_, prec_)), p(p_), R(R_), prec(prec_), fin(in_type(prec_)), fout(out_type(prec_)), s(s_) {
    ws = static_cast<char*>(workspace);
    Ug = static_cast<double2*>(U);
    rec = reinterpret_cast<ScaleRec*>(ws + l.rec);
    rec2 = reinterpret_cast<ScaleRec*>(ws + l.rec2);
    unit = reinterpret_cast<ScaleRec*>(ws + l.unit);
    part = reinterpret_cast<double*>(ws + l.part);
    partY = reinterpret_cast<double*>(ws + l.partY);
    trc = reinterpret_cast<double2*>(ws + l.trc);
    series_elems = static_cast<size_t>(l.nord) * l.E;
    // slot maps: Q_mn (m != n) -> 0..11, R_mn (m < n) -> 12..17, W_mn (m < n) -> 18..23
    int q = 0, pr = 0;
    for (int m = 0; m < 4; ++m)
      for (int nn = 0; nn < 4; ++nn) {
        qslot[m][nn] = (m != nn) ? q++ : -1;
        pair[m][nn] = (m < nn) ? pr++ : -1;
      }
  }

  double2* Useries(int r, int mu) const { return Ug + (static_cast<size_t>(r) * 4 + mu) * series_elems; }
  char* Ut(int r, int mu) const { return ws + l.Ut + (static_cast<size_t>(r) * 4 + mu) * l.fin; }
  char* G(int r, int slot) const { return ws + l.G + (static_cast<size_t>(r) * 24 + slot) * l.fout; }
  char* Xt(int r, int slot) const { return ws + l.Xt + (static_cast<size_t>(r) * 24 + slot) * l.fin; }
  double2* Mser(int r, int mu) const {
    return reinterpret_cast<double2*>(ws + l.M + (static_cast<size_t>(r) * 4 + mu) * l.tser);
  }
  // powers Y^j, j = 1..b, slot j - 1
  double2* Ypt(int r, int mu, int j) const {
    return reinterpret_cast<double2*>(ws + l.Ypt + ((static_cast<size_t>(r) * 4 + mu) * l.b + (j - 1)) * l.tser);
  }
  char* Ypf(int r, int mu, int j) const {
    return ws + l.Ypf + ((static_cast<size_t>(r) * 4 + mu) * l.b + (j - 1)) * l.fin;
  }
  char* Zf(int r, int mu) const { return ws + l.Z + (static_cast<size_t>(r) * 4 + mu) * l.fin; }

  // ---- rescale factor from the norms of all link series (and the unit
  //      record), then the forward transforms of the links
  pm_status links_forward() {
    const int E = l.E, nord = l.nord, L = l.L, n = l.n;
    NormArgs na{};
    for (int r = 0; r < R; ++r)
      for (int mu = 0; mu < 4; ++mu) {
        if (na.njobs == kMaxTransformJobs) {
          pm_status e = st(timed(PM_PHASE_RESCALE, s, [&] { return launch_norms(na, nord, s); }));
          if (e) return e;
          na.njobs = 0;
        }
        NormJob& j = na.jobs[na.njobs++];
        j.src = Useries(r, mu);
        j.partial = part + (static_cast<size_t>(r) * 4 + mu) * nord * kNormChunks;
        j.E = E;
        j.nord = nord;
      }
    pm_status e = st(timed(PM_PHASE_RESCALE, s, [&] { return launch_norms(na, nord, s); }));
    if (e) return e;
    ScaleArgs sa{};
    sa.njobs = 2;
    sa.jobs[0].partA = part;
    sa.jobs[0].partB = part;
    sa.jobs[0].rec = rec;
    sa.jobs[0].nord = nord;
    sa.jobs[0].L = L;
    sa.jobs[0].fixed_s = 0.0;
    sa.jobs[0].nser = 4 * R;
    sa.jobs[1] = sa.jobs[0];
    sa.jobs[1].rec = unit;
    sa.jobs[1].fixed_s = 1.0;
    sa.jobs[1].nser = 1;
    e = st(timed(PM_PHASE_RESCALE, s, [&] { return launch_scale(sa, s); }));
    if (e) return e;

    FwdArgs fa{};
    for (int r = 0; r < R; ++r)
      for (int mu = 0; mu < 4; ++mu) {
        if (fa.njobs == kMaxTransformJobs) {
          e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fa, L, E, fin, s); }));
          if (e) return e;
          fa.njobs = 0;
        }
        FwdJob& j = fa.jobs[fa.njobs++];
        j.src = Useries(r, mu);
        j.dst = Ut(r, mu);
        j.rec = rec;
        j.E = E;
        j.nord = nord;
        j.n = n;
      }
    return st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fa, L, E, fin, s); }));
  }

  // ---- staples: M_m of every replica and direction (unscaled time domain)
  //      and the traces Tr M^(k)
  pm_status staples() {
    const int n = l.n, E = l.E, nord = l.nord, L = l.L;
    // first wave: Q, R, W, re-truncated in Fourier space
    {
      GemmBatch nn{fin, s, 0}, nc{fin, s, 1}, cn{fin, s, 2};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m)
          for (int q = 0; q < 4; ++q) {
            if (m == q) continue;
            nn.add(Ut(r, m), Ut(r, q), G(r, qslot[m][q]), n, L);
            if (m < q) {
              nc.add(Ut(r, m), Ut(r, q), G(r, 12 + pair[m][q]), n, L);
              cn.add(Ut(r, m), Ut(r, q), G(r, 18 + pair[m][q]), n, L);
            }
          }
      nn.flush();
      nc.flush();
      cn.flush();
      if (nn.status || nc.status || cn.status) return PM_ERR_DEVICE;
      RetruncBatch rt{&l, fout, fin, s};
      rt.a.nadd = 0;
      rt.a.idcoef = make_double2(0.0, 0.0);
      for (int r = 0; r < R; ++r)
        for (int slot = 0; slot < 24; ++slot) rt.add(G(r, slot), Xt(r, slot), nullptr, nullptr, 0);
      rt.flush();
      if (rt.status) return rt.status;
    }
    // second wave: P (6) into G slots 0..5, T (12) into G slots 6..17
    {
      GemmBatch nc{fin, s, 1}, nn{fin, s, 0}, cc{fin, s, 3};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m)
          for (int q = 0; q < 4; ++q) {
            if (m == q) continue;
            if (m < q) {
              nc.add(Xt(r, qslot[m][q]), Xt(r, qslot[q][m]), G(r, pair[m][q]), n, L);               // P_mq
              nn.add(Xt(r, 12 + pair[m][q]), Xt(r, 18 + pair[m][q]), G(r, 6 + qslot[m][q]), n, L);  // T_mq
            } else {
              cc.add(Xt(r, 12 + pair[q][m]), Xt(r, 18 + pair[q][m]), G(r, 6 + qslot[m][q]), n, L);  // T_mq, m > q
            }
          }
      nc.flush();
      nn.flush();
      cc.flush();
      if (nn.status || nc.status || cc.status) return PM_ERR_DEVICE;
    }
    // M_m: weighted sum of P and T, back to the (unscaled) time domain
    {
      CombineArgs ca{};
      auto flush = [&]() -> pm_status {
        if (ca.njobs == 0) return PM_OK;
        pm_status e = st(timed(PM_PHASE_INVERSE, s, [&] { return launch_inv_combine(ca, L, E, fout, s); }));
        ca.njobs = 0;
        return e;
      };
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) {
          if (ca.njobs == kMaxCombineJobs) { pm_status e = flush(); if (e) return e; }
          CombineJob& j = ca.jobs[ca.njobs++];
          j.nsrc = 0;
          for (int q = 0; q < 4; ++q) {
            if (q == m) continue;
            if (q > m) {
              j.src[j.nsrc] = G(r, pair[m][q]);
              j.coef[j.nsrc++] = twist(p, m, q);
            } else {
              const double2 z = twist(p, q, m);
              j.src[j.nsrc] = G(r, pair[q][m]);
              j.coef[j.nsrc++] = make_double2(-z.x, -z.y);
            }
            const double2 z = twist(p, m, q);
            j.src[j.nsrc] = G(r, 6 + qslot[m][q]);
            j.coef[j.nsrc++] = make_double2(z.x, -z.y);
          }
          j.dst = Mser(r, m);
          j.rec = rec;
          j.E = E;
          j.nord = nord;
          j.kmin = 0;
        }
      pm_status e = flush();
      if (e) return e;
    }
    // traces
    TraceArgs ta{};
    for (int r = 0; r < R; ++r)
      for (int m = 0; m < 4; ++m) {
        if (ta.njobs == kMaxTransformJobs) {
          pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_trace(ta, nord, s); }));
          if (e) return e;
          ta.njobs = 0;
        }
        TraceJob& j = ta.jobs[ta.njobs++];
        j.src = Mser(r, m);
        j.out = trc + (static_cast<size_t>(r) * 4 + m) * nord;
        j.n = n;
        j.nord = nord;
      }
    return st(timed(PM_PHASE_OTHER, s, [&] { return launch_trace(ta, nord, s); }));
  }

  // ---- action series S^(k) = 12 N delta_k0 - 2 Re sum_{m<n} z_mn Tr P_mn^(k)
  //      (eq. (1) at beta = 1 expanded in g, the plaquettes
  //      P_mn = U_m U_n U_m^+ U_n^+ = Q_mn * Q_nm^+) into S [R][nord]
  pm_status action(double* S) {
    const int n = l.n, E = l.E, nord = l.nord, L = l.L;
    {
      GemmBatch nn{fin, s, 0};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m)
          for (int q = 0; q < 4; ++q)
            if (m != q) nn.add(Ut(r, m), Ut(r, q), G(r, qslot[m][q]), n, L);
      nn.flush();
      if (nn.status) return PM_ERR_DEVICE;
      RetruncBatch rt{&l, fout, fin, s};
      rt.a.nadd = 0;
      rt.a.idcoef = make_double2(0.0, 0.0);
      for (int r = 0; r < R; ++r)
        for (int slot = 0; slot < 12; ++slot) rt.add(G(r, slot), Xt(r, slot), nullptr, nullptr, 0);
      rt.flush();
      if (rt.status) return rt.status;
      GemmBatch nc{fin, s, 1};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m)
          for (int q = m + 1; q < 4; ++q) nc.add(Xt(r, qslot[m][q]), Xt(r, qslot[q][m]), G(r, pair[m][q]), n, L);
      nc.flush();
      if (nc.status) return PM_ERR_DEVICE;
    }
    // sum_{m<n} z_mn P_mn back to the time domain, one series per replica
    {
      CombineArgs ca{};
      auto flush = [&]() -> pm_status {
        if (ca.njobs == 0) return PM_OK;
        pm_status e = st(timed(PM_PHASE_INVERSE, s, [&] { return launch_inv_combine(ca, L, E, fout, s); }));
        ca.njobs = 0;
        return e;
      };
      for (int r = 0; r < R; ++r) {
        if (ca.njobs == kMaxCombineJobs) { pm_status e = flush(); if (e) return e; }
        CombineJob& j = ca.jobs[ca.njobs++];
        j.nsrc = 0;
        for (int m = 0; m < 4; ++m)
          for (int q = m + 1; q < 4; ++q) {
            j.src[j.nsrc] = G(r, pair[m][q]);
            j.coef[j.nsrc++] = twist(p, m, q);
          }
        j.dst = Mser(r, 0);
        j.rec = rec;
        j.E = E;
        j.nord = nord;
        j.kmin = 0;
      }
      pm_status e = flush();
      if (e) return e;
    }
    return traces_to(S, 12.0 * n, -2.0);
  }

  // ---- a x b Wilson loops W^(k) = 1/(6N) sum_{m<n} Re z_mn^{ab}
  //      Tr (U_m^a U_n^b (U_m^+)^a (U_n^+)^b)^(k) into W [R][nord]; the loop of
  //      plane (m, n) is A * B^+ with A = U_m^a U_n^b and B = U_n^b U_m^a
  pm_status wilson(int wa, int wb, double* W) {
    const int n = l.n, E = l.E, nord = l.nord, L = l.L;
    const int jmax = std::max(wa, wb);
    // powers U^j (j <= 4) in Fourier space: Xt slots 12 + 4 (j - 2) + m
    auto pw = [&](int r, int m, int j) -> const void* { return j == 1 ? Ut(r, m) : Xt(r, 12 + 4 * (j - 2) + m); };
    for (int j = 2; j <= jmax; ++j) {
      GemmBatch g{fin, s, 0};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) g.add(pw(r, m, j - 1), Ut(r, m), G(r, m), n, L);
      g.flush();
      if (g.status) return g.status;
      RetruncBatch rt{&l, fout, fin, s};
      rt.a.nadd = 0;
      rt.a.idcoef = make_double2(0.0, 0.0);
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) rt.add(G(r, m), Xt(r, 12 + 4 * (j - 2) + m), nullptr, nullptr, 0);
      rt.flush();
      if (rt.status) return rt.status;
    }
    // A_mn = U_m^a U_n^b into slot (m, n), B_mn = U_n^b U_m^a into slot (n, m), m < n
    {
      GemmBatch g{fin, s, 0};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m)
          for (int q = m + 1; q < 4; ++q) {
            g.add(pw(r, m, wa), pw(r, q, wb), G(r, qslot[m][q]), n, L);
            g.add(pw(r, q, wb), pw(r, m, wa), G(r, qslot[q][m]), n, L);
          }
      g.flush();
      if (g.status) return g.status;
      RetruncBatch rt{&l, fout, fin, s};
      rt.a.nadd = 0;
      rt.a.idcoef = make_double2(0.0, 0.0);
      for (int r = 0; r < R; ++r)
        for (int slot = 0; slot < 12; ++slot) rt.add(G(r, slot), Xt(r, slot), nullptr, nullptr, 0);
      rt.flush();
      if (rt.status) return rt.status;
      GemmBatch nc{fin, s, 1};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m)
          for (int q = m + 1; q < 4; ++q) nc.add(Xt(r, qslot[m][q]), Xt(r, qslot[q][m]), G(r, pair[m][q]), n, L);
      nc.flush();
      if (nc.status) return PM_ERR_DEVICE;
    }
    {
      CombineArgs ca{};
      auto flush = [&]() -> pm_status {
        if (ca.njobs == 0) return PM_OK;
        pm_status e = st(timed(PM_PHASE_INVERSE, s, [&] { return launch_inv_combine(ca, L, E, fout, s); }));
        ca.njobs = 0;
        return e;
      };
      const double ang = 2.0 * M_PI * p->k * wa * wb / p->L;   // z^{ab} for m < n
      for (int r = 0; r < R; ++r) {
        if (ca.njobs == kMaxCombineJobs) { pm_status e = flush(); if (e) return e; }
        CombineJob& j = ca.jobs[ca.njobs++];
        j.nsrc = 0;
        for (int m = 0; m < 4; ++m)
          for (int q = m + 1; q < 4; ++q) {
            j.src[j.nsrc] = G(r, pair[m][q]);
            j.coef[j.nsrc++] = make_double2(std::cos(ang), std::sin(ang));
          }
        j.dst = Mser(r, 0);
        j.rec = rec;
        j.E = E;
        j.nord = nord;
        j.kmin = 0;
      }
      pm_status e = flush();
      if (e) return e;
    }
    return traces_to(W, 0.0, 1.0 / (6.0 * n));
  }

  // out[r][k] = c0 delta_k0 + c1 Re Tr Mser(r, 0)^(k)
  pm_status traces_to(double* out, double c0, double c1) {
    const int n = l.n, nord = l.nord;
    TraceArgs ta{};
    ActionArgs aa{};
    aa.c0 = c0;
    aa.c1 = c1;
    aa.nord = nord;
    for (int r = 0; r < R; ++r) {
      if (ta.njobs == kMaxTransformJobs) {
        pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_trace(ta, nord, s); }));
        if (e) return e;
        ta.njobs = 0;
      }
      TraceJob& j = ta.jobs[ta.njobs++];
      j.src = Mser(r, 0);
      j.out = trc + static_cast<size_t>(r) * nord;
      j.n = n;
      j.nord = nord;
    }
    pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_trace(ta, nord, s); }));
    if (e) return e;
    aa.tr = trc;
    aa.S = out;
    aa.count = R * nord;
    return st(timed(PM_PHASE_OTHER, s, [&] { return launch_action(aa, s); }));
  }

  // ---- force pass.  Langevin (P == nullptr): Y^1 = i X from the force and
  //      the noise.  MD: P^(k) += kick F^(k) (k >= 1) and, when write_y,
  //      Y^1 = i dt P (unscaled).
  pm_status force(const double2* eta, double2* P, double kick, double dt, bool write_y) {
    const int n = l.n, nord = l.nord;
    ForceArgs fa{};
    fa.md = P ? 1 : 0;
    fa.eps = p->eps;
    fa.noise_amp = std::sqrt(2.0 * p->eps);
    fa.kick = kick;
    fa.dt = dt;
    for (int r = 0; r < R; ++r)
      for (int m = 0; m < 4; ++m) {
        if (fa.njobs == kMaxForceJobs) {
          pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_force(fa, n, nord, s); }));
          if (e) return e;
          fa.njobs = 0;
        }
        ForceJob& j = fa.jobs[fa.njobs++];
        j.M = Mser(r, m);
        j.tr = trc + (static_cast<size_t>(r) * 4 + m) * nord;
        j.eta = eta ? eta + (static_cast<size_t>(r) * 4 + m) * l.E : nullptr;
        j.P = P ? P + (static_cast<size_t>(r) * 4 + m) * series_elems : nullptr;
        j.Y = write_y ? Ypt(r, m, 1) : nullptr;
        j.rec = unit;                  // Y unscaled; rescaled by s' before the exponential
        j.n = n;
        j.nord = nord;
      }
    return st(timed(PM_PHASE_OTHER, s, [&] { return launch_force(fa, n, nord, s); }));
  }

  // ---- gauge-fixing exponent (after links_forward): with V_m = U_m^(0),
  //      G = sum_m (U_m V_m^+ - V_m^+ U_m) and
  //      Y = -(alpha/2) [(G - G^+) - Tr(G - G^+)/N] into Ypt(r, 0, 1), one per replica
  pm_status gauge_exponent(double alpha) {
    const int n = l.n, E = l.E, nord = l.nord, L = l.L;
    // V_m: the order-0 coefficient alone, i.e. the same matrix at every mode
    {
      FwdArgs fw{};
      auto flush = [&]() -> pm_status {
        pm_status e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fw, L, E, fin, s); }));
        fw.njobs = 0;
        return e;
      };
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) {
          if (fw.njobs == kMaxTransformJobs) { pm_status e = flush(); if (e) return e; }
          FwdJob& j = fw.jobs[fw.njobs++];
          j.src = Useries(r, m);
          j.dst = Xt(r, m);
          j.rec = rec;
          j.E = E;
          j.nord = 1;
          j.n = n;
        }
      pm_status e = flush();
      if (e) return e;
    }
    {
      GemmBatch nc{fin, s, 1}, cn{fin, s, 2};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) {
          nc.add(Ut(r, m), Xt(r, m), G(r, m), n, L);        // U_m V_m^+
          cn.add(Xt(r, m), Ut(r, m), G(r, 4 + m), n, L);    // V_m^+ U_m
        }
      nc.flush();
      cn.flush();
      if (nc.status || cn.status) return PM_ERR_DEVICE;
    }
    // G in the (unscaled) time domain
    {
      CombineArgs ca{};
      auto flush = [&]() -> pm_status {
        if (ca.njobs == 0) return PM_OK;
        pm_status e = st(timed(PM_PHASE_INVERSE, s, [&] { return launch_inv_combine(ca, L, E, fout, s); }));
        ca.njobs = 0;
        return e;
      };
      for (int r = 0; r < R; ++r) {
        if (ca.njobs == kMaxCombineJobs) { pm_status e = flush(); if (e) return e; }
        CombineJob& j = ca.jobs[ca.njobs++];
        j.nsrc = 8;
        for (int m = 0; m < 4; ++m) {
          j.src[m] = G(r, m);
          j.coef[m] = make_double2(1.0, 0.0);
          j.src[4 + m] = G(r, 4 + m);
          j.coef[4 + m] = make_double2(-1.0, 0.0);
        }
        j.dst = Mser(r, 0);
        j.rec = rec;
        j.E = E;
        j.nord = nord;
        j.kmin = 0;
      }
      pm_status e = flush();
      if (e) return e;
    }
    TraceArgs ta{};
    for (int r = 0; r < R; ++r) {
      if (ta.njobs == kMaxTransformJobs) {
        pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_trace(ta, nord, s); }));
        if (e) return e;
        ta.njobs = 0;
      }
      TraceJob& j = ta.jobs[ta.njobs++];
      j.src = Mser(r, 0);
      j.out = trc + static_cast<size_t>(r) * 4 * nord;
      j.n = n;
      j.nord = nord;
    }
    pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_trace(ta, nord, s); }));
    if (e) return e;
    // Y = -eps (D - Tr D / N), D = G - G^+, with eps = alpha / 2 and no noise
    ForceArgs fa{};
    fa.md = 0;
    fa.eps = 0.5 * alpha;
    fa.noise_amp = 0.0;
    for (int r = 0; r < R; ++r) {
      if (fa.njobs == kMaxForceJobs) {
        e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_force(fa, n, nord, s); }));
        if (e) return e;
        fa.njobs = 0;
      }
      ForceJob& j = fa.jobs[fa.njobs++];
      j.M = Mser(r, 0);
      j.tr = trc + static_cast<size_t>(r) * 4 * nord;
      j.eta = nullptr;
      j.P = nullptr;
      j.Y = Ypt(r, 0, 1);
      j.rec = unit;
      j.n = n;
      j.nord = nord;
    }
    return st(timed(PM_PHASE_OTHER, s, [&] { return launch_force(fa, n, nord, s); }));
  }

  // ---- exponential of Y (Y^1 in Ypt(.,.,1), scaled) into Zf, then the link
  //      update U_m <- E_m * U_m (orders >= 1); nexp == 1: one exponent per
  //      replica for all m; conj_update: U_m <- E * U_m * E^+
  pm_status exp_and_update() {
    const int n = l.n, E = l.E, nord = l.nord, L = l.L, b = l.b;
    // s' from the norms of Y (all replicas and directions) against those of
    // the links, then Y <- Y(s' g) in place
    {
      NormArgs na{};
      auto flush = [&]() -> pm_status {
        pm_status e = st(timed(PM_PHASE_RESCALE, s, [&] { return launch_norms(na, nord, s); }));
        na.njobs = 0;
        return e;
      };
      for (int r = 0; r < R; ++r)
        for (int mu = 0; mu < nexp; ++mu) {
          if (na.njobs == kMaxTransformJobs) { pm_status e = flush(); if (e) return e; }
          NormJob& j = na.jobs[na.njobs++];
          j.src = Ypt(r, mu, 1);
          j.partial = partY + (static_cast<size_t>(r) * nexp + mu) * nord * kNormChunks;
          j.E = E;
          j.nord = nord;
        }
      pm_status e = flush();
      if (e) return e;
      ScaleArgs sa{};
      sa.njobs = 1;
      sa.jobs[0].partA = partY;
      sa.jobs[0].partB = part;
      sa.jobs[0].rec = rec2;
      sa.jobs[0].nord = nord;
      sa.jobs[0].L = L;
      sa.jobs[0].fixed_s = 0.0;
      sa.jobs[0].nser = nexp * R;
      sa.jobs[0].nser_b = 4 * R;
      e = st(timed(PM_PHASE_RESCALE, s, [&] { return launch_scale(sa, s); }));
      if (e) return e;
      SeriesScaleArgs ss{};
      auto flush2 = [&]() -> pm_status {
        pm_status e2 = st(timed(PM_PHASE_OTHER, s, [&] { return launch_series_scale(ss, nord, s); }));
        ss.njobs = 0;
        return e2;
      };
      for (int r = 0; r < R; ++r)
        for (int mu = 0; mu < nexp; ++mu) {
          if (ss.njobs == kMaxSeriesScaleJobs) { e = flush2(); if (e) return e; }
          SeriesScaleJob& j = ss.jobs[ss.njobs++];
          j.x = Ypt(r, mu, 1);
          j.rec = rec2;
          j.E = E;
          j.nord = nord;
        }
      e = flush2();
      if (e) return e;
    }
    // Fourier coefficients of Y (already scaled: unit record)
    {
      FwdArgs fw{};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < nexp; ++m) {
          if (fw.njobs == kMaxTransformJobs) {
            pm_status e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fw, L, E, fin, s); }));
            if (e) return e;
            fw.njobs = 0;
          }
          FwdJob& j = fw.jobs[fw.njobs++];
          j.src = Ypt(r, m, 1);
          j.dst = Ypf(r, m, 1);
          j.rec = unit;
          j.E = E;
          j.nord = nord;
          j.n = n;
        }
      pm_status e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fw, L, E, fin, s); }));
      if (e) return e;
    }
    // powers Y^2 .. Y^b
    for (int j = 2; j <= b; ++j) {
      GemmBatch g{fin, s, 0};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < nexp; ++m) g.add(Ypf(r, m, j - 1), Ypf(r, m, 1), G(r, m), n, L);
      g.flush();
      if (g.status) return g.status;
      RetruncBatch rt{&l, fout, fin, s};
      rt.a.nadd = 0;
      rt.a.idcoef = make_double2(0.0, 0.0);
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < nexp; ++m) rt.add(G(r, m), Ypf(r, m, j), Ypt(r, m, j), nullptr, 0);
      rt.flush();
      if (rt.status) return rt.status;
    }
    // E = sum_q (Y^b)^q B_q(Y) by Horner in Y^b, each step at the length
    // of the orders it still needs (ExpPlan)
    {
      const int nt = nord - 1;
      const ExpPlan pl = exp_plan(nt);
      const int Q = pl.Q;
      auto cfac = [&](int jj) {
        if (jj > nt) return 0.0;
        double f = 1.0;
        for (int t = 2; t <= jj; ++t) f *= t;
        return 1.0 / f;
      };
      const size_t ystride = l.tser / sizeof(double2);   // elements between Y^i and Y^(i+1)
      // Y^b at every shorter length in use (G slots 4.. are free after the
      // staples): truncated at L'/2 - 1 orders, so no product wraps around
      int nshort = 0, shortlen[8];
      for (int q = 0; q < Q; ++q) {
        const int lq = pl.len[q];
        bool seen = lq == L;
        for (int i = 0; i < nshort; ++i) seen = seen || shortlen[i] == lq;
        if (!seen) shortlen[nshort++] = lq;
      }
      auto ybf = [&](int r, int m, int lq) -> const void* {
        if (lq == L) return Ypf(r, m, b);
        for (int i = 0; i < nshort; ++i)
          if (shortlen[i] == lq) return G(r, 4 + 4 * i + m);
        return nullptr;
      };
      for (int i = 0; i < nshort; ++i) {
        FwdArgs fw{};
        auto flush = [&]() -> pm_status {
          pm_status e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fw, shortlen[i], E, fin, s); }));
          fw.njobs = 0;
          return e;
        };
        for (int r = 0; r < R; ++r)
          for (int m = 0; m < nexp; ++m) {
            if (fw.njobs == kMaxTransformJobs) { pm_status e = flush(); if (e) return e; }
            FwdJob& j = fw.jobs[fw.njobs++];
            j.src = Ypt(r, m, b);
            j.dst = G(r, 4 + 4 * i + m);
            j.rec = unit;
            j.E = E;
            j.nord = std::min(nord, shortlen[i] / 2);
            j.n = n;
          }
        pm_status e = flush();
        if (e) return e;
      }
      for (int q = Q; q >= 0; --q) {
        const int lprod = q < Q ? pl.len[q] : 0;             // length of this step's product
        const int lnext = q > 0 ? pl.len[q - 1] : L;          // length the result is transformed at
        if (q < Q) {
          GemmBatch g{fin, s, 0};
          for (int r = 0; r < R; ++r)
            for (int m = 0; m < nexp; ++m) g.add(ybf(r, m, lprod), Zf(r, m), G(r, m), n, lprod);
          g.flush();
          if (g.status) return g.status;
        }
        RetruncBatch rt{&l, fout, fin, s};
        rt.lin = q < Q ? lprod : lnext;
        rt.lout = lnext;
        rt.nord = std::min(nord, nt - q * b + 1);
        rt.a.nadd = b - 1;
        for (int i = 1; i < b; ++i) rt.a.coef[i - 1] = make_double2(cfac(q * b + i), 0.0);
        rt.a.idcoef = make_double2(cfac(q * b), 0.0);
        for (int r = 0; r < R; ++r)
          for (int m = 0; m < nexp; ++m)
            rt.add(q < Q ? static_cast<const void*>(G(r, m)) : nullptr, Zf(r, m), nullptr,
                   b > 1 ? Ypt(r, m, 1) : nullptr, ystride);
        rt.flush();
        if (rt.status) return rt.status;
      }
    }
    // link update U_m <- E_m * U_m (orders >= 1), with U transformed again
    // in the variable s'
    {
      FwdArgs fa{};
      for (int r = 0; r < R; ++r)
        for (int mu = 0; mu < 4; ++mu) {
          if (fa.njobs == kMaxTransformJobs) {
            pm_status e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fa, L, E, fin, s); }));
            if (e) return e;
            fa.njobs = 0;
          }
          FwdJob& j = fa.jobs[fa.njobs++];
          j.src = Useries(r, mu);
          j.dst = Ut(r, mu);
          j.rec = rec2;
          j.E = E;
          j.nord = nord;
          j.n = n;
        }
      pm_status e = st(timed(PM_PHASE_FORWARD, s, [&] { return launch_forward(fa, L, E, fin, s); }));
      if (e) return e;
      auto ez = [&](int r, int m) { return Zf(r, nexp == 1 ? 0 : m); };
      GemmBatch g{fin, s, 0};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) g.add(ez(r, m), Ut(r, m), G(r, m), n, L);
      g.flush();
      if (g.status) return g.status;
      if (conj_update) {
        // (E U_m) re-truncated in Fourier space, then times E^+ (the
        // conjugated operand: mode (L - p) mod L, conjugate-transposed)
        RetruncBatch rt{&l, fout, fin, s};
        rt.a.nadd = 0;
        rt.a.idcoef = make_double2(0.0, 0.0);
        for (int r = 0; r < R; ++r)
          for (int m = 0; m < 4; ++m) rt.add(G(r, m), Xt(r, 4 + m), nullptr, nullptr, 0);
        rt.flush();
        if (rt.status) return rt.status;
        GemmBatch gc{fin, s, 1};
        for (int r = 0; r < R; ++r)
          for (int m = 0; m < 4; ++m) gc.add(Xt(r, 4 + m), ez(r, m), G(r, m), n, L);
        gc.flush();
        if (gc.status) return gc.status;
      }
      CombineArgs ca{};
      for (int r = 0; r < R; ++r)
        for (int m = 0; m < 4; ++m) {
          if (ca.njobs == kMaxCombineJobs) {
            pm_status e = st(timed(PM_PHASE_INVERSE, s, [&] { return launch_inv_combine(ca, L, E, fout, s); }));
            if (e) return e;
            ca.njobs = 0;
          }
          CombineJob& j = ca.jobs[ca.njobs++];
          j.nsrc = 1;
          j.src[0] = G(r, m);
          j.coef[0] = make_double2(1.0, 0.0);
          j.dst = Useries(r, m);
          j.rec = rec2;
          j.E = E;
          j.nord = nord;
          j.kmin = 1;
        }
      return st(timed(PM_PHASE_INVERSE, s, [&] { return launch_inv_combine(ca, L, E, fout, s); }));
    }
  }
};

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t ab = reinterpret_cast<uintptr_t>(a), bb = reinterpret_cast<uintptr_t>(b);
  return ab < bb + nb && bb < ab + na;
}

}  // namespace

size_t nspt_workspace_bytes(int replicas, const nspt_params* p, int prec) {
  if (!valid_params(replicas, p, prec)) return 0;
  return layout(replicas, p, prec).total;
}

pm_status nspt_step(void* U, const void* eta, int R, const nspt_params* p, int prec, void* workspace,
                    size_t workspace_bytes, hipStream_t s) {
  if (!valid_params(R, p, prec)) return PM_ERR_INVALID;
  if (!U || !eta || !workspace) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(U) % 16 || reinterpret_cast<uintptr_t>(eta) % 16 ||
      reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return PM_ERR_INVALID;
  const Layout l = layout(R, p, prec);
  if (workspace_bytes < l.total) return PM_ERR_WORKSPACE;
  const size_t ub = static_cast<size_t>(R) * 4 * l.nord * l.E * 16, nb = static_cast<size_t>(R) * 4 * l.E * 16;
  if (overlaps(workspace, l.total, U, ub) || overlaps(workspace, l.total, eta, nb) || overlaps(U, ub, eta, nb))
    return PM_ERR_INVALID;

  Run run(U, R, p, prec, workspace, s);
  pm_status e = run.links_forward();
  if (!e) e = run.staples();
  if (!e) e = run.force(static_cast<const double2*>(eta), nullptr, 0.0, 0.0, true);
  if (!e) e = run.exp_and_update();
  return e;
}

pm_status nspt_noise(void* eta, int R, int n, unsigned long long seed, unsigned long long step, hipStream_t s) {
  if (!eta || R < 1 || R > 1024 || n < 1 || n > PM_MAX_N) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(eta) % 16) return PM_ERR_INVALID;
  NoiseArgs na{};
  na.eta = static_cast<double2*>(eta);
  na.seed = seed;
  na.step = step;
  na.n = n;
  na.count = 4 * R;
  return st(timed(PM_PHASE_OTHER, s, [&] { return launch_noise(na, s); }));
}

pm_status nspt_steps(void* U, int R, const nspt_params* p, unsigned long long seed, unsigned long long step0,
                     int nsteps, int prec, void* workspace, size_t workspace_bytes, hipStream_t s) {
  if (!valid_params(R, p, prec)) return PM_ERR_INVALID;
  if (!U || !workspace || nsteps < 1 || nsteps > kMaxMdSteps) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(U) % 16 || reinterpret_cast<uintptr_t>(workspace) % kAlign) return PM_ERR_INVALID;
  const Layout l = layout(R, p, prec);
  if (workspace_bytes < l.total) return PM_ERR_WORKSPACE;
  const size_t ub = static_cast<size_t>(R) * 4 * l.nord * l.E * 16;
  if (overlaps(workspace, l.total, U, ub)) return PM_ERR_INVALID;
  double2* eta = reinterpret_cast<double2*>(static_cast<char*>(workspace) + l.eta);
  Run run(U, R, p, prec, workspace, s);
  pm_status e = PM_OK;
  for (int t = 0; t < nsteps && !e; ++t) {
    e = nspt_noise(eta, R, p->n, seed, step0 + static_cast<unsigned long long>(t), s);
    if (!e) e = run.links_forward();
    if (!e) e = run.staples();
    if (!e) e = run.force(eta, nullptr, 0.0, 0.0, true);
    if (!e) e = run.exp_and_update();
  }
  return e;
}

pm_status nspt_gauge(void* U, int R, const nspt_params* p, double alpha, int prec, void* workspace,
                     size_t workspace_bytes, hipStream_t s) {
  if (!valid_params(R, p, prec)) return PM_ERR_INVALID;
  if (!U || !workspace || !std::isfinite(alpha) || alpha < 0.0) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(U) % 16 || reinterpret_cast<uintptr_t>(workspace) % kAlign) return PM_ERR_INVALID;
  const Layout l = layout(R, p, prec);
  if (workspace_bytes < l.total) return PM_ERR_WORKSPACE;
  const size_t ub = static_cast<size_t>(R) * 4 * l.nord * l.E * 16;
  if (overlaps(workspace, l.total, U, ub)) return PM_ERR_INVALID;
  if (alpha == 0.0) return PM_OK;   // Omega = 1
  Run run(U, R, p, prec, workspace, s);
  run.nexp = 1;
  run.conj_update = true;
  pm_status e = run.links_forward();
  if (!e) e = run.gauge_exponent(alpha);
  if (!e) e = run.exp_and_update();
  return e;
}

pm_status nspt_series_action(const void* U, int R, const nspt_params* p, int prec, double* S, void* workspace,
                             size_t workspace_bytes, hipStream_t s) {
  if (!valid_params(R, p, prec)) return PM_ERR_INVALID;
  if (!U || !S || !workspace) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(U) % 16 || reinterpret_cast<uintptr_t>(S) % 8 ||
      reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return PM_ERR_INVALID;
  const Layout l = layout(R, p, prec);
  if (workspace_bytes < l.total) return PM_ERR_WORKSPACE;
  const size_t ub = static_cast<size_t>(R) * 4 * l.nord * l.E * 16, sb = static_cast<size_t>(R) * l.nord * 8;
  if (overlaps(workspace, l.total, U, ub) || overlaps(workspace, l.total, S, sb) || overlaps(U, ub, S, sb))
    return PM_ERR_INVALID;
  Run run(const_cast<void*>(U), R, p, prec, workspace, s);   // U is only read
  pm_status e = run.links_forward();
  if (!e) e = run.action(S);
  return e;
}

pm_status nspt_wilson(const void* U, int R, const nspt_params* p, int wa, int wb, int prec, double* W,
                      void* workspace, size_t workspace_bytes, hipStream_t s) {
  if (!valid_params(R, p, prec)) return PM_ERR_INVALID;
  if (wa < 1 || wa > 4 || wb < 1 || wb > 4) return PM_ERR_INVALID;
  if (!U || !W || !workspace) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(U) % 16 || reinterpret_cast<uintptr_t>(W) % 8 ||
      reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return PM_ERR_INVALID;
  const Layout l = layout(R, p, prec);
  if (workspace_bytes < l.total) return PM_ERR_WORKSPACE;
  const size_t ub = static_cast<size_t>(R) * 4 * l.nord * l.E * 16, wbytes = static_cast<size_t>(R) * l.nord * 8;
  if (overlaps(workspace, l.total, U, ub) || overlaps(workspace, l.total, W, wbytes) || overlaps(U, ub, W, wbytes))
    return PM_ERR_INVALID;
  Run run(const_cast<void*>(U), R, p, prec, workspace, s);   // U is only read
  pm_status e = run.links_forward();
  if (!e) e = run.wilson(wa, wb, W);
  return e;
}

pm_status nspt_md(void* U, void* P, const void* eta, int R, const nspt_params* p, int nsteps, int prec,
                  void* workspace, size_t workspace_bytes, hipStream_t s) {
  if (!valid_params(R, p, prec)) return PM_ERR_INVALID;
  if (!U || !P || !workspace || nsteps < 1 || nsteps > kMaxMdSteps) return PM_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(U) % 16 || reinterpret_cast<uintptr_t>(P) % 16 ||
      reinterpret_cast<uintptr_t>(eta) % 16 || reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return PM_ERR_INVALID;
  const Layout l = layout(R, p, prec);
  if (workspace_bytes < l.total) return PM_ERR_WORKSPACE;
  const size_t ub = static_cast<size_t>(R) * 4 * l.nord * l.E * 16, nb = static_cast<size_t>(R) * 4 * l.E * 16;
  if (overlaps(workspace, l.total, U, ub) || overlaps(workspace, l.total, P, ub) || overlaps(U, ub, P, ub))
    return PM_ERR_INVALID;
  if (eta && (overlaps(workspace, l.total, eta, nb) || overlaps(U, ub, eta, nb) || overlaps(P, ub, eta, nb)))
    return PM_ERR_INVALID;

  double2* Pg = static_cast<double2*>(P);
  if (eta) {
    RefreshArgs ra{};
    for (int r = 0; r < R; ++r)
      for (int m = 0; m < 4; ++m) {
        if (ra.njobs == kMaxRefreshJobs) {
          pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_refresh(ra, s); }));
          if (e) return e;
          ra.njobs = 0;
        }
        RefreshJob& j = ra.jobs[ra.njobs++];
        j.P = Pg + (static_cast<size_t>(r) * 4 + m) * l.nord * l.E;
        j.eta = static_cast<const double2*>(eta) + (static_cast<size_t>(r) * 4 + m) * l.E;
        j.E = l.E;
        j.nord = l.nord;
      }
    pm_status e = st(timed(PM_PHASE_OTHER, s, [&] { return launch_refresh(ra, s); }));
    if (e) return e;
  }
  const double dt = p->eps;
  Run run(U, R, p, prec, workspace, s);
  // leapfrog: half kick, (drift, kick) x (nsteps - 1), drift, half kick;
  // every kick but the last also forms the exponent of the next drift
  pm_status e = run.links_forward();
  if (!e) e = run.staples();
  if (!e) e = run.force(nullptr, Pg, 0.5 * dt, dt, true);
  for (int i = 0; i < nsteps && !e; ++i) {
    const bool last = i == nsteps - 1;
    e = run.exp_and_update();
    if (!e) e = run.links_forward();
    if (!e) e = run.staples();
    if (!e) e = run.force(nullptr, Pg, last ? 0.5 * dt : dt, dt, !last);
  }
  return e;
}

}  // namespace pm
