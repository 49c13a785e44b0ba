// Host runtime of the polymat library: argument validation, workspace
// planning and the launch sequence of each C-ABI entry point.
//
// Nothing here allocates device memory or synchronises: every call checks its
// arguments, carves the caller's workspace into per-product regions and
// enqueues kernels on the caller's stream.
#include "polymat.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "pm_common.h"
#include "pm_kernels.h"
#include "pm_nspt.h"
#include "pm_pipeline.h"

namespace {

using namespace pm;

constexpr size_t kAlign = 256;
// polymat_mul takes the direct form up to this order (FP64).  Measured at
// N = 225: ntrunc = 0 direct 0.033 ms vs transform path 0.047 ms; ntrunc = 1
// 0.063 vs 0.051 ms (one product alone fills few work-groups in the direct form).
constexpr int kNaiveMaxNtrunc = 0;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int transform_length(int ntrunc) {
  if (ntrunc < 0 || ntrunc > PM_MAX_NTRUNC) return 0;
  const int need = 2 * (ntrunc + 1);
  int L = 4;
  while (L < need) L *= 2;
  return L;
}

FourierType fourier_type(int prec) {
  return prec == PM_PREC_FP64 ? kF64 : (prec == PM_PREC_FP32 ? kF32 : kBF16Split);
}

// Bytes of the Fourier coefficients of one operand over L modes.
size_t operand_bytes(int n, int L, int prec) {
  const size_t E = static_cast<size_t>(n) * n;
  switch (prec) {
    case PM_PREC_FP64: return E * L * 16;
    case PM_PREC_FP32: return E * L * 8;
    default: return static_cast<size_t>(bf16_ld(n)) * n * 8 * L;   // 8-byte split entries, rows padded to ld
  }
}
// Bytes of the product coefficients over L modes (FP64 or FP32 complex).
size_t result_bytes(int n, int L, int prec) {
  const size_t E = static_cast<size_t>(n) * n;
  return E * L * (prec == PM_PREC_FP64 ? 16 : 8);
}

struct ProductLayout {
  size_t rec, pipe, partA, partB, At, Bt, Ct, total;
};

ProductLayout product_layout(int n, int ntrunc, int prec) {
  ProductLayout l{};
  const int L = transform_length(ntrunc);
  const size_t part = static_cast<size_t>(ntrunc + 1) * kNormChunks * sizeof(double);
  size_t off = 0;
  l.rec = off;   off += align_up(sizeof(ScaleRec));
  l.pipe = off;  off += align_up(sizeof(PipeSlot));
  l.partA = off; off += align_up(part);
  l.partB = off; off += align_up(part);
  l.At = off;    off += align_up(operand_bytes(n, L, prec));
  l.Bt = off;    off += align_up(operand_bytes(n, L, prec));
  l.Ct = off;    off += align_up(result_bytes(n, L, prec));
  l.total = off;
  return l;
}

bool valid_prec(int p) { return p == PM_PREC_FP64 || p == PM_PREC_FP32 || p == PM_PREC_BF16X3; }
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

struct Range { uintptr_t b, e; };
bool overlaps(Range x, Range y) { return x.b < y.e && y.b < x.e; }
Range range_of(const void* p, size_t bytes) {
  uintptr_t b = reinterpret_cast<uintptr_t>(p);
  return Range{b, b + bytes};
}
size_t series_bytes(int n, int ntrunc) { return static_cast<size_t>(n) * n * (ntrunc + 1) * 16; }

pm_status check_problem_shape(const void* A, const void* B, const void* C, int n, int ntrunc,
                              double scale) {
  if (!A || !B || !C) return PM_ERR_INVALID;
  if (!aligned(A, 16) || !aligned(B, 16) || !aligned(C, 16)) return PM_ERR_INVALID;
  if (n < 1 || n > PM_MAX_N) return PM_ERR_INVALID;
  if (ntrunc < 0) return PM_ERR_INVALID;
  if (ntrunc > PM_MAX_NTRUNC) return PM_ERR_UNSUPPORTED;
  if (!std::isfinite(scale) || scale < 0.0) return PM_ERR_INVALID;
  return PM_OK;
}

pm_status from_hip(hipError_t e) { return e == hipSuccess ? PM_OK : PM_ERR_DEVICE; }

// Finiteness check of the product entry points (polymat_check_enable).
std::atomic<bool> g_check{false};

int env_int(const char* name, int dflt) {
  const char* e = getenv(name);
  if (!e || !*e) return dflt;
  return atoi(e);
}

// POLYMAT_PIPELINE=1 routes FP64 batches through the persistent one-launch
// pipeline (pm_pipeline.hip) instead of the staged launches; it is off by
// default because on MI355X it is slower (the fused kernel's 128-register
// budget and its per-ticket release fences cost more than the overlap of
// transforms and products gains).  POLYMAT_PIPE_SPIN_LIMIT bounds each of its
// waits (polls before the launch gives up and sets its abort flag).  Both are
// read at every call.
bool pipeline_enabled() { return env_int("POLYMAT_PIPELINE", 0) == 1; }
unsigned int pipeline_spin_limit() {
  const int v = env_int("POLYMAT_PIPE_SPIN_LIMIT", 1 << 20);
  return v < 0 ? 0u : static_cast<unsigned int>(v);
}

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// ------------------------------------------------------------ phase timing

struct TimingRec { int phase; hipEvent_t a, b; };
std::atomic<bool> g_timing{false};
std::mutex g_tmu;
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t pooled_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Enqueue the whole FFT-CONV pipeline for a list of validated problems whose
// workspace regions are given.
struct Planned {
  pm_problem pr;
  int L;
  char* ws;        // base of this product's region
  ProductLayout lay;
};

pm_status enqueue_products(const std::vector<Planned>& items, int prec, hipStream_t st) {
  const FourierType ft = fourier_type(prec);

  // 1. per-order norms of the operands whose s is chosen on the device
  {
    NormArgs na{};
    int max_nord = 0;
    auto flush = [&]() -> pm_status {
      if (na.njobs == 0) return PM_OK;
      pm_status s = from_hip(timed(PM_PHASE_RESCALE, st, [&] { return launch_norms(na, max_nord, st); }));
      na.njobs = 0;
      max_nord = 0;
      return s;
    };
    for (const Planned& it : items) {
      if (it.pr.scale > 0.0) continue;
      const int nord = it.pr.ntrunc + 1;
      const int E = it.pr.n * it.pr.n;
      for (int side = 0; side < 2; ++side) {
        if (na.njobs == kMaxTransformJobs) { pm_status s = flush(); if (s) return s; }
        NormJob& j = na.jobs[na.njobs++];
        j.src = static_cast<const double2*>(side == 0 ? it.pr.A : it.pr.B);
        j.partial = reinterpret_cast<double*>(it.ws + (side == 0 ? it.lay.partA : it.lay.partB));
        j.E = E;
        j.nord = nord;
        max_nord = std::max(max_nord, nord);
      }
    }
    pm_status s = flush();
    if (s) return s;
  }
  // 2. the scale record (s^k and s^-k / L tables) of every product
  {
    ScaleArgs sa{};
    for (const Planned& it : items) {
      if (sa.njobs == kMaxTransformJobs) {
        pm_status s = from_hip(timed(PM_PHASE_RESCALE, st, [&] { return launch_scale(sa, st); }));
        if (s) return s;
        sa.njobs = 0;
      }
      ScaleJob& j = sa.jobs[sa.njobs++];
      j.partA = reinterpret_cast<const double*>(it.ws + it.lay.partA);
      j.partB = reinterpret_cast<const double*>(it.ws + it.lay.partB);
      j.rec = reinterpret_cast<ScaleRec*>(it.ws + it.lay.rec);
      j.nord = it.pr.ntrunc + 1;
      j.L = it.L;
      j.fixed_s = it.pr.scale;
      j.nser = 1;
    }
    pm_status s = from_hip(timed(PM_PHASE_RESCALE, st, [&] { return launch_scale(sa, st); }));
    if (s) return s;
  }
  // 3. forward transforms, one launch per transform length (and per 64 jobs)
  std::map<int, std::vector<const Planned*>> byL;
  for (const Planned& it : items) byL[it.L].push_back(&it);
  for (auto& kv : byL) {
    FwdArgs fa{};
    int maxE = 0;
    auto flush = [&]() -> pm_status {
      if (fa.njobs == 0) return PM_OK;
      pm_status s = from_hip(timed(PM_PHASE_FORWARD, st, [&] { return launch_forward(fa, kv.first, maxE, ft, st); }));
      fa.njobs = 0;
      maxE = 0;
      return s;
    };
    for (const Planned* it : kv.second) {
      for (int side = 0; side < 2; ++side) {
        if (fa.njobs == kMaxTransformJobs) { pm_status s = flush(); if (s) return s; }
        FwdJob& j = fa.jobs[fa.njobs++];
        j.src = static_cast<const double2*>(side == 0 ? it->pr.A : it->pr.B);
        j.dst = it->ws + (side == 0 ? it->lay.At : it->lay.Bt);
        j.rec = reinterpret_cast<const ScaleRec*>(it->ws + it->lay.rec);
        j.E = it->pr.n * it->pr.n;
        j.nord = it->pr.ntrunc + 1;
        j.n = it->pr.n;
        maxE = std::max(maxE, j.E);
      }
    }
    pm_status s = flush();
    if (s) return s;
  }
  // 4. mode-wise products, one launch per (operand form, tile configuration,
  // matrix size): the tiles of one launch then cost the same, so the equal
  // shares of tiles that the XCD-contiguous tile order gives the eight XCDs
  // are equal shares of work (a launch mixing sizes leaves the XCDs that hold
  // the large problems' tiles running after the others)
  {
    std::vector<int> sizes;
    for (const Planned& it : items) sizes.push_back(it.pr.n);
    std::sort(sizes.begin(), sizes.end(), std::greater<int>());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    const int ncfg = gemm_num_configs(ft);
    for (int nsz : sizes) {
    for (int form = 0; form < 4; ++form) {
      for (int cfg = 0; cfg < ncfg; ++cfg) {
        GemmArgs ga{};
        const GemmShape sh = gemm_shape(ft, cfg);
        auto flush = [&]() -> pm_status {
          if (ga.njobs == 0) return PM_OK;
          pm_status s = from_hip(timed(PM_PHASE_PRODUCT, st, [&] { return launch_gemm(ga, ft, cfg, st); }));
          ga.njobs = 0;
          ga.total_tiles = 0;
          return s;
        };
        for (const Planned& it : items) {
          if (it.pr.n != nsz || it.pr.op_a * 2 + it.pr.op_b != form || gemm_config(ft, it.pr.n, it.L) != cfg) continue;
          if (ga.njobs == kMaxGemmJobs) { pm_status s = flush(); if (s) return s; }
          GemmJob& j = ga.jobs[ga.njobs++];
          j.A = it.ws + it.lay.At;
          j.B = it.ws + it.lay.Bt;
          j.C = it.ws + it.lay.Ct;
          j.n = it.pr.n;
          j.L = it.L;
          j.opA = it.pr.op_a;
          j.opB = it.pr.op_b;
          j.tiles_m = (it.pr.n + sh.bm - 1) / sh.bm;
          j.tiles_n = (it.pr.n + sh.bn - 1) / sh.bn;
          j.tile_begin = ga.total_tiles;
          ga.total_tiles += j.tiles_m * j.tiles_n * it.L;
        }
        pm_status s = flush();
        if (s) return s;
      }
    }
    }
  }
  // 5. inverse transforms, truncation and unscaling into C
  for (auto& kv : byL) {
    InvArgs ia{};
    int maxE = 0;
    auto flush = [&]() -> pm_status {
      if (ia.njobs == 0) return PM_OK;
      pm_status s = from_hip(timed(PM_PHASE_INVERSE, st, [&] { return launch_inverse(ia, kv.first, maxE, ft, st); }));
      ia.njobs = 0;
      maxE = 0;
      return s;
    };
    for (const Planned* it : kv.second) {
      if (ia.njobs == kMaxTransformJobs) { pm_status s = flush(); if (s) return s; }
      InvJob& j = ia.jobs[ia.njobs++];
      j.src = it->ws + it->lay.Ct;
      j.dst = static_cast<double2*>(it->pr.C);
      j.rec = reinterpret_cast<ScaleRec*>(it->ws + it->lay.rec);
      j.E = it->pr.n * it->pr.n;
      j.nord = it->pr.ntrunc + 1;
      maxE = std::max(maxE, j.E);
    }
    pm_status s = flush();
    if (s) return s;
  }
  return PM_OK;
}

// Compute units of the device that runs `st` (cached per device).
int device_cus(hipStream_t st) {
  static std::mutex mu;
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (st != nullptr && hipStreamGetDevice(st, &dev) != hipSuccess) return 0;
  if (dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lk(mu);
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 0;
    cus[dev] = v;
  }
  return cus[dev];
}

// True when no problem's C overlaps an operand of another problem: the
// pipeline writes the first results while later problems are still being
// read, so cross-problem aliasing keeps the batch on the staged launches.
bool pipeline_alias_free(const std::vector<Planned>& items) {
  if (items.size() > 256) return false;
  for (size_t i = 0; i < items.size(); ++i) {
    const Range c = range_of(items[i].pr.C, series_bytes(items[i].pr.n, items[i].pr.ntrunc));
    for (size_t j = 0; j < items.size(); ++j) {
      if (i == j) continue;
      const size_t sb = series_bytes(items[j].pr.n, items[j].pr.ntrunc);
      if (overlaps(c, range_of(items[j].pr.A, sb)) || overlaps(c, range_of(items[j].pr.B, sb))) return false;
    }
  }
  return true;
}

// The whole FFT-CONV of a batch of FP64 products in one persistent launch per
// kMaxPipeProblems problems (plus one small set-up launch per
// kPipeInitChunk problems that writes the problem descriptors and clears the
// counters).  The control block of each launch is returned in ctl (for the
// status read-back of the finiteness check).
pm_status enqueue_pipeline(const std::vector<Planned>& items, hipStream_t st, std::vector<const PipeSlot*>* ctl) {
  const int cus = device_cus(st);
  if (cus <= 0) return PM_ERR_DEVICE;
  for (size_t c0 = 0; c0 < items.size(); c0 += kMaxPipeProblems) {
    const int cn = static_cast<int>(std::min(items.size() - c0, static_cast<size_t>(kMaxPipeProblems)));
    // largest product work first
    std::vector<int> order(cn);
    for (int k = 0; k < cn; ++k) order[k] = k;
    auto work = [&](int k) {
      const Planned& it = items[c0 + k];
      return static_cast<double>(it.L) * it.pr.n * it.pr.n * it.pr.n;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    PipeArgs pa{};
    std::vector<PipeProblem> probs(cn);
    for (int k = 0; k < cn; ++k) {
      const Planned& it = items[c0 + order[k]];
      PipeProblem& p = probs[k];
      p.A = (const PM_GLOBAL double2*)(it.pr.A);
      p.B = (const PM_GLOBAL double2*)(it.pr.B);
      p.C = (PM_GLOBAL double2*)(it.pr.C);
      p.At = (PM_GLOBAL double2*)(it.ws + it.lay.At);
      p.Bt = (PM_GLOBAL double2*)(it.ws + it.lay.Bt);
      p.Ct = (PM_GLOBAL double2*)(it.ws + it.lay.Ct);
      p.partA = (PM_GLOBAL double*)(it.ws + it.lay.partA);
      p.partB = (PM_GLOBAL double*)(it.ws + it.lay.partB);
      p.rec = (PM_GLOBAL ScaleRec*)(it.ws + it.lay.rec);
      p.scale = it.pr.scale;
      p.n = it.pr.n;
      p.nord = it.pr.ntrunc + 1;
      p.ops = it.pr.op_a | (it.pr.op_b << 1);
      pa.slot[k] = reinterpret_cast<PipeSlot*>(it.ws + it.lay.pipe);
    }
    for (int i0 = 0; i0 < cn; i0 += kPipeInitChunk) {
      PipeInitArgs ia{};
      ia.count = std::min(kPipeInitChunk, cn - i0);
      for (int j = 0; j < ia.count; ++j) {
        ia.probs[j] = probs[i0 + j];
        ia.slot[j] = pa.slot[i0 + j];
      }
      ia.ctl = pa.slot[0];
      ia.reset_ctl = i0 == 0;
      pm_status s = from_hip(timed(PM_PHASE_PIPELINE, st, [&] { return launch_pipeline_init(ia, st); }));
      if (s) return s;
    }
    // ticket order: iteration i holds SCALE(i-1), NORM(i), FWD(i-2), GEMM(i-3), INV(i-5)
    unsigned int t = 0;
    int ns = 0;
    auto add = [&](int stage, int k) {
      if (k < 0 || k >= cn) return;
      const unsigned int c = pipe_count(probs[k], stage);
      if (c == 0) return;
      pa.segs[ns].start = t;
      pa.segs[ns].stage = static_cast<unsigned short>(stage);
      pa.segs[ns].prob = static_cast<unsigned short>(k);
      ++ns;
      t += c;
    };
    for (int i = 0; i < cn + 5; ++i) {
      add(kStScale, i - 1);
      add(kStNorm, i);
      add(kStFwd, i - 2);
      add(kStGemm, i - 3);
      add(kStInv, i - 5);
    }
    pa.nseg = ns;
    pa.total = t;
    pa.spin_limit = pipeline_spin_limit();
    pm_status s = from_hip(timed(PM_PHASE_PIPELINE, st, [&] { return launch_pipeline(pa, 2 * cus, st); }));
    if (s) return s;
    if (ctl) ctl->push_back(pa.slot[0]);
  }
  return PM_OK;
}

pm_status plan_batch(const pm_problem* problems, int count, int prec, char* ws, size_t ws_bytes,
                     std::vector<Planned>& out, size_t* need_out) {
  if (!problems || count < 1 || count > PM_MAX_BATCH || !valid_prec(prec)) return PM_ERR_INVALID;
  size_t off = 0;
  out.clear();
  out.reserve(count);
  for (int i = 0; i < count; ++i) {
    const pm_problem& p = problems[i];
    pm_status s = check_problem_shape(p.A, p.B, p.C, p.n, p.ntrunc, p.scale);
    if (s) return s;
    if ((p.op_a != PM_OP_N && p.op_a != PM_OP_C) || (p.op_b != PM_OP_N && p.op_b != PM_OP_C))
      return PM_ERR_INVALID;
    Planned it;
    it.pr = p;
    it.L = transform_length(p.ntrunc);
    it.lay = product_layout(p.n, p.ntrunc, prec);
    it.ws = ws ? ws + off : nullptr;
    off += it.lay.total;
    out.push_back(it);
  }
  if (need_out) *need_out = off;
  if (!ws) return PM_OK;
  if (!aligned(ws, kAlign)) return PM_ERR_INVALID;
  if (ws_bytes < off) return PM_ERR_WORKSPACE;
  const Range wr = range_of(ws, off);
  for (const Planned& it : out) {
    const size_t sb = series_bytes(it.pr.n, it.pr.ntrunc);
    if (overlaps(wr, range_of(it.pr.A, sb)) || overlaps(wr, range_of(it.pr.B, sb)) ||
        overlaps(wr, range_of(it.pr.C, sb)))
      return PM_ERR_INVALID;
  }
  return PM_OK;
}

// ------------------------------------------- allocation-free single product
//
// polymat_mul_noalloc carves its workspace out of this file-scope device
// array instead of a caller's buffer.  Each GPU the library runs on holds
// its own copy (allocated with the code object, kept until the process
// ends); host code never uses the array's name as an address: the device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = static_cast<size_t>(PM_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device of `st` (looked up once per device).
pm_status scratch_address(hipStream_t st, void** out) {
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return PM_ERR_DEVICE;
  dev = cur;
  if (st != nullptr && hipStreamGetDevice(st, &dev) != hipSuccess) return PM_ERR_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return PM_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return PM_ERR_DEVICE;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr) return PM_ERR_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PM_OK;
}

}  // namespace

namespace pm {

PhaseMark phase_begin(int phase, hipStream_t st) {
  PhaseMark m{phase, nullptr};
  if (!g_timing.load(std::memory_order_relaxed)) return m;
  std::lock_guard<std::mutex> lk(g_tmu);
  m.a = pooled_event();
  if (m.a) (void)hipEventRecord(m.a, st);
  return m;
}

void phase_end(const PhaseMark& m, hipStream_t st) {
  if (!m.a) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  hipEvent_t b = pooled_event();
  if (!b) {
    g_pool.push_back(m.a);
    return;
  }
  (void)hipEventRecord(b, st);
  g_recs.push_back(TimingRec{m.phase, m.a, b});
}

}  // namespace pm

extern "C" {

int polymat_abi_version(void) { return 1; }

pm_status polymat_check_enable(int on) {
  g_check.store(on != 0);
  return PM_OK;
}

pm_status polymat_timing_enable(int on) {
  g_timing.store(on != 0);
  return PM_OK;
}

pm_status polymat_timing_read(double* ms, int* launches) {
  std::vector<TimingRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    recs.swap(g_recs);
  }
  double acc[PM_NUM_PHASES] = {0};
  int cnt[PM_NUM_PHASES] = {0};
  pm_status st = PM_OK;
  for (const TimingRec& r : recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      st = PM_ERR_DEVICE;
    } else if (r.phase >= 0 && r.phase < PM_NUM_PHASES) {
      acc[r.phase] += t;
      cnt[r.phase] += 1;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    for (const TimingRec& r : recs) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
    }
  }
  for (int i = 0; i < PM_NUM_PHASES; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
  return st;
}

const char* polymat_strerror(pm_status status) {
  switch (status) {
    case PM_OK: return "success";
    case PM_ERR_INVALID: return "invalid argument";
    case PM_ERR_WORKSPACE: return "workspace too small";
    case PM_ERR_DEVICE: return "HIP device error";
    case PM_ERR_UNSUPPORTED: return "unsupported size or mode";
    case PM_ERR_NONFINITE: return "non-finite value in an operand or the result";
    default: return "unknown status";
  }
}

int polymat_transform_length(int ntrunc) { return transform_length(ntrunc); }

size_t polymat_workspace_size(int n, int ntrunc, int precision, int count) {
  if (n < 1 || n > PM_MAX_N || ntrunc < 0 || ntrunc > PM_MAX_NTRUNC || !valid_prec(precision) ||
      count < 1 || count > PM_MAX_BATCH)
    return 0;
  return product_layout(n, ntrunc, precision).total * static_cast<size_t>(count);
}

size_t polymat_batched_workspace_size(const pm_problem* problems, int count, int precision) {
  std::vector<Planned> items;
  size_t need = 0;
  if (plan_batch(problems, count, precision, nullptr, 0, items, &need) != PM_OK) return 0;
  return need;
}

pm_status polymat_mul_batched(const pm_problem* problems, int count, int precision, void* workspace,
                              size_t workspace_bytes, void* stream) {
  if (!workspace) return PM_ERR_INVALID;
  std::vector<Planned> items;
  pm_status s = plan_batch(problems, count, precision, static_cast<char*>(workspace), workspace_bytes,
                           items, nullptr);
  if (s) return s;
  // two problems must not write overlapping outputs
  std::vector<Range> outs;
  outs.reserve(items.size());
  for (const Planned& it : items) outs.push_back(range_of(it.pr.C, series_bytes(it.pr.n, it.pr.ntrunc)));
  std::sort(outs.begin(), outs.end(), [](const Range& a, const Range& b) { return a.b < b.b; });
  for (size_t i = 1; i < outs.size(); ++i)
    if (outs[i].b < outs[i - 1].e) return PM_ERR_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool check = g_check.load(std::memory_order_relaxed);
  if (check && stream_capturing(st)) return PM_ERR_INVALID;
  std::vector<const PipeSlot*> ctl;
  if (precision == PM_PREC_FP64 && pipeline_enabled() && gemm_uses_g3() && pipeline_alias_free(items))
    s = enqueue_pipeline(items, st, &ctl);
  else
    s = enqueue_products(items, precision, st);
  if (s || !check) return s;
  // read back the status words of every product's scale record (and the
  // abort flag of every pipeline launch: a wait that ran out)
  if (hipStreamSynchronize(st) != hipSuccess) return PM_ERR_DEVICE;
  for (const PipeSlot* c : ctl) {
    unsigned int ab = 0u;
    if (hipMemcpy(&ab, &c->abort, sizeof(ab), hipMemcpyDeviceToHost) != hipSuccess || ab != 0u)
      return PM_ERR_DEVICE;
  }
  for (const Planned& it : items) {
    unsigned int flags[2] = {0u, 0u};
    const char* rec = it.ws + it.lay.rec + offsetof(ScaleRec, in_bad);
    if (hipMemcpy(flags, rec, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess) return PM_ERR_DEVICE;
    if (flags[0] || flags[1]) return PM_ERR_NONFINITE;
  }
  return PM_OK;
}

pm_status polymat_mul_naive(const void* A, const void* B, void* C, int n, int ntrunc, int op_a, int op_b,
                            void* stream) {
  if (!A || !B || !C || !aligned(A, 16) || !aligned(B, 16) || !aligned(C, 16)) return PM_ERR_INVALID;
  if (n < 1 || n > PM_MAX_N || ntrunc < 0) return PM_ERR_INVALID;
  if (ntrunc > PM_MAX_NTRUNC) return PM_ERR_UNSUPPORTED;
  if ((op_a != PM_OP_N && op_a != PM_OP_C) || (op_b != PM_OP_N && op_b != PM_OP_C)) return PM_ERR_INVALID;
  const size_t sb = series_bytes(n, ntrunc);
  if (overlaps(range_of(C, sb), range_of(A, sb)) || overlaps(range_of(C, sb), range_of(B, sb)))
    return PM_ERR_INVALID;
  GemmArgs ga{};
  ga.njobs = 1;
  GemmJob& j = ga.jobs[0];
  j.A = A;
  j.B = B;
  j.C = C;
  j.n = n;
  j.L = ntrunc + 1;
  j.opA = op_a;
  j.opB = op_b;
  j.tiles_m = j.tiles_n = (n + kConvTile - 1) / kConvTile;
  j.tile_begin = 0;
  ga.total_tiles = j.tiles_m * j.tiles_n * j.L;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return from_hip(timed(PM_PHASE_PRODUCT, st, [&] { return launch_conv(ga, st); }));
}

pm_status polymat_mul(const void* A, const void* B, void* C, int n, int ntrunc, int precision,
                      double scale, void* workspace, size_t workspace_bytes, void* stream) {
  // A single-order FP64 product (a plain matrix product) takes the direct
  // form of eq. (5): one N x N product instead of L = 4 mode products plus the
  // transforms.  The arguments are validated as for the transform path.
  if (precision == PM_PREC_FP64 && ntrunc >= 0 && ntrunc <= kNaiveMaxNtrunc && n >= 1 && n <= PM_MAX_N && A &&
      B && C && !g_check.load(std::memory_order_relaxed)) {
    const size_t sb = series_bytes(n, ntrunc);
    if (!overlaps(range_of(C, sb), range_of(A, sb)) && !overlaps(range_of(C, sb), range_of(B, sb))) {
      if (!std::isfinite(scale) || scale < 0.0) return PM_ERR_INVALID;
      const size_t need = polymat_workspace_size(n, ntrunc, precision, 1);
      if (need == 0 || !workspace || !aligned(workspace, kAlign)) return PM_ERR_INVALID;
      if (workspace_bytes < need) return PM_ERR_WORKSPACE;
      const Range wr = range_of(workspace, need);
      if (overlaps(wr, range_of(A, sb)) || overlaps(wr, range_of(B, sb)) || overlaps(wr, range_of(C, sb)))
        return PM_ERR_INVALID;
      return polymat_mul_naive(A, B, C, n, ntrunc, PM_OP_N, PM_OP_N, stream);
    }
  }
  pm_problem p;
  p.A = A;
  p.B = B;
  p.C = C;
  p.n = n;
  p.ntrunc = ntrunc;
  p.op_a = PM_OP_N;
  p.op_b = PM_OP_N;
  p.scale = scale;
  return polymat_mul_batched(&p, 1, precision, workspace, workspace_bytes, stream);
}

pm_status polymat_mul_noalloc(const void* A, const void* B, void* C, int n, int ntrunc, int precision,
                              double scale, void* stream) {
  // sizes first: a product whose workspace exceeds the built-in array is
  // rejected before any HIP call
  if (n < 1 || n > PM_MAX_N || ntrunc < 0 || !valid_prec(precision)) return PM_ERR_INVALID;
  if (ntrunc > PM_MAX_NTRUNC) return PM_ERR_UNSUPPORTED;
  const size_t need = polymat_workspace_size(n, ntrunc, precision, 1);
  if (need == 0) return PM_ERR_INVALID;
  if (need > kNoAllocBytes) return PM_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  const pm_status s = scratch_address(st, &ws);
  if (s) return s;
  return polymat_mul(A, B, C, n, ntrunc, precision, scale, ws, kNoAllocBytes, stream);
}

size_t polymat_transform_workspace_size(void) { return align_up(sizeof(ScaleRec)); }

static pm_status transform_common(const void* X, const void* Y, int n, int ntrunc, double scale,
                                  void* workspace, size_t workspace_bytes) {
  if (!X || !Y || !aligned(X, 16) || !aligned(Y, 16)) return PM_ERR_INVALID;
  if (n < 1 || n > PM_MAX_N || ntrunc < 0) return PM_ERR_INVALID;
  if (ntrunc > PM_MAX_NTRUNC) return PM_ERR_UNSUPPORTED;
  if (!std::isfinite(scale) || scale <= 0.0) return PM_ERR_INVALID;
  if (!workspace || !aligned(workspace, kAlign)) return PM_ERR_INVALID;
  if (workspace_bytes < polymat_transform_workspace_size()) return PM_ERR_WORKSPACE;
  return PM_OK;
}

pm_status polymat_forward_transform(const void* A, void* At, int n, int ntrunc, double scale,
                                    void* workspace, size_t workspace_bytes, void* stream) {
  pm_status s = transform_common(A, At, n, ntrunc, scale, workspace, workspace_bytes);
  if (s) return s;
  const int L = transform_length(ntrunc);
  const size_t E = static_cast<size_t>(n) * n;
  const Range wr = range_of(workspace, polymat_transform_workspace_size());
  if (overlaps(wr, range_of(A, series_bytes(n, ntrunc))) || overlaps(wr, range_of(At, E * L * 16)) ||
      overlaps(range_of(A, series_bytes(n, ntrunc)), range_of(At, E * L * 16)))
    return PM_ERR_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  ScaleArgs sa{};
  sa.njobs = 1;
  sa.jobs[0].rec = static_cast<ScaleRec*>(workspace);
  sa.jobs[0].nord = ntrunc + 1;
  sa.jobs[0].L = L;
  sa.jobs[0].fixed_s = scale;
  sa.jobs[0].nser = 1;
  s = from_hip(launch_scale(sa, st));
  if (s) return s;
  FwdArgs fa{};
  fa.njobs = 1;
  fa.jobs[0].src = static_cast<const double2*>(A);
  fa.jobs[0].dst = At;
  fa.jobs[0].rec = static_cast<const ScaleRec*>(workspace);
  fa.jobs[0].E = n * n;
  fa.jobs[0].nord = ntrunc + 1;
  fa.jobs[0].n = n;
  return from_hip(launch_forward(fa, L, n * n, kF64, st));
}

pm_status polymat_inverse_transform(const void* Ct, void* C, int n, int ntrunc, double scale,
                                    void* workspace, size_t workspace_bytes, void* stream) {
  pm_status s = transform_common(Ct, C, n, ntrunc, scale, workspace, workspace_bytes);
  if (s) return s;
  const int L = transform_length(ntrunc);
  const size_t E = static_cast<size_t>(n) * n;
  const Range wr = range_of(workspace, polymat_transform_workspace_size());
  if (overlaps(wr, range_of(C, series_bytes(n, ntrunc))) || overlaps(wr, range_of(Ct, E * L * 16)) ||
      overlaps(range_of(C, series_bytes(n, ntrunc)), range_of(Ct, E * L * 16)))
    return PM_ERR_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  ScaleArgs sa{};
  sa.njobs = 1;
  sa.jobs[0].rec = static_cast<ScaleRec*>(workspace);
  sa.jobs[0].nord = ntrunc + 1;
  sa.jobs[0].L = L;
  sa.jobs[0].fixed_s = scale;
  sa.jobs[0].nser = 1;
  s = from_hip(launch_scale(sa, st));
  if (s) return s;
  InvArgs ia{};
  ia.njobs = 1;
  ia.jobs[0].src = Ct;
  ia.jobs[0].dst = static_cast<double2*>(C);
  ia.jobs[0].rec = static_cast<ScaleRec*>(workspace);
  ia.jobs[0].E = n * n;
  ia.jobs[0].nord = ntrunc + 1;
  return from_hip(launch_inverse(ia, L, n * n, kF64, st));
}

size_t nspt_workspace_size(int replicas, const nspt_params* params, int precision) {
  return pm::nspt_workspace_bytes(replicas, params, precision);
}

pm_status nspt_langevin_step(void* U, const void* eta, int replicas, const nspt_params* params,
                             int precision, void* workspace, size_t workspace_bytes, void* stream) {
  return pm::nspt_step(U, eta, replicas, params, precision, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream));
}

pm_status nspt_action(const void* U, int replicas, const nspt_params* params, int precision, double* S,
                      void* workspace, size_t workspace_bytes, void* stream) {
  return pm::nspt_series_action(U, replicas, params, precision, S, workspace, workspace_bytes,
                                static_cast<hipStream_t>(stream));
}

pm_status nspt_wilson_loop(const void* U, int replicas, const nspt_params* params, int a, int b, int precision,
                           double* W, void* workspace, size_t workspace_bytes, void* stream) {
  return pm::nspt_wilson(U, replicas, params, a, b, precision, W, workspace, workspace_bytes,
                         static_cast<hipStream_t>(stream));
}

pm_status nspt_noise(void* eta, int replicas, int n, unsigned long long seed, unsigned long long step,
                     void* stream) {
  return pm::nspt_noise(eta, replicas, n, seed, step, static_cast<hipStream_t>(stream));
}

pm_status nspt_langevin_steps(void* U, int replicas, const nspt_params* params, unsigned long long seed,
                              unsigned long long step0, int nsteps, int precision, void* workspace,
                              size_t workspace_bytes, void* stream) {
  return pm::nspt_steps(U, replicas, params, seed, step0, nsteps, precision, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

pm_status nspt_gauge_fix(void* U, int replicas, const nspt_params* params, double alpha, int precision,
                         void* workspace, size_t workspace_bytes, void* stream) {
  return pm::nspt_gauge(U, replicas, params, alpha, precision, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

pm_status nspt_md_trajectory(void* U, void* P, const void* eta, int replicas, const nspt_params* params,
                             int nsteps, int precision, void* workspace, size_t workspace_bytes,
                             void* stream) {
  return pm::nspt_md(U, P, eta, replicas, params, nsteps, precision, workspace, workspace_bytes,
                     static_cast<hipStream_t>(stream));
}

}  // extern "C"
