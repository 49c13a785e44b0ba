// Tile-configuration table and dispatch of the mode-wise complex products.
//
// Each precision has a small set of compiled tile shapes; the shape used for
// a matrix size comes from the table in pm_gemm_tuning.h, written by the
// autotuner (paper_2001_02835_amd/autotune.py) from measurements on MI355X.
// POLYMAT_GEMM_CONFIG=<index> in the environment forces one shape (read once
// per process), which is how the autotuner measures them.
#include <cstdlib>

#include "pm_gemm_impl.h"
#include "pm_gemm_tuning.h"

namespace pm {

hipError_t launch_gemm_f64(const GemmArgs& a, int cfg, bool g3, hipStream_t s);
hipError_t launch_gemm_f32(const GemmArgs& a, int cfg, bool g3, hipStream_t s);
hipError_t launch_gemm_conv_f64(const GemmArgs& a, bool g3, hipStream_t s);

namespace {

struct Shape { int wm, wn, wgm, wgn; };
constexpr Shape kShapes[] = {
#define PM_SHAPE(I, WM, WN, WGM, WGN) {WM, WN, WGM, WGN},
    PM_GEMM_CONFIGS(PM_SHAPE)
#undef PM_SHAPE
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int env_int(const char* name, int dflt) {
  const char* e = getenv(name);
  if (!e || !*e) return dflt;
  return atoi(e);
}

// Three-product complex form on by default; POLYMAT_GEMM_4M=1 selects the
// four-product form.
const bool g_gemm_g3 = env_int("POLYMAT_GEMM_4M", 0) != 1;
const int g_force_cfg = env_int("POLYMAT_GEMM_CONFIG", -1);

}  // namespace

bool gemm_uses_g3() { return g_gemm_g3; }

int gemm_num_configs(FourierType t) { return t == kBF16Split ? 1 : kNumShapes; }

GemmShape gemm_shape(FourierType t, int cfg) {
  if (t == kBF16Split) return GemmShape{gemm_tile_bf16(), gemm_tile_bf16()};
  const Shape& sh = kShapes[cfg];
  return GemmShape{16 * sh.wm * sh.wgm, 16 * sh.wn * sh.wgn};
}

int gemm_config(FourierType t, int n, int L) {
  if (t == kBF16Split) return 0;
  if (g_force_cfg >= 0 && g_force_cfg < kNumShapes) return g_force_cfg;
  const TuneRow* rows = t == kF64 ? kTune_fp64 : kTune_fp32;
  const int nrows = t == kF64 ? static_cast<int>(sizeof(kTune_fp64) / sizeof(TuneRow))
                              : static_cast<int>(sizeof(kTune_fp32) / sizeof(TuneRow));
  for (int i = 0; i < nrows; ++i)
    if (n <= rows[i].n_max && L <= rows[i].l_max) return rows[i].cfg;
  return rows[nrows - 1].cfg;
}

hipError_t launch_conv(const GemmArgs& a, hipStream_t s) {
  if (a.njobs <= 0 || a.total_tiles <= 0) return hipSuccess;
  return launch_gemm_conv_f64(a, g_gemm_g3, s);
}

hipError_t launch_gemm(const GemmArgs& a, FourierType t, int cfg, hipStream_t s) {
  if (a.njobs <= 0 || a.total_tiles <= 0) return hipSuccess;
  if (t == kF64) return launch_gemm_f64(a, cfg, g_gemm_g3, s);
  if (t == kF32) return launch_gemm_f32(a, cfg, g_gemm_g3, s);
  return launch_gemm_bf16(a, s);
}

}  // namespace pm
