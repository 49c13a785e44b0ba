// Tile configuration per matrix size for the mode-wise products, measured
// on MI355X by paper_2001_02835_amd/autotune.py (fastest of the compiled
// shapes for a batch of 4 products, ntrunc = 31).  {n_max, config}: the first
// row with n <= n_max applies.
#pragma once

namespace pm {

struct TuneRow { int n_max, cfg; };
constexpr TuneRow kTune_fp64[] = {{92, 2}, {145, 2}, {197, 2}, {257, 2}, {1073741824, 2}};
constexpr TuneRow kTune_fp32[] = {{92, 2}, {145, 2}, {197, 2}, {257, 2}, {1073741824, 2}};

}  // namespace pm
