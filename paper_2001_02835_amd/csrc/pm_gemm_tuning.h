// Tile configuration per matrix size for the mode-wise products, measured
// on MI355X by paper_2001_02835_amd/autotune.py (fastest of the compiled
// shapes for a batch of 4 products, ntrunc = 31).  {n_max, config}: the first
// row with n <= n_max applies.
#pragma once

namespace pm {

struct TuneRow { int n_max, cfg; };
constexpr TuneRow kTune_fp64[] = {{92, 6}, {145, 2}, {197, 2}, {257, 6}, {1073741824, 6}};
constexpr TuneRow kTune_fp32[] = {{92, 6}, {145, 1}, {197, 6}, {257, 5}, {1073741824, 6}};

}  // namespace pm
