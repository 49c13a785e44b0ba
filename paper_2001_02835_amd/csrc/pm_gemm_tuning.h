// Tile configuration per matrix size and transform length for the mode-wise
// products, measured on MI355X by paper_2001_02835_amd/autotune.py (fastest
// of the compiled shapes for a batch of 4 products at ntrunc = 15, 31, 63).
// {n_max, l_max, config}: the first row with n <= n_max and L <= l_max applies.
#pragma once

namespace pm {

struct TuneRow { int n_max, l_max, cfg; };
constexpr TuneRow kTune_fp64[] = {{1073741824, 1073741824, 2}};
constexpr TuneRow kTune_fp32[] = {{92, 32, 2}, {92, 64, 2}, {92, 1073741824, 2}, {145, 32, 2}, {145, 64, 1}, {145, 1073741824, 1}, {197, 32, 2}, {197, 64, 2}, {197, 1073741824, 2}, {257, 32, 2}, {257, 64, 2}, {257, 1073741824, 2}, {1073741824, 32, 2}, {1073741824, 64, 2}, {1073741824, 1073741824, 2}};

}  // namespace pm
