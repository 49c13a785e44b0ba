"""Host-side check of the product kernels' tile order (pm_common.h,
tile_in_mode): for every matrix size up to 600 and every tile shape the
kernels use, the work-groups of one mode cover each tile exactly once, and
every full tile comes before every edge or corner tile.  Compiled for the
host only with hipcc (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_02835_amd", "csrc")

PROG = r"""
#include "pm_common.h"
#include <cstdio>
#include <vector>
int main() {
  const int shapes[][2] = {{32, 32}, {64, 64}, {128, 64}, {64, 128}, {32, 64}, {64, 32}, {128, 128}};
  for (const auto& sh : shapes)
    for (int n = 1; n <= 600; ++n) {
      const int bm = sh[0], bn = sh[1];
      const int tmc = (n + bm - 1) / bm, tnc = (n + bn - 1) / bn;
      std::vector<int> seen(tmc * tnc, 0);
      int last_full = -1, first_short = tmc * tnc;
      for (int rem = 0; rem < tmc * tnc; ++rem) {
        int tm = -1, tn = -1;
        pm::tile_in_mode(rem, n, tmc, tnc, bm, bn, tm, tn);
        if (tm < 0 || tm >= tmc || tn < 0 || tn >= tnc) { std::printf("out of range n=%d\n", n); return 1; }
        seen[tm * tnc + tn]++;
        const bool full = (tm + 1) * bm <= n && (tn + 1) * bn <= n;
        if (full) last_full = rem; else if (rem < first_short) first_short = rem;
      }
      for (int v : seen)
        if (v != 1) { std::printf("not a permutation n=%d bm=%d bn=%d\n", n, bm, bn); return 1; }
      if (last_full > first_short) { std::printf("edge tile before a full tile n=%d\n", n); return 1; }
    }
  std::printf("ok\n");
  return 0;
}
"""


def test_tile_order_is_a_permutation_with_full_tiles_first(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    src = tmp_path / "tile_order.cpp"
    exe = tmp_path / "tile_order"
    src.write_text(PROG)
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1", "-std=c++17", f"-I{CSRC}",
                        f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
