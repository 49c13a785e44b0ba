"""Tile-shape autotuner for the mode-wise product kernels.

Run on an MI355X after building the library:

    python -m paper_2001_02835_amd.autotune [--out table.h] [--sizes 64,121,169,225,289]

For every compiled tile configuration (forced with POLYMAT_GEMM_CONFIG in a
child process) it times the product phase of a batch of 4 products for each
matrix size, transform length (ntrunc = 15, 31, 63: L = 32, 64, 128) and
precision, checks the configuration's products against a direct FP64
evaluation, and writes a C header with the fastest configuration per size
and length interval.  The committed csrc/pm_gemm_tuning.h was produced this
way.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NUM_CONFIGS = 6
NTRUNCS = (15, 31, 63)


def measure(sizes, steps=20):
    """Child process: time the product phase for every size (current config)."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import synth
    import paper_2001_02835_amd as pm
    dev = "cuda:0"
    out = {}
    for n in sizes:
        # correctness of the configuration: a short series product through the
        # batched call (always the transform path, so the forced tile shape
        # computes every mode product) against the convolution of eq. (5)
        # evaluated directly with numpy
        ntc = 3
        a0 = synth.random_series(synth.rng_for(3, n, 0), n, ntc)
        b0 = synth.random_series(synth.rng_for(3, n, 1), n, ntc)
        ref = np.stack([sum(a0[l] @ b0[k - l] for l in range(k + 1)) for k in range(ntc + 1)])
        for prec in ("fp64", "fp32"):
            chk = [dict(A=torch.from_numpy(a0).to(dev), B=torch.from_numpy(b0).to(dev),
                        C=torch.empty((ntc + 1, n, n), dtype=torch.complex128, device=dev))]
            pm.polymat_mul_batched(chk, precision=prec)
            got = chk[0]["C"].cpu().numpy()
            err = float(max(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(ntc + 1)))
            if err > (1e-12 if prec == "fp64" else 1e-5):
                raise SystemExit(f"config gives wrong products ({prec}, n={n}, err={err})")
        for nt in NTRUNCS:
            items = []
            for i in range(4):
                a = torch.from_numpy(synth.random_series(synth.rng_for(2, i, 0), n, nt, 0.5)).to(dev)
                b = torch.from_numpy(synth.random_series(synth.rng_for(2, i, 1), n, nt, 0.5)).to(dev)
                items.append(dict(A=a, B=b, C=torch.empty_like(a)))
            for prec in ("fp64", "fp32"):
                ws = pm.workspace(pm.batched_workspace_size(items, prec), dev)
                for _ in range(3):
                    pm.polymat_mul_batched(items, prec, ws=ws)
                torch.cuda.synchronize()
                pm.timing_read()
                pm.timing_enable(True)
                for _ in range(steps):
                    pm.polymat_mul_batched(items, prec, ws=ws)
                torch.cuda.synchronize()
                pm.timing_enable(False)
                out[f"{prec}:{n}:{pm.transform_length(nt)}"] = pm.timing_read()["product"][0] / steps
                del ws
            del items
    print(json.dumps(out))


def header(table) -> str:
    lines = ["// Tile configuration per matrix size and transform length for the mode-wise",
             "// products, measured on MI355X by paper_2001_02835_amd/autotune.py (fastest",
             "// of the compiled shapes for a batch of 4 products at ntrunc = 15, 31, 63).",
             "// {n_max, l_max, config}: the first row with n <= n_max and L <= l_max applies.",
             "#pragma once", "", "namespace pm {", "", "struct TuneRow { int n_max, l_max, cfg; };"]
    for prec, rows in table.items():
        body = ", ".join(f"{{{m}, {lm}, {c}}}" for m, lm, c in rows)
        lines.append(f"constexpr TuneRow kTune_{prec}[] = {{{body}}};")
    lines += ["", "}  // namespace pm", ""]
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="64,121,169,225,289")
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "pm_gemm_tuning.h"))
    ap.add_argument("--child", action="store_true")
    a = ap.parse_args(argv)
    sizes = [int(x) for x in a.sizes.split(",")]
    if a.child:
        measure(sizes)
        return 0
    results = {}
    for cfg in range(NUM_CONFIGS):
        env = dict(os.environ, POLYMAT_GEMM_CONFIG=str(cfg))
        r = subprocess.run([sys.executable, "-m", "paper_2001_02835_amd.autotune", "--child", "--sizes", a.sizes],
                           env=env, capture_output=True, text=True, cwd=ROOT, timeout=600)
        if r.returncode != 0:
            print(f"config {cfg}: failed\n{r.stderr[-2000:]}", file=sys.stderr)
            continue
        results[cfg] = json.loads(r.stdout.strip().splitlines()[-1])
        print(f"config {cfg}: {results[cfg]}", flush=True)
    lengths = sorted({int(k.split(":")[2]) for r in results.values() for k in r})
    table = {}
    for prec in ("fp64", "fp32"):
        rows = []
        for i, n in enumerate(sizes):
            n_max = (n + sizes[i + 1]) // 2 if i + 1 < len(sizes) else 1 << 30
            for j, L in enumerate(lengths):
                best = min(results, key=lambda c: results[c][f"{prec}:{n}:{L}"])
                l_max = L if j + 1 < len(lengths) else 1 << 30
                rows.append((n_max, l_max, best))
        if len({c for _, _, c in rows}) == 1:     # one shape everywhere: one row
            rows = [(1 << 30, 1 << 30, rows[0][2])]
        table[prec] = rows
    with open(a.out, "w") as f:
        f.write(header(table))
    print(f"wrote {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
