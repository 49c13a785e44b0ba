"""Throughput of FFT-CONV truncated matrix-series products on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Headline workload (one step): a batch of 4 truncated series products, one
per link direction, with N = 225 (SU(225)), ntrunc = 31 (orders g^0..g^31,
transform length 64), complex128 coefficients with i.i.d. N(0,1) real and
imaginary parts times 0.5^k at order k, FP64 mode-wise products, rescaling
chosen on the device.  Inputs are resident in HBM before the timed region.
The value is products per second over the K timed steps, which run after the
other workloads of the line (the GPU at its running clock); the same W + K
steps timed right after start-up are reported as cold_start.

Also reported: the same metric at ntrunc = 63 (N = 225, entries times 1.3^k)
for the FP64, FP32 and split-BF16 product precisions, the time per phase,
the roofline position of the dominant kernel (the mode-wise products,
timed with HIP events around each of its launches on the launch stream),
and the FP64 CPU oracle (naive star product) on the host cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "poly-matrix mults/s at SU(225) O(g^31),O(g^63); split-BF16 vs FP64 MFMA"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0


GEMM_SOURCES = ("pm_gemm_impl.h", "pm_gemm_f64.hip", "pm_gemm.hip", "pm_gemm_tuning.h", "pm_common.h")


def _code_only(text: str) -> str:
    """C++ source without comments and blank lines (comment edits leave the
    compiled kernel and its counters unchanged)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def gemm_source_hash() -> str:
    """Hash of the code (comments stripped) that defines the FP64 product
    kernel and its shape choice."""
    h = hashlib.sha256()
    for name in GEMM_SOURCES:
        with open(os.path.join(ROOT, "paper_2001_02835_amd", "csrc", name)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel_key: str):
    """HBM traffic of the dominant kernel from the committed counter summary,
    or None if there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        rec = d.get(kernel_key)
        if not rec or rec.get("source_sha256_16") != gemm_source_hash():
            return None
        return rec.get("hbm_bytes_per_launch")
    except Exception:
        return None


def make_inputs(torch, synth, cfg, count, n, nt, ratio, dev):
    items = []
    for i in range(count):
        a = torch.from_numpy(synth.random_series(synth.rng_for(cfg, i, 0), n, nt, ratio)).to(dev)
        b = torch.from_numpy(synth.random_series(synth.rng_for(cfg, i, 1), n, nt, ratio)).to(dev)
        c = torch.empty_like(a)
        items.append(dict(A=a, B=b, C=c, scale=0.0))
    return items


def time_steps(torch, pm, items, prec, steps, warmup, ws, timing=False):
    """ms per step over `steps` un-instrumented steps; with timing, the per-phase
    HIP-event times come from a second pass of `steps` steps (the events around
    every launch add about 8 us per launch, so they stay out of the first pass)."""
    for _ in range(warmup):
        pm.polymat_mul_batched(items, prec, ws=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pm.polymat_mul_batched(items, prec, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    phases = None
    if timing:
        pm.timing_read()           # discard anything recorded before
        pm.timing_enable(True)
        for _ in range(steps):
            pm.polymat_mul_batched(items, prec, ws=ws)
        torch.cuda.synchronize()
        pm.timing_enable(False)
        phases = pm.timing_read()
    return ms, phases


def bench_uneven(torch, synth, pm, dev, steps):
    """64 independent products with N drawn from {64,121,169,225,289} and ntrunc
    from {15,31,63} (entries N(0,1)*0.7^k), one batched call per step."""
    shapes = synth.uneven_batch_shapes(synth.rng_for(4, 0), 64)
    items = []
    for i, (n, nt) in enumerate(shapes):
        a = torch.from_numpy(synth.random_series(synth.rng_for(4, 1 + i, 0), n, nt, 0.7)).to(dev)
        b = torch.from_numpy(synth.random_series(synth.rng_for(4, 1 + i, 1), n, nt, 0.7)).to(dev)
        items.append(dict(A=a, B=b, C=torch.empty_like(a), scale=0.0))
    useful = sum(pm.transform_length(nt) * 8.0 * n ** 3 for n, nt in shapes)
    res = {"workload": "64 products, N in {64,121,169,225,289}, ntrunc in {15,31,63}, entries N(0,1)*0.7^k, "
                       "one batched call (staged launches: norms, scale, forward per transform length, products "
                       "per matrix size, inverse per transform length)",
           "useful_gflop_per_batch": round(useful / 1e9, 1)}
    for prec in ("fp64", "bf16x3"):
        ws = pm.workspace(pm.batched_workspace_size(items, prec), dev)
        ms, ph = time_steps(torch, pm, items, prec, steps, 1, ws, timing=True)
        res[prec] = {"ms_per_batch": round(ms, 3), "mults_per_s": round(64 / (ms * 1e-3), 1),
                     "useful_tflops": round(useful / (ms * 1e-3) / 1e12, 2),
                     "phase_ms_per_batch": {k: round(v[0] / steps, 3) for k, v in ph.items() if v[1]}}
        if prec == "fp64":
            # the same batch through the opt-in persistent one-launch pipeline
            # (set-up launches, then every step of every product in one launch)
            os.environ["POLYMAT_PIPELINE"] = "1"
            try:
                pms, _ = time_steps(torch, pm, items, prec, steps, 1, ws)
                res["fp64_one_launch_pipeline"] = {"ms_per_batch": round(pms, 3),
                                                   "useful_tflops": round(useful / (pms * 1e-3) / 1e12, 2),
                                                   "note": "opt-in (POLYMAT_PIPELINE=1); the staged launches are "
                                                           "the default"}
            except Exception as exc:   # reported, not fatal: the staged figures above stand
                res["fp64_one_launch_pipeline"] = {"error": str(exc)}
            finally:
                del os.environ["POLYMAT_PIPELINE"]
        del ws
    return res


def bench_nspt(torch, synth, pm, dev, steps):
    """NSPT Euler-Langevin step: 8 replicas x 4 links, SU(225) (L=15, k=4), ntrunc=31,
    eps=0.01, started at the twisted vacuum and evolved by warm-up steps; the same
    step replayed from a captured HIP graph; steps with the noise drawn on the
    device; then one stochastic gauge-fixing step (alpha = 0.1) on the same links."""
    import numpy as np
    L, k, nt, eps, R = 15, 4, 31, 0.01, 8
    n = L * L
    u = torch.from_numpy(synth.vacuum_links(L, k, nt, replicas=R)).to(dev)
    rng = synth.rng_for(5, 0)
    noise = [torch.from_numpy(synth.langevin_noise(rng, R, n)).to(dev) for _ in range(2)]
    prm = pm.nspt_params(L, k, nt, eps)
    res = {"workload": "8 replicas x 4 links, N=225 (L=15, k=4), ntrunc=31, eps=0.01, FP64 links"}
    for prec in ("fp64", "bf16x3"):
        ws = pm.workspace(pm.nspt_workspace_size(R, prm, prec), dev)
        for i in range(2):
            pm.nspt_langevin_step(u, noise[i % 2], prm, prec, ws=ws)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            pm.nspt_langevin_step(u, noise[i % 2], prm, prec, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # phases from a second, instrumented pass
        pm.timing_read()
        pm.timing_enable(True)
        for i in range(steps):
            pm.nspt_langevin_step(u, noise[i % 2], prm, prec, ws=ws)
        torch.cuda.synchronize()
        pm.timing_enable(False)
        ph = pm.timing_read()
        # the same step captured once into a HIP graph and replayed
        try:
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                pm.nspt_langevin_step(u, noise[0], prm, prec, ws=ws)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                pm.nspt_langevin_step(u, noise[0], prm, prec, ws=ws)
            graph.replay()
            torch.cuda.synchronize()
            e0.record()
            for i in range(steps):
                graph.replay()
            e1.record()
            torch.cuda.synchronize()
            graph_ms = round(e0.elapsed_time(e1) / steps, 3)
            del graph
        except Exception as exc:   # report, do not fail the bench line
            graph_ms = f"capture failed: {exc}"
        # the same number of steps in one call with the noise drawn on the device
        e0.record()
        pm.nspt_langevin_steps(u, prm, 2024, 0, steps, prec, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        dev_noise_ms = round(e0.elapsed_time(e1) / steps, 3)
        # one stochastic gauge-fixing step (alpha = 0.1) on the evolved links
        pm.nspt_gauge_fix(u, prm, 0.1, prec, ws=ws)
        torch.cuda.synchronize()
        e0.record()
        for i in range(steps):
            pm.nspt_gauge_fix(u, prm, 0.1, prec, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / steps
        res[prec] = {"ms_per_step": round(ms, 3), "steps_per_s": round(1e3 / ms, 3),
                     "replica_steps_per_s": round(R * 1e3 / ms, 2),
                     "phase_ms_per_step": {kk: round(v[0] / steps, 3) for kk, v in ph.items() if v[1]},
                     "graph_ms_per_step": graph_ms, "device_noise_ms_per_step": dev_noise_ms,
                     "gauge_fix_ms": round(gms, 3)}
        del ws
    return res


def bench_md(torch, synth, pm, dev, nsteps):
    """NSPT molecular-dynamics trajectory (leapfrog, momentum refresh): 8 replicas
    x 4 links, SU(225) (L=15, k=4), ntrunc=31, dt=0.05, started at the twisted
    vacuum and evolved by a short warm-up trajectory; one timed trajectory of
    `nsteps` MD steps (the paper's unit is a trajectory of 40 MD steps), then
    one more with HIP events around every launch for the phase times."""
    L, k, nt, dt, R = 15, 4, 31, 0.05, 8
    n = L * L
    u = torch.from_numpy(synth.vacuum_links(L, k, nt, replicas=R)).to(dev)
    P = torch.zeros_like(u)
    rng = synth.rng_for(6, 0)
    noise = [torch.from_numpy(synth.langevin_noise(rng, R, n)).to(dev) for _ in range(2)]
    prm = pm.nspt_params(L, k, nt, dt)
    res = {"workload": f"8 replicas x 4 links, N=225 (L=15, k=4), ntrunc=31, leapfrog dt=0.05, "
                       f"{nsteps} MD steps per trajectory with momentum refresh, FP64 links"}
    for prec in ("fp64", "bf16x3"):
        ws = pm.workspace(pm.nspt_workspace_size(R, prm, prec), dev)
        pm.nspt_md_trajectory(u, P, prm, min(nsteps, 2), eta=noise[0], precision=prec, ws=ws)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        pm.nspt_md_trajectory(u, P, prm, nsteps, eta=noise[1], precision=prec, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        # phases from a second, instrumented trajectory
        pm.timing_read()
        pm.timing_enable(True)
        pm.nspt_md_trajectory(u, P, prm, nsteps, eta=noise[0], precision=prec, ws=ws)
        torch.cuda.synchronize()
        pm.timing_enable(False)
        ph = pm.timing_read()
        res[prec] = {"ms_per_trajectory": round(ms, 2), "ms_per_md_step": round(ms / nsteps, 3),
                     "force_evaluations": nsteps + 1,
                     "phase_ms_per_trajectory": {kk: round(v[0], 3) for kk, v in ph.items() if v[1]},
                     "paper_run_estimate_s": {"trajectories": 10, "md_steps": 40,
                                              "seconds": round(10 * 40 * ms / nsteps / 1e3, 2),
                                              "from": f"one measured trajectory of {nsteps} MD steps"}}
        del ws
    return res


def bench_crossover(torch, synth, pm, dev, reps=20):
    """Naive-CONV (direct eq. (5)) against FFT-CONV for one FP64 product at
    N=225 and growing ntrunc (entries N(0,1)*0.5^k): where the transform pays."""
    n = 225
    res = {"workload": "1 product N=225, FP64, entries N(0,1)*0.5^k; ms per product (in_chain_fftconv_ms: "
                       "forward + product + inverse phases, the cost of one product inside a Fourier-space chain)",
           "points": []}
    for nt in (0, 1, 2, 3, 5, 7, 15, 31):
        a = torch.from_numpy(synth.random_series(synth.rng_for(7, nt, 0), n, nt, 0.5)).to(dev)
        b = torch.from_numpy(synth.random_series(synth.rng_for(7, nt, 1), n, nt, 0.5)).to(dev)
        c = torch.empty_like(a)
        items = [dict(A=a, B=b, C=c)]
        ws = pm.workspace(pm.batched_workspace_size(items, "fp64"), dev)
        t = {}
        for name, fn in (("naive", lambda: pm.polymat_mul_naive(a, b, C=c)),
                         ("fftconv", lambda: pm.polymat_mul_batched(items, "fp64", ws=ws))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            t[name] = e0.elapsed_time(e1) / reps
        # phases of the FFT-CONV call: inside a chain of products that stays in
        # Fourier space (the Horner steps of the series exponential) a product
        # costs its product phase plus one re-truncation (an inverse and a
        # forward transform in one pass), without the rescale
        pm.timing_read()
        pm.timing_enable(True)
        for _ in range(reps):
            pm.polymat_mul_batched(items, "fp64", ws=ws)
        torch.cuda.synchronize()
        pm.timing_enable(False)
        ph = {k: round(v[0] / reps, 4) for k, v in pm.timing_read().items() if v[1]}
        res["points"].append({"ntrunc": nt, "naive_ms": round(t["naive"], 4), "fftconv_ms": round(t["fftconv"], 4),
                              "naive_products": (nt + 1) * (nt + 2) // 2, "fft_modes": pm.transform_length(nt),
                              "fftconv_phase_ms": ph,
                              "in_chain_fftconv_ms": round(ph.get("forward", 0.0) + ph.get("product", 0.0)
                                                           + ph.get("inverse", 0.0), 4)})
        del ws
    return res


def cpu_fftconv(a, b, workers):
    """FFT-CONV on the host CPU, the analogue of the paper's CPU FFT-CONV
    (its Section 3 comparison): order-axis FFTs of the zero-padded operands
    with scipy.fft over `workers` threads, one complex128 matrix product per
    frequency (BLAS), the inverse FFT, truncation.  A timing baseline only:
    nothing on the GPU path uses it."""
    import numpy as np
    import scipy.fft as sfft
    nt1 = a.shape[0]
    L = 4
    while L < 2 * nt1:
        L *= 2
    at = sfft.fft(a, n=L, axis=0, workers=workers)
    bt = sfft.fft(b, n=L, axis=0, workers=workers)
    ct = np.empty_like(at)
    for p in range(L):
        np.matmul(at[p], bt[p], out=ct[p])
    return sfft.ifft(ct, axis=0, workers=workers)[:nt1]


def cpu_baseline(seconds: float, gpu_c2=None, gpu_c3=None):
    """The FP64 oracle (naive star product, BLAS matmul per term) on the host
    cores, on the four headline products (the same seeded inputs as the GPU
    step) in turn until `seconds` have elapsed; beside it the CPU FFT-CONV
    baseline on the same products.  The oracle's first result of each product
    (and one oracle product of the ntrunc = 63 workload) also gives the
    per-order error of the GPU results passed in."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import synth
    from oracle import series as ser

    n, nt = 225, 31
    ops = [(synth.random_series(synth.rng_for(2, i, 0), n, nt, 0.5),
            synth.random_series(synth.rng_for(2, i, 1), n, nt, 0.5)) for i in range(4)]
    ser.star(ops[0][0][:2], ops[0][1][:2])            # warm the BLAS pool
    refs = [None] * 4
    done, t0 = 0, time.perf_counter()
    while True:
        i = done % 4
        c = ser.star(*ops[i])
        if refs[i] is None:
            refs[i] = c
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds and done >= 4:
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    ncpu = os.cpu_count() or 1
    out = {
        "value": done / el, "unit": "mults/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{done} products N=225 ntrunc=31 (the four headline products in turn, entries N(0,1)*0.5^k), "
                  f"naive O(ntrunc^2) star product with numpy complex128 matmul, {el:.1f} s on {ncpu} host CPUs",
    }
    # the paper-analog CPU FFT-CONV on the same products
    cpu_fftconv(*ops[0], ncpu)
    fdone, t0 = 0, time.perf_counter()
    ferr = 0.0
    while True:
        i = fdone % 4
        c = cpu_fftconv(*ops[i], ncpu)
        if fdone < 4:
            ferr = max(ferr, float(order_errors(c, refs[i]).max()))
        fdone += 1
        fel = time.perf_counter() - t0
        if fel >= seconds / 4 and fdone >= 4:
            break
    out["fftconv"] = {"value": round(fdone / fel, 2), "unit": "mults/s", "threads": ncpu,
                      "kind": "CPU FFT-CONV (scipy.fft workers + per-frequency BLAS matmul), not tuned",
                      "sample": f"{fdone} products N=225 ntrunc=31 in {fel:.1f} s",
                      "max_per_order_error_vs_oracle": float(f"{ferr:.3e}")}
    errs = {}
    if gpu_c2 is not None:
        e = np.stack([order_errors(gpu_c2[i], refs[i]) for i in range(4)])
        errs["n225_nt31_x4_fp64"] = {"max": float(f"{e.max():.3e}"), "order_of_max": int(e.max(axis=0).argmax())}
    if gpu_c3:
        a3 = synth.random_series(synth.rng_for(3, 0, 0), 225, 63, 1.3)
        b3 = synth.random_series(synth.rng_for(3, 0, 1), 225, 63, 1.3)
        ref3 = ser.star(a3, b3)
        for prec, c in gpu_c3.items():
            e = order_errors(c, ref3)
            errs[f"n225_nt63_{prec}"] = {"max": float(f"{e.max():.3e}"), "order_of_max": int(e.argmax()),
                                         "median": float(f"{np.median(e):.3e}")}
    return out, errs


def order_errors(c, ref):
    """e_k = ||C^(k) - C_ref^(k)||_F / ||C_ref^(k)||_F for every order k."""
    import numpy as np
    num = np.sqrt(np.sum(np.abs(c - ref) ** 2, axis=(-2, -1)))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(-2, -1)))
    return num / np.where(den > 0, den, 1.0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extra", action="store_true", help="skip the ntrunc = 63 precision lines")
    ap.add_argument("--precision-only", action="store_true",
                    help="of the extra lines, run only the ntrunc = 63 precision comparison")
    ap.add_argument("--nspt-steps", type=int, default=3)
    ap.add_argument("--md-steps", type=int, default=40, help="leapfrog steps of the timed MD trajectory")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the series products of this workload are not "
              "sharded across GPUs here (run with --gpus 1).", file=sys.stderr)
        return 2

    import torch
    import synth
    import paper_2001_02835_amd as pm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = "cuda:0"
    pm.lib()   # fails loudly if the library is missing

    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- headline inputs: 4 products N=225 ntrunc=31, FP64
    n, nt, count = 225, 31, 4
    L = pm.transform_length(nt)
    items = make_inputs(torch, synth, 2, count, n, nt, 0.5, dev)
    ws = pm.workspace(pm.batched_workspace_size(items, "fp64"), dev)
    # The same step timed right after start-up (W warm-up steps, then K steps).
    # The GPU's clock is still rising from idle here: the first few tens of
    # milliseconds of work run slower than the steady state.
    cold_ms, _ = time_steps(torch, pm, items, "fp64", args.steps, args.warmup, ws)

    extras = {}
    # ---- ntrunc = 63: FP64 vs FP32 vs split-BF16 on the same GPU
    gpu_c3 = {}
    if not args.no_extra:
        n3, nt3 = 225, 63
        items3 = make_inputs(torch, synth, 3, 1, n3, nt3, 1.3, dev)
        extra = {}
        for prec in ("fp64", "fp32", "bf16x3"):
            try:
                ws3 = pm.workspace(pm.batched_workspace_size(items3, prec), dev)
                st3 = max(args.steps // 4, 10)
                # 100 warm-up products (20-40 ms of work) after the allocation
                # and host copies between the precisions, so that each
                # precision is timed at the GPU's running clock
                ms3, ph3 = time_steps(torch, pm, items3, prec, st3, 100, ws3, timing=True)
                gpu_c3[prec] = items3[0]["C"].cpu().numpy()
                pms3, pl3 = ph3["product"]
                fl3 = pm.transform_length(nt3) * 8.0 * n3 ** 3
                ach = fl3 / (pms3 * 1e-3 / max(pl3, 1)) / 1e12
                # matrix-core flops issued per useful flop: the three-product
                # complex form (FP64, FP32 by default) issues 3 real products
                # instead of 4; split BF16 issues 4 real products x 3 split terms
                four_m = os.environ.get("POLYMAT_GEMM_4M") == "1"
                issued = ach * (3.0 if prec == "bf16x3" else (1.0 if four_m else 0.75))
                extra[prec] = {"mults_per_s": round(1e3 / ms3, 1), "ms_per_mult": round(ms3, 4),
                               "product_kernel_useful_tflops": round(ach, 2),
                               "product_kernel_issued_tflops": round(issued, 2),
                               "product_kernel_frac_of_peak": round(ach / PEAK[prec], 4),
                               "product_kernel_issued_frac_of_peak": round(issued / PEAK[prec], 4),
                               "phase_ms_per_mult": {k: round(v[0] / st3, 4) for k, v in ph3.items() if v[1]}}
                del ws3
            except Exception as exc:   # a precision that is not built reports why
                extra[prec] = {"error": str(exc)}
        extras["ntrunc63"] = {"workload": "1 product N=225 ntrunc=63 (L=128), entries N(0,1)*1.3^k, auto rescale",
                           **extra}

    if not args.no_extra and not args.precision_only:
        # the crossover's single small products leave the GPU idle between
        # calls, so it runs before the long workloads; the MD trajectory, the
        # longest, comes right before the headline
        def guarded(fn, *a):
            # an extra line that fails reports its error; the headline still runs
            try:
                return fn(*a)
            except Exception as exc:
                torch.cuda.synchronize()
                return {"error": str(exc)}
        crossover = guarded(bench_crossover, torch, synth, pm, dev)
        extras["batched_uneven"] = guarded(bench_uneven, torch, synth, pm, dev, max(args.steps // 20, 3))
        extras["nspt_step"] = guarded(bench_nspt, torch, synth, pm, dev, args.nspt_steps)
        extras["nspt_md"] = guarded(bench_md, torch, synth, pm, dev, args.md_steps)
        extras["naive_vs_fftconv"] = crossover

    # ---- headline, timed after the other workloads (the GPU at its running
    #      clock, as in a long NSPT run): W warm-up steps, then K timed steps
    ms, phases = time_steps(torch, pm, items, "fp64", args.steps, args.warmup, ws, timing=True)
    value = count / (ms * 1e-3)

    flops_step = count * L * 8.0 * n ** 3             # useful flops of one step (8 N^3 per mode)
    pms, plaunch = phases["product"]
    kernel = "k_cgemm2<double> (FP64 MFMA mode-wise products, 3-product complex form)"
    work = f"{count} products x {L} modes x 8*{n}^3 flop = {flops_step/1e9:.2f} GFLOP per launch"
    achieved = flops_step * args.steps / (pms * 1e-3) / 1e12
    traffic = load_traffic("k_cgemm_f64_c2")
    # matrix-core flops issued per useful flop: the three-product complex form
    # issues 3 real products where the useful count has 4
    issued_ratio = 1.0 if os.environ.get("POLYMAT_GEMM_4M") == "1" else 0.75
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["fp64"], 4), "traffic": traffic, "kernel": kernel,
                "algorithmic_work": work, "avg_launch_ms": round(pms / max(plaunch, 1), 4),
                "launches_per_step": plaunch // args.steps,
                "issued_achieved": round(achieved * issued_ratio, 2),
                "issued_frac": round(achieved * issued_ratio / PEAK["fp64"], 4),
                "issued_note": "MFMA flops actually issued: 6 N^3 per mode (3-product complex form) "
                               "against the 8 N^3 useful count"}
    gpu_c2 = [it["C"].cpu().numpy() for it in items]
    phase_ms = {k: round(v[0] / args.steps, 4) for k, v in phases.items() if v[1]}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "mults/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "4 truncated series products (one per direction), SU(225) N=225, "
                               "ntrunc=31 (L=64), complex128, entries N(0,1)*0.5^k, FP64 MFMA, auto rescale",
                   "n": n, "ntrunc": nt, "products_per_step": count, "precision": "fp64"},
        "roofline": roofline,
        "phase_ms_per_step": phase_ms,
        "timing": "value and ms_per_step from the K timed steps (no instrumentation), run after the other "
                  "workloads of this line so that the GPU is at its running clock; phases and roofline from "
                  "K further steps with HIP events around every launch on its stream",
        "cold_start": {"ms_per_step": round(cold_ms, 4), "mults_per_s": round(count / (cold_ms * 1e-3), 1),
                       "note": "the same W warm-up and K timed steps run first, right after start-up, "
                               "while the GPU clock still rises from idle"},
    }

    out.update(extras)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["per_order_error"] = cpu_baseline(args.cpu_seconds, gpu_c2, gpu_c3)
        out["per_order_error"]["metric"] = ("max over orders k of ||C_k - C_k^oracle||_F / ||C_k^oracle||_F, "
                                            "GPU results of the timed workloads against the FP64 oracle")
    out["context"] = ("paper: GPU FFT-CONV 9x faster than CPU FFT-CONV for the whole NSPT run at SU(225), "
                      "O(g^31), on 4xP100 vs 2xXeon 6154 (no absolute product rate published)")
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
