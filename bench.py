#!/usr/bin/env python3
"""THIIM benchmark on one MI355X.

Workload (default): the 512 x 512 x 512 production-size problem -- three
seeded layers (eps' in [1,16], eps'' in [0,0.5]) with a textured interface
(amplitude 4 cells), 200 SiO2-like spheres (eps = 2.1) in the last layer,
6-plane graded PML in z, periodic x/y, normal-incidence x-polarised source,
lambda = 600 nm at 20 nm cells -- 100 THIIM iterations in complex128.

One step = the whole hot path on the resident inputs: coefficient assembly
(thiim_create), 100 iterations (thiim_iterate) and the FP64 residual
(thiim_residual).  The value is lattice-site updates per second (GLUP/s:
nx*ny*nz*100 / step time).  The dominant kernel's roofline entry uses the
average duration of one iteration launch measured with HIP events on the
library's stream, and the algorithmic bytes of that sweep per cell update.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--kernel fused]
       [--size 512] [--iters 100] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# algorithmic HBM bytes per cell and iteration, complex128, 40-array layout
BYTES_PER_LUP = {
    "naive": 1024,   # two sweeps: (26 reads + 6 writes) x 16 B each
    "fused": 832,    # one pass: 40 reads + 12 writes, x 16 B
    "blocked": 416,  # one pass per two iterations: 40 reads + 12 writes, x 16 B
}
ITERS_PER_LAUNCH = {"naive": 0.5, "fused": 1, "blocked": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_kernel_run(torch, thiim, pb, kernel, iters, steps, warmup, tile=(0, 0),
                    z_chunk=0):
    """Runs warmup + steps whole-job steps; returns timings."""
    stream = torch.cuda.current_stream()
    step_ms, iter_ms, res = [], [], None
    for s in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver = thiim.Solver(pb, kernel=kernel, tile=tile, z_chunk=z_chunk,
                              stream=stream)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        solver.iterate(iters)
        ev1.record(stream)
        res = solver.residual()       # synchronising
        t1 = time.perf_counter()
        solver.close()
        if s >= warmup:
            step_ms.append((t1 - t0) * 1e3)
            iter_ms.append(ev0.elapsed_time(ev1) / iters)
        log(f"[bench] {kernel} step {s} ({'warmup' if s < warmup else 'timed'}): "
            f"{(t1 - t0) * 1e3:.1f} ms, {ev0.elapsed_time(ev1) / iters:.3f} ms/iteration, "
            f"residual {res:.3e}")
    return step_ms, iter_ms, res


def cpu_baseline(pb_full, budget_s=15.0):
    """The CPU oracle on a bounded sample of the same workload: the first
    planes of the 512^3 geometry (PML, source, first layer) as their own grid,
    iterated on all host cores."""
    import numpy as np

    import oracle
    from paper_1510_05218_amd import inputs

    nzs = 24
    eps = np.ascontiguousarray(pb_full.eps[:nzs])
    src = {k: np.ascontiguousarray(v[:nzs]) for k, v in pb_full.sources.items()}
    sig_e = pb_full.sig_e[:nzs].copy()
    sig_h = pb_full.sig_h[:nzs].copy()
    coef = oracle.coeffs(eps, sig_e, sig_h, src, pb_full.omega, pb_full.tau)
    x = oracle.zero_fields(eps.shape)
    t = time.perf_counter()
    oracle.iterate(coef, x, 1)
    one = time.perf_counter() - t
    n = max(1, min(200, int(budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.iterate(coef, x, n)
    dt = time.perf_counter() - t
    cells = eps.size
    del inputs
    return {
        "value": cells * n / dt / 1e9,
        "unit": "GLUP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{eps.shape[2]}x{eps.shape[1]}x{nzs} leading planes of the "
                  f"workload, {n} iterations, {dt:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel", default="blocked", choices=["naive", "fused", "blocked"])
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--compare", default="fused,naive",
                    help="comma list of extra kernels timed for context")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 4 GiB device copy first (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py: this THIIM build runs on one GPU only; the multi-GPU "
                 "(z-slab) decomposition is a design note, not implemented.")

    import torch

    from paper_1510_05218_amd import inputs, thiim

    if not torch.cuda.is_available():
        sys.exit("bench.py needs an MI355X GPU")
    thiim.lib()
    n = args.size
    log(f"[bench] generating {n}^3 workload")
    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200 if n >= 128 else 0)
    N = n ** 3
    # inputs resident in HBM before any timed region
    dev = inputs.Problem(**{**pb.__dict__})
    dev.eps = torch.from_numpy(pb.eps).cuda()
    dev.sources = {k: torch.from_numpy(v).cuda() for k, v in pb.sources.items()}
    torch.cuda.synchronize()

    if args.calib_copy:
        a = torch.empty(2 ** 32, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 4 GiB read + 4 GiB written")
        del a, b
        torch.cuda.empty_cache()

    results = {}
    for kernel in [args.kernel] + [k for k in args.compare.split(",") if k and k != args.kernel]:
        step_ms, iter_ms, res = time_kernel_run(torch, thiim, dev, kernel, args.iters,
                                                args.steps if kernel == args.kernel else 1,
                                                args.warmup if kernel == args.kernel else 1)
        results[kernel] = (step_ms, iter_ms, res)
        torch.cuda.empty_cache()

    step_ms, iter_ms, res = results[args.kernel]
    ms_per_step = sum(step_ms) / len(step_ms)
    it_ms = sum(iter_ms) / len(iter_ms)
    glups = N * args.iters / (ms_per_step * 1e-3) / 1e9
    # dominant kernel: the sweep (two launches per iteration for naive, one per
    # iteration for fused, one per two iterations for blocked)
    ipl = ITERS_PER_LAUNCH[args.kernel]
    bytes_per_launch = BYTES_PER_LUP[args.kernel] * N * ipl
    achieved = bytes_per_launch / (it_ms * ipl * 1e-3) / 1e9
    extra = {}
    for k, (sm, im, r) in results.items():
        extra[k] = {"ms_per_iteration": sum(im) / len(im),
                    "sweep_glups": N / (sum(im) / len(im) * 1e-3) / 1e9,
                    "alg_bytes_per_lup": BYTES_PER_LUP[k],
                    "final_rel_residual": r}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(pb)
    out = {
        "metric": "THIIM GLUP/s (512^3, complex128, 100 iterations)",
        "value": glups,
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"thiim_{n}x{n}x{n}_layered_textured_spheres_pml6",
                   "iterations": args.iters, "kernel": args.kernel,
                   "precision": "fp64 complex"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": cpu,
        "kernels": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
