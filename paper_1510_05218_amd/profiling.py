"""Summaries of rocprofv3 output for the THIIM sweeps.

* ``kernel_stats_md``: the ``--kernel-trace --stats`` CSV as a markdown table
  with achieved algorithmic bandwidth per kernel.
* ``counters_md``: occupancy, wait shares and instruction mix per kernel from
  ``--pmc`` runs of SQ counters and MeanOccupancyPerCU.
* ``traffic_summary``: per-dispatch ``FETCH_SIZE`` / ``WRITE_SIZE`` (KiB) from
  two ``--pmc`` runs, each scaled by what the same counter reads for a plain
  device copy of known size run in the same process (the calibration copy of
  ``bench.py --calib-copy``).  The result records a hash of the kernel
  sources; ``bench.py`` reports the traffic only while that hash matches.

* ``run_kernels``: the workload of the counter runs -- every sweep kernel on
  the n^3 benchmark problem from a dense random state.
* ``run_mixed``: a GPU workload for profiling the complex64 inner sweeps --
  two defect-correction steps of the mixed-precision solver on the n^3
  benchmark problem, with T = 2 and with T = 3 inner passes.
* ``run_solve``: time to relative residual 1e-8 on the n^3 benchmark
  problem, mixed solver against the plain FP64 iteration.
* ``run_c3``: the mixed solver on the n^3 benchmark problem to 1e-8 and on
  to 1e-10; the error of the 1e-8 solution against the 1e-10 one.
* ``run_c5``: time to the adjoint gradient on the 128 x 128 x 256 stack.
* ``run_spectral``: the full batched spectral sweep (32 wavelengths x 4
  geometries up to 192 x 192 x 384) to 1e-8 in resident waves.

Usage:
    python -m paper_1510_05218_amd.profiling traffic FETCH.csv WRITE.csv N OUT.json CMD [FS WS]
    python -m paper_1510_05218_amd.profiling stats STATS.csv N OUT.md CMD [NAME,NAME...]
    python -m paper_1510_05218_amd.profiling counters SQ.csv OCC.csv OUT.md CMD [NAME,...]
    python -m paper_1510_05218_amd.profiling run_kernels [n]
    python -m paper_1510_05218_amd.profiling run_mixed [n]
    python -m paper_1510_05218_amd.profiling run_solve [n]
    python -m paper_1510_05218_amd.profiling run_c3 [n]
    python -m paper_1510_05218_amd.profiling run_c5
    python -m paper_1510_05218_amd.profiling run_spectral [waves]
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 2 ** 32  # the calibration copy reads and writes 4 GiB

# Algorithmic HBM bytes per cell and launch (each value read or written once;
# Src arrays only on source planes, so not counted); see bench.py.  Keys are
# kernel names as short_name() prints them.
ALG_BYTES_PER_CELL = {
    # FP64 sweeps, complex128 (16 B per value)
    "k_naive_h<FullCoefs>": 480,             # 12 t/c + 12 fields read, 6 written
    "k_naive_e<FullCoefs>": 480,
    "k_naive_h<CompactCoefs>": 288,          # 12 fields read, 6 written
    "k_naive_e<CompactCoefs>": 304,          # + eps
    "k_fused<64,8,FullCoefs>": 768,          # 24 t/c + 12 read, 12 written
    "k_fused<64,8,CompactCoefs>": 400,       # eps + 12 read, 12 written
    # (k_fused_res, the fused pass that forms the residual on the way, moves
    # the same bytes per cell, but thiim_create also launches it on the few
    # planes a source reaches: its average launch covers no fixed cell count)
    # full storage: each stage reads its planes' 24 t/c arrays
    "k_blocked<64,8,2,Pol64<FullCoefs>>": 1152,
    "k_blocked<32,16,2,Pol64<CompactCoefs>>": 400,
    "k_blocked<64,8,2,Pol64<CompactCoefs>>": 400,
    # transposed sweep: 12 lam + eps + 3 g read, 12 written
    "k_adjoint<64,8,AdjPol64<false>>": 448,
    # batched passes: the same per-cell bytes, over all problems of a launch
    "k_blocked_batch<32,16,2>": 400,
    "k_fused_batch<64,8>": 400,
    # with a source on every part (defect correction): 12 lam + eps + 12 G
    "k_adjoint<64,8,AdjPol64<true>>": 592,
    # complex64 transposed inner sweep: 12 lam + 16 B record + 12 G read,
    # 12 lam written
    "k_adjoint<64,8,AdjPol32>": 304,
    # its two-iteration blocked form (per pass) keeps lam, its source and the
    # window sum in pair-equal form (a symmetric pair stored once): the bytes
    # of the forward inner passes, 162 at 512^3 (165 at 128 x 128 x 256, where
    # the PML planes weigh more), 258 for the instances that also sum into the
    # window accumulator
    "k_adjoint32_blocked<32,24,2,false,true>": 162,
    "k_adjoint32_blocked<32,24,2,true,true>": 258,
    "k_adjoint32_blocked<32,16,2,false,false>": 162,
    # complex64 inner sweeps (8 B per value) in pair-sum form: per H and E
    # side 3 d + 3 r read and 3 d written where the split pairs are symmetric,
    # 5 of each on the PML planes, + the 16 B record: 160 B off the PML, 162
    # at 512^3 with 6-plane PMLs (13 H and 12 E planes not symmetric)
    "k_blocked<32,16,3,Pol32>": 162,
    "k_blocked<32,32,2,Pol32R>": 162,
    # two-sweep passes with the pass source r_T = (I + M) r read once, at the
    # last stage (the same algorithmic bytes)
    "k_blocked<32,32,2,Pol32L>": 162,
    "k_inner32_batch<32,24,2,Pol32L>": 162,
    "k_inner32_batch<32,16,3,Pol32>": 162,
    # the last Kp passes of a correction also read and write the window sum
    # (6 complex64 values in pair-sum form): + 96 B
    "k_blocked<32,32,2,WithAcc<Pol32L>>": 258,
    "k_blocked<32,16,3,WithAcc<Pol32>>": 258,
    "k_inner32_batch<32,24,2,WithAcc<Pol32L>>": 258,
    "k_inner32_batch<32,16,3,WithAcc<Pol32>>": 258,
}


def code_balance(rx, ry, t, b_read, b_write, nx, ny):
    """Modelled HBM bytes per lattice-site update of a temporally blocked
    sweep with overlapped tiles (the GPU form of the paper's Eq. 12): regions
    of rx x ry columns store their centre (rx - 2t) x (ry - 2t) after t
    iterations per pass; each pass reads b_read bytes for every region cell
    (ring included, tiles rounded up to cover nx x ny) and writes b_write
    bytes per stored cell."""
    ox, oy = rx - 2 * t, ry - 2 * t
    tiles_x, tiles_y = -(-nx // ox), -(-ny // oy)
    read_per_cell = b_read * tiles_x * tiles_y * rx * ry / (nx * ny)
    return (read_per_cell + b_write) / t


# The temporally blocked sweeps of the measured bytes-per-update table: name,
# storage / precision, iterations per pass T, region (rx, ry), bytes read per
# region column and pass (b_read), bytes written per stored column (b_write)
# -- the GPU form of the paper's code-balance model, Eq. 12 -- with T = 1 the
# fused single-iteration sweep (its halo is a one-column ring of E sums).
BALANCE_CASES = [
    ("k_fused<64,8,CompactCoefs>", "FP64 compact", 1, None, 208, 192),
    ("k_blocked<32,16,2,Pol64<CompactCoefs>>", "FP64 compact", 2, (32, 16), 208, 192),
    ("k_fused<64,8,FullCoefs>", "FP64 40-array", 1, None, 576, 192),
    # each stage reads its planes' 24 t/c arrays: 12 fields + 2 x 24 t/c
    ("k_blocked<64,8,2,Pol64<FullCoefs>>", "FP64 40-array", 2, (64, 8), 960, 192),
    # complex64 pair-sum form off the PML: d 48 + source 48 + record 16 read,
    # d 48 written; the two-sweep form reads the record at both stages (+16)
    ("k_blocked<32,32,2,Pol32L>", "complex64 inner", 2, (32, 32), 128, 48),
    ("k_blocked<32,16,3,Pol32>", "complex64 inner", 3, (32, 16), 112, 48),
]


def balance_table(traffic_json, n=512):
    """Markdown table: measured counter bytes per lattice update of each
    sweep in BALANCE_CASES (rocprofv3 FETCH_SIZE + WRITE_SIZE per launch / T /
    cells, from a traffic summary) against the overlapped-tile code-balance
    model at n x n planes (T = 1: bytes read + written per cell)."""
    t = json.load(open(traffic_json))
    lines = ["| sweep | storage / precision | T | region | model B/LUP | measured B/LUP | "
             "measured / model |", "|---|---|---|---|---|---|---|"]
    rows = []
    for name, what, T, region, br, bw in BALANCE_CASES:
        k = t["kernels"].get(name)
        if k is None:
            continue
        model = (br + bw) if region is None else code_balance(region[0], region[1], T, br, bw,
                                                              n, n)
        meas = k["bytes_per_cell"] / T
        rows.append((name, what, T, region, model, meas))
        reg = "-" if region is None else f"{region[0]} x {region[1]}"
        lines.append(f"| {name} | {what} | {T} | {reg} | {model:.1f} | {meas:.1f} | "
                     f"{meas / model:.2f} |")
    return "\n".join(lines) + "\n", rows


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def short_name(kernel_name: str) -> str:
    """'void thiim::k_blocked<32, 16, 2, thiim::Pol64<thiim::CompactCoefs> >(...)'
    -> 'k_blocked<32,16,2,Pol64<CompactCoefs>>'."""
    n = kernel_name.split("(")[0].replace("void ", "").replace("thiim::", "")
    return n.replace(" ", "").strip()


def _per_kernel(path):
    agg = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            agg[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]) * 1024.0)
    return agg


def _calibration(agg, expected):
    for name, vals in agg.items():
        if "copyBuffer" in name or "copy_kernel" in name or "elementwise_kernel" in name:
            big = max(vals)
            if big > 0.25 * expected:
                return big / expected
    raise RuntimeError("calibration copy not found in the counter file")


def traffic_summary(fetch_csv, write_csv, n_cells, out_json, command, scales=None):
    """scales = (fetch, write) counter factors measured in another run of the
    same part, for runs without a calibration copy."""
    fetch, write = _per_kernel(fetch_csv), _per_kernel(write_csv)
    if scales is None:
        f_scale = _calibration(fetch, CALIB_BYTES)
        w_scale = _calibration(write, CALIB_BYTES)
    else:
        f_scale, w_scale = scales
    kernels = {}
    for name in sorted(set(fetch) & set(write)):
        if not name.startswith("k_"):
            continue
        fb = sum(fetch[name]) / len(fetch[name]) / f_scale
        wb = sum(write[name]) / len(write[name]) / w_scale
        kernels[name] = {
            "dispatches": len(fetch[name]),
            "read_bytes_per_launch": fb,
            "write_bytes_per_launch": wb,
            "bytes_per_launch": fb + wb,
            "bytes_per_cell": (fb + wb) / n_cells,
            "alg_bytes_per_cell": ALG_BYTES_PER_CELL.get(name),
        }
    out = {"source_hash": source_hash(), "cells": n_cells,
           "fetch_counter_scale": f_scale, "write_counter_scale": w_scale,
           "command": command, "kernels": kernels}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def kernel_stats_md(stats_csv, n_cells, out_md, command, only=None):
    """only: comma-separated substrings; keep the kernels whose name holds one
    (n_cells must then be the cells one launch of each kept kernel covers)."""
    rows = list(csv.DictReader(open(stats_csv)))
    if only:
        keys = only.split(",")
        rows = [r for r in rows if any(k in r["Name"] for k in keys)]
    lines = ["# THIIM kernels: rocprofv3 kernel statistics", "",
             "Command:", "", "```", command, "```", "",
             (f"Grid: {n_cells} cells.  Achieved = algorithmic bytes per launch / average "
              "duration." if n_cells > 1 else
              "Launches over problem sets of different sizes: no bandwidth computed."), "",
             "| kernel | calls | avg (ms) | min (ms) | max (ms) | alg. B/cell | achieved GB/s |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = short_name(r["Name"])
        avg = float(r["AverageNs"]) / 1e6
        b = ALG_BYTES_PER_CELL.get(name)
        gbs = f"{b * n_cells / (avg * 1e-3) / 1e9:.0f}" if b and n_cells > 1 else "-"
        lines.append(f"| {name} | {r['Calls']} | {avg:.3f} | {float(r['MinNs']) / 1e6:.3f} | "
                     f"{float(r['MaxNs']) / 1e6:.3f} | {b if b else '-'} | {gbs} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters_md(sq_csv, occ_csv, out_md, command, only=None):
    """Per-kernel averages of a ``--pmc`` run of the SQ counters (waves, wave
    cycles, cycles waiting on memory / on instruction issue, VALU and LDS
    instructions, LDS bank conflicts) and of one of MeanOccupancyPerCU, as a
    markdown table: waves resident per CU, the share of wave time spent
    waiting, VALU instructions per wave, and LDS instructions and bank
    conflicts per wave."""
    def load(path):
        agg = defaultdict(lambda: defaultdict(list))
        for r in csv.DictReader(open(path)):
            agg[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return agg

    sq, occ = load(sq_csv), load(occ_csv)
    keys = sorted(k for k in sq if k.startswith("k_"))
    if only:
        keys = [k for k in keys if any(o in k for o in only.split(","))]
    lines = ["# THIIM kernels: occupancy, waits and instruction mix (rocprofv3 --pmc)", "",
             "Command (one run per counter set):", "", "```", command, "```", "",
             "Per launch, averaged over launches: occupancy = MeanOccupancyPerCU (waves "
             "resident per CU, of at most 32); wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES (share "
             "of wave time waiting on memory or LDS counters); issue = "
             "SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (waiting for an instruction to issue); "
             "VALU, LDS = instructions per wave; conflicts = SQ_LDS_BANK_CONFLICT cycles "
             "per wave.", "",
             "| kernel | launches | waves | occupancy | wait | issue | VALU/wave | LDS/wave | "
             "conflicts/wave |", "|---|---|---|---|---|---|---|---|---|"]
    for k in keys:
        d = sq[k]

        def g(c, d=d):
            return sum(d[c]) / len(d[c]) if c in d else float("nan")

        waves = g("SQ_WAVES")
        o = occ.get(k, {}).get("MeanOccupancyPerCU", [])
        oc = f"{sum(o) / len(o):.1f}" if o else "-"
        lines.append(f"| {k} | {len(d['SQ_WAVES'])} | {waves:.0f} | {oc} | "
                     f"{g('SQ_WAIT_ANY') / g('SQ_WAVE_CYCLES'):.2f} | "
                     f"{g('SQ_WAIT_INST_ANY') / g('SQ_WAVE_CYCLES'):.2f} | "
                     f"{g('SQ_INSTS_VALU') / waves:.0f} | {g('SQ_INSTS_LDS') / waves:.0f} | "
                     f"{g('SQ_LDS_BANK_CONFLICT') / waves:.0f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def run_kernels(n=512, m=180):
    """Workload of the counter runs: a calibration copy of 4 GiB, then every
    sweep kernel on the n^3 benchmark problem from a dense state (unit-variance random fields, so that no part
    of the grid holds zeros), a few launches each -- the FP64 naive, fused
    and blocked sweeps on compact and on the 28-array storage, then one
    mixed-precision correction (m inner sweeps) with two- and with
    three-sweep inner passes.  Prints one line per block."""
    import torch

    from . import inputs, thiim

    # the counters' calibration: a plain copy of CALIB_BYTES (read and written)
    a = torch.empty(CALIB_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200 if n >= 128 else 0)
    dev = inputs.Problem(**{**pb.__dict__})
    dev.eps = torch.from_numpy(pb.eps).cuda()
    dev.sources = {k: torch.from_numpy(v).cuda() for k, v in pb.sources.items()}

    def dense(s):
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        shape = (12, n, n, n)
        x = torch.complex(torch.randn(shape, dtype=torch.float64, device="cuda", generator=g),
                          torch.randn(shape, dtype=torch.float64, device="cuda", generator=g))
        s.set_fields(x)
        del x
        torch.cuda.empty_cache()

    for storage in ("compact", "full"):
        for kernel, its in (("naive", 2), ("fused", 4), ("blocked", 8)):
            s = thiim.Solver(dev, storage=storage, kernel=kernel)
            dense(s)
            s.iterate(its)
            torch.cuda.synchronize()
            s.close()
            torch.cuda.empty_cache()
            print(json.dumps({"storage": storage, "kernel": kernel, "iterations": its}),
                  flush=True)
    for t_block in (0, 3):
        s = thiim.Solver(dev, storage="compact", precision="mixed", t_block=t_block)
        dense(s)
        s.solve(1e-30, 1 + m, m)
        torch.cuda.synchronize()
        s.close()
        torch.cuda.empty_cache()
        print(json.dumps({"mixed_t_block": t_block, "inner_sweeps": m}), flush=True)


def run_mixed(n=512):
    """Two correction steps (FP64 residual sweep + 40 / 60 inner sweeps) of
    the mixed solver with T = 2 and T = 3 inner passes on the n^3 problem."""
    import time

    import torch

    from . import inputs, thiim

    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200 if n >= 128 else 0)
    dev = inputs.Problem(**{**pb.__dict__})
    dev.eps = torch.from_numpy(pb.eps).cuda()
    dev.sources = {k: torch.from_numpy(v).cuda() for k, v in pb.sources.items()}
    for T, m in ((2, 41), (3, 61)):
        s = thiim.Solver(dev, storage="compact", precision="mixed", t_block=T)
        torch.cuda.synchronize()
        t = time.time()
        rc, it, r = s.solve(1e-30, 2, m)
        torch.cuda.synchronize()
        print(json.dumps({"T": T, "sweeps": it, "s": round(time.time() - t, 3)}), flush=True)
        s.close()
        torch.cuda.empty_cache()


def run_solve_512(n=512, tol=1e-8, fp64_budget=40000):
    """Time to solution on the n^3 benchmark workload (textured, 200 lossless
    spheres): the mixed solver (2000 inner sweeps per correction) to
    tol, then the plain FP64 iteration to tol or fp64_budget iterations.  Both
    run in slices so that every slice prints its progress."""
    import time

    import torch

    from . import inputs, thiim

    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200 if n >= 128 else 0)
    dev = inputs.Problem(**{**pb.__dict__})
    dev.eps = torch.from_numpy(pb.eps).cuda()
    dev.sources = {k: torch.from_numpy(v).cuda() for k, v in pb.sources.items()}
    out = {"grid": f"{n}^3", "tol": tol}
    m = 2000
    s = thiim.Solver(dev, storage="compact", precision="mixed")
    torch.cuda.synchronize()
    t0 = time.time()
    sweeps, r = 0, 1.0
    while r > tol and sweeps < 400000:
        rc, it, r = s.solve(tol, 3 * (m + 1), m)
        sweeps += it
        print(json.dumps({"mixed_sweeps": sweeps, "rel_res": r, "s": round(time.time() - t0, 1)}),
              flush=True)
    out["mixed"] = {"sweeps": sweeps, "rel_res": r, "seconds": time.time() - t0}
    xm = s.fields()
    pm = xm[0::2] + xm[1::2]
    del xm
    s.close()
    torch.cuda.empty_cache()
    s = thiim.Solver(dev, storage="compact")
    torch.cuda.synchronize()
    t0 = time.time()
    its, r = 0, 1.0
    while r > tol and its < fp64_budget:
        rc, it, r = s.solve(tol, 2000, 500)
        its += it
        print(json.dumps({"fp64_iterations": its, "rel_res": r, "s": round(time.time() - t0, 1)}),
              flush=True)
    out["fp64"] = {"iterations": its, "rel_res": r, "seconds": time.time() - t0}
    x64 = s.fields()
    p64 = x64[0::2] + x64[1::2]
    del x64
    out["physical_rel_diff"] = float(torch.linalg.vector_norm(pm - p64) /
                                     torch.linalg.vector_norm(p64))
    s.close()
    print(json.dumps(out), flush=True)


def run_c3(n=512, tol=1e-8, ref_tol=1e-10, m=2000):
    """The mixed solver (m inner sweeps per correction) on the n^3
    benchmark workload to tol, then the same context on to ref_tol: the
    second iterate is the FP64 fixed point to ref_tol (its residual is the
    FP64 one), and the relative 2-norm difference of the physical fields is
    the error of the tol solution.  Slices of three corrections print their
    progress."""
    import time

    import torch

    from . import inputs, thiim

    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200 if n >= 128 else 0)
    dev = inputs.Problem(**{**pb.__dict__})
    dev.eps = torch.from_numpy(pb.eps).cuda()
    dev.sources = {k: torch.from_numpy(v).cuda() for k, v in pb.sources.items()}
    out = {"grid": f"{n}^3", "tol": tol, "ref_tol": ref_tol, "inner_sweeps": m}
    s = thiim.Solver(dev, storage="compact", precision="mixed")
    torch.cuda.synchronize()
    t0 = time.time()
    sweeps, r, snap = 0, 1.0, None
    for goal in (tol, ref_tol):
        while r > goal and sweeps < 1000000:
            rc, it, r = s.solve(goal, 3 * (m + 1), m)
            sweeps += it
            print(json.dumps({"sweeps": sweeps, "rel_res": r, "s": round(time.time() - t0, 1)}),
                  flush=True)
        out[f"to_{goal:g}"] = {"sweeps": sweeps, "rel_res": r, "seconds": time.time() - t0}
        x = s.fields()
        p = x[0::2] + x[1::2]
        del x
        if snap is None:
            snap = p
        else:
            out["error_vs_ref"] = float(torch.linalg.vector_norm(snap - p) /
                                        torch.linalg.vector_norm(p))
        torch.cuda.empty_cache()
    s.close()
    print(json.dumps(out), flush=True)


def run_c5(tol=1e-10, m=2000):
    """Time to the gradient on the adjoint configuration: a 128 x 128 x 256
    textured stack (seed 20, eps'' in [0.1, 0.5]), J over the middle layer;
    the forward state by the mixed solver and the adjoint by averaged defect
    correction with complex64 inner sweeps, both to tol."""
    import time

    import numpy as np
    import torch

    from . import inputs, thiim

    pb = inputs.solar_cell(128, 128, 256, seed=20, npml=6, loss_range=(0.1, 0.5))
    w = (pb.eps == pb.layers[1][2]).astype(np.float64)
    s = thiim.Solver(pb, storage="compact", precision="mixed", adjoint=True)
    torch.cuda.synchronize()
    t0 = time.time()
    rc, n_fw, r = s.solve(tol, 2000000, m)
    t1 = time.time()
    rc2, J, grad, n_adj, ar = s.adjoint_grad(w, tol=tol, max_it=2000000, check_every=m)
    t2 = time.time()
    s.close()
    print(json.dumps({"grid": "128x128x256", "tol": tol, "forward_status": rc,
                      "forward_sweeps": n_fw, "forward_s": t1 - t0, "adjoint_status": rc2,
                      "adjoint_sweeps": n_adj, "adjoint_s": t2 - t1, "J": J,
                      "gradient_total_s": t2 - t0}), flush=True)


SPECTRAL_GEOMETRIES = [(64, 64, 64, 10), (96, 96, 128, 11), (128, 128, 256, 12),
                       (192, 192, 384, 13)]


def run_spectral(waves_spec="0,1,2:3a:3b:3c", n_wl=32, tol=1e-8, m=2000):
    """The batched spectral sweep: n_wl wavelengths 300-1100 nm x the four
    seeded geometries, solved to tol by the batched mixed-precision solver in
    resident waves (a wave is a list of geometry indices; '3a', '3b', '3c'
    split geometry 3's wavelengths in three), each wave in slices of three
    corrections so that every slice prints its progress."""
    import time

    import torch

    from . import inputs, thiim

    wls = [300.0 + 800.0 * i / (n_wl - 1) for i in range(n_wl)]
    total_t, total_cells, solved = 0.0, 0, 0
    for wave in waves_spec.split(":"):
        probs = []
        for part in wave.split(","):
            gi = int(part[0])
            sel = wls
            if len(part) > 1:
                j = "abc".index(part[1])
                sel = wls[j::3]
            nx, ny, nz, seed = SPECTRAL_GEOMETRIES[gi]
            probs += [inputs.solar_cell(nx, ny, nz, seed=seed, npml=6, wavelength_nm=wl)
                      for wl in sel]
        cells = sum(p.eps.size for p in probs)
        t0 = time.time()
        bt = thiim.Batch(probs, precision="mixed")
        res = None
        while res is None or res.max() > tol:
            rc, its, res = bt.solve(tol, 3 * (m + 1), m)
            print(json.dumps({"wave": wave, "problems": len(probs), "converged":
                              int((res <= tol).sum()), "max_res": float(res.max()),
                              "s": round(time.time() - t0, 1)}), flush=True)
        bt.synchronize()
        dt = time.time() - t0
        bt.close()
        torch.cuda.empty_cache()
        total_t += dt
        total_cells += cells
        solved += len(probs)
        print(json.dumps({"wave_done": wave, "cells": cells, "seconds": dt}), flush=True)
    print(json.dumps({"problems": solved, "cells": total_cells, "seconds": total_t,
                      "solves_per_s": solved / total_t}), flush=True)


def main(argv):
    if argv[0] == "traffic":
        fetch, write, n, out, cmd = argv[1:6]
        scales = (float(argv[6]), float(argv[7])) if len(argv) > 7 else None
        print(json.dumps(traffic_summary(fetch, write, int(n), out, cmd, scales), indent=1))
    elif argv[0] == "stats":
        stats, n, out, cmd = argv[1:5]
        kernel_stats_md(stats, int(n), out, cmd, argv[5] if len(argv) > 5 else None)
        print(open(out).read())
    elif argv[0] == "balance":
        md, _ = balance_table(argv[1])
        print(md)
    elif argv[0] == "counters":
        sq, occ, out, cmd = argv[1:5]
        counters_md(sq, occ, out, cmd, argv[5] if len(argv) > 5 else None)
        print(open(out).read())
    elif argv[0] == "run_kernels":
        run_kernels(int(argv[1]) if len(argv) > 1 else 512)
    elif argv[0] == "run_mixed":
        run_mixed(int(argv[1]) if len(argv) > 1 else 512)
    elif argv[0] == "run_solve":
        run_solve_512(int(argv[1]) if len(argv) > 1 else 512)
    elif argv[0] == "run_c3":
        run_c3(int(argv[1]) if len(argv) > 1 else 512)
    elif argv[0] == "run_c5":
        run_c5()
    elif argv[0] == "run_spectral":
        run_spectral(argv[1] if len(argv) > 1 else "0,1,2:3a:3b:3c")
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
