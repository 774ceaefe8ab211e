"""Throughput benchmark of the batched BDF solver on one MI355X.

One step = one full solve of a batch of cells of the 500-species /
6000-reaction network from t = 0 to t_end (rates, starting step, every BDF
step attempt with its Newton-matrix factorisations, Newton iterations and
step control), inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--cells C] [--precision fp64|fp32_lu]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3


def _oracle_cell(args):
    net_name, cells, i = args
    import synth
    from oracle import bdf, chem
    net = synth.network_for_config(net_name)
    ch = chem.cell_chemistry(net, cells.cell(i))
    r = bdf.solve(ch, cells.x0[i], cells.t_end[i], 1e-6, 1e-20)
    return r.status


def cpu_baseline(net_name, cells, n_sample):
    """The oracle, untuned, one cell per process on the host cores."""
    procs = max(1, min(os.cpu_count() or 1, 16, n_sample))
    import synth  # noqa: F401  (warm the network cache before forking)
    synth.network_for_config(net_name)
    sample = cells.subset(np.arange(n_sample))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs, initializer=_single_thread_blas) as pool:
        st = pool.map(_oracle_cell, [(net_name, sample, i) for i in range(n_sample)])
    wall = time.perf_counter() - t0
    ok = sum(1 for s in st if s == 0)
    return {"value": ok / wall, "unit": "cell-solves/s", "cores": procs, "kind": "oracle",
            "sample": f"first {n_sample} cells of the timed batch, one process per cell, wall {wall:.1f} s"}


def _single_thread_blas():
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["OMP_NUM_THREADS"] = "1"


def recorded_traffic():
    """Per-unit HBM bytes from the last rocprofv3 counter passes (profiles/traffic.json),
    or None when the kernel sources have changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.join(ROOT, "profiles"))
    import summarize
    rec = json.load(open(path))
    return rec if rec.get("source_hash") == summarize.source_hash() else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=4096)
    ap.add_argument("--network", default="net500", choices=["small", "net200", "net500"])
    ap.add_argument("--t-end-yr", type=float, default=1e6)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_lu"])
    ap.add_argument("--seed", type=int, default=3001)
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one elementwise kernel reading and writing 256 MiB "
                         "(a reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the cells are independent and this build runs on one "
              "MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_10558_amd as ab
    import synth

    dev = torch.device("cuda:0")
    net = synth.network_for_config(args.network)
    cells = synth.sample_cells(net, args.cells, seed=args.seed, t_end_yr=args.t_end_yr)
    g = ab.Network.from_text(net.to_text())
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    inp = [t(cells.T), t(cells.n_H), t(cells.A_V), t(cells.zeta), t(cells.G0), t(cells.x0), t(cells.t_end)]
    opts = ab.make_options(rtol=1e-6, atol=1e-20, precision=args.precision)

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)     # elementwise kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        ab.solve(g, *inp, options=opts)
    torch.cuda.synchronize()
    ab.profile_read(reset=True)
    ab.profile_enable(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, status, st = ab.solve(g, *inp, options=opts, with_stats=True)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ab.profile_enable(False)
    prof = ab.profile_read(reset=True)

    ok = int((status == 0).sum().item())
    total = ok * args.steps
    value = total / wall
    S, R = net.n_species, net.n_reactions
    allst = np.concatenate(stats)
    n_lu = float(allst["n_lu"].sum())
    n_newton = float((allst["n_rhs"] - 2).sum())
    n_att = float(allst["n_attempts"].sum())
    # algorithmic work per unit
    lu_flop = 2.0 / 3.0 * S ** 3                      # one factorisation
    elt = 8 if args.precision == "fp64" else 4
    newton_bytes = S * S * elt                         # factor read by the triangular solves
    rhs_bytes = (2 * S + R) * 8                        # x and k read, residual written
    control_bytes = 2 * 8 * S * 8                      # difference table read + write
    kern = {}
    for name, (launches, ms) in prof.items():
        kern[name] = {"launches": launches, "ms": round(ms, 3)}
    dom = max(("factor", "newton", "control", "rhs"), key=lambda k: prof[k][1])
    if dom == "factor":
        peak = FP64_MFMA_PEAK_TFLOPS if args.precision == "fp64" else FP32_MFMA_PEAK_TFLOPS
        ach = n_lu * lu_flop / (prof["factor"][1] * 1e-3) / 1e12
        roof = {"kernel": "k_factor", "bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": None}
    elif dom == "newton":
        ach = n_newton * newton_bytes / (prof["newton"][1] * 1e-3) / 1e9
        roof = {"kernel": "k_newton_solve", "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    elif dom == "rhs":
        ach = n_newton * rhs_bytes / (prof["rhs"][1] * 1e-3) / 1e9
        roof = {"kernel": "k_newton_rhs", "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    else:
        ach = n_att * control_bytes / (prof["control"][1] * 1e-3) / 1e9
        roof = {"kernel": "k_control", "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    rec = recorded_traffic()
    if rec is not None and args.precision == "fp64":
        if roof["kernel"] == "k_factor":
            roof["traffic"] = round(rec["k_factor_bytes_per_lu"] * n_lu / max(1, prof["factor"][0]))
        elif roof["kernel"] == "k_newton_solve":
            roof["traffic"] = round(rec["k_newton_solve_bytes_per_iteration"] * n_newton / max(1, prof["newton"][0]))
        roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    # secondary figures for the other two hot kernels
    if prof["factor"][1] > 0:
        kern["factor"]["tflops"] = round(n_lu * lu_flop / (prof["factor"][1] * 1e-3) / 1e12, 3)
    if prof["newton"][1] > 0:
        kern["newton"]["gbs"] = round(n_newton * newton_bytes / (prof["newton"][1] * 1e-3) / 1e9, 1)
    if prof["rhs"][1] > 0:
        kern["rhs"]["gbs"] = round(n_newton * rhs_bytes / (prof["rhs"][1] * 1e-3) / 1e9, 1)

    out = {
        "metric": "cell-solves/sec to t_end at rtol 1e-6, 500-sp net",
        "value": round(value, 3),
        "unit": "cell-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (f32 LU)",
        "data": "synthetic",
        "config": {"workload": f"{args.network}: {S} species / {R} reactions, batch of {args.cells} cells, "
                               f"t_end {args.t_end_yr:g} yr, rtol 1e-6 atol 1e-20, {args.precision} Newton LU",
                   "cells": args.cells, "species": S, "reactions": R, "precision": args.precision,
                   "parallelism": "one GPU, cells across workgroups"},
        "work": {"cells_ok": ok, "factorisations": int(n_lu), "newton_iterations": int(n_newton),
                 "step_attempts": int(n_att)},
        "kernels": kern,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        n = min(args.cpu_sample, args.cells)
        out["cpu_baseline"] = cpu_baseline(args.network, cells, n)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
