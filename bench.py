"""Throughput benchmark of the batched BDF solver on one MI355X.

One step = one full solve of a batch of cells of the 500-species /
6000-reaction network from t = 0 to t_end (rates, starting step, every BDF
step attempt with its Newton-matrix factorisations, Newton iterations and
step control), inputs resident in HBM.  After the timed steps the default run
also serves a Poisson request stream on the same network in both precision
forms (throughput with p50/p99 latency) and times the right-hand-side kernel
on its own.  Prints one JSON line.

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
    return i, r.status, r.x


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(net_name, cells, n_sample):
    """The oracle, untuned, one cell per single-threaded process on the host
    cores (at most 16 processes).  Called before anything touches the GPU, so
    the worker processes are forked from a process without GPU state.  Returns
    the baseline record and the oracle's abundances of the sampled cells."""
    procs = max(1, min(os.cpu_count() or 1, 16, n_sample))
    import synth  # noqa: F401  (warm the network cache before forking)
    synth.network_for_config(net_name)
    sample = cells.subset(np.arange(n_sample))
    t0 = time.perf_counter()
    res = [None] * n_sample
    with mp.get_context("fork").Pool(procs, initializer=_single_thread_blas) as pool:
        for k, (i, st, x) in enumerate(pool.imap_unordered(_oracle_cell, [(net_name, sample, i)
                                                                         for i in range(n_sample)])):
            res[i] = (st, x)
            print(f"[bench] oracle cell {k + 1}/{n_sample} done at {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    ok = sum(1 for s, _ in res if s == 0)
    rec = {"value": ok / wall, "unit": "cell-solves/s", "cores": procs, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"first {n_sample} cells of the timed batch, {procs} single-threaded processes "
                     f"(one cell per task), wall {wall:.1f} s"}
    return rec, np.array([x for _, x in res])


def max_rel_err(x, ref, floor=1e-12):
    """max |x - ref| / ref over entries with ref > floor (the abundance parity measure)."""
    m = ref > floor
    return float(np.max(np.abs(x[m] - ref[m]) / ref[m])) if m.any() else 0.0


def _single_thread_blas():
    # one BLAS / OpenMP thread per worker process: the environment covers
    # libraries loaded later, threadpool_limits those already loaded
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import scipy.linalg  # noqa: F401
    import scipy.sparse  # noqa: F401
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def recorded_traffic():
    """Per-unit HBM bytes from the last rocprofv3 counter passes (profiles/traffic.json),
    or None when the kernel sources have changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_2511_10558_amd import profile_summary
    rec = json.load(open(path))
    return rec if rec.get("source_hash") == profile_summary.source_hash() else None


def serve_stream(args, net, g, n_requests, precisions):
    """Poisson arrivals of requests of 1..1024 cells with horizons log-uniform
    in 1e3..1e7 yr on one server per precision form.  A closed-loop pass (every
    request queued at once) gives the saturated throughput; the open-loop pass
    offers 0.8 of it (unless --rate is given) and yields the latency
    percentiles.  Returns the record of every pass."""
    import paper_2511_10558_amd as ab
    import synth
    reqs = synth.request_stream(net, n_requests, seed=args.seed, rate_per_s=1.0)
    warm = synth.request_stream(net, 16, seed=args.seed + 1, rate_per_s=1.0)
    unit_arrivals = np.array([r.arrival_s for r in reqs])
    n_cells = sum(r.cells.n for r in reqs)
    mean_cells = n_cells / len(reqs)

    def submit(srv, cells):
        return srv.submit(cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0, cells.x0, cells.t_end)

    def one_pass(precision, arrivals, label):
        with ab.Server(g, precision=precision, check_every=args.check_every, lu_reuse=args.lu_reuse) as srv:
            wid = [submit(srv, r.cells) for r in warm]
            got = 0
            while got < len(wid):
                got += len(srv.poll(timeout_ms=500))
            info0 = srv.info()
            t0 = srv.clock()
            ids, done, i = {}, {}, 0
            last_note = 0.0
            while len(done) < len(reqs):
                now = srv.clock() - t0
                if now - last_note > 15.0:
                    last_note = now
                    print(f"[serve] {precision} {label}: {now:.0f} s, {i} submitted, {len(done)} complete",
                          file=sys.stderr, flush=True)
                while i < len(reqs) and arrivals[i] <= now:
                    ids[submit(srv, reqs[i].cells)] = i
                    i += 1
                wait = 200 if i >= len(reqs) else max(0, min(200, int((arrivals[i] - now) * 1e3)))
                for c in srv.poll(max_n=512, timeout_ms=wait):
                    done[ids[c["id"]]] = c
            info1 = srv.info()
        t_end = max(c["t_done"] for c in done.values()) - t0
        lat = np.array([done[j]["t_done"] - (t0 + arrivals[j]) for j in range(len(reqs))])
        failed = sum(c["n_failed"] for c in done.values())
        busy = info1["busy_slot_seconds"] - info0["busy_slot_seconds"]
        return {"cell_solves_per_s": round((n_cells - failed) / t_end, 3), "window_s": round(t_end, 3),
                "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                "mean_latency_s": round(float(lat.mean()), 4), "failed_cells": int(failed),
                "slots": int(info1["slots"]), "mean_occupied_slots": round(busy / t_end, 1)}

    out = {"workload": f"{args.network} serving: {len(reqs)} Poisson requests after 16 warm-up requests, "
                       f"{n_cells} cells (1..1024 per request, mean {mean_cells:.1f}), t_end log-uniform "
                       "1e3..1e7 yr, rtol 1e-6 atol 1e-20"
                       + (f", factorisation kept while |c/c_lu - 1| <= {args.lu_reuse:g}" if args.lu_reuse else ""),
           "requests": len(reqs), "cells": n_cells, "seed": args.seed, "lu_reuse": args.lu_reuse, "passes": {}}
    # closed loops first; then every form is offered the same open-loop stream,
    # at 0.8 of the first form's saturated throughput, so that their latencies
    # compare at equal load
    rate = args.rate
    for prec in precisions:
        out["passes"][prec] = {}
        if args.rate <= 0:
            closed = one_pass(prec, np.zeros(len(reqs)), "closed loop")
            out["passes"][prec]["closed_loop"] = closed
            if rate <= 0:
                rate = 0.8 * closed["cell_solves_per_s"] / mean_cells
    out["arrival_rate_req_per_s"] = round(rate, 4)
    for prec in precisions:
        res = out["passes"][prec]
        res["open_loop"] = one_pass(prec, unit_arrivals / rate, "open loop")
        print(f"[serve] {prec}: {json.dumps(res)}", file=sys.stderr, flush=True)
    if "fp64" in out["passes"] and "fp32_lu" in out["passes"]:
        a, b = out["passes"]["fp64"], out["passes"]["fp32_lu"]
        if "closed_loop" in a:
            out["fp32_lu_speedup_saturated"] = round(b["closed_loop"]["cell_solves_per_s"] /
                                                     a["closed_loop"]["cell_solves_per_s"], 4)
        out["fp32_lu_p50_ratio_same_load"] = round(b["open_loop"]["p50_latency_s"] / a["open_loop"]["p50_latency_s"], 4)
        out["fp32_lu_p99_ratio_same_load"] = round(b["open_loop"]["p99_latency_s"] / a["open_loop"]["p99_latency_s"], 4)
    return out


def run_serve(args):
    """Serving workload on its own (--workload serve)."""
    import paper_2511_10558_amd as ab
    import synth
    net = synth.network_for_config(args.network)
    g = ab.Network.from_text(net.to_text())
    rec = serve_stream(args, net, g, args.requests, args.serve_precisions.split(","))
    first = rec["passes"][args.serve_precisions.split(",")[0]]["open_loop"]
    out = {"metric": "served cell-solves/sec (Poisson request stream, 500-sp net) with p50/p99 latency",
           "value": first["cell_solves_per_s"], "unit": "cell-solves/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "p50_latency_s": first["p50_latency_s"], "p99_latency_s": first["p99_latency_s"],
           "config": {"workload": rec.pop("workload"), "requests": rec["requests"], "cells": rec["cells"],
                      "seed": rec["seed"], "lu_reuse": rec["lu_reuse"]},
           **{k: v for k, v in rec.items() if k not in ("requests", "cells", "seed", "lu_reuse")}}
    print(json.dumps(out))


def rhs_standalone(net, g, inp, net_name, n_rep=20):
    """The right-hand-side kernel on its own (abdf_rhs over the batch's cells,
    rates from abdf_rates, abundances x0): algorithmic bytes (x and k read, f
    written) per average launch, each launch's start and end recorded as HIP
    events by its own dispatch inside the library (the rhs_eval timer
    family)."""
    import torch
    import paper_2511_10558_amd as ab
    k = ab.rates(g, *inp[:5])
    x = inp[5]
    C = x.shape[0]
    ab.rhs(g, k, x)
    torch.cuda.synchronize()
    ab.profile_read(reset=True)
    ab.profile_enable(True)
    for _ in range(n_rep):
        ab.rhs(g, k, x)
    ab.profile_enable(False)
    launches, total_ms = ab.profile_read(reset=True)["rhs_eval"]
    ms = total_ms / max(1, launches)
    byt = C * (2 * net.n_species + net.n_reactions) * 8
    ach = byt / (ms * 1e-3) / 1e9
    # HBM bytes per launch from the counter passes, when they were taken on
    # this network with the current kernels
    rec = recorded_traffic()
    traffic = None
    if rec is not None and "k_rhs_bytes_per_cell" in rec and rec.get("network") == net_name:
        traffic = round(rec["k_rhs_bytes_per_cell"] * C)
    # every network bench.py offers fits the streaming kernel
    return {"kernel": "k_rhs_stream (abdf_rhs, standalone)", "bound": "hbm", "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "cells": C, "avg_launch_ms": round(ms, 4),
            "work": f"(2 S + R) x 8 B = {(2 * net.n_species + net.n_reactions) * 8} B per cell-evaluation",
            **({"traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}
               if traffic is not None else {})}


def run_adjoint(args):
    """Differentiation workload: record 256 cells of the 500-species network to
    1e6 yr, then the discrete adjoint of the loss sum of log x over 10 seeded
    target species with respect to log alpha of every reaction."""
    import torch
    import paper_2511_10558_amd as ab
    import synth
    dev = torch.device("cuda:0")
    net = synth.network_for_config("net500")
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, args.adj_cells, seed=5001, t_end_yr=1e6)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    inp = [t(cells.T), t(cells.n_H), t(cells.A_V), t(cells.zeta), t(cells.G0), t(cells.x0), t(cells.t_end)]
    # targets: 10 seeded species above 1e-12 in every cell at t_end
    x_plain, st_plain = ab.solve(g, *inp)
    xp = x_plain.cpu().numpy()
    eligible = np.flatnonzero((xp > 1e-12).all(axis=0))
    targets = np.sort(np.random.default_rng(5002).choice(eligible, 10, replace=False))
    torch.cuda.synchronize()
    ab.profile_read(reset=True)
    ab.profile_enable(True)
    t0 = time.perf_counter()
    x, status, tape = ab.solve_record(g, *inp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] recorded forward: {t1 - t0:.1f} s", file=sys.stderr, flush=True)
    dLdx = torch.zeros_like(x)
    dLdx[:, targets] = 1.0 / x[:, targets]
    gsum, gcell, _, gphi = tape.adjoint(dLdx, per_cell=True, phys_grad=True)   # gphi: dL/d(T, n_H, A_V, zeta, G0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ab.profile_enable(False)
    prof = ab.profile_read(reset=True)
    ok = int((status == 0).sum().item())
    out = {"metric": "gradient cell-solves/sec (forward with step tape + discrete adjoint), 500-sp net",
           "phys_gradient_abs_mean": [float(v) for v in gphi.abs().mean(dim=0).cpu()],
           "value": round(ok / (t2 - t0), 3), "unit": "cell-solves/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "dtype": "f64",
           "config": {"workload": f"net500 differentiation: {args.adj_cells} cells, t_end 1e6 yr, rtol 1e-6 "
                                  "atol 1e-20, d(sum of log x over 10 targets)/d log alpha for all 6000 reactions "
                                  "and d/d(T, n_H, A_V, zeta, G0) per cell",
                      "cells": args.adj_cells, "targets": targets.tolist()},
           "forward_record_s": round(t1 - t0, 3), "reverse_s": round(t2 - t1, 3),
           "checkpoint_bytes": tape.nbytes, "cells_ok": ok,
           "forward_equals_plain_solve": bool(torch.equal(x, x_plain)),
           "kernels": {k: {"launches": v[0], "ms": round(v[1], 3)} for k, v in prof.items()}}
    tape.free()
    gold_path = os.path.join(ROOT, "tests", "golden", "adjoint_net500.json")
    if os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        n = len(gold["cells"])
        gt, gr = np.array(gold["targets"]), np.array(gold["reactions"])
        sub = [v[:n].contiguous() for v in inp]
        xs, _ = ab.solve(g, *sub)
        d = torch.zeros_like(xs)
        d[:, gt] = 1.0 / xs[:, gt]
        _, _, _, gc, _, gpc = ab.solve_adjoint(g, *sub, d, per_cell=True, phys_grad=True)
        gc = gc.cpu().numpy()

        def err(gv, ref, top):
            ref = np.asarray(ref)
            return float(np.max(np.abs(gv - ref) / np.maximum(np.abs(ref), 1e-3 * top)))
        e_sens, e_cs, e_fd, e_own = [], [], [], []
        for c, r in enumerate(gold["cells"]):
            sens, cs, fd = np.array(r["sens"]), np.array(r["cs"]), np.array(r["fd"])
            top = np.abs(cs).max()
            e_sens.append(err(gc[c, gr], sens, top))
            e_cs.append(err(gc[c, gr], cs, top))
            e_fd.append(err(gc[c, gr], fd, top))
            e_own.append(float(np.max(np.abs(fd - cs)) / top))
        # references: the oracle's forward sensitivities, the complex-step
        # derivative of its frozen map, and central differences of that map
        # replayed in extended precision; entry errors relative to the entry
        # with a floor of 1e-3 of the largest
        out["check"] = {"cells": n, "reactions": len(gr),
                        "max_rel_err_vs_oracle_forward_sensitivities": max(e_sens),
                        "max_rel_err_vs_complex_step": max(e_cs),
                        "max_rel_err_vs_central_differences": max(e_fd),
                        "oracle_central_differences_vs_complex_step_over_max_gradient": max(e_own)}
        phys_path = os.path.join(ROOT, "tests", "golden", "phys_net500.json")
        pg = json.load(open(phys_path)) if os.path.exists(phys_path) else None
        if pg is not None and pg["targets"] == gold["targets"]:
            m = len(pg["cells"])
            gp = gpc[:m].cpu().numpy()
            e_ps, e_pf, e_po = [], [], []
            for c, r in enumerate(pg["cells"]):
                # phi_j dL/dphi_j (dL/dA_V for the extinction): one dimensionless scale
                cl = cells.cell(c)
                w = np.array([cl["T"], cl["n_H"], 1.0, cl["zeta"], cl["G0"]])
                sens, fd, gv = np.array(r["sens"]) * w, np.array(r["fd"]) * w, gp[c] * w
                top = np.abs(sens).max()
                e_ps.append(err(gv, sens, top))
                e_pf.append(float(np.max(np.abs(gv - fd)) / top))
                e_po.append(float(np.max(np.abs(sens - fd)) / top))
            out["check_phys"] = {"cells": m, "params": pg["params"],
                                 "max_rel_err_vs_oracle_forward_sensitivities": max(e_ps),
                                 "max_abs_err_vs_central_differences_over_max_gradient": max(e_pf),
                                 "oracle_sensitivities_vs_central_differences_over_max_gradient": max(e_po)}
    print(json.dumps(out))


def run_single(args):
    """One cell of the 12-species network (n_H 1e4, T 10 K, A_V 0, t_end 1e6 yr):
    the latency of a whole solve, its steps, and its error against the oracle."""
    import torch
    import paper_2511_10558_amd as ab
    import synth
    from oracle import bdf, chem
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    # CPU baseline: the oracle on the same cell, one thread (its result also
    # gives the error of the GPU solve)
    t0 = time.perf_counter()
    ref = bdf.solve(chem.cell_chemistry(net, cells.cell(0)), cells.x0[0], cells.t_end[0], 1e-6, 1e-20)
    cpu_us = (time.perf_counter() - t0) * 1e6
    dev = torch.device("cuda:0")
    g = ab.Network.from_text(net.to_text())
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    inp = [t(cells.T), t(cells.n_H), t(cells.A_V), t(cells.zeta), t(cells.G0), t(cells.x0), t(cells.t_end)]
    opts = ab.make_options(rtol=1e-6, atol=1e-20)
    for _ in range(max(1, args.warmup)):
        ab.solve(g, *inp, options=opts)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(1, args.steps) * 10):
        t0 = time.perf_counter()
        x, st, stats = ab.solve(g, *inp, options=opts, with_stats=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    xg = x[0].cpu().numpy()
    m = ref.x > 1e-12
    out = {"metric": "single-cell solve latency, 12-species network", "value": round(float(np.median(times)) * 1e6, 1),
           "unit": "us", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "12 species / 40 reactions, one cell n_H 1e4 T 10 K A_V 0, t_end 1e6 yr, "
                                  "rtol 1e-6 atol 1e-20", "repeats": len(times)},
           "steps": int(stats["n_steps"][0]), "oracle_steps": int(ref.stats.n_steps),
           "max_rel_err_vs_oracle": float(np.max(np.abs(xg[m] - ref.x[m]) / ref.x[m])),
           "status": int(st[0]),
           "cpu_baseline": {"value": round(cpu_us, 1), "unit": "us", "cores": 1, "kind": "oracle",
                            "sample": "the same cell, one solve"}}
    print(json.dumps(out))


def run_ceilings(args):
    """Measured ceilings of this GPU for the roofline denominators: a plain
    device copy (HBM) and a large FP64 / FP32 matrix product (rocBLAS through
    torch), next to the vendor peaks used in the roofline."""
    import torch
    dev = torch.device("cuda:0")
    res = {}
    n = 1 << 28                              # 2 GiB of doubles
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    res["copy_GBs"] = round(2 * 8 * n * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    for name, dt in (("dgemm_TFLOPs", torch.float64), ("sgemm_TFLOPs", torch.float32)):
        m = 8192
        x = torch.randn(m, m, dtype=dt, device=dev)
        y = torch.randn(m, m, dtype=dt, device=dev)
        for _ in range(3):
            torch.matmul(x, y)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            torch.matmul(x, y)
        e1.record()
        torch.cuda.synchronize()
        res[name] = round(2 * m ** 3 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e12, 2)
        del x, y
    out = {"metric": "measured ceilings (copy, FP64 and FP32 GEMM)", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "2 GiB device copy; 8192^3 torch.matmul in FP64 and FP32"},
           "vendor_peaks": {"hbm_GBs": HBM_PEAK_GBS, "fp64_mfma_TFLOPs": FP64_MFMA_PEAK_TFLOPS,
                            "fp32_mfma_TFLOPs": FP32_MFMA_PEAK_TFLOPS}, **res}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch", choices=["batch", "serve", "adjoint", "single", "ceilings"])
    ap.add_argument("--requests", type=int, default=256, help="serve: requests after the warm-up")
    ap.add_argument("--batch-serve-requests", type=int, default=96,
                    help="requests of the serving pass that follows the batch steps (0: none)")
    ap.add_argument("--rate", type=float, default=0.0, help="serve: arrival rate [requests/s]; 0 = 0.8 x saturation")
    ap.add_argument("--serve-precisions", default="fp64,fp32_lu")
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--adj-cells", type=int, default=256)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=4096)
    ap.add_argument("--network", default="net500", choices=["small", "net200", "net500"])
    ap.add_argument("--t-end-yr", type=float, default=1e6)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_lu"])
    ap.add_argument("--seed", type=int, default=3001)
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lu-reuse", type=float, default=0.3,
                    help="keep a factorisation while |c/c_lu - 1| <= this (0: refactor whenever c changes)")
    ap.add_argument("--no-compare-reuse", dest="compare_reuse", action="store_false",
                    help="skip the run with the other factorisation policy (0 if --lu-reuse > 0, else 0.3)")
    ap.add_argument("--no-compare-fp32", dest="compare_fp32", action="store_false",
                    help="skip the FP32-LU run of the same batch")
    ap.add_argument("--method", default="bdf", choices=["bdf", "esdirk5"],
                    help="integrator of the timed solve (the ESDIRK runs with lu_reuse 0)")
    ap.add_argument("--no-compare-esdirk", dest="compare_esdirk", action="store_false",
                    help="skip the ESDIRK solve of the same batch")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one elementwise kernel reading and writing 256 MiB "
                         "(a reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the cells are independent and this benchmark runs on one "
              "MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "adjoint":
        return run_adjoint(args)
    if args.workload == "single":
        return run_single(args)
    if args.workload == "ceilings":
        return run_ceilings(args)
    import synth
    net = synth.network_for_config(args.network)
    cells = synth.sample_cells(net, args.cells, seed=args.seed, t_end_yr=args.t_end_yr)
    cpu_rec = None
    if not args.no_cpu_baseline:
        # on rank 0 at one GPU only, before the GPU is initialised
        n_cpu = min(args.cpu_sample, args.cells)
        print(f"[bench] oracle on {n_cpu} cells", file=sys.stderr, flush=True)
        cpu_rec, xo = cpu_baseline(args.network, cells, n_cpu)
    import torch
    import paper_2511_10558_amd as ab

    dev = torch.device("cuda:0")
    g = ab.Network.from_text(net.to_text())
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    inp = [t(cells.T), t(cells.n_H), t(cells.A_V), t(cells.zeta), t(cells.G0), t(cells.x0), t(cells.t_end)]
    opts = ab.make_options(rtol=1e-6, atol=1e-20, precision=args.precision,
                           lu_reuse=args.lu_reuse if args.method == "bdf" else 0.0, method=args.method)

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)     # elementwise kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        del src, dst
    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        ab.solve(g, *inp, options=opts)
        torch.cuda.synchronize()
        progress(f"warmup {w + 1}/{args.warmup}: {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    ab.profile_read(reset=True)
    ab.profile_enable(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, status, st = ab.solve(g, *inp, options=opts, with_stats=True)
        stats.append(st)
        progress(f"step {k + 1}/{args.steps} done at {time.perf_counter() - t0:.1f} s")
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
    # the counters were taken on one network in FP64; other workloads report none
    if rec is not None and args.precision == "fp64" and rec.get("network") == args.network:
        if roof["kernel"] == "k_factor":
            roof["traffic"] = round(rec["k_factor_bytes_per_lu"] * n_lu / max(1, prof["factor"][0]))
        elif roof["kernel"] == "k_newton_solve":
            roof["traffic"] = round(rec["k_newton_solve_bytes_per_iteration"] * n_newton / max(1, prof["newton"][0]))
        roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    # secondary figures for the other two hot kernels
    if prof["factor"][1] > 0:
        kern["factor"]["tflops"] = round(n_lu * lu_flop / (prof["factor"][1] * 1e-3) / 1e12, 3)
    # Newton iterations run on two streams (cells that factor on the solver's
    # stream, the others beside the factorisation), so per-kernel bandwidths of
    # the Newton kernels come from the rocprofv3 summary, not from these spans.

    out = {
        "metric": ("cell-solves/sec to t_end at rtol 1e-6, 500-sp net; p50/p99 latency; FP32-LU vs FP64"
                   if args.network == "net500" else f"cell-solves/sec to t_end at rtol 1e-6, {S}-sp net"),
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
                               f"t_end {args.t_end_yr:g} yr, rtol 1e-6 atol 1e-20, {args.precision} Newton LU"
                               + (f", factorisation kept while |c/c_lu - 1| <= {args.lu_reuse:g}"
                                  if args.lu_reuse and args.method == "bdf" else "")
                               + (", Kvaerno 5(4) ESDIRK" if args.method == "esdirk5" else ""),
                   "cells": args.cells, "species": S, "reactions": R, "precision": args.precision,
                   "method": args.method,
                   "parallelism": "one GPU, cells across workgroups"},
        "work": {"cells_ok": ok, "factorisations": int(n_lu), "newton_iterations": int(n_newton),
                 "step_attempts": int(n_att)},
        "kernels": kern,
        "roofline": roof,
    }
    x64 = x.cpu().numpy()
    if args.compare_fp32 and args.precision == "fp64":
        # the same batch with the Newton-matrix LU in FP32 (residuals, norms, control in FP64)
        o32 = ab.make_options(rtol=1e-6, atol=1e-20, precision="fp32_lu", lu_reuse=args.lu_reuse)
        ab.solve(g, *inp, options=o32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x32, st32 = ab.solve(g, *inp, options=o32)
        torch.cuda.synchronize()
        w32 = time.perf_counter() - t0
        ok32 = int((st32 == 0).sum().item())
        progress(f"fp32_lu solve: {w32:.1f} s")
        out["fp32_lu"] = {"value": round(ok32 / w32, 3), "unit": "cell-solves/s", "cells_ok": ok32,
                          "speedup_vs_fp64": round((ok32 / w32) / value, 4),
                          "max_rel_dev_from_fp64_gpu": max_rel_err(x32.cpu().numpy(), x64)}
    if args.compare_reuse and args.method == "bdf":
        # the same batch with the other factorisation policy: refactor whenever c
        # changes (the oracle's), or keep factorisations across small changes of c
        other = 0.0 if args.lu_reuse > 0 else 0.3
        o_r = ab.make_options(rtol=1e-6, atol=1e-20, precision=args.precision, lu_reuse=other)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xr, str_, sr = ab.solve(g, *inp, options=o_r, with_stats=True)
        torch.cuda.synchronize()
        wr = time.perf_counter() - t0
        okr = int((str_ == 0).sum().item())
        progress(f"lu_reuse {other} solve: {wr:.1f} s")
        out["lu_reuse_other"] = {"lu_reuse": other, "value": round(okr / wr, 3), "unit": "cell-solves/s",
                                 "cells_ok": okr, "ratio_to_value": round((okr / wr) / value, 4),
                                 "factorisations": int(sr["n_lu"].sum()),
                                 "max_rel_dev_from_headline_gpu": max_rel_err(xr.cpu().numpy(), x64)}
    if args.compare_esdirk and args.precision == "fp64" and args.method == "bdf":
        # the same batch integrated with Kvaerno's 5(4) ESDIRK (FP64 factors,
        # one factorisation per step attempt)
        o_rk = ab.make_options(rtol=1e-6, atol=1e-20, precision="fp64", method="esdirk5")
        ab.profile_read(reset=True)
        ab.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xk, stk, sk = ab.solve(g, *inp, options=o_rk, with_stats=True)
        torch.cuda.synchronize()
        wk = time.perf_counter() - t0
        ab.profile_enable(False)
        pk = ab.profile_read(reset=True)
        okk = int((stk == 0).sum().item())
        progress(f"esdirk5 solve: {wk:.1f} s")
        nk_lu = float(sk["n_lu"].sum())
        out["esdirk5"] = {"value": round(okk / wk, 3), "unit": "cell-solves/s", "cells_ok": okk,
                          "ratio_to_value": round((okk / wk) / value, 4),
                          "factorisations": int(nk_lu), "newton_iterations": int((sk["n_rhs"] - 2).sum()),
                          "steps": int(sk["n_steps"].sum()), "step_attempts": int(sk["n_attempts"].sum()),
                          "k_factor_tflops": round(nk_lu * lu_flop / max(1e-9, pk["factor"][1] * 1e-3) / 1e12, 3),
                          "kernels": {k: {"launches": v[0], "ms": round(v[1], 3)} for k, v in pk.items()},
                          "max_rel_dev_from_bdf_gpu": max_rel_err(xk.cpu().numpy(), x64)}
    out["roofline_rhs"] = rhs_standalone(net, g, inp, args.network)
    progress(f"standalone right-hand side: {out['roofline_rhs']['achieved']} GB/s")
    if args.batch_serve_requests > 0 and args.network == "net500":
        # the serving half of the metric: p50/p99 latency, FP32-LU against FP64
        rec = serve_stream(args, net, g, args.batch_serve_requests, ["fp64", "fp32_lu"])
        p64, p32 = rec["passes"]["fp64"]["open_loop"], rec["passes"]["fp32_lu"]["open_loop"]
        out["p50_latency_s"], out["p99_latency_s"] = p64["p50_latency_s"], p64["p99_latency_s"]
        out["serving"] = rec
        out["serving"]["summary"] = {
            "fp64": {"served_cell_solves_per_s": p64["cell_solves_per_s"], "p50_s": p64["p50_latency_s"],
                     "p99_s": p64["p99_latency_s"]},
            "fp32_lu": {"served_cell_solves_per_s": p32["cell_solves_per_s"], "p50_s": p32["p50_latency_s"],
                        "p99_s": p32["p99_latency_s"]}}
    if cpu_rec is not None:
        n = len(xo)
        out["cpu_baseline"] = cpu_rec
        out["parity_vs_oracle"] = {"cells": n, "max_rel_err_fp64": max_rel_err(x64[:n], xo)}
        if "fp32_lu" in out:
            out["parity_vs_oracle"]["max_rel_err_fp32_lu"] = max_rel_err(x32.cpu().numpy()[:n], xo)
        if "esdirk5" in out:
            # a different method at the same tolerance: agreement at the tolerance's reach
            out["parity_vs_oracle"]["max_rel_err_esdirk5_vs_bdf_oracle"] = max_rel_err(xk.cpu().numpy()[:n], xo)
        if "lu_reuse_other" in out:
            out["parity_vs_oracle"][f"max_rel_err_lu_reuse_{other:g}"] = max_rel_err(xr.cpu().numpy()[:n], xo)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
