"""Writes adjoint_net500.json: oracle gradients of the differentiation workload
(500 species / 6000 reactions, t_end 1e6 yr, rtol 1e-6, atol 1e-20) for the
first cells of its seeded batch.

Loss L = sum over 10 target species of log x_s(t_end).  For each cell the
oracle's own accepted (h, q) sequence is frozen (its recorded run), each
corrector solved exactly, and the file holds, for 50 seeded reactions r, three
independent values of dL/dlog alpha_r of that map:
  sens: the oracle's discrete forward sensitivities (FP64)
  cs:   the complex-step derivative Im L(log alpha_r + i h) / h, h = 1e-30
        (Squire & Trapp, SIAM Review 40, 1998): no difference is formed, so
        no cancellation
  fd:   central differences with step 1e-6 in log alpha_r, each replay run
        in x86 extended precision (64-bit significand) with Newton iterated
        until the weighted correction is below 1e-12, so that the rounding
        noise the map amplifies stays far below the difference quotient
Only the oracle is called.  Run from the repository root:
    python tests/golden/make_adjoint_golden.py [--cells 2] [--procs 7]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import bdf, chem  # noqa: E402

N_CELLS_BATCH = 256
SEED_CELLS, SEED_TARGETS, SEED_REACTIONS = 5001, 5002, 5003
N_TARGETS, N_REACTIONS = 10, 50
DELTA = 1e-6          # central-difference step in log alpha
H_CS = 1e-30          # complex step
NEWTON_FP64 = 5       # full Newton from the predictor: FP64 iterates reach the rounding floor within 3
NEWTON_EXT = 50       # extended precision: iterated until the weighted correction is below 1e-12
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_net500.json")

_state = {}


def _setup(n_cells):
    net = synth.network_for_config("net500")
    cells = synth.sample_cells(net, N_CELLS_BATCH, seed=SEED_CELLS, t_end_yr=1e6).subset(np.arange(n_cells))
    runs = []
    for c in range(n_cells):
        ch = chem.cell_chemistry(net, cells.cell(c))
        runs.append(bdf.solve(ch, cells.x0[c], cells.t_end[c], 1e-6, 1e-20, record=True))
    return net, cells, runs


def _init(n_cells):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)          # one BLAS thread per worker process
    _state["setup"] = _setup(n_cells)


def _task(args):
    kind, c, r, sign = args
    net, cells, runs = _state["setup"]
    k = chem.cell_chemistry(net, cells.cell(c)).k
    if kind == "fd":
        k = k.astype(np.longdouble)
        k[r] *= np.exp(np.longdouble(sign * DELTA))
        x = bdf.replay(chem.Chemistry(net, k), cells.x0[c], runs[c].history, max_newton=NEWTON_EXT)
    else:
        k = k.astype(np.complex128)
        k[r] *= np.exp(1j * H_CS)
        x = bdf.replay(chem.Chemistry(net, k), cells.x0[c], runs[c].history, max_newton=NEWTON_FP64)
    return (kind, c, r, sign), x


def _sens_task(args):
    c, reactions = args
    net, cells, runs = _state["setup"]
    ch = chem.cell_chemistry(net, cells.cell(c))
    rs = np.asarray(reactions)
    x, S = bdf.replay(ch, cells.x0[c], runs[c].history, max_newton=NEWTON_FP64,
                      sens_dfdp=lambda y: ch.df_dlogalpha(y)[:, rs].toarray())
    return ("sens", c, -1, 0), (x, S)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=2)
    ap.add_argument("--procs", type=int, default=7)
    args = ap.parse_args()
    net, cells, runs = _setup(args.cells)
    xs = np.array([r.x for r in runs])
    # targets: species above 1e-12 in every cell at t_end
    eligible = np.flatnonzero((xs > 1e-12).all(axis=0))
    targets = np.sort(np.random.default_rng(SEED_TARGETS).choice(eligible, N_TARGETS, replace=False))
    reactions = np.sort(np.random.default_rng(SEED_REACTIONS).choice(net.n_reactions, N_REACTIONS, replace=False))
    tasks = [("fd", c, int(r), s) for c in range(args.cells) for r in reactions for s in (1, -1)]
    tasks += [("cs", c, int(r), 0) for c in range(args.cells) for r in reactions]
    res = {}
    t0 = time.time()
    with mp.get_context("fork").Pool(args.procs, initializer=_init, initargs=(args.cells,)) as pool:
        for key, val in pool.imap_unordered(_sens_task, [(c, reactions.tolist()) for c in range(args.cells)]):
            res[key] = val
        for n, (key, val) in enumerate(pool.imap_unordered(_task, tasks)):
            res[key] = val
            print(f"{n + 1}/{len(tasks)} replays at {time.time() - t0:.0f} s", flush=True)
    out = {"workload": "net500 differentiation: 500 species / 6000 reactions, t_end 1e6 yr, rtol 1e-6, atol 1e-20",
           "seeds": {"cells": SEED_CELLS, "targets": SEED_TARGETS, "reactions": SEED_REACTIONS},
           "batch_cells": N_CELLS_BATCH, "fd_step_log_alpha": DELTA, "complex_step": H_CS,
           "newton_fp64": NEWTON_FP64, "newton_extended": NEWTON_EXT,
           "targets": targets.tolist(), "reactions": reactions.tolist(), "cells": []}
    for c in range(args.cells):
        x, S = res[("sens", c, -1, 0)]
        g_sens = (S[targets] / x[targets, None]).sum(axis=0)
        g_fd, g_cs = [], []
        for r in reactions:
            xp, xm = res[("fd", c, int(r), 1)], res[("fd", c, int(r), -1)]
            g_fd.append(float(np.sum(np.log(xp[targets]) - np.log(xm[targets])) / (2 * DELTA)))
            xc = res[("cs", c, int(r), 0)]
            g_cs.append(float(np.sum(np.log(xc[targets])).imag / H_CS))
        g_fd, g_cs = np.array(g_fd), np.array(g_cs)
        top = np.abs(g_sens).max()
        out["cells"].append({"index": c, "n_steps": runs[c].stats.n_steps, "x_end_targets": x[targets].tolist(),
                             "sens": g_sens.tolist(), "cs": g_cs.tolist(), "fd": g_fd.tolist()})
        print(f"cell {c}: steps {runs[c].stats.n_steps}, max |g| {top:.3e}; over max |g|: "
              f"|sens - cs| {np.max(np.abs(g_sens - g_cs)) / top:.2e}, |fd - cs| {np.max(np.abs(g_fd - g_cs)) / top:.2e}, "
              f"|fd - sens| {np.max(np.abs(g_fd - g_sens)) / top:.2e}")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
