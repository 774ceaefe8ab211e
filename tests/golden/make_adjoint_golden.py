"""Writes adjoint_net500.json: oracle gradients of the differentiation workload
(500 species / 6000 reactions, t_end 1e6 yr, rtol 1e-6, atol 1e-20) for the
first cells of its seeded batch.

Loss L = sum over 10 target species of log x_s(t_end).  For each cell the
oracle's own accepted (h, q) sequence is frozen (its recorded run) and the
file holds, for 50 seeded reactions r:
  sens: dL/dlog alpha_r from the oracle's discrete forward sensitivities
  fd:   central differences of the frozen map with step 1e-6 in log alpha_r,
        for the first N_FD of them (seeded order)
Only the oracle is called.  Run from the repository root:
    python tests/golden/make_adjoint_golden.py [--cells 2] [--procs 8]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import bdf, chem  # noqa: E402

N_CELLS_BATCH = 256
SEED_CELLS, SEED_TARGETS, SEED_REACTIONS = 5001, 5002, 5003
N_TARGETS, N_REACTIONS, N_FD = 10, 50, 20
DELTA = 1e-6
MAX_NEWTON = 4        # full Newton from the predictor reaches rounding level within these
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


def _fd_task(args):
    c, r, sign = args
    net, cells, runs = _state["setup"]
    ch = chem.cell_chemistry(net, cells.cell(c))
    k = ch.k.copy()
    k[r] *= np.exp(sign * DELTA)
    return bdf.replay(chem.Chemistry(net, k), cells.x0[c], runs[c].history, max_newton=MAX_NEWTON)


def _sens_task(args):
    c, reactions = args
    net, cells, runs = _state["setup"]
    ch = chem.cell_chemistry(net, cells.cell(c))
    rs = np.asarray(reactions)
    x, S = bdf.replay(ch, cells.x0[c], runs[c].history, max_newton=MAX_NEWTON,
                      sens_dfdp=lambda y: ch.df_dlogalpha(y)[:, rs].toarray())
    return x, S


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=2)
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    net, cells, runs = _setup(args.cells)
    xs = np.array([r.x for r in runs])
    # targets: species above 1e-12 in every cell at t_end
    eligible = np.flatnonzero((xs > 1e-12).all(axis=0))
    targets = np.sort(np.random.default_rng(SEED_TARGETS).choice(eligible, N_TARGETS, replace=False))
    drawn = np.random.default_rng(SEED_REACTIONS).choice(net.n_reactions, N_REACTIONS, replace=False)
    reactions = np.sort(drawn)
    fd_reactions = np.sort(drawn[:N_FD])
    with mp.get_context("fork").Pool(args.procs, initializer=_init, initargs=(args.cells,)) as pool:
        sens = pool.map(_sens_task, [(c, reactions.tolist()) for c in range(args.cells)])
        tasks = [(c, int(r), s) for c in range(args.cells) for r in fd_reactions for s in (1, -1)]
        fd_x = pool.map(_fd_task, tasks)
    out = {"workload": "net500 differentiation: 500 species / 6000 reactions, t_end 1e6 yr, rtol 1e-6, atol 1e-20",
           "seeds": {"cells": SEED_CELLS, "targets": SEED_TARGETS, "reactions": SEED_REACTIONS},
           "batch_cells": N_CELLS_BATCH, "fd_step_log_alpha": DELTA, "max_newton": MAX_NEWTON,
           "targets": targets.tolist(), "reactions": reactions.tolist(), "fd_reactions": fd_reactions.tolist(),
           "cells": []}
    it = iter(fd_x)
    for c in range(args.cells):
        x, S = sens[c]
        g_sens = (S[targets] / x[targets, None]).sum(axis=0)
        g_fd = []
        for _ in fd_reactions:
            xp, xm = next(it), next(it)
            g_fd.append(float(np.sum(np.log(xp[targets]) - np.log(xm[targets])) / (2 * DELTA)))
        out["cells"].append({"index": c, "n_steps": runs[c].stats.n_steps, "x_end_targets": x[targets].tolist(),
                             "sens": g_sens.tolist(), "fd": g_fd})
        sel = np.searchsorted(reactions, fd_reactions)
        print(f"cell {c}: steps {runs[c].stats.n_steps}, max |sens - fd| / max |sens| = "
              f"{np.max(np.abs(g_sens[sel] - np.array(g_fd))) / np.max(np.abs(g_sens)):.2e}")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
