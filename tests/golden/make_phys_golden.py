"""Writes phys_net500.json: oracle gradients of the differentiation workload's
loss with respect to each cell's physical parameters (T, n_H, A_V, zeta, G0)
for the first cells of its seeded batch (500 species / 6000 reactions, t_end
1e6 yr, rtol 1e-6, atol 1e-20; the batch, targets and loss of
make_adjoint_golden.py).

For each cell the oracle's own accepted (h, q) sequence is frozen and the file
holds, per parameter phi_j:
  sens: dL/dphi_j from the oracle's discrete forward sensitivities with
        d f / d phi_j = sum_r nu_r rate_r d log k_r / d phi_j
  fd:   central differences of the frozen map, step 1e-6 phi_j (1e-6 for A_V)
Only the oracle is called.  Run from the repository root:
    python tests/golden/make_phys_golden.py [--cells 2] [--procs 8]
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
SEED_CELLS, SEED_TARGETS = 5001, 5002
N_TARGETS = 10
REL_STEP = 1e-6
MAX_NEWTON = 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "phys_net500.json")

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
    threadpool_limits(1)
    _state["setup"] = _setup(n_cells)


def _step(cell, j):
    name = chem.PHYS_PARAMS[j]
    return REL_STEP if name == "A_V" else REL_STEP * cell[name]


def _fd_task(args):
    c, j, sign = args
    net, cells, runs = _state["setup"]
    cell = dict(cells.cell(c))
    cell[chem.PHYS_PARAMS[j]] += sign * _step(cells.cell(c), j)
    return bdf.replay(chem.cell_chemistry(net, cell), cells.x0[c], runs[c].history, max_newton=MAX_NEWTON)


def _sens_task(c):
    net, cells, runs = _state["setup"]
    cell = cells.cell(c)
    ch = chem.cell_chemistry(net, cell)
    D = chem.log_rate_derivatives(net, **cell)
    return bdf.replay(ch, cells.x0[c], runs[c].history, max_newton=MAX_NEWTON,
                      sens_dfdp=lambda y: ch.df_dlogalpha(y) @ D)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=2)
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    net, cells, runs = _setup(args.cells)
    xs = np.array([r.x for r in runs])
    eligible = np.flatnonzero((xs > 1e-12).all(axis=0))
    targets = np.sort(np.random.default_rng(SEED_TARGETS).choice(eligible, N_TARGETS, replace=False))
    with mp.get_context("fork").Pool(args.procs, initializer=_init, initargs=(args.cells,)) as pool:
        sens = pool.map(_sens_task, range(args.cells))
        tasks = [(c, j, s) for c in range(args.cells) for j in range(5) for s in (1, -1)]
        fd_x = pool.map(_fd_task, tasks)
    out = {"workload": "net500 differentiation: 500 species / 6000 reactions, t_end 1e6 yr, rtol 1e-6, atol 1e-20",
           "seeds": {"cells": SEED_CELLS, "targets": SEED_TARGETS}, "batch_cells": N_CELLS_BATCH,
           "params": list(chem.PHYS_PARAMS), "fd_rel_step": REL_STEP, "fd_step_A_V": REL_STEP,
           "max_newton": MAX_NEWTON, "targets": targets.tolist(), "cells": []}
    it = iter(fd_x)
    for c in range(args.cells):
        x, S = sens[c]
        g_sens = (S[targets] / x[targets, None]).sum(axis=0)
        g_fd = []
        for j in range(5):
            xp, xm = next(it), next(it)
            g_fd.append(float(np.sum(np.log(xp[targets]) - np.log(xm[targets])) / (2 * _step(cells.cell(c), j))))
        out["cells"].append({"index": c, "sens": g_sens.tolist(), "fd": g_fd})
        print(f"cell {c}: sens {np.array2string(g_sens, precision=4)}, fd {np.array2string(np.array(g_fd), precision=4)}")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
