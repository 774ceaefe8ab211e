"""Steady state of the rate equations by damped Newton (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The mass-action system conserves every element and the charge, so f(x) = 0
has a family of solutions; the one reached from x0 also satisfies
W_e . x = W_e . x0 for each conserved quantity e.  One row of f per conserved
quantity is replaced by that linear law (the row of the species carrying the
largest share |W_e,i x_i| not already used), which makes the root isolated.
"""
from __future__ import annotations

import numpy as np


def _replace_rows(W, x):
    used = []
    rows = []
    for e in range(W.shape[0]):
        if not np.any(W[e]):
            continue
        share = np.abs(W[e] * x)
        share[used] = -1.0
        i = int(np.argmax(share))
        used.append(i)
        rows.append(e)
    return used, rows


def steady_state(chem, W, x0, x_start, tol=1e-14, max_iter=200, floor=1e-25):
    """Root of f with the conservation laws of x0 substituted for dependent rows.

    Species below `floor` in x_start (never produced, so their rows and columns
    of J vanish and the root is not isolated in them) are held at their start
    values; the Newton iteration runs over the others.
    Returns (x, converged, iterations)."""
    W = np.asarray(W, dtype=float)
    target = W @ x0
    x = np.asarray(x_start, dtype=float).copy()
    act = np.nonzero(np.abs(x) > floor)[0]
    used, erows = _replace_rows(W[:, act], x[act])
    used = [int(act[i]) for i in used]

    def F(y):
        r = chem.f(y)
        for i, e in zip(used, erows):
            r[i] = W[e] @ y - target[e]
        return r

    def JF(y):
        J = chem.jac(y)
        for i, e in zip(used, erows):
            J[i] = W[e]
        return J

    r = F(x)
    for it in range(1, max_iter + 1):
        delta = np.zeros_like(x)
        delta[act] = np.linalg.solve(JF(x)[np.ix_(act, act)], -r[act])
        lam = 1.0
        nr = np.linalg.norm(r[act])
        while True:
            y = x + lam * delta
            ry = F(y)
            if np.linalg.norm(ry[act]) < nr or lam < 1e-6:
                break
            lam *= 0.5
        x, r = y, ry
        if np.max(np.abs(lam * delta[act]) / np.maximum(np.abs(x[act]), 1e-300)) < tol or np.linalg.norm(r[act]) == 0:
            return x, True, it
    return x, False, max_iter
