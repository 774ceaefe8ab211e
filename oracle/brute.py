"""Brute-force fixed-step reference integrator for tiny networks (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Three-stage Radau IIA (order 5, L-stable, stiffly accurate; Hairer & Wanner,
Solving ODEs II, Sec. IV.5) on a geometric time grid, each step's stage system
solved by full Newton to rounding level.  The step count is doubled until two
successive runs agree to `rel`, so the answer does not depend on any step-size
controller.  Only meant for a handful of species (dense 3S x 3S Newton).
"""
from __future__ import annotations

import numpy as np

_S6 = np.sqrt(6.0)
RADAU_A = np.array([
    [(88 - 7 * _S6) / 360, (296 - 169 * _S6) / 1800, (-2 + 3 * _S6) / 225],
    [(296 + 169 * _S6) / 1800, (88 + 7 * _S6) / 360, (-2 - 3 * _S6) / 225],
    [(16 - _S6) / 36, (16 + _S6) / 36, 1.0 / 9.0],
])


def _step(chem, y, h):
    S = y.shape[0]
    Z = np.zeros((3, S))          # stage increments z_i = Y_i - y
    I3S = np.eye(3 * S)
    for _ in range(60):
        F = np.array([chem.f(y + Z[i]) for i in range(3)])
        G = (Z - h * RADAU_A @ F).ravel()
        Js = [chem.jac(y + Z[i]) for i in range(3)]
        JG = I3S.copy()
        for i in range(3):
            for j in range(3):
                JG[i * S:(i + 1) * S, j * S:(j + 1) * S] -= h * RADAU_A[i, j] * Js[j]
        dZ = np.linalg.solve(JG, -G).reshape(3, S)
        Z = Z + dZ
        if np.max(np.abs(dZ)) <= 1e-15 * max(1.0, np.max(np.abs(y + Z[2]))):
            break
    return y + Z[2]


def integrate(chem, x0, t_end, n_steps, t_first):
    """n_steps Radau IIA steps on the grid 0, t_first*g, ..., t_end with
    geometric spacing between t_first and t_end."""
    grid = np.concatenate([[0.0], np.geomspace(t_first, t_end, n_steps)])
    y = np.asarray(x0, dtype=float).copy()
    for a, b in zip(grid[:-1], grid[1:]):
        y = _step(chem, y, b - a)
    return y


def converged_solution(chem, x0, t_end, t_first, rel=1e-10, floor=1e-14,
                       n0=400, max_doublings=6):
    """Double the step count until successive results agree to `rel` on every
    component above `floor`.  Returns (x, n_steps, achieved_rel)."""
    prev = integrate(chem, x0, t_end, n0, t_first)
    n = n0
    achieved = np.inf
    for _ in range(max_doublings):
        n *= 2
        cur = integrate(chem, x0, t_end, n, t_first)
        m = np.abs(cur) > floor
        achieved = float(np.max(np.abs(cur[m] - prev[m]) / np.abs(cur[m]))) if m.any() else 0.0
        prev = cur
        if achieved <= rel:
            break
    return prev, n, achieved
