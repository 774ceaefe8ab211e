"""Kvaerno's fifth-order ESDIRK method for one cell (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper integrates its networks with Kvaerno's fifth-order stiff method
(Sec. 4): the seven-stage singly diagonally implicit Runge-Kutta method with an
explicit first stage of Kvaerno ("Singly diagonally implicit Runge-Kutta
methods with an explicit first stage", BIT Numer. Math. 44, 2004).  Its
tableau has diagonal gamma = 0.26 and stage order 2; both the fifth-order
result (stage 7) and the embedded fourth-order result (stage 6) are stages of
their own (stiffly accurate, c_6 = c_7 = 1), so the error estimate is
Y_7 - Y_6 = sum_j (A[6, j] - A[5, j]) h F_j.

One step from (t_n, x_n) with step h, F_j = f(Y_j), G_j = h F_j:
  Y_1 = x_n (explicit stage; F_1 = f(x_n), carried over from the previous
        step's last stage, FSAL)
  Y_i = x_n + sum_{j<i} A[i, j] G_j + gamma h f(Y_i),   i = 2..7,
each implicit stage solved by the modified Newton iteration of the BDF oracle
(bdf._newton: the same rate tests and tolerance, at most NEWTON_MAXITER = 10
iterations) on M = I - h gamma J(x_n),
with J and the factorisation formed once per step attempt.  A stage starts
from its own equation with the previous stage's G in place of G_i,
Y_i^0 = x_n + sum_{j<i} A[i, j] G_j + gamma G_{i-1}.  A converged stage gives
G_i from its own equation,
G_i = (Y_i - x_n - sum_{j<i} A[i, j] G_j) / gamma, so no extra evaluation of f
is made; x_{n+1} = Y_7 and the next step's F_1 = G_7 / h.

Step control (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4): the
weighted RMS norm err of the estimate with weights atol + rtol max(|x_n|,
|x_{n+1}|); accept when err <= 1; the next step is h * min(10, max(0.2,
0.9 err^(-1/5))), with no increase on the step after a rejection; a corrector
failure halves h.  Readings where the paper and Kvaerno leave freedom (the
stage starting points, the Newton test, the controller constants) are listed
in the design notes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import bdf
from .bdf import (BAD_INPUT, MAX_STEPS, NONFINITE, OK, STEP_TOO_SMALL, U_ROUND, Result, Stats, newton_tolerance,
                  wrms)

GAMMA = 0.26
STAGES = 7
ORDER = 5
SAFETY = 0.9
MIN_FACTOR = 0.2
MAX_FACTOR = 10.0
# Newton iterations per stage: with the BDF corrector's 4, half the attempts on
# the networks' cells end in a corrector failure while the error estimate would
# allow the step; 10 leaves almost none
NEWTON_MAXITER = 10


def tableau():
    """Kvaerno's 7-stage 5(4) ESDIRK coefficients A (7 x 7, lower triangular
    with A[0, 0] = 0 and A[i, i] = gamma for i >= 1).  Rows 6 and 7 are the
    embedded and the advancing method's weights."""
    g = GAMMA
    rows = [
        [0.0],
        [g, g],
        [0.13, 0.84033320996790809, g],
        [0.22371961478320505, 0.47675532319799699, -0.06470895363112615, g],
        [0.16648564323248321, 0.10450018841591720, 0.03631482272098715, -0.13090704451073998, g],
        [0.13855640231268224, 0.0, -0.04245337201752043, 0.02446657898003141, 0.61943039072480676, g],
        [0.13659751177640291, 0.0, -0.05496908796538376, -0.04118626728321046, 0.62993304899016403,
         0.06962479448202728, g],
    ]
    A = np.zeros((STAGES, STAGES))
    for i, r in enumerate(rows):
        A[i, : len(r)] = r
    return A


A = tableau()
C = A.sum(axis=1)
E = A[6] - A[5]          # weights of the error estimate Y_7 - Y_6


def step(chem, x, F1, h, lu, tol, rtol, atol, stats, maxiter=NEWTON_MAXITER):
    """One step attempt from x with stage derivative F1 = f(x) and the factor
    `lu` of I - h gamma J.  Returns (ok, x_new, G, err_vec): ok False when a
    stage's corrector failed; G[j] = h F_{j+1}; err_vec = Y_7 - Y_6."""
    c = h * GAMMA
    G = [h * F1]
    y_prev = x
    for i in range(1, STAGES):
        s = np.zeros_like(x)
        for j in range(i):
            s = s + A[i, j] * G[j]
        start = x + s + GAMMA * G[i - 1]
        psi = start - x - s
        scale = atol + rtol * np.abs(start)
        conv, _m, y, d = bdf._newton(chem, lu, c, psi, start, scale, tol, stats, maxiter=maxiter)
        if not conv:
            return False, None, G, None
        G.append((psi + d) / GAMMA)
        y_prev = y
    e = np.zeros_like(x)
    for j in range(STAGES):
        e = e + E[j] * G[j]
    return True, y_prev, G, e


def solve(chem, x0, t_end, rtol=1e-6, atol=1e-20, max_steps=100000, newton_tol=None,
          h0=0.0, h_max=0.0, record=False) -> Result:
    """Integrate dx/dt = f(x) from t = 0 to t_end with Kvaerno's 5(4) pair.

    The arguments mean what they mean for bdf.solve (atol scalar or per
    species; h0 > 0 replaces the starting-step heuristic, run here for order
    5; h_max > 0 bounds every step).  Counters: n_attempts step attempts,
    n_lu factorisations (one per attempt), n_jac Jacobians (one per accepted
    point a step starts from), n_rhs evaluations of f (Newton iterations plus
    the initial and trial evaluations)."""
    x0 = np.asarray(x0, dtype=float)
    S = x0.shape[0]
    stats = Stats()
    stats.order = ORDER
    hist = [] if record else None
    atol = np.asarray(atol, dtype=float) if np.ndim(atol) else float(atol)
    if not (np.all(np.isfinite(x0)) and np.isfinite(t_end) and t_end >= 0 and rtol > 0
            and np.all(np.isfinite(atol)) and np.all(np.asarray(atol) >= 0)):
        return Result(x0.copy(), BAD_INPUT, 0.0, stats, hist)
    if t_end == 0.0:
        return Result(x0.copy(), OK, 0.0, stats, hist)
    tol = newton_tolerance(rtol) if newton_tol is None else newton_tol
    F1 = chem.f(x0)
    stats.n_rhs += 1
    if not np.all(np.isfinite(F1)):
        return Result(x0.copy(), NONFINITE, 0.0, stats, hist)
    h = bdf.initial_step(chem.f, x0, F1, t_end, rtol, atol, order=ORDER)
    stats.n_rhs += 1
    if h0 > 0.0:
        h = min(h0, t_end)
    if h_max > 0.0:
        h = min(h, h_max)
    x = x0.copy()
    t = 0.0
    J = None
    rejected = False
    status = OK
    I = np.eye(S)
    while True:
        if stats.n_attempts >= max_steps:
            status = MAX_STEPS
            break
        stats.n_attempts += 1
        if h < 10.0 * U_ROUND * abs(t):
            status = STEP_TOO_SMALL
            break
        landing = False
        if t + h >= t_end:
            h = t_end - t
            landing = True
        if J is None:
            J = chem.jac(x)
            stats.n_jac += 1
        lu = sla.lu_factor(I - (h * GAMMA) * J)
        stats.n_lu += 1
        ok, x_new, G, e = step(chem, x, F1, h, lu, tol, rtol, atol, stats)
        if not ok:
            stats.n_newton_fail += 1
            h = 0.5 * h
            rejected = True
            continue
        err = wrms(e, atol + rtol * np.maximum(np.abs(x), np.abs(x_new)))
        if not np.isfinite(err):
            status = NONFINITE
            break
        if err > 1.0:
            stats.n_err_reject += 1
            h = h * max(MIN_FACTOR, SAFETY * err ** (-1.0 / ORDER))
            rejected = True
            continue
        # accept
        t = t_end if landing else t + h
        stats.n_steps += 1
        if record:
            hist.append((h, ORDER, t, x_new.copy()))
        x = x_new
        F1 = G[STAGES - 1] / h
        J = None
        if not np.all(np.isfinite(x)):
            status = NONFINITE
            break
        if landing:
            break
        fac = MAX_FACTOR if err == 0.0 else min(MAX_FACTOR, max(MIN_FACTOR, SAFETY * err ** (-1.0 / ORDER)))
        if rejected:
            fac = min(1.0, fac)
            rejected = False
        h = h * fac
        if h_max > 0.0:
            h = min(h, h_max)
    stats.h = h
    return Result(x, status, t, stats, hist)
