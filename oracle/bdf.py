"""Variable-order, variable-step BDF for one cell (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names BDF as the standard stiff integrator of astrochemistry codes
(Sec. 1).  This is the quasi-constant-step BDF in backward-difference form of
Shampine & Reichelt ("The MATLAB ODE Suite", SIAM J. Sci. Comput. 18, 1997,
Sec. 2.1-2.3) with kappa = 0 (plain BDF, no NDF correction), orders 1..5.

Notation (one cell):
  D[j]   j-th backward difference of the solution on the current uniform grid
         of spacing h (D[0] = x_n); rows 0..q+2 are live at order q.
  gamma_q = sum_{j=1..q} 1/j,  E_q = 1/(q+1) (local error constant).
  c = h / gamma_q.  The corrector solves  d = c f(x_p + d) - psi  with
  x_p = sum_{j<=q} D[j], psi = sum_{j=1..q} gamma_j D[j] / gamma_q, by
  modified Newton on the matrix M = I - c J.

Readings where the method leaves freedom are fixed in the module constants
below and listed in the design notes (Newton tolerance and iteration cap,
safety factor, step-ratio limits, order-tie rule, landing on t_end).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

U_ROUND = 2.0 ** -52
MAX_ORDER = 5
NEWTON_MAXITER = 4
MIN_FACTOR = 0.2
MAX_FACTOR = 10.0

# per-cell status codes
OK = 0
STEP_TOO_SMALL = 1
MAX_STEPS = 2
NONFINITE = 3
BAD_INPUT = 4


def gamma_coefficients():
    """gamma[q] = sum_{j=1..q} 1/j for q = 0..MAX_ORDER+1 (cumulative, in order)."""
    g = [0.0]
    acc = 0.0
    for j in range(1, MAX_ORDER + 2):
        acc += 1.0 / j
        g.append(acc)
    return np.array(g)


def error_constants():
    """E[q] = 1/(q+1) for q = 0..MAX_ORDER+1."""
    return np.array([1.0 / (q + 1) for q in range(MAX_ORDER + 2)])


GAMMA = gamma_coefficients()
ERRC = error_constants()


def newton_tolerance(rtol):
    return max(10.0 * U_ROUND / rtol, min(0.03, rtol ** 0.5))


def safety_factor(n_newton):
    return 0.9 * (2 * NEWTON_MAXITER + 1) / (2 * NEWTON_MAXITER + n_newton)


def interp_matrix(q, rho):
    """R(rho): R[i, j] = prod_{m=1..i} (m - 1 - rho*j) / m for i, j in 0..q.

    D' = (R(rho) R(1))^T D re-expresses the backward differences of the
    interpolating polynomial on a grid of spacing rho*h (Shampine & Reichelt,
    Sec. 2.3)."""
    R = np.ones((q + 1, q + 1))
    for i in range(1, q + 1):
        for j in range(q + 1):
            R[i, j] = R[i - 1, j] * (i - 1 - rho * j) / i
    return R


def rescale(D, q, rho):
    """In place: rows 0..q of D moved from spacing h to spacing rho*h."""
    RU = interp_matrix(q, rho) @ interp_matrix(q, 1.0)
    D[: q + 1] = RU.T @ D[: q + 1]


def wrms(v, scale):
    """Weighted root-mean-square norm sqrt(mean(|v/scale|^2)) (|.| the modulus
    for the complex iterates of complex-step replays)."""
    return float(np.sqrt(np.mean(np.abs(v / scale) ** 2)))


def initial_step(f, x0, f0, t_span, rtol, atol, ft=None, order=1):
    """Starting step of Hairer, Norsett & Wanner (Solving ODEs I, Sec. II.4) for
    a method of the given order (1: BDF's first step; 5: the fifth-order
    Runge-Kutta method).  ft(t, x), if given, is the right-hand side at time t
    (for the trial evaluation at t = h0); otherwise f(x)."""
    scale = atol + rtol * np.abs(x0)
    d0 = wrms(x0, scale)
    d1 = wrms(f0, scale)
    if d0 < 1e-5 or d1 < 1e-5:
        h0 = 1e-6
    else:
        h0 = 0.01 * d0 / d1
    h0 = min(h0, t_span)
    f1 = ft(h0, x0 + h0 * f0) if ft is not None else f(x0 + h0 * f0)
    d2 = wrms(f1 - f0, scale) / h0
    if max(d1, d2) <= 1e-15:
        h1 = max(1e-6, h0 * 1e-3)
    else:
        h1 = (0.01 / max(d1, d2)) ** (1.0 / (order + 1))
    return min(100.0 * h0, h1, t_span)


def _growth(err, order_plus_one):
    if err == 0.0:
        return np.inf
    if not np.isfinite(err):
        return 0.0
    return err ** (-1.0 / order_plus_one)


@dataclasses.dataclass
class Stats:
    n_steps: int = 0         # accepted steps
    n_attempts: int = 0      # step attempts (accepted + rejected + Newton failures)
    n_err_reject: int = 0
    n_newton_fail: int = 0
    n_rhs: int = 0
    n_jac: int = 0
    n_lu: int = 0
    n_newton_iter: int = 0
    order: int = 1
    h: float = 0.0


@dataclasses.dataclass
class Result:
    x: np.ndarray
    status: int
    t: float
    stats: Stats
    history: list | None = None   # accepted (h, q, t_new, x_new) when recorded


def _newton(chem, lu, c, psi, x_p, scale, tol, stats, maxiter=NEWTON_MAXITER):
    """Modified Newton on d = c f(x_p + d) - psi with the factor of I - cJ."""
    d = np.zeros_like(x_p)
    x = x_p.copy()
    eta_old = None
    for m in range(1, maxiter + 1):
        fx = chem.f(x)
        stats.n_rhs += 1
        stats.n_newton_iter += 1
        if not np.all(np.isfinite(fx)):
            return False, m, x, d
        delta = sla.lu_solve(lu, c * fx - psi - d)
        eta = wrms(delta, scale)
        theta = None if eta_old is None else eta / eta_old
        if theta is not None and (
            theta >= 1.0 or theta ** (maxiter - m) / (1.0 - theta) * eta > tol
        ):
            return False, m, x, d
        x = x + delta
        d = d + delta
        if eta == 0.0 or (theta is not None and theta / (1.0 - theta) * eta < tol):
            return True, m, x, d
        eta_old = eta
    return False, maxiter, x, d


def solve(chem, x0, t_end, rtol=1e-6, atol=1e-20, max_steps=100000,
          newton_tol=None, record=False, max_order=MAX_ORDER, h0=0.0, h_max=0.0) -> Result:
    """Integrate dx/dt = f(x) from t = 0 to t_end with adaptive order and step.

    chem provides f and jac; if it also provides at(t), the rate
    coefficients depend on time: every step attempt from t to t + h uses those
    at t + h (the corrector equation is evaluated there), the Jacobian is taken
    at the attempt where it is refreshed, and the starting step's trial
    evaluation at t = h0.

    atol is a scalar or one absolute tolerance per species.  max_order
    (1..5) caps the order the order selection may reach; 1 leaves
    the implicit Euler method under the same error and step control.  h0 > 0
    replaces the starting-step heuristic's result; h_max > 0 bounds every step
    (the starting step, and each increase chosen with the order)."""
    if not 1 <= max_order <= MAX_ORDER:
        raise ValueError("max_order must be in 1..5")
    x0 = np.asarray(x0, dtype=float)
    S = x0.shape[0]
    stats = Stats()
    at = getattr(chem, "at", None)
    chem_at = at if at is not None else (lambda t: chem)
    hist = [] if record else None
    atol = np.asarray(atol, dtype=float) if np.ndim(atol) else float(atol)
    if not (np.all(np.isfinite(x0)) and np.isfinite(t_end) and t_end >= 0 and rtol > 0
            and np.all(np.isfinite(atol)) and np.all(np.asarray(atol) >= 0)):
        return Result(x0.copy(), BAD_INPUT, 0.0, stats, hist)
    if t_end == 0.0:
        return Result(x0.copy(), OK, 0.0, stats, hist)
    tol = newton_tolerance(rtol) if newton_tol is None else newton_tol
    ch0 = chem_at(0.0)
    f0 = ch0.f(x0)
    stats.n_rhs += 1
    if not np.all(np.isfinite(f0)):
        # rates overflow at the initial state: no step can be taken
        return Result(x0.copy(), NONFINITE, 0.0, stats, hist)
    h = initial_step(ch0.f, x0, f0, t_end, rtol, atol,
                     ft=(lambda t, y: chem_at(t).f(y)) if at is not None else None)
    stats.n_rhs += 1
    if h0 > 0.0:
        h = min(h0, t_end)
    if h_max > 0.0:
        h = min(h, h_max)
    D = np.zeros((MAX_ORDER + 3, S))
    D[0] = x0
    D[1] = h * f0
    q = 1
    n_equal = 0
    t = 0.0
    J = ch0.jac(x0)
    stats.n_jac += 1
    j_fresh = True
    lu, c_lu = None, None
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
            if t + h > t_end:
                rho = (t_end - t) / h
                rescale(D, q, rho)
                h = t_end - t
                n_equal = 0
            landing = True
        # predictor and corrector constants
        x_p = D[0].copy()
        for j in range(1, q + 1):
            x_p = x_p + D[j]
        psi = np.zeros(S)
        for j in range(1, q + 1):
            psi = psi + GAMMA[j] * D[j]
        psi = psi / GAMMA[q]
        c = h / GAMMA[q]
        ch = chem_at(t + h)
        if lu is None or c != c_lu:
            lu = sla.lu_factor(I - c * J)
            c_lu = c
            stats.n_lu += 1
        scale = atol + rtol * np.abs(x_p)
        converged, m, x_new, d = _newton(ch, lu, c, psi, x_p, scale, tol, stats)
        if not converged:
            stats.n_newton_fail += 1
            if not j_fresh:
                J = ch.jac(x_p)
                stats.n_jac += 1
                j_fresh = True
                lu = None
                continue
            h = 0.5 * h
            rescale(D, q, 0.5)
            n_equal = 0
            lu = None
            continue
        safety = safety_factor(m)
        scale_e = atol + rtol * np.maximum(np.abs(D[0]), np.abs(x_new))
        err = wrms(ERRC[q] * d, scale_e)
        if not np.isfinite(err):
            status = NONFINITE
            break
        if err > 1.0:
            stats.n_err_reject += 1
            rho = max(MIN_FACTOR, safety * _growth(err, q + 1))
            h = h * rho
            rescale(D, q, rho)
            n_equal = 0
            lu = None
            continue
        # accept
        t = t_end if landing else t + h
        stats.n_steps += 1
        if record:
            hist.append((h, q, t, x_new.copy()))
        D[q + 2] = d - D[q + 1]
        D[q + 1] = d
        for j in range(q, -1, -1):
            D[j] = D[j] + D[j + 1]
        n_equal += 1
        j_fresh = False
        if not np.all(np.isfinite(D[0])):
            status = NONFINITE
            break
        if landing:
            break
        if n_equal < q + 1:
            continue
        e_m = wrms(ERRC[q - 1] * D[q], scale_e) if q > 1 else np.inf
        e_p = wrms(ERRC[q + 1] * D[q + 2], scale_e) if q < max_order else np.inf
        rhos = [_growth(e_m, q), _growth(err, q + 1), _growth(e_p, q + 2)]
        best = 1
        if rhos[0] > rhos[best]:
            best = 0
        if rhos[2] > rhos[best]:
            best = 2
        q = q + best - 1
        rho = min(MAX_FACTOR, safety * rhos[best])
        if h_max > 0.0:
            rho = min(rho, h_max / h)
        h = h * rho
        rescale(D, q, rho)
        n_equal = 0
        lu = None
    stats.order = q
    stats.h = h
    return Result(D[0].copy(), status, t, stats, hist)


def replay(chem, x0, history, newton_atol=1e-12, rtol=1e-6, atol=1e-20,
           sens_dfdp=None, max_newton=50):
    """Frozen-sequence BDF: the accepted (h, q) sequence of a recorded run, each
    corrector solved by full Newton until the weighted correction norm is below
    `newton_atol` (or `max_newton` iterations).  This is the discrete map whose
    exact derivative the adjoint computes.

    The arithmetic follows the coefficients' type: FP64; complex (a rate
    coefficient perturbed by i h gives the complex-step derivative of the map,
    Im L / h, free of cancellation); or np.longdouble (x86 extended precision:
    the state, residuals and difference tables are carried with a 64-bit
    significand while each Newton correction is solved in FP64, so the
    iteration converges to the extended-precision corrector solution).

    sens_dfdp(x) -> (S x P) array of d f / d p: if given, the discrete forward
    sensitivities S = dx/dp are carried along (difference array D_S with the
    structure of D, rescaled with it; each step solves
    (I - c J(x_{n+1})) S_{n+1} = S_p - psi_S + c df/dp(x_{n+1})).
    Returns x_end, or (x_end, S_end) with sensitivities."""
    work = np.result_type(np.asarray(chem.k).dtype, np.float64)
    lin = np.complex128 if np.issubdtype(work, np.complexfloating) else np.float64
    x0 = np.asarray(x0).astype(work)
    S = x0.shape[0]
    I = np.eye(S)
    D = np.zeros((MAX_ORDER + 3, S), dtype=work)
    D[0] = x0
    h0 = history[0][0]
    D[1] = h0 * chem.f(x0)
    DS = None
    if sens_dfdp is not None:
        fp0 = np.asarray(sens_dfdp(x0))
        DS = np.zeros((MAX_ORDER + 3, S, fp0.shape[1]))
        DS[1] = h0 * fp0
    h_prev, q_prev = h0, history[0][1]
    for n, (h, q, *_rest) in enumerate(history):
        if n > 0 and (h != h_prev or q != q_prev):
            rho = h / h_prev
            rescale(D, q, rho)
            if DS is not None:
                RU = interp_matrix(q, rho) @ interp_matrix(q, 1.0)
                DS[: q + 1] = np.einsum("ji,jsp->isp", RU, DS[: q + 1])
        x_p = D[: q + 1].sum(axis=0)
        psi = (GAMMA[1: q + 1] @ D[1: q + 1]) / GAMMA[q]
        c = h / GAMMA[q]
        scale = atol + rtol * np.abs(x_p)
        x = x_p.copy()
        for _ in range(max_newton):
            g = x - x_p - c * chem.f(x) + psi
            delta = np.linalg.solve((I - c * chem.jac(x)).astype(lin), (-g).astype(lin))
            x = x + delta
            if wrms(delta, scale) <= newton_atol:
                break
        d = x - x_p
        if DS is not None:
            SP = DS[: q + 1].sum(axis=0)
            psiS = np.einsum("j,jsp->sp", GAMMA[1: q + 1], DS[1: q + 1]) / GAMMA[q]
            rhs = SP - psiS + c * np.asarray(sens_dfdp(x))
            Snew = np.linalg.solve(I - c * chem.jac(x), rhs)
            dS = Snew - SP
            DS[q + 2] = dS - DS[q + 1]
            DS[q + 1] = dS
            for j in range(q, -1, -1):
                DS[j] = DS[j] + DS[j + 1]
        D[q + 2] = d - D[q + 1]
        D[q + 1] = d
        for j in range(q, -1, -1):
            D[j] = D[j] + D[j + 1]
        h_prev, q_prev = h, q
    if DS is not None:
        return D[0].copy(), DS[0].copy()
    return D[0].copy()
