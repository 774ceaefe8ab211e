"""Pins for the oracle's BDF integrator (CPU only).

Each pin comes from outside the oracle: backward differences of polynomials,
implicit Euler, closed-form solutions of one-reaction systems, the matrix
exponential of a linear network, and conservation laws.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import bdf, chem
from tests import tiny_nets

YEAR = synth.YEAR_S
CELL = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)


def _backward_differences(p, t, h, q):
    """nabla^j p(t) on the grid t, t-h, ..., t-q*h for j = 0..q."""
    vals = np.array([p(t - i * h) for i in range(q + 1)])
    out = [vals[0]]
    cur = vals
    for _ in range(q):
        cur = cur[:-1] - cur[1:]
        out.append(cur[0])
    return np.array(out)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_rescale_is_regridding_of_the_interpolating_polynomial(q):
    rng = np.random.default_rng(q)
    coef = rng.normal(size=q + 1)
    p = np.polynomial.Polynomial(coef)
    t, h = 0.7, 0.13
    for rho in (0.2, 0.5, 1.0, 1.7, 10.0):
        D = np.zeros((bdf.MAX_ORDER + 3, 1))
        D[: q + 1, 0] = _backward_differences(p, t, h, q)
        bdf.rescale(D, q, rho)
        want = _backward_differences(p, t, rho * h, q)
        np.testing.assert_allclose(D[: q + 1, 0], want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_harmonic_and_error_constants_make_bdf_exact_on_polynomials():
    # sum_{j=1..q} (1/j) nabla^j y(t_{n+1}) = h y'(t_{n+1}) for deg y <= q is the BDF
    # formula; gamma_q is the coefficient of the newest correction in it and
    # E_q = 1/(q+1) is the coefficient of nabla^{q+1} y in its local error.
    for q in range(1, 6):
        gam = sum(1.0 / j for j in range(1, q + 1))
        assert bdf.GAMMA[q] == pytest.approx(gam, rel=1e-15)
        # exactness on t^q
        h, t1 = 0.1, 1.0
        y = lambda s: s ** q
        dif = _backward_differences(y, t1, h, q)
        lhs = sum(dif[j] / j for j in range(1, q + 1))
        assert lhs == pytest.approx(h * q * t1 ** (q - 1), rel=1e-10)
        # local error of the order-q formula on t^{q+1} is h^{q+1} (q+1)! / (q+1) ... scaled
        y2 = lambda s: s ** (q + 1)
        dif2 = _backward_differences(y2, t1, h, q + 1)
        resid = sum(dif2[j] / j for j in range(1, q + 1)) - h * (q + 1) * t1 ** q
        assert resid == pytest.approx(-bdf.ERRC[q] * dif2[q + 1], rel=1e-8)


def test_first_step_is_implicit_euler():
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    res = bdf.solve(ch, np.array([1.0, 0.0]), 5.0 / k, 1e-6, 1e-20, record=True)
    h, q, t, x = res.history[0]
    assert q == 1
    assert x[0] == pytest.approx(1.0 / (1.0 + h * k), rel=1e-14)
    assert x[1] == pytest.approx(1.0 - 1.0 / (1.0 + h * k), rel=1e-12)


def test_order_cap_one_is_implicit_euler_throughout():
    # max_order 1: every accepted step stays at order 1, and on the linear
    # decay each step multiplies x_A by 1 / (1 + k h), so x_A(t_end) is the
    # product over the recorded steps
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    res = bdf.solve(ch, np.array([1.0, 0.0]), 5.0 / k, 1e-6, 1e-20, record=True, max_order=1)
    assert res.status == bdf.OK and len(res.history) > 10
    assert all(q == 1 for (_h, q, _t, _x) in res.history)
    want = np.prod([1.0 / (1.0 + k * h) for (h, _q, _t, _x) in res.history])
    assert res.x[0] == pytest.approx(want, rel=1e-12)
    assert res.x[1] == pytest.approx(1.0 - want, rel=1e-12)
    # a cap of two on the 12-species network: orders stay <= 2, and an
    # uncapped run reaches higher ones
    small = synth.network_for_config("small")
    cells = synth.single_cell(small)
    chs = chem.cell_chemistry(small, cells.cell(0))
    r2 = bdf.solve(chs, cells.x0[0], cells.t_end[0], 1e-6, 1e-20, record=True, max_order=2)
    r5 = bdf.solve(chs, cells.x0[0], cells.t_end[0], 1e-6, 1e-20, record=True)
    assert r2.status == bdf.OK and max(q for (_h, q, _t, _x) in r2.history) == 2
    assert max(q for (_h, q, _t, _x) in r5.history) > 2
    with pytest.raises(ValueError):
        bdf.solve(ch, np.array([1.0, 0.0]), 1.0, max_order=6)


def test_step_bounds():
    # h0 is the first step taken, h_max bounds every step, and the solution is
    # still the exponential to the tolerance's reach
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    t_end, h0, h_max = 5.0 / k, 1e-9 / k, 5.0 / (400 * k)
    res = bdf.solve(ch, np.array([1.0, 0.0]), t_end, 1e-8, 1e-30, record=True, h0=h0, h_max=h_max)
    assert res.status == bdf.OK
    assert res.history[0][0] == h0
    assert all(h <= h_max * (1 + 1e-12) for (h, _q, _t, _x) in res.history)
    assert len(res.history) >= 400
    np.testing.assert_allclose(res.x, [np.exp(-5.0), -np.expm1(-5.0)], rtol=1e-6)
    free = bdf.solve(ch, np.array([1.0, 0.0]), t_end, 1e-8, 1e-30, record=True)
    assert max(h for (h, _q, _t, _x) in free.history) > h_max


def test_per_species_atol():
    # a vector of the scalar everywhere is the scalar run exactly; a huge atol on
    # B leaves the control to A, whose value stays the exponential
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    x0 = np.array([1.0, 0.0])
    a = bdf.solve(ch, x0, 5.0 / k, 1e-8, 1e-30)
    b = bdf.solve(ch, x0, 5.0 / k, 1e-8, np.array([1e-30, 1e-30]))
    assert np.array_equal(a.x, b.x) and a.stats.n_attempts == b.stats.n_attempts
    c = bdf.solve(ch, x0, 5.0 / k, 1e-8, np.array([1e-30, 1.0]))
    assert c.status == bdf.OK
    assert c.x[0] == pytest.approx(np.exp(-5.0), rel=1e-6)
    assert bdf.solve(ch, x0, 5.0 / k, 1e-8, np.array([1e-30, -1.0])).status == bdf.BAD_INPUT


def test_decay_matches_exponential():
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    # global relative error of x_A grows with the number of e-folds integrated
    for kt, tol in ((0.3, 1e-8), (5.0, 1e-8), (20.0, 1e-7)):
        res = bdf.solve(ch, np.array([1.0, 0.0]), kt / k, 1e-10, 1e-30)
        assert res.status == bdf.OK
        assert res.t == kt / k
        want = np.array([np.exp(-kt), -np.expm1(-kt)])
        np.testing.assert_allclose(res.x, want, rtol=tol)
    # and at the production tolerance within the tolerance's reach
    res = bdf.solve(ch, np.array([1.0, 0.0]), 5.0 / k, 1e-6, 1e-20)
    np.testing.assert_allclose(res.x, [np.exp(-5.0), -np.expm1(-5.0)], rtol=1e-4)


@pytest.mark.parametrize("a0,b0", [(3e-4, 1e-4), (1e-4, 1e-4), (1e-4, 5e-4)])
def test_association_matches_closed_form(a0, b0):
    net = tiny_nets.association(1e-9)
    ch = chem.cell_chemistry(net, CELL)
    kp = ch.k[0]          # already multiplied by n_H
    t = 3.0 / (kp * max(a0, b0))
    res = bdf.solve(ch, np.array([a0, b0, 0.0]), t, 1e-10, 1e-30)
    d = a0 - b0
    if d == 0:
        a = a0 / (1 + kp * a0 * t)
    else:
        a = d / (1 - (b0 / a0) * np.exp(-kp * d * t))
    want = np.array([a, a - d, a0 - a])
    np.testing.assert_allclose(res.x, want, rtol=1e-8)


def test_first_order_network_matches_matrix_exponential():
    net = tiny_nets.first_order()
    cell = dict(T=20.0, n_H=1e3, A_V=0.5, zeta=1e-16, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    K = ch.jac(np.zeros(net.n_species))     # constant: all reactions are one-body
    x0 = np.zeros(net.n_species)
    x0[net.index("H2")] = 0.5
    x0[net.index("CO")] = 1e-4
    t = 1e6 * YEAR
    res = bdf.solve(ch, x0, t, 1e-10, 1e-30)
    want = sla.expm(t * K) @ x0
    m = want > 1e-12
    np.testing.assert_allclose(res.x[m], want[m], rtol=1e-8)


def test_small_network_conserves_elements_and_charge():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    res = bdf.solve(ch, cells.x0[0], cells.t_end[0], 1e-6, 1e-20, record=True)
    assert res.status == bdf.OK
    W = net.conservation_matrix().astype(float)
    w0 = W @ cells.x0[0]
    for (_h, _q, _t, x) in res.history[:: max(1, len(res.history) // 20)] + [res.history[-1]]:
        # relative to the conserved quantity's own terms, with a rounding floor
        # set by the whole state (the linear solves mix all species)
        bound = 1e-12 * (np.abs(W) @ np.abs(x)) + 1e-15 * np.abs(x).sum()
        assert np.all(np.abs(W @ x - w0) <= bound)


def test_order_and_step_adapt_on_smooth_problem():
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    res = bdf.solve(ch, np.array([1.0, 0.0]), 30.0 / k, 1e-8, 1e-30, record=True)
    orders = [q for (_h, q, _t, _x) in res.history]
    assert max(orders) >= 4
    assert res.stats.n_steps < 1000


def test_status_codes():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0 = cells.x0[0]
    assert bdf.solve(ch, x0, cells.t_end[0], max_steps=3).status == bdf.MAX_STEPS
    assert bdf.solve(ch, x0, cells.t_end[0], rtol=0.0).status == bdf.BAD_INPUT
    bad = x0.copy()
    bad[1] = np.nan
    assert bdf.solve(ch, bad, cells.t_end[0]).status == bdf.BAD_INPUT
    r = bdf.solve(ch, x0, 0.0)
    assert r.status == bdf.OK and np.array_equal(r.x, x0)


def test_recorded_history_holds_the_accepted_states():
    # each record is (h, q, t, x) after the accepted step: the last equals the result,
    # and the times advance by the recorded steps to t_end
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    t_end = 4.0 / ch.k[0]
    res = bdf.solve(ch, np.array([1.0, 0.0]), t_end, 1e-6, 1e-20, record=True)
    assert np.allclose(res.history[-1][3], res.x, rtol=1e-14, atol=0)
    assert res.history[-1][2] == t_end
    t = 0.0
    for h, q, t_rec, _x in res.history[:-1]:
        t += h
        assert t_rec == pytest.approx(t, rel=1e-12)


def _hnw_linear(y0, lam, sc, t_span):
    """The starting step of Hairer, Norsett & Wanner (Solving ODEs I, Sec. II.4,
    order p = 1) for y' = lam y, written with the exact derivatives of the linear
    problem: y' = lam y0, y'' = lam^2 y0 (the algorithm estimates the latter by a
    difference quotient over one explicit Euler step, which is exact here up to
    rounding)."""
    rms = lambda v: np.sqrt(np.mean((v / sc) ** 2))
    d0, d1, d2 = rms(y0), rms(lam * y0), rms(lam ** 2 * y0)
    h0 = 1e-6 if (d0 < 1e-5 or d1 < 1e-5) else 0.01 * d0 / d1
    h0 = min(h0, t_span)
    h1 = max(1e-6, 1e-3 * h0) if max(d1, d2) <= 1e-15 else (0.01 / max(d1, d2)) ** 0.5
    return min(100.0 * h0, h1, t_span), d0, d1, d2, h0


@pytest.mark.parametrize("case", ["curvature", "cap_100_h0", "t_span", "tiny_state", "no_motion"])
def test_initial_step_on_linear_problem(case):
    # each case makes a different term of the starting-step rule decide
    y0 = np.array([1.0, 2.0, 3.0])
    rtol, atol, t_span = 1e-3, 0.0, 1e9
    lam = np.array([-1e3, -2e3, -3e3])
    if case == "cap_100_h0":        # weights dominated by atol: d0 = 1e-3, |lam| = 5
        y0, atol, rtol, lam = np.full(3, 1e-9), 1e-6, 1e-12, np.full(3, -5.0)
    elif case == "t_span":
        t_span = 1e-7
    elif case == "tiny_state":      # d0 < 1e-5: h0 = 1e-6
        y0, atol = np.full(3, 1e-12), 1e-6
    elif case == "no_motion":       # f = 0
        lam = np.zeros(3)
    sc = atol + rtol * np.abs(y0)
    f = lambda y: lam * y
    h = bdf.initial_step(f, y0, f(y0), t_span, rtol, atol)
    want, d0, d1, d2, h0 = _hnw_linear(y0, lam, sc, t_span)
    assert h == pytest.approx(want, rel=1e-12)
    if case == "curvature":
        # the defining condition of the order-1 rule: h^2 max(d1, d2) = 0.01
        assert d2 > d1 and h < 100 * h0
        assert h * h * max(d1, d2) == pytest.approx(0.01, rel=1e-12)
    elif case == "cap_100_h0":
        assert h == pytest.approx(100.0 * 0.01 * d0 / d1, rel=1e-12)
        assert h * h * max(d1, d2) < 0.01
    elif case == "t_span":
        assert h == t_span
    elif case == "tiny_state":
        assert d0 < 1e-5 and h0 == 1e-6
    else:
        assert h == 1e-6


def test_oracle_conservation_drift_on_connected_networks():
    # W f = 0 and W (I - c J) = W, so W x is conserved in exact arithmetic; the
    # oracle's FP64 LAPACK solves at the condition numbers of the connected
    # 200-species network (up to ~1e7) let it drift.  This measures that drift
    # on the cells behind the conservation bars of the GPU tests: cell 2840 of
    # the seeded 4096-cell batch (the largest drift found in that batch) and the
    # cells of the small-batch parity test.  The GPU bars are set above the
    # oracle's own: 1e-12 sum_i |W_ei x_i| + 1e-8 |x|_1 for the small batches,
    # 1e-7 |x|_1 over the 4096-cell batch.
    from threadpoolctl import threadpool_limits
    net = synth.network_for_config("net200")
    W = net.conservation_matrix().astype(float)

    def drift(cells, c):
        with threadpool_limits(1):
            r = bdf.solve(chem.cell_chemistry(net, cells.cell(c)), cells.x0[c], cells.t_end[c], 1e-6, 1e-20)
        assert r.status == bdf.OK
        return float(np.max(np.abs(W @ r.x - W @ cells.x0[c]))) / np.abs(r.x).sum(), r.x

    big = synth.sample_cells(net, 4096, seed=2001, t_end_yr=1e6)
    d2840, x = drift(big, 2840)
    # far above 1e-12 of the conserved totals, and within the GPU's batch bar
    assert 1e-9 < d2840 < 1e-7 / 4
    assert np.max(np.abs(W @ x - W @ big.x0[2840]) / (np.abs(W) @ np.abs(x))) > 1e-9
    small = synth.sample_cells(net, 6, seed=2001)
    for c in range(small.n):
        d, x = drift(small, c)
        assert d <= 1e-8, (c, d)


def test_finite_time_blow_up_ends_with_step_too_small():
    # A + B -> C from x_A = x_B = a0 < 0 (abundances are never clipped): x_A' =
    # -k' x_A^2 has x_A(t) = a0 / (1 + k' a0 t), which blows up at t* = 1 / (k' |a0|).
    # The step control shrinks h towards t* until h < 10 u t: STEP_TOO_SMALL,
    # with the blow-up time the solution implies, t + 1 / (k' |x_A|), at t*
    net = tiny_nets.association(1e-9)
    ch = chem.cell_chemistry(net, dict(T=300.0, n_H=1e4, A_V=0.0, zeta=1e-17, G0=1.0))
    kp, a0 = ch.k[0], -1e-4
    t_star = 1.0 / (kp * abs(a0))
    r = bdf.solve(ch, np.array([a0, a0, 0.0]), 2 * t_star, 1e-6, 1e-20)
    assert r.status == bdf.STEP_TOO_SMALL
    assert r.stats.h < 10 * bdf.U_ROUND * r.t
    assert abs(r.t - t_star) <= 1e-4 * t_star and r.t < t_star
    assert abs(r.t + 1.0 / (kp * abs(r.x[0])) - t_star) <= 1e-4 * t_star
    assert r.x[0] == r.x[1] and abs(r.x[2] + r.x[0] - a0) <= 1e-12 * abs(r.x[0])


def test_rates_overflowing_at_the_initial_state_end_as_nonfinite():
    net = tiny_nets.association(1e-9)
    ch = chem.cell_chemistry(net, dict(T=300.0, n_H=1e4, A_V=0.0, zeta=1e-17, G0=1.0))
    x0 = np.array([1e200, 1e200, 0.0])
    with np.errstate(over="ignore", invalid="ignore"):
        r = bdf.solve(ch, x0, 1e10, 1e-6, 1e-20)
    assert r.status == bdf.NONFINITE and r.t == 0.0 and np.array_equal(r.x, x0)


def _expansion_integral(t, t_c, p):
    """int_0^t (1 + s / t_c)^(-p) ds."""
    if p == 1.0:
        return t_c * np.log1p(t / t_c)
    return t_c * ((1.0 + t / t_c) ** (1.0 - p) - 1.0) / (1.0 - p)


@pytest.mark.parametrize("p", [0.5, 1.0, 1.5, 2.0])
def test_decay_under_falling_ionisation_rate(p):
    # A -> B by cosmic rays with zeta(t) = zeta0 (1 + t / t_c)^(-p):
    # x_A(t) = exp(-alpha zeta0 int_0^t (1 + s / t_c)^(-p) ds)
    net = tiny_nets.decay(2.0)
    cell = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)
    k0 = 2.0 * cell["zeta"]
    t_end = 3.0 / k0
    t_c = 0.5 * t_end
    ch = chem.TrajectoryChemistry(net, cell, t_c, [0.0, 0.0, 0.0, p, 0.0])
    r = bdf.solve(ch, np.array([1.0, 0.0]), t_end, 1e-10, 1e-30)
    want = np.exp(-k0 * _expansion_integral(t_end, t_c, p))
    assert r.status == bdf.OK
    np.testing.assert_allclose(r.x, [want, 1.0 - want], rtol=1e-7)


def test_association_under_expanding_density():
    # A + B -> C, two-body coefficient k n_H with n_H(t) = n_H0 (1 + t/t_c)^-2:
    # for a0 = b0, 1/a - 1/a0 = k n_H0 int_0^t (1 + s/t_c)^-2 ds
    net = tiny_nets.association(1e-9)
    cell = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)
    kp = chem.rate_coefficients(net, **cell)[0]
    a0 = 2e-4
    t_end = 5.0 / (kp * a0)
    t_c = 0.3 * t_end
    ch = chem.TrajectoryChemistry(net, cell, t_c, [0.0, 2.0, 1.0, 0.0, 0.0])
    r = bdf.solve(ch, np.array([a0, a0, 0.0]), t_end, 1e-10, 1e-30)
    a = a0 / (1.0 + a0 * kp * _expansion_integral(t_end, t_c, 2.0))
    assert r.status == bdf.OK
    np.testing.assert_allclose(r.x, [a, a, a0 - a], rtol=1e-7)


def test_constant_trajectory_is_the_autonomous_solve():
    # t_c = 0 (and all exponents 0) leave the conditions constant: the same
    # steps and the same result bit for bit as the autonomous solve
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    cell = cells.cell(0)
    ref = bdf.solve(chem.cell_chemistry(net, cell), cells.x0[0], cells.t_end[0], 1e-6, 1e-20)
    for t_c, p in ((0.0, [0.7, 2.0, 1.0, 0.0, 0.0]), (1e10, [0.0] * 5)):
        r = bdf.solve(chem.TrajectoryChemistry(net, cell, t_c, p), cells.x0[0], cells.t_end[0], 1e-6, 1e-20)
        assert np.array_equal(r.x, ref.x) and r.stats.n_steps == ref.stats.n_steps
    tr = chem.TrajectoryChemistry(net, cell, 1e10, [0.7, 2.0, 1.0, 0.5, 0.0])
    ph = tr.phi(1e10)
    assert ph["T"] == pytest.approx(cell["T"] * 2 ** -0.7) and ph["n_H"] == pytest.approx(cell["n_H"] / 4)
    assert ph["G0"] == cell["G0"] and tr.phi(0.0) == cell


def test_initial_step_takes_the_trial_evaluation_at_h0():
    # y' = lam(t) y with lam(t) = lam0 (1 + t / tau)^-2: the trial evaluation
    # of the starting-step rule is f(h0, y0 + h0 f0) = lam(h0) (1 + h0 lam0) y0,
    # so d2 = |lam(h0) (1 + h0 lam0) - lam0| d0 / h0 exactly (up to rounding)
    y0 = np.array([1.0, 2.0, 3.0])
    rtol, atol = 1e-3, 0.0
    lam0, tau = -2e3, 1e-4
    lam = lambda t: lam0 * (1.0 + t / tau) ** -2
    sc = atol + rtol * np.abs(y0)
    rms = lambda v: np.sqrt(np.mean((v / sc) ** 2))
    d0, d1 = rms(y0), rms(lam0 * y0)
    h0 = 0.01 * d0 / d1
    d2 = abs(lam(h0) * (1.0 + h0 * lam0) - lam0) * d0 / h0
    want = min(100 * h0, (0.01 / max(d1, d2)) ** 0.5, 1e9)
    h = bdf.initial_step(lambda y: lam0 * y, y0, lam0 * y0, 1e9, rtol, atol, ft=lambda t, y: lam(t) * y)
    assert h == pytest.approx(want, rel=1e-12)
    assert h != pytest.approx(bdf.initial_step(lambda y: lam0 * y, y0, lam0 * y0, 1e9, rtol, atol), rel=1e-3)
