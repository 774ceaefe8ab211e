"""Pins for the oracle's ESDIRK integrator (CPU only).

The tableau is pinned by Butcher's order conditions (every rooted tree up to
five nodes, enumerated here), by its structure (explicit first stage, singly
diagonal, stiffly accurate, stage order 2) and by its stability function; the
integrator by the observed convergence order on closed-form problems, by the
closed forms themselves and by conservation of elements and charge.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import bdf, brute, chem, esdirk
from tests import tiny_nets

YEAR = synth.YEAR_S
CELL = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)


# ---------------------------------------------------------------- Butcher trees
def rooted_trees(n):
    """All rooted trees with n nodes, each a sorted tuple of its subtrees."""
    if n == 1:
        return [()]
    out = set()

    def forests(m, smallest):
        # multisets of trees with m nodes in total, listed in non-decreasing order
        if m == 0:
            yield ()
            return
        for k in range(1, m + 1):
            for t in rooted_trees(k):
                key = (k, t)
                if smallest is not None and key < smallest:
                    continue
                for rest in forests(m - k, key):
                    yield (t,) + rest

    for f in forests(n - 1, None):
        out.add(tuple(sorted(f)))
    return sorted(out)


def order_of(t):
    return 1 + sum(order_of(s) for s in t)


def density(t):
    """gamma(t) = |t| prod gamma(children)."""
    g = order_of(t)
    for s in t:
        g *= density(s)
    return g


def internal_weights(t, A):
    """Phi_i(t): the product over the children of (A Phi(child))_i."""
    v = np.ones(A.shape[0])
    for s in t:
        v = v * (A @ internal_weights(s, A))
    return v


def test_tree_counts():
    # the number of rooted trees with n nodes (Cayley): 1, 1, 2, 4, 9, 20
    assert [len(rooted_trees(n)) for n in range(1, 7)] == [1, 1, 2, 4, 9, 20]


@pytest.mark.parametrize("row,order", [(6, 5), (5, 4)])
def test_tableau_satisfies_the_order_conditions(row, order):
    A, b = esdirk.A, esdirk.A[row]
    for n in range(1, order + 1):
        for t in rooted_trees(n):
            assert b @ internal_weights(t, A) == pytest.approx(1.0 / density(t), abs=2e-16), (n, t)
    # and no more: some tree of the next order is missed by a clear margin
    worst = max(abs(b @ internal_weights(t, A) - 1.0 / density(t)) for t in rooted_trees(order + 1))
    assert worst > 1e-4


def test_tableau_structure():
    A, c, g = esdirk.A, esdirk.C, esdirk.GAMMA
    assert np.all(A[0] == 0.0)
    assert np.all(np.triu(A, 1) == 0.0)
    assert np.all(np.diag(A)[1:] == g)
    # stiffly accurate pair: the results are stages, both at the step's end
    assert c[5] == pytest.approx(1.0, abs=1e-15) and c[6] == pytest.approx(1.0, abs=1e-15)
    # stage order 2 on every stage: A c = c^2 / 2
    np.testing.assert_allclose(A @ c, c ** 2 / 2, atol=2e-16)
    assert abs(esdirk.E.sum()) < 1e-15 and np.all(esdirk.E == A[6] - A[5])


class Linear:
    """x' = lam x (componentwise), with its exact Jacobian."""

    def __init__(self, lam):
        self.lam = np.asarray(lam, dtype=complex)
        self.k = self.lam

    def f(self, x):
        return self.lam * x

    def jac(self, x):
        return np.diag(self.lam)


def stability(z):
    """R(z) of one step, from the integrator's own step on x' = z x, h = 1."""
    lin = Linear([z])
    lu = sla.lu_factor(np.eye(1) - esdirk.GAMMA * lin.jac(None))
    ok, x, _G, _e = esdirk.step(lin, np.array([1.0 + 0j]), lin.f(np.array([1.0 + 0j])), 1.0, lu,
                                1e-14, 1e-8, 0.0, bdf.Stats(), maxiter=20)
    assert ok
    return x[0]


def test_stability_function():
    # e^z to fifth order: the defect shrinks as z^6
    d1, d2 = abs(stability(-0.1) - np.exp(-0.1)), abs(stability(-0.05) - np.exp(-0.05))
    assert 5.6 < np.log2(d1 / d2) < 6.4
    # L-stable: |R| -> 0 at infinity
    assert abs(stability(-1e8)) < 1e-6
    # A-stable: |R| <= 1 on the imaginary axis and in the left half-plane
    for y in np.logspace(-2, 4, 60):
        assert abs(stability(1j * y)) <= 1.0 + 1e-12
    rng = np.random.default_rng(3)
    for z in -np.abs(rng.normal(size=40)) * 30 + 1j * rng.normal(size=40) * 30:
        assert abs(stability(z)) <= 1.0 + 1e-12


def _assoc_exact(a0, b0, kp, t):
    d = a0 - b0
    a = d / (1 - (b0 / a0) * np.exp(-kp * d * t))
    return np.array([a, a - d, a0 - a])


def _fixed_steps(ch, x0, t_end, n):
    """n equal steps, the stage equations solved to rounding level."""
    h = t_end / n
    x, F1 = x0.copy(), ch.f(x0)
    st = bdf.Stats()
    for _ in range(n):
        lu = sla.lu_factor(np.eye(x.size) - h * esdirk.GAMMA * ch.jac(x))
        ok, x, G, e = esdirk.step(ch, x, F1, h, lu, 1e-13, 1e-8, 1e-30, st, maxiter=60)
        assert ok
        F1 = G[-1] / h
    return x, e


def test_convergence_order_on_association():
    net = tiny_nets.association(1e-9)
    ch = chem.cell_chemistry(net, CELL)
    kp = ch.k[0]
    a0, b0 = 3e-4, 1e-4
    t = 3.0 / (kp * a0)
    x0 = np.array([a0, b0, 0.0])
    want = _assoc_exact(a0, b0, kp, t)
    errs = [np.abs(_fixed_steps(ch, x0, t, n)[0] - want).max() for n in (6, 12, 24)]
    p1, p2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert 4.6 < p1 < 5.6 and 4.6 < p2 < 5.6, (errs, p1, p2)
    # the embedded difference of one step from the same point shrinks as h^5
    # (the fourth-order method's local error)
    e = []
    for h in (t / 8, t / 16, t / 32):
        lu = sla.lu_factor(np.eye(3) - h * esdirk.GAMMA * ch.jac(x0))
        ok, _x, _G, ev = esdirk.step(ch, x0, ch.f(x0), h, lu, 1e-13, 1e-8, 1e-30, bdf.Stats(), maxiter=60)
        e.append(np.abs(ev).max())
    assert 4.5 < np.log2(e[1] / e[2]) < 5.5, e


def test_decay_matches_exponential():
    net = tiny_nets.decay(2.0)
    ch = chem.cell_chemistry(net, CELL)
    k = ch.k[0]
    for kt, rtol, tol in ((0.3, 1e-10, 1e-8), (20.0, 1e-10, 1e-7), (5.0, 1e-6, 1e-4)):
        res = esdirk.solve(ch, np.array([1.0, 0.0]), kt / k, rtol, 1e-30)
        assert res.status == esdirk.OK and res.t == kt / k
        np.testing.assert_allclose(res.x, [np.exp(-kt), -np.expm1(-kt)], rtol=tol)


@pytest.mark.parametrize("a0,b0", [(3e-4, 1e-4), (1e-4, 5e-4)])
def test_association_matches_closed_form(a0, b0):
    net = tiny_nets.association(1e-9)
    ch = chem.cell_chemistry(net, CELL)
    kp = ch.k[0]
    t = 3.0 / (kp * max(a0, b0))
    res = esdirk.solve(ch, np.array([a0, b0, 0.0]), t, 1e-10, 1e-30)
    assert res.status == esdirk.OK
    np.testing.assert_allclose(res.x, _assoc_exact(a0, b0, kp, t), rtol=1e-8)


def test_first_order_network_matches_matrix_exponential():
    net = tiny_nets.first_order()
    cell = dict(T=20.0, n_H=1e3, A_V=0.5, zeta=1e-16, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    K = ch.jac(np.zeros(net.n_species))
    x0 = np.zeros(net.n_species)
    x0[net.index("H2")] = 0.5
    x0[net.index("CO")] = 1e-4
    t = 1e6 * YEAR
    res = esdirk.solve(ch, x0, t, 1e-10, 1e-30)
    want = sla.expm(t * K) @ x0
    m = want > 1e-12
    np.testing.assert_allclose(res.x[m], want[m], rtol=1e-8)


def test_small_network_conserves_elements_and_charge_and_agrees_with_bdf():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0, t_end = cells.x0[0], cells.t_end[0]
    res = esdirk.solve(ch, x0, t_end, 1e-6, 1e-20, record=True)
    assert res.status == esdirk.OK and res.t == t_end
    W = net.conservation_matrix().astype(float)
    w0 = W @ x0
    for (_h, _q, _t, x) in res.history:
        bound = 1e-12 * (np.abs(W) @ np.abs(x)) + 1e-15 * np.abs(x).sum()
        assert np.all(np.abs(W @ x - w0) <= bound)
    # the element totals' rounding-level drift aside, the BDF oracle at a tight
    # tolerance is the reference here; the brute-force comparison is slow
    ref = bdf.solve(ch, x0, t_end, 1e-11, 1e-30).x
    m = ref > 1e-12 * x0.sum()
    np.testing.assert_allclose(res.x[m], ref[m], rtol=1e-3)
    tight = esdirk.solve(ch, x0, t_end, 1e-10, 1e-30)
    np.testing.assert_allclose(tight.x[m], ref[m], rtol=2e-6)


@pytest.mark.slow
def test_small_network_against_brute_force_radau():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0, t_end = cells.x0[0], cells.t_end[0]
    ref, _n, achieved = brute.converged_solution(ch, x0, t_end, t_first=10.0, rel=1e-10)
    assert achieved <= 1e-10
    m = ref > 1e-12
    tight = esdirk.solve(ch, x0, t_end, 1e-10, 1e-30).x
    assert np.max(np.abs(tight[m] - ref[m]) / ref[m]) <= 1e-7
    loose = esdirk.solve(ch, x0, t_end, 1e-6, 1e-20).x
    assert np.max(np.abs(loose[m] - ref[m]) / ref[m]) <= 1e-4


def test_counters_and_controller():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    res = esdirk.solve(ch, cells.x0[0], cells.t_end[0], 1e-6, 1e-20, record=True)
    st = res.stats
    assert st.n_attempts == st.n_steps + st.n_err_reject + st.n_newton_fail
    assert st.n_lu == st.n_attempts            # one factorisation per attempt
    assert st.n_jac == st.n_steps              # at x0 and after every accepted step but the last
    assert st.n_rhs == st.n_newton_iter + 2    # the initial and trial evaluations
    assert st.n_newton_iter >= 6 * st.n_attempts - 6 * st.n_newton_fail
    hs = np.array([h for (h, _q, _t, _x) in res.history])
    # accepted steps never grow by more than the factor bound
    assert np.all(hs[1:-1] <= esdirk.MAX_FACTOR * hs[:-2] * (1 + 1e-15))
    ts = np.array([t for (_h, _q, t, _x) in res.history])
    assert ts[-1] == cells.t_end[0] and np.all(np.diff(ts) > 0)


def test_status_codes():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0 = cells.x0[0]
    assert esdirk.solve(ch, x0, cells.t_end[0], max_steps=3).status == esdirk.MAX_STEPS
    assert esdirk.solve(ch, x0, cells.t_end[0], rtol=0.0).status == esdirk.BAD_INPUT
    r = esdirk.solve(ch, x0, 0.0)
    assert r.status == esdirk.OK and np.array_equal(r.x, x0)
    # rates overflowing at the initial state: no step is taken
    cha = chem.cell_chemistry(tiny_nets.association(1e-9), dict(T=300.0, n_H=1e4, A_V=0.0, zeta=1e-17, G0=1.0))
    xb = np.array([1e200, 1e200, 0.0])
    with np.errstate(over="ignore", invalid="ignore"):
        r = esdirk.solve(cha, xb, 1e10, 1e-6, 1e-20)
    assert r.status == esdirk.NONFINITE and r.t == 0.0 and np.array_equal(r.x, xb)


def test_finite_time_blow_up_ends_with_step_too_small():
    # A + B -> C from x_A = x_B = a0 < 0: x_A(t) = a0 / (1 + k' a0 t) blows up at
    # t* = 1 / (k' |a0|); the controller shrinks h towards t* until h < 10 u t
    ch = chem.cell_chemistry(tiny_nets.association(1e-9), dict(T=300.0, n_H=1e4, A_V=0.0, zeta=1e-17, G0=1.0))
    kp, a0 = ch.k[0], -1e-4
    t_star = 1.0 / (kp * abs(a0))
    r = esdirk.solve(ch, np.array([a0, a0, 0.0]), 2 * t_star, 1e-6, 1e-20)
    assert r.status == esdirk.STEP_TOO_SMALL
    assert r.stats.h < 10 * bdf.U_ROUND * r.t
    assert abs(r.t - t_star) <= 1e-4 * t_star and r.t < t_star
    assert abs(r.t + 1.0 / (kp * abs(r.x[0])) - t_star) <= 1e-4 * t_star


def test_initial_step_for_the_fifth_order_method():
    # y' = lam y: the rule's defining condition for order 5 is h^6 max(d1, d2) = 0.01
    # (slow enough modes that the 100 h0 cap does not decide)
    y0 = np.array([1.0, 2.0, 3.0])
    lam = np.array([-1.0, -2.0, -3.0])
    rtol, atol = 1e-3, 0.0
    sc = atol + rtol * np.abs(y0)
    rms = lambda v: np.sqrt(np.mean((v / sc) ** 2))
    d0, d1, d2 = rms(y0), rms(lam * y0), rms(lam ** 2 * y0)
    h = bdf.initial_step(lambda y: lam * y, y0, lam * y0, 1e9, rtol, atol, order=5)
    assert h < 100 * 0.01 * d0 / d1
    assert h ** 6 * max(d1, d2) == pytest.approx(0.01, rel=1e-10)
