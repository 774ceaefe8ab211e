"""Pins of the oracle against steady states, brute force and sensitivities (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import bdf, brute, chem, steady
from tests import tiny_nets

YEAR = synth.YEAR_S


def test_dimer_steady_state_closed_form():
    # H + H -> H2 (k1' = alpha n_H) and H2 -> 2H (k2): k1' x^2 = k2 (1 - x)/2 with
    # x = x_H and x_H + 2 x_H2 = 1; the positive root of 2 k1' x^2 + k2 x - k2 = 0.
    net = tiny_nets.dimer(alpha_f=1e-11, alpha_d=5e-12, gamma_d=1.0)
    cell = dict(T=20.0, n_H=100.0, A_V=1.0, zeta=1e-17, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    k1, k2 = ch.k
    x = (-k2 + np.sqrt(k2 * k2 + 8 * k1 * k2)) / (4 * k1)
    want = np.array([x, (1 - x) / 2])
    x0 = np.array([1.0, 0.0])
    W = net.conservation_matrix()
    ss, ok, _ = steady.steady_state(ch, W, x0, np.array([0.5, 0.25]))
    assert ok
    np.testing.assert_allclose(ss, want, rtol=1e-12)
    res = bdf.solve(ch, x0, 1e12 * YEAR, 1e-10, 1e-30)
    np.testing.assert_allclose(res.x, want, rtol=1e-8)


def test_long_time_bdf_reaches_newton_steady_state():
    # A dense, shielded cell settles within 1e7 yr.  (Much longer horizons are
    # out of reach of this Newton test in FP64: at steps with h k ~ 1e7 the
    # residual c f(x) carries rounding noise of the gross rates above the
    # corrections, the contraction ratio reaches 1 and attempts are rejected.)
    net = synth.large_network(80, 400, seed=11, mix=(0.85, 0.05, 0.1))
    cells = synth.sample_cells(net, 1, seed=12)
    cells.n_H[:], cells.T[:], cells.A_V[:] = 1e5, 20.0, 10.0
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0 = cells.x0[0]
    res = bdf.solve(ch, x0, 1e7 * YEAR, 1e-8, 1e-30)
    assert res.status == bdf.OK
    ss, ok, _ = steady.steady_state(ch, net.conservation_matrix(), x0, res.x)
    assert ok
    m = ss > 1e-12
    assert np.max(np.abs(res.x[m] - ss[m]) / ss[m]) <= 1e-6
    assert np.max(np.abs(ch.f(ss))) <= 1e-20 + 1e-12 * np.max(np.abs(ch.f(x0)))


@pytest.mark.slow
def test_small_network_against_brute_force_radau():
    net = synth.network_for_config("small")
    cells = synth.single_cell(net)
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0, t_end = cells.x0[0], cells.t_end[0]
    ref, n, achieved = brute.converged_solution(ch, x0, t_end, t_first=10.0, rel=1e-10)
    assert achieved <= 1e-10
    m = ref > 1e-12
    tight = bdf.solve(ch, x0, t_end, 1e-10, 1e-30).x
    assert np.max(np.abs(tight[m] - ref[m]) / ref[m]) <= 1e-7
    loose = bdf.solve(ch, x0, t_end, 1e-6, 1e-20).x
    assert np.max(np.abs(loose[m] - ref[m]) / ref[m]) <= 1e-4


def test_decay_sensitivity_closed_form():
    # x_A = exp(-kt): d log x_A / d log alpha = -kt;
    # x_B = 1 - exp(-kt): d log x_B / d log alpha = kt e^{-kt} / (1 - e^{-kt}).
    net = tiny_nets.decay(2.0)
    cell = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    k = ch.k[0]
    t = 3.0 / k
    res = bdf.solve(ch, np.array([1.0, 0.0]), t, 1e-10, 1e-30, record=True)
    x, Sx = bdf.replay(ch, np.array([1.0, 0.0]), res.history,
                       sens_dfdp=lambda y: ch.df_dlogalpha(y).toarray())
    kt = k * t
    assert Sx[0, 0] / x[0] == pytest.approx(-kt, rel=1e-6)
    assert Sx[1, 0] / x[1] == pytest.approx(kt * np.exp(-kt) / -np.expm1(-kt), rel=1e-6)


def test_first_order_sensitivity_matches_expm_frechet():
    net = tiny_nets.first_order()
    cell = dict(T=20.0, n_H=1e3, A_V=0.5, zeta=1e-16, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    S = net.n_species
    K = ch.jac(np.zeros(S))
    x0 = np.zeros(S)
    x0[net.index("H2")] = 0.5
    x0[net.index("CO")] = 1e-4
    t = 3e4 * YEAR
    res = bdf.solve(ch, x0, t, 1e-9, 1e-30, record=True)
    x, Sx = bdf.replay(ch, x0, res.history, sens_dfdp=lambda y: ch.df_dlogalpha(y).toarray())
    want = np.zeros_like(Sx)
    for r in range(net.n_reactions):
        # K depends linearly on alpha_r: dK/dlog alpha_r = nu[:, r] (d rate_r/dx)
        nu = chem.stoichiometry(net).toarray()[:, r:r + 1]
        drow = chem.rate_derivative(net, ch.k, np.zeros(S)).toarray()[r:r + 1]
        dK = nu @ drow
        _, L = sla.expm_frechet(t * K, t * dK)
        want[:, r] = L @ x0
    # entries are compared on the scale of the largest gradient entry
    assert np.max(np.abs(Sx - want)) <= 1e-6 * np.abs(want).max()


def test_sensitivity_is_exact_derivative_of_frozen_map():
    # d log x / d log alpha from the discrete forward sensitivities against central
    # differences of the frozen-sequence map, for the reactions that move the
    # solution most; compared on the scale of the largest log-gradient entry.
    net = synth.network_for_config("small")
    cells = synth.single_cell(net, t_end_yr=1e5)
    ch = chem.cell_chemistry(net, cells.cell(0))
    x0, t_end = cells.x0[0], cells.t_end[0]
    res = bdf.solve(ch, x0, t_end, 1e-6, 1e-20, record=True)
    x, Sx = bdf.replay(ch, x0, res.history, sens_dfdp=lambda y: ch.df_dlogalpha(y).toarray())
    m = x > 1e-12
    G = Sx[m] / x[m, None]
    reacts = np.argsort(-np.abs(G).max(axis=0))[:4]
    delta = 1e-4
    gscale = np.abs(G).max()
    for r in reacts:
        kp, km = ch.k.copy(), ch.k.copy()
        kp[r] *= np.exp(delta)
        km[r] *= np.exp(-delta)
        xp = bdf.replay(chem.Chemistry(net, kp), x0, res.history)
        xm = bdf.replay(chem.Chemistry(net, km), x0, res.history)
        fd = (np.log(xp[m]) - np.log(xm[m])) / (2 * delta)
        assert np.max(np.abs(fd - G[:, r])) <= 1e-5 * gscale


def test_phys_gradient_decay_closed_form():
    # A -> B by cosmic rays, k = alpha zeta: d log x_A / d zeta = -alpha t, and
    # no other parameter enters
    net = tiny_nets.decay(2.0)
    cell = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    t = 3.0 / ch.k[0]
    res = bdf.solve(ch, np.array([1.0, 0.0]), t, 1e-10, 1e-30, record=True)
    x, Sx = bdf.replay(ch, np.array([1.0, 0.0]), res.history,
                       sens_dfdp=lambda y: ch.df_dlogalpha(y).toarray())
    gphi = chem.phys_gradient(net, cell, Sx[0] / x[0])
    assert gphi[3] == pytest.approx(-2.0 * t, rel=1e-6)
    assert np.all(gphi[[0, 1, 2, 4]] == 0)


def test_phys_gradient_first_order_matches_expm_frechet():
    # x(t) = expm(tK) x0 with K linear in every k_r: for a parameter phi,
    # dK/dphi = sum_r (d log k_r / d phi) dK/dlog alpha_r and dx/dphi is the
    # Frechet derivative of expm along t dK/dphi applied to x0
    net = tiny_nets.first_order()
    cell = dict(T=20.0, n_H=1e3, A_V=0.5, zeta=1e-16, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    S = net.n_species
    K = ch.jac(np.zeros(S))
    x0 = np.zeros(S)
    x0[net.index("H2")] = 0.5
    x0[net.index("CO")] = 1e-4
    t = 3e4 * YEAR
    w = np.random.default_rng(11).uniform(-1, 1, S)
    res = bdf.solve(ch, x0, t, 1e-9, 1e-30, record=True)
    x, Sx = bdf.replay(ch, x0, res.history, sens_dfdp=lambda y: ch.df_dlogalpha(y).toarray())
    gphi = chem.phys_gradient(net, cell, w @ Sx)
    D = chem.log_rate_derivatives(net, **cell)
    nu = chem.stoichiometry(net).toarray()
    drate = chem.rate_derivative(net, ch.k, np.zeros(S)).toarray()
    for j in (2, 3, 4):      # A_V, zeta, G0 (no two-body reaction: T, n_H do not enter)
        dK = sum(D[r, j] * np.outer(nu[:, r], drate[r]) for r in range(net.n_reactions))
        _, L = sla.expm_frechet(t * K, t * dK)
        want = w @ (L @ x0)
        assert gphi[j] == pytest.approx(want, rel=1e-6, abs=1e-12 * abs(want))
    assert gphi[0] == 0 and gphi[1] == 0


def test_phys_gradient_is_derivative_of_frozen_map():
    # every parameter of the 12-species cell against central differences of the
    # frozen-sequence map in that parameter (the rates are recomputed)
    net = synth.network_for_config("small")
    cells = synth.single_cell(net, t_end_yr=1e5)
    cell = cells.cell(0)
    ch = chem.cell_chemistry(net, cell)
    x0, t_end = cells.x0[0], cells.t_end[0]
    res = bdf.solve(ch, x0, t_end, 1e-6, 1e-20, record=True)
    x, Sx = bdf.replay(ch, x0, res.history, sens_dfdp=lambda y: ch.df_dlogalpha(y).toarray())
    m = np.flatnonzero(x > 1e-12)
    gphi = chem.phys_gradient(net, cell, (Sx[m] / x[m, None]).sum(axis=0))
    for j, name in enumerate(chem.PHYS_PARAMS):
        if name == "A_V":
            continue     # no photo reaction in this network: A_V and G0 do not enter
        d = 1e-4 * cell[name]
        up, dn = dict(cell), dict(cell)
        up[name] += d
        dn[name] -= d
        xp = bdf.replay(chem.cell_chemistry(net, up), x0, res.history)
        xm = bdf.replay(chem.cell_chemistry(net, dn), x0, res.history)
        fd = (np.log(xp[m]).sum() - np.log(xm[m]).sum()) / (2 * d)
        assert gphi[j] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(gphi[j]) + 1e-300), name
