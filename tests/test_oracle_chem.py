"""Pins for the oracle's rate laws, right-hand side and Jacobian (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import chem
from tests import tiny_nets

CELL = dict(T=50.0, n_H=1e4, A_V=2.0, zeta=1.3e-17, G0=1.0)


def _one(rtype, alpha, beta, gamma):
    if rtype == synth.TWO_BODY:
        net = tiny_nets.association(alpha, beta, gamma)
    else:
        net = synth.make_network("one", [("A", {"C": 1, "O": 1}, 0), ("B", {"C": 1, "O": 1}, 0)],
                                 [(rtype, ["A"], ["B"], alpha, beta, gamma)])
    return net


def k_of(net, **kw):
    cell = dict(CELL)
    cell.update(kw)
    return chem.rate_coefficients(net, **cell)[0]


def test_two_body_reduces_to_alpha_nH_without_temperature_terms():
    # Sec. 2 Kooij-Arrhenius with beta = gamma = 0: the rate coefficient is alpha;
    # in fractional-abundance units it is multiplied by n_H.
    net = _one(synth.TWO_BODY, 3e-10, 0.0, 0.0)
    for T in (10.0, 77.0, 300.0):
        assert k_of(net, T=T, n_H=2e5) == pytest.approx(3e-10 * 2e5, rel=1e-15)


def test_two_body_power_law_in_temperature():
    # gamma = 0: log k is linear in log T with slope beta (the T/300 power law).
    for beta in (-0.7, 0.4, 1.0):
        net = _one(synth.TWO_BODY, 1e-10, beta, 0.0)
        k1, k2 = k_of(net, T=20.0), k_of(net, T=180.0)
        slope = (np.log(k2) - np.log(k1)) / (np.log(180.0) - np.log(20.0))
        assert slope == pytest.approx(beta, abs=1e-12)


def test_two_body_temperature_factor_is_one_at_300K():
    a = k_of(_one(synth.TWO_BODY, 1e-10, 0.8, 0.0), T=300.0)
    b = k_of(_one(synth.TWO_BODY, 1e-10, -0.3, 0.0), T=300.0)
    assert a == pytest.approx(b, rel=1e-15)


def test_two_body_arrhenius_slope_in_inverse_temperature():
    # beta = 0: log k is linear in 1/T with slope -gamma.
    for gamma in (5.0, 80.0, 200.0):
        net = _one(synth.TWO_BODY, 1e-10, 0.0, gamma)
        k1, k2 = k_of(net, T=40.0), k_of(net, T=250.0)
        slope = (np.log(k2) - np.log(k1)) / (1 / 250.0 - 1 / 40.0)
        assert slope == pytest.approx(-gamma, rel=1e-10)


def test_cosmic_ray_rate_is_alpha_zeta_and_ignores_other_physics():
    net = _one(synth.COSMIC_RAY, 2.5, 0.0, 0.0)
    assert k_of(net, zeta=4e-16) == pytest.approx(2.5 * 4e-16, rel=1e-15)
    base = k_of(net)
    assert k_of(net, T=250.0, n_H=10.0, A_V=15.0, G0=3.0) == base


def test_photo_rate_extinction_law():
    net = _one(synth.PHOTO, 4e-10, 0.0, 2.2)
    assert k_of(net, A_V=0.0, G0=1.0) == pytest.approx(4e-10, rel=1e-15)
    assert k_of(net, A_V=0.0, G0=3.0) == pytest.approx(1.2e-9, rel=1e-15)
    k1, k2 = k_of(net, A_V=1.0), k_of(net, A_V=7.0)
    assert (np.log(k2) - np.log(k1)) / 6.0 == pytest.approx(-2.2, rel=1e-12)
    assert k_of(net, T=250.0, n_H=10.0, zeta=1e-15) == k_of(net)


def test_single_reaction_right_hand_sides():
    # decay A -> B: A lost and B gained at rate k x_A
    net = tiny_nets.decay(2.0)
    k = chem.rate_coefficients(net, **CELL)
    f = chem.Chemistry(net, k).f(np.array([0.3, 0.1]))
    assert f[0] == pytest.approx(-k[0] * 0.3, rel=1e-15)
    assert f[1] == pytest.approx(k[0] * 0.3, rel=1e-15)
    # association A + B -> C
    net = tiny_nets.association(1e-10)
    k = chem.rate_coefficients(net, **CELL)
    f = chem.Chemistry(net, k).f(np.array([0.2, 0.5, 0.0]))
    r = k[0] * 0.2 * 0.5
    np.testing.assert_allclose(f, [-r, -r, r], rtol=1e-15)
    # identical reactants H + H -> H2: rate k x_H^2, H consumed twice
    net = tiny_nets.dimer(alpha_d=0.0)
    k = chem.rate_coefficients(net, **CELL)
    f = chem.Chemistry(net, k).f(np.array([0.4, 0.3]))
    r = k[0] * 0.4 * 0.4
    np.testing.assert_allclose(f, [-2 * r, r], rtol=1e-15)


@pytest.mark.parametrize("name", ["small", "net200", "net500"])
def test_rhs_conserves_elements_and_charge(name):
    net = synth.network_for_config(name)
    W = net.conservation_matrix().astype(float)
    rng = np.random.default_rng(3)
    ch = chem.cell_chemistry(net, CELL)
    nu = chem.stoichiometry(net)
    for _ in range(3):
        x = np.exp(rng.uniform(-30, 0, net.n_species))
        f = ch.f(x)
        rate = chem.reaction_rates(net, ch.k, x)
        bound = 1e-15 * (np.abs(W) @ (abs(nu) @ rate)) + 1e-300
        assert np.all(np.abs(W @ f) <= 4 * bound)


@pytest.mark.parametrize("name", ["small", "net200", "net500"])
def test_jacobian_matches_central_differences(name):
    # f is at most quadratic in x, so central differences carry no truncation error.
    net = synth.network_for_config(name)
    ch = chem.cell_chemistry(net, CELL)
    rng = np.random.default_rng(5)
    x = np.exp(rng.uniform(-20, 0, net.n_species))
    J = ch.jac(x)
    absnu = abs(chem.stoichiometry(net))
    eps = np.finfo(float).eps
    cols = rng.choice(net.n_species, size=min(25, net.n_species), replace=False)
    for j in cols:
        dx = 0.1 * x[j]
        e = np.zeros_like(x)
        e[j] = dx
        fp, fm = ch.f(x + e), ch.f(x - e)
        fd = (fp - fm) / (2 * dx)
        # rounding bound of the two sums, divided by the step
        terms = absnu @ (chem.reaction_rates(net, ch.k, x + e) + chem.reaction_rates(net, ch.k, x - e))
        bound = 1e-12 * np.abs(J[:, j]).max() + 8 * eps * terms / (2 * dx) + 1e-300
        assert np.all(np.abs(fd - J[:, j]) <= bound)


def test_df_dlogalpha_matches_finite_difference():
    # f is linear in each k_r and d/dlog alpha_r = k_r d/dk_r, so a central
    # difference in k_r with a finite relative step is exact up to rounding.
    net = synth.network_for_config("small")
    rng = np.random.default_rng(8)
    x = np.exp(rng.uniform(-10, 0, net.n_species))
    k = chem.rate_coefficients(net, **CELL)
    G = chem.Chemistry(net, k).df_dlogalpha(x).toarray()
    absnu = abs(chem.stoichiometry(net))
    eps = np.finfo(float).eps
    for r in rng.choice(net.n_reactions, 6, replace=False):
        kp, km = k.copy(), k.copy()
        kp[r] *= 1.5
        km[r] *= 0.5
        fd = (chem.Chemistry(net, kp).f(x) - chem.Chemistry(net, km).f(x)) / 1.0
        terms = absnu @ (chem.reaction_rates(net, kp, x) + chem.reaction_rates(net, km, x))
        assert np.all(np.abs(fd - G[:, r]) <= 8 * eps * terms + 1e-300)


def test_log_rate_derivatives_match_central_differences():
    # every rate law is smooth in each parameter: a central difference of log k
    # with relative step 1e-5 agrees with the analytic derivative to ~1e-9
    net = synth.network_for_config("net200")
    D = chem.log_rate_derivatives(net, **CELL)
    for j, name in enumerate(chem.PHYS_PARAMS):
        step = 1e-5 * (abs(CELL[name]) if CELL[name] != 0 else 1.0)
        up, dn = dict(CELL), dict(CELL)
        up[name] += step
        dn[name] -= step
        fd = (np.log(chem.rate_coefficients(net, **up)) - np.log(chem.rate_coefficients(net, **dn))) / (2 * step)
        scale = np.abs(D[:, j]).max()
        assert np.all(np.abs(fd - D[:, j]) <= 1e-7 * scale + 1e-12 * np.abs(fd)), name
    # each law depends only on its own parameters
    two, cr, ph = (net.rtype == t for t in (synth.TWO_BODY, synth.COSMIC_RAY, synth.PHOTO))
    assert np.all(D[cr][:, [0, 1, 2, 4]] == 0) and np.all(D[ph][:, [0, 1, 3]] == 0)
    assert np.all(D[two][:, 2:] == 0)


def test_cosmic_ray_photon_rates():
    # photorates by cosmic-ray-induced photons scale with zeta and (T/300)^beta,
    # are independent of n_H, A_V and G0, and grow as 1 / (1 - albedo); their
    # log-derivatives match central differences
    from tests import tiny_nets
    net = tiny_nets.four_types(albedo=0.6)
    crp = net.rtype == synth.CR_PHOTON
    assert crp.sum() == 3
    k0 = chem.rate_coefficients(net, **CELL)
    moved = dict(CELL, n_H=3 * CELL["n_H"], A_V=CELL["A_V"] + 2.0, G0=5.0)
    assert np.array_equal(chem.rate_coefficients(net, **moved)[crp], k0[crp])
    k2 = chem.rate_coefficients(net, **dict(CELL, zeta=2 * CELL["zeta"]))
    np.testing.assert_allclose(k2[crp], 2 * k0[crp], rtol=1e-15)
    kt = chem.rate_coefficients(net, **dict(CELL, T=2 * CELL["T"]))
    np.testing.assert_allclose(kt[crp] / k0[crp], 2.0 ** net.beta[crp], rtol=1e-14)
    dark = tiny_nets.four_types(albedo=0.0)
    np.testing.assert_allclose(k0[crp] / chem.rate_coefficients(dark, **CELL)[crp], 1 / 0.4, rtol=1e-15)
    D = chem.log_rate_derivatives(net, **CELL)
    for j, name in enumerate(chem.PHYS_PARAMS):
        step = 1e-5 * (abs(CELL[name]) if CELL[name] != 0 else 1.0)
        up, dn = dict(CELL), dict(CELL)
        up[name] += step
        dn[name] -= step
        fd = (np.log(chem.rate_coefficients(net, **up)) - np.log(chem.rate_coefficients(net, **dn))) / (2 * step)
        scale = max(np.abs(D[:, j]).max(), 1e-300)
        assert np.all(np.abs(fd - D[:, j]) <= 1e-7 * scale + 1e-12 * np.abs(fd)), name
    assert np.all(D[crp][:, [1, 2, 4]] == 0)


@pytest.mark.parametrize("where", ["generic", "zeta0", "G00"])
def test_rate_parameter_derivatives_match_central_differences(where):
    # dk/dphi of every law against central differences of k itself, including
    # cells where zeta = 0 or G0 = 0 switch a family of reactions off (k is
    # linear in zeta and in G0, so there the difference quotient is exact up to
    # rounding); where k != 0 it equals k d log k / dphi
    from tests import tiny_nets
    net = tiny_nets.four_types(albedo=0.3)
    cell = dict(CELL, zeta=0.0) if where == "zeta0" else dict(CELL, G0=0.0) if where == "G00" else dict(CELL)
    D = chem.rate_parameter_derivatives(net, **cell)
    for j, name in enumerate(chem.PHYS_PARAMS):
        step = 1e-5 * (abs(cell[name]) if cell[name] != 0 else 1.0)
        up, dn = dict(cell), dict(cell)
        up[name] += step
        dn[name] -= step
        fd = (chem.rate_coefficients(net, **up) - chem.rate_coefficients(net, **dn)) / (2 * step)
        scale = max(np.abs(D[:, j]).max(), 1e-300)
        assert np.all(np.abs(fd - D[:, j]) <= 1e-7 * scale + 1e-12 * np.abs(fd)), name
    k = chem.rate_coefficients(net, **cell)
    on = k != 0
    L = chem.log_rate_derivatives(net, **cell) if where == "generic" else None
    if L is not None:
        np.testing.assert_allclose(D[on], k[on, None] * L[on], rtol=1e-14, atol=0)
    if where == "zeta0":
        cr = np.isin(net.rtype, [synth.COSMIC_RAY, synth.CR_PHOTON])
        assert np.all(k[cr] == 0) and np.all(D[cr, 3] > 0)
    if where == "G00":
        ph = net.rtype == synth.PHOTO
        assert np.all(k[ph] == 0) and np.all(D[ph, 4] > 0)
