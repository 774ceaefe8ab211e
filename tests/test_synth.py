"""Seeded synthetic inputs: determinism, integer conservation, reaction mix."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("name,S,R,mix", [
    ("small", 12, 40, (30, 10, 0)),
    ("net200", 200, 2500, (2000, 250, 250)),
    ("net500", 500, 6000, (4800, 600, 600)),
])
def test_network_shape_mix_and_conservation(name, S, R, mix):
    net = synth.network_for_config(name)
    assert net.n_species == S and net.n_reactions == R
    assert tuple(np.bincount(net.rtype, minlength=3)) == mix
    W = net.conservation_matrix()
    for r in range(R):
        re = [i for i in net.reactants[r] if i >= 0]
        pr = [i for i in net.products[r] if i >= 0]
        assert 1 <= len(re) <= 2 and 1 <= len(pr) <= 3
        assert np.array_equal(W[:, re].sum(1), W[:, pr].sum(1))
        assert sorted(re) != sorted(pr)
    keys = {(tuple(net.reactants[r]), tuple(net.products[r])) for r in range(R)}
    assert len(keys) == R


def test_small_network_reactant_rules():
    net = synth.network_for_config("small")
    e = net.index("e-")
    for r in range(net.n_reactions):
        re = [i for i in net.reactants[r] if i >= 0]
        assert e not in re
        if net.rtype[r] == synth.TWO_BODY:
            assert not all(net.charge[i] != 0 for i in re)
    # every neutral single-reactant ionisation is among the cosmic-ray reactions
    cr = [r for r in range(net.n_reactions) if net.rtype[r] == synth.COSMIC_RAY]
    assert len(cr) == 10


def test_generation_is_deterministic():
    a = synth.large_network(200, 2500, seed=200)
    b = synth.network_for_config("net200")
    assert a.to_text() == b.to_text()
    c1 = synth.sample_cells(a, 16, seed=3)
    c2 = synth.sample_cells(a, 16, seed=3)
    assert np.array_equal(c1.T, c2.T) and np.array_equal(c1.x0, c2.x0)


def test_cells_ranges():
    net = synth.network_for_config("net200")
    c = synth.sample_cells(net, 2000, seed=9)
    assert c.n_H.min() >= 1e2 and c.n_H.max() <= 1e6
    assert c.T.min() >= 10 and c.T.max() <= 300
    assert c.A_V.min() >= 0 and c.A_V.max() <= 20
    assert c.zeta.min() >= 1e-17 and c.zeta.max() <= 1e-15
    assert np.all(c.G0 == 1.0)
    # atomic start conserves: H nuclei = 1
    W = net.conservation_matrix()
    assert np.allclose(W[0] @ c.x0[0], 1.0)


def test_request_stream_sizes():
    net = synth.network_for_config("small")
    reqs = synth.cells.request_stream(net, 200, seed=4, rate_per_s=10.0)
    sizes = np.array([r.cells.n for r in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 1024
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) >= 0)
    t_end = np.array([r.cells.t_end[0] for r in reqs]) / synth.YEAR_S
    assert t_end.min() >= 1e3 and t_end.max() <= 1e7


def test_network_text_is_round_trip_exact():
    net = synth.network_for_config("small")
    txt = net.to_text()
    lines = txt.splitlines()
    start = lines.index("reactions 40") + 1
    for r, line in enumerate(lines[start:start + 40]):
        a, b, g = (float(v) for v in line.split()[-3:])
        assert (a, b, g) == (net.alpha[r], net.beta[r], net.gamma[r])
