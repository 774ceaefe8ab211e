"""Request server with continuous batching (GPU).

Each cell's arithmetic does not depend on its neighbours in the batch, so a
request's results must be bitwise the same alone, in a mix of requests that
arrive while others run, and from the batch entry point at the same
tolerances.
"""
import time

import numpy as np
import pytest

import synth
from oracle import bdf, chem
from tests.gpu_util import device, rel_err_above, solve_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ab():
    import paper_2511_10558_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def net200():
    return synth.network_for_config("net200")


def _submit(srv, cells, **kw):
    return srv.submit(cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0, cells.x0, cells.t_end, **kw)


def _drain(srv, n, timeout_s=120.0):
    out = {}
    t0 = time.time()
    while len(out) < n:
        for c in srv.poll(timeout_ms=200):
            out[c["id"]] = c
        assert time.time() - t0 < timeout_s, "server did not complete the requests in time"
    return out


def _stream(net, seeds_sizes_tends):
    return [synth.sample_cells(net, n, seed=s, t_end_yr=te) for s, n, te in seeds_sizes_tends]


def test_served_results_equal_batch_results_bitwise(ab, dev, net200):
    g = ab.Network.from_text(net200.to_text())
    reqs = _stream(net200, [(11, 5, 1e4), (12, 17, 1e6), (13, 2, 3e3)])
    with ab.Server(g) as srv:
        ids = [_submit(srv, c) for c in reqs]
        done = _drain(srv, len(ids))
    for rid, cells in zip(ids, reqs):
        c = done[rid]
        assert not c["cancelled"] and c["n_failed"] == 0
        assert c["t_submit"] <= c["t_first_admit"] <= c["t_done"]
        xb, sb, stb = solve_cells(ab, g, cells, dev)
        assert (c["status"] == sb).all()
        assert np.array_equal(c["x"], xb), "served result differs from the batch solve"
        assert np.array_equal(c["stats"]["n_steps"], stb["n_steps"])


def test_served_results_follow_the_method_options(ab, dev, net200):
    # the server applies the solve options (order cap, step bounds) exactly as
    # the batch entry point does
    g = ab.Network.from_text(net200.to_text())
    reqs = _stream(net200, [(21, 3, 1e5), (22, 4, 1e6)])
    opts = dict(max_order=2, h0=10.0, h_max=1e11)
    with ab.Server(g, **opts) as srv:
        ids = [_submit(srv, c) for c in reqs]
        done = _drain(srv, len(ids))
    for rid, cells in zip(ids, reqs):
        c = done[rid]
        assert c["n_failed"] == 0
        xb, sb, stb = solve_cells(ab, g, cells, dev, **opts)
        assert (c["status"] == sb).all() and (stb["order"] <= 2).all()
        assert np.array_equal(c["x"], xb)
        assert np.array_equal(c["stats"]["n_steps"], stb["n_steps"])
    # per-species absolute tolerances, read when the server is created
    import torch
    av = torch.tensor(np.exp(np.random.default_rng(5).uniform(np.log(1e-22), np.log(1e-18), net200.n_species)),
                      dtype=torch.float64, device=dev)
    with ab.Server(g, atol_species=av) as srv:
        rid = _submit(srv, reqs[0])
        c = _drain(srv, 1)[rid]
    xb, sb, _ = solve_cells(ab, g, reqs[0], dev, atol_species=av)
    assert (c["status"] == sb).all() and np.array_equal(c["x"], xb)


def test_result_alone_equals_result_in_the_mix(ab, dev, net200):
    g = ab.Network.from_text(net200.to_text())
    probe = synth.sample_cells(net200, 9, seed=21, t_end_yr=2e5)
    with ab.Server(g) as srv:
        pid0 = _submit(srv, probe)
        a = _drain(srv, 1)[pid0]
    others = _stream(net200, [(31, 40, 1e7), (32, 3, 1e3), (33, 25, 1e5), (34, 60, 1e6)])
    # a small pool, so cells wait for slots and freed slots are refilled mid-run
    with ab.Server(g, max_slots=24) as srv:
        ids = [_submit(srv, others[0]), _submit(srv, others[1])]
        time.sleep(0.05)
        pid = _submit(srv, probe)
        time.sleep(0.02)
        ids += [_submit(srv, others[2]), _submit(srv, others[3])]
        done = _drain(srv, 5)
        info = srv.info()
    m = done[pid]
    assert np.array_equal(m["x"], a["x"])
    assert np.array_equal(m["status"], a["status"])
    assert np.array_equal(m["stats"]["n_attempts"], a["stats"]["n_attempts"])
    assert info["slots"] == 24 and info["completed_requests"] == 5
    assert info["completed_cells"] == 9 + sum(c.n for c in others)
    assert info["occupied"] == 0 and info["queued_cells"] == 0
    for rid, cells in zip(ids, others):
        assert (done[rid]["status"] == 0).all()


def test_served_cells_match_the_oracle(ab, dev, net200):
    g = ab.Network.from_text(net200.to_text())
    cells = synth.sample_cells(net200, 3, seed=41, t_end_yr=1e6)
    with ab.Server(g) as srv:
        rid = _submit(srv, cells)
        c = _drain(srv, 1)[rid]
    for i in range(cells.n):
        ref = bdf.solve(chem.cell_chemistry(net200, cells.cell(i)), cells.x0[i], cells.t_end[i], 1e-6, 1e-20)
        assert c["status"][i] == 0
        assert rel_err_above(c["x"][i], ref.x) <= 1e-4


def test_per_request_tolerances(ab, dev):
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 3, seed=51, t_end_yr=1e5)
    with ab.Server(g) as srv:
        r_tight = _submit(srv, cells, rtol=1e-9, atol=1e-25)
        r_default = _submit(srv, cells)
        done = _drain(srv, 2)
    xt, _, _ = solve_cells(ab, g, cells, dev, rtol=1e-9, atol=1e-25)
    xd, _, _ = solve_cells(ab, g, cells, dev)
    assert np.array_equal(done[r_tight]["x"], xt)
    assert np.array_equal(done[r_default]["x"], xd)
    assert done[r_tight]["stats"]["n_steps"].sum() > done[r_default]["stats"]["n_steps"].sum()


def test_empty_bad_and_cancelled_requests(ab, dev, net200):
    g = ab.Network.from_text(net200.to_text())
    cells = synth.sample_cells(net200, 4, seed=61, t_end_yr=1e4)
    bad = synth.sample_cells(net200, 3, seed=62, t_end_yr=1e4)
    bad.T[1] = -5.0
    big = synth.sample_cells(net200, 200, seed=63, t_end_yr=1e7)
    with ab.Server(g, max_slots=16) as srv:
        e = _submit(srv, synth.sample_cells(net200, 0, seed=1))
        b = _submit(srv, bad)
        k = _submit(srv, big)
        srv.cancel(k)
        ok = _submit(srv, cells)
        done = _drain(srv, 4)
        with pytest.raises(ab.AbdfError):
            srv.cancel(10 ** 9)
    assert done[e]["n_cells"] == 0
    assert list(done[b]["status"]) == [0, 4, 0] and done[b]["n_failed"] == 1
    assert done[k]["cancelled"]
    assert (done[ok]["status"] == 0).all()
    xb, _, _ = solve_cells(ab, g, cells, dev)
    assert np.array_equal(done[ok]["x"], xb)


def test_fp32_lu_server(ab, dev, net200):
    g = ab.Network.from_text(net200.to_text())
    cells = synth.sample_cells(net200, 6, seed=71, t_end_yr=1e6)
    with ab.Server(g, precision="fp32_lu") as srv:
        rid = _submit(srv, cells)
        c = _drain(srv, 1)[rid]
    xb, sb, _ = solve_cells(ab, g, cells, dev, precision="fp32_lu")
    assert np.array_equal(c["x"], xb) and (c["status"] == 0).all()


@pytest.mark.parametrize("precision", ["fp64", "fp32_lu"])
def test_net500_result_alone_equals_result_in_a_large_mix(ab, dev, precision):
    # The served configuration: the 500-species network, the benchmark's
    # factorisation policy, a pool of 96 slots kept full by overlapping
    # requests (at 32 or more occupied slots an attempt runs on two streams,
    # residual and correction kernels apart; alone, the probe's 4 cells run on
    # one stream with every Newton iteration in one fused launch).  The probe's
    # results are bitwise the same both ways and match the oracle
    net = synth.network_for_config("net500")
    g = ab.Network.from_text(net.to_text())
    opts = dict(precision=precision, lu_reuse=0.3)
    probe = synth.sample_cells(net, 4, seed=91, t_end_yr=3e5)
    with ab.Server(g, **opts) as srv:
        pid0 = _submit(srv, probe)
        a = _drain(srv, 1)[pid0]
    others = _stream(net, [(92, 80, 1e6), (93, 50, 1e5), (94, 60, 3e5), (95, 30, 1e6)])
    with ab.Server(g, max_slots=96, **opts) as srv:
        ids = [_submit(srv, others[0]), _submit(srv, others[1])]
        time.sleep(0.05)
        pid = _submit(srv, probe)
        ids += [_submit(srv, others[2]), _submit(srv, others[3])]
        done = _drain(srv, 5, timeout_s=300.0)
        info = srv.info()
    m = done[pid]
    assert (a["status"] == 0).all() and (m["status"] == 0).all()
    assert m["t_first_admit"] < max(done[r]["t_done"] for r in ids)      # it ran beside the others
    assert np.array_equal(m["x"], a["x"]), "served result differs alone and in the mix"
    assert np.array_equal(m["stats"]["n_attempts"], a["stats"]["n_attempts"])
    assert info["slots"] == 96 and info["completed_cells"] == 4 + sum(c.n for c in others)
    for rid in ids:
        assert (done[rid]["status"] == 0).all()
    for i in range(2):
        ref = bdf.solve(chem.cell_chemistry(net, probe.cell(i)), probe.x0[i], probe.t_end[i], 1e-6, 1e-20)
        assert rel_err_above(m["x"][i], ref.x) <= 1e-4, (i, rel_err_above(m["x"][i], ref.x))
