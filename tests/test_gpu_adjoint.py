"""Discrete adjoint of the recorded BDF solve (GPU).

The adjoint differentiates the frozen-sequence map of the GPU's own run.  It
is checked against closed forms and library routines where the gradient is
known exactly, against the oracle's discrete forward sensitivities (the same
map on the oracle's own step sequence), and against central differences of
that map.  Gradient bar (reading C-18): |g - g_ref| <= 1e-3 max(|g_ref|,
1e-3 max_r |g_ref,r|).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import bdf, chem
from tests import tiny_nets
from tests.gpu_util import device, solve_cells, t

pytestmark = pytest.mark.gpu
YEAR = synth.YEAR_S
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_net500.json")


@pytest.fixture(scope="module")
def ab():
    import paper_2511_10558_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return device()


def grad_ok(g, ref):
    """max |g - ref| / max(|ref|, 1e-3 max |ref|); an all-zero reference needs g = 0."""
    g, ref = np.asarray(g, float), np.asarray(ref, float)
    top = np.abs(ref).max()
    if top == 0.0:
        return 0.0 if not np.any(g) else np.inf
    scale = np.maximum(np.abs(ref), 1e-3 * top)
    return float(np.max(np.abs(g - ref) / scale))


def cells_for(net, cell, x0, t_end):
    return synth.Cells(np.array([cell["T"]]), np.array([cell["n_H"]]), np.array([cell["A_V"]]),
                       np.array([cell["zeta"]]), np.array([cell["G0"]]), np.asarray(x0, float)[None, :],
                       np.array([t_end]))


def adjoint(ab, g, cells, dLdx, dev, **kw):
    args = [t(v, dev) for v in (cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0, cells.x0, cells.t_end)]
    x, st, gs, gc, dx0, _ = ab.solve_adjoint(g, *args, t(dLdx, dev), per_cell=True, x0_grad=True, **kw)
    return (x.cpu().numpy(), st.cpu().numpy(), gs.cpu().numpy(), gc.cpu().numpy(), dx0.cpu().numpy())


def log_loss_grad(x, targets):
    d = np.zeros_like(x)
    d[..., targets] = 1.0 / x[..., targets]
    return d


def test_decay_gradient_closed_form(ab, dev):
    # x_A = exp(-kt): d log x_A / d log alpha = -kt; x_B = 1 - exp(-kt):
    # d log x_B / d log alpha = kt e^{-kt} / (1 - e^{-kt})
    net = tiny_nets.decay(2.0)
    g = ab.Network.from_text(net.to_text())
    cell = dict(T=30.0, n_H=1e4, A_V=1.0, zeta=1.3e-17, G0=1.0)
    k = chem.cell_chemistry(net, cell).k[0]
    cells = cells_for(net, cell, [1.0, 0.0], 3.0 / k)
    kt = 3.0
    for sp, want in ((0, -kt), (1, kt * np.exp(-kt) / -np.expm1(-kt))):
        x, st, gs, _, _ = adjoint(ab, g, cells, np.eye(2)[sp][None, :], dev, rtol=1e-10, atol=1e-30)
        assert st[0] == 0
        assert gs[0] / x[0, sp] == pytest.approx(want, rel=1e-6)


def test_first_order_network_matches_expm_frechet(ab, dev):
    # x(t) = expm(tK) x0 with K linear in every alpha_r: dx/dlog alpha_r is the
    # Frechet derivative of expm along t dK_r, and dL/dx0 = expm(tK)^T w.
    net = tiny_nets.first_order()
    g = ab.Network.from_text(net.to_text())
    cell = dict(T=20.0, n_H=1e3, A_V=0.5, zeta=1e-16, G0=1.0)
    ch = chem.cell_chemistry(net, cell)
    S, R = net.n_species, net.n_reactions
    K = ch.jac(np.zeros(S))
    x0 = np.zeros(S)
    x0[net.index("H2")] = 0.5
    x0[net.index("CO")] = 1e-4
    tt = 3e4 * YEAR
    w = np.random.default_rng(7).uniform(-1, 1, S)
    x, st, gs, _, dx0 = adjoint(ab, g, cells_for(net, cell, x0, tt), w[None, :], dev, rtol=1e-9, atol=1e-30)
    assert st[0] == 0
    nu = chem.stoichiometry(net).toarray()
    drow = chem.rate_derivative(net, ch.k, np.zeros(S)).toarray()
    want = np.array([w @ (sla.expm_frechet(tt * K, tt * np.outer(nu[:, r], drow[r]))[1] @ x0) for r in range(R)])
    assert np.max(np.abs(gs - want)) <= 1e-6 * np.abs(want).max()
    # dL/dx0: the frozen map is linear in x0 for a linear ODE, so its
    # transpose also follows from replaying the oracle's step sequence on unit
    # vectors; both approximate expm(tK)^T w to the integration accuracy.
    # (The map amplifies rounding in its high difference rows by many orders
    # of magnitude, which is what this checks the reverse sweep survives.)
    res = bdf.solve(ch, x0, tt, 1e-9, 1e-30, record=True)
    frozen = np.array([w @ bdf.replay(ch, np.eye(S)[j], res.history, max_newton=8) for j in range(S)])
    exact = sla.expm(tt * K).T @ w
    assert np.max(np.abs(dx0[0] - frozen)) <= 1e-6 * np.abs(frozen).max()
    assert np.max(np.abs(dx0[0] - exact)) <= 1e-6 * np.abs(exact).max()


def oracle_log_gradient(net, cells, c, targets, reactions, rtol=1e-6, atol=1e-20):
    ch = chem.cell_chemistry(net, cells.cell(c))
    res = bdf.solve(ch, cells.x0[c], cells.t_end[c], rtol, atol, record=True)
    rs = np.asarray(reactions)
    x, S = bdf.replay(ch, cells.x0[c], res.history, max_newton=8,
                      sens_dfdp=lambda y: ch.df_dlogalpha(y)[:, rs].toarray())
    return (S[targets] / x[targets, None]).sum(axis=0), x


def test_small_network_matches_oracle_sensitivities(ab, dev):
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    cells = synth.single_cell(net, t_end_yr=1e5)
    xg, st, *_ = solve_cells(ab, g, cells, dev)
    targets = np.flatnonzero(xg[0] > 1e-12)
    x, st, gs, gc, _ = adjoint(ab, g, cells, log_loss_grad(xg, targets), dev)
    assert st[0] == 0 and np.array_equal(x, xg), "recording changed the forward result"
    ref, _ = oracle_log_gradient(net, cells, 0, targets, np.arange(net.n_reactions))
    assert grad_ok(gs, ref) <= 1e-3
    assert np.array_equal(gc[0], gs)


def test_net200_cell_matches_oracle_sensitivities(ab, dev):
    net = synth.network_for_config("net200")
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 1, seed=2001, t_end_yr=1e5)
    xg, _, _ = solve_cells(ab, g, cells, dev)
    targets = np.sort(np.random.default_rng(5).choice(np.flatnonzero(xg[0] > 1e-12), 6, replace=False))
    x, st, gs, _, _ = adjoint(ab, g, cells, log_loss_grad(xg, targets), dev)
    assert st[0] == 0
    ref, _ = oracle_log_gradient(net, cells, 0, targets, np.arange(net.n_reactions))
    assert np.count_nonzero(ref) >= 10
    assert grad_ok(gs, ref) <= 1e-3


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle gradients of the 500-species workload not generated")
def test_net500_matches_oracle_sensitivities_and_central_differences(ab, dev):
    gold = json.load(open(GOLDEN))
    net = synth.network_for_config("net500")
    g = ab.Network.from_text(net.to_text())
    n = len(gold["cells"])
    cells = synth.sample_cells(net, gold["batch_cells"], seed=gold["seeds"]["cells"], t_end_yr=1e6)
    cells = cells.subset(np.arange(n))
    targets, reactions = np.array(gold["targets"]), np.array(gold["reactions"])
    xg, _, _ = solve_cells(ab, g, cells, dev)
    x, st, gs, gc, _ = adjoint(ab, g, cells, log_loss_grad(xg, targets), dev)
    assert (st == 0).all()
    for c, rec in enumerate(gold["cells"]):
        sens, cs, fd = np.array(rec["sens"]), np.array(rec["cs"]), np.array(rec["fd"])
        top = np.abs(cs).max()
        # the references of the golden file: the oracle's forward sensitivities,
        # the complex-step derivative of its frozen map and central differences
        # of that map replayed in extended precision.  The differences stay
        # within 1.5e-6 of the largest entry of the complex-step values (1.2e-6
        # measured), which bounds what any entry-wise comparison can resolve;
        # the GPU also differentiates its own step sequence, which differs from
        # the oracle's at the tolerance (rtol 1e-6).  Bar, entry by entry over
        # all 50 reactions: 1e-3 of the entry plus 2e-6 of the largest
        assert np.max(np.abs(fd - cs)) <= 1.5e-6 * top and np.max(np.abs(sens - cs)) <= 1e-7 * top
        for ref in (sens, cs, fd):
            assert np.all(np.abs(gc[c, reactions] - ref) <= 1e-3 * np.abs(ref) + 2e-6 * top)
        assert np.all(np.isfinite(gc[c]))
    assert np.allclose(gs, gc.sum(axis=0), rtol=1e-12, atol=0)


def test_autograd_function_matches_solve_adjoint(ab, dev):
    import torch
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 3, seed=81, t_end_yr=1e5)
    log_alpha = torch.tensor(np.log(net.alpha), dtype=torch.float64, device=dev, requires_grad=True)
    x0 = t(cells.x0, dev).requires_grad_(True)
    phys = [t(v, dev) for v in (cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0)]
    x, st = ab.solve_diff(g, *phys, x0, t(cells.t_end, dev), log_alpha)
    targets = [g_i for g_i in range(net.n_species) if (x[:, g_i] > 1e-12).all()]
    loss = torch.log(x[:, targets]).sum()
    loss.backward()
    assert (st == 0).all()
    # the same through the one-call entry point with alpha = exp(log alpha)
    alpha = torch.exp(log_alpha.detach())
    dLdx = torch.zeros_like(x)
    dLdx[:, targets] = 1.0 / x.detach()[:, targets]
    x2, _, gs, _, dx0, _ = ab.solve_adjoint(g, *phys, x0.detach(), t(cells.t_end, dev), dLdx, alpha=alpha,
                                         x0_grad=True)
    assert torch.equal(x2, x.detach())
    assert torch.equal(log_alpha.grad, gs)
    assert torch.equal(x0.grad, dx0)


def test_tape_is_linear_in_the_loss_gradient_and_reusable(ab, dev):
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 4, seed=91, t_end_yr=3e4)
    args = [t(v, dev) for v in (cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0, cells.x0, cells.t_end)]
    x, st, tape = ab.solve_record(g, *args)
    xb, _, _ = solve_cells(ab, g, cells, dev)
    assert np.array_equal(x.cpu().numpy(), xb)
    assert tape.nbytes > 0
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(2, 4, net.n_species))
    ga, gca, da, _ = tape.adjoint(t(a, dev), per_cell=True, x0_grad=True)
    gb, _, db, _ = tape.adjoint(t(b, dev), x0_grad=True)
    gab, _, dab, _ = tape.adjoint(t(a + b, dev), x0_grad=True)
    ga2, _, _, _ = tape.adjoint(t(a, dev))
    assert torch_equal(ga, ga2)
    scale = max(float(ga.abs().max()), float(gb.abs().max()))
    assert float((gab - ga - gb).abs().max()) <= 1e-10 * scale
    assert float((dab - da - db).abs().max()) <= 1e-10 * max(float(da.abs().max()), float(db.abs().max()))
    assert float((gca.sum(0) - ga).abs().max()) <= 1e-12 * float(ga.abs().max())
    tape.free()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_failed_and_empty_cells_contribute_nothing(ab, dev):
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 3, seed=93, t_end_yr=1e4)
    cells.T[1] = -1.0          # bad input
    cells.t_end[2] = 0.0       # nothing to integrate: dL/dx0 = dL/dx
    dLdx = np.random.default_rng(4).normal(size=(3, net.n_species))
    x, st, gs, gc, dx0 = adjoint(ab, g, cells, dLdx, dev)
    assert list(st) == [0, 4, 0]
    assert not gc[1].any() and not dx0[1].any()
    assert not gc[2].any() and np.array_equal(dx0[2], dLdx[2])
    alone = adjoint(ab, g, cells.subset([0]), dLdx[:1], dev)
    assert np.array_equal(alone[3][0], gc[0]) and np.array_equal(alone[4][0], dx0[0])


def _record_and_sweep(ab, g, args, dLdx, cap, sweeps=1):
    import torch
    x, st, tape = ab.solve_record(g, *args, max_tape_steps=cap)
    outs = [tape.adjoint(dLdx, per_cell=True, x0_grad=True, phys_grad=True) for _ in range(sweeps)]
    torch.cuda.synchronize()
    tape.free()
    return x.cpu().numpy(), st.cpu().numpy(), [[v.cpu().numpy() for v in o] for o in outs]


@pytest.mark.parametrize("name,n,seed,t_end_yr,cap", [("small", 3, 95, 1e5, 7), ("net200", 40, 96, 1e6, 150)])
def test_cells_longer_than_the_tape_are_swept_in_windows(ab, dev, name, n, seed, t_end_yr, cap):
    # a tape far shorter than the cells' step counts: the forward solve still
    # reaches t_end, and the windowed sweep (forward re-runs of each window,
    # the adjoint state carried between windows) gives bitwise the gradients
    # of a tape that holds every step, sweep after sweep.  The batch mixes in a
    # cell with no steps (t_end = 0) and one with bad input (zero gradients);
    # the 40-cell batch runs the two-stream attempts in its re-runs
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, n, seed=seed, t_end_yr=t_end_yr)
    cells.t_end[1] = 0.0
    cells.T[2] = -5.0
    args = [t(v, dev) for v in (cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0, cells.x0, cells.t_end)]
    dLdx = t(np.random.default_rng(seed).normal(size=cells.x0.shape), dev)
    xf, sf, (gf,) = _record_and_sweep(ab, g, args, dLdx, 100000)
    xw, sw, gw = _record_and_sweep(ab, g, args, dLdx, cap, sweeps=2)
    assert sf[2] == 4 and sf[1] == 0 and (np.delete(sf, 2) == 0).all()
    assert np.array_equal(sw, sf) and np.array_equal(xw, xf)
    _, _, tp, stats = ab.solve_record(g, *args, max_tape_steps=cap, with_stats=True)
    tp.free()
    assert stats["n_steps"].max() > 3 * cap          # several windows
    for run in gw:
        for a, b in zip(run, gf):
            assert np.array_equal(a, b)
    assert not gw[0][1][2].any()
