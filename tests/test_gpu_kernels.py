"""Kernel-level parity of the HIP path against the oracle (GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import chem
from tests.gpu_util import device, t

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


@pytest.fixture(scope="module")
def ab():
    import paper_2511_10558_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return device()


def test_matrix_core_layouts(ab, dev):
    ab.selftest()


@pytest.mark.parametrize("name", ["small", "net200", "net500"])
def test_rates_match_oracle(ab, dev, name):
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 37, seed=11)
    k = ab.rates(g, t(cells.T, dev), t(cells.n_H, dev), t(cells.A_V, dev), t(cells.zeta, dev),
                 t(cells.G0, dev)).cpu().numpy()
    for c in range(cells.n):
        ref = chem.rate_coefficients(net, **cells.cell(c))
        np.testing.assert_allclose(k[c], ref, rtol=1e-13, atol=0)


def test_four_rate_laws_match_oracle(ab, dev):
    # two-body, cosmic-ray, photo and cosmic-ray-induced photon rates, then the
    # physical-parameter gradient contraction, and a solve of the network
    from tests import tiny_nets
    net = tiny_nets.four_types(albedo=0.6)
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 9, seed=4)
    args = [t(v, dev) for v in (cells.T, cells.n_H, cells.A_V, cells.zeta, cells.G0)]
    k = ab.rates(g, *args).cpu().numpy()
    gl = np.random.default_rng(8).normal(size=(cells.n, net.n_reactions))
    gphi = ab.phys_gradient(g, *args, t(gl, dev)).cpu().numpy()
    for c in range(cells.n):
        np.testing.assert_allclose(k[c], chem.rate_coefficients(net, **cells.cell(c)), rtol=1e-13, atol=0)
        want = chem.phys_gradient(net, cells.cell(c), gl[c])
        np.testing.assert_allclose(gphi[c], want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    from tests.gpu_util import rel_err_above, solve_cells
    from oracle import bdf
    x, status, _ = solve_cells(ab, g, cells, dev)
    for c in range(3):
        ref = bdf.solve(chem.cell_chemistry(net, cells.cell(c)), cells.x0[c], cells.t_end[c], 1e-6, 1e-20)
        assert status[c] == 0 and ref.status == bdf.OK
        assert rel_err_above(x[c], ref.x) <= 1e-4


@pytest.mark.parametrize("name", ["small", "net200", "net500"])
def test_rhs_matches_oracle(ab, dev, name):
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 19, seed=12)
    rng = np.random.default_rng(13)
    x = np.exp(rng.uniform(np.log(1e-20), 0.0, (cells.n, net.n_species)))
    x[:, 0] = 0.0                       # an exactly-zero species
    K = np.array([chem.rate_coefficients(net, **cells.cell(c)) for c in range(cells.n)])
    f = ab.rhs(g, t(K, dev), t(x, dev)).cpu().numpy()
    absnu = abs(chem.stoichiometry(net))
    for c in range(cells.n):
        ch = chem.Chemistry(net, K[c])
        ref = ch.f(x[c])
        bound = 16 * EPS * (absnu @ chem.reaction_rates(net, K[c], x[c]))
        assert np.all(np.abs(f[c] - ref) <= bound + 1e-300)


@pytest.mark.parametrize("n_rx", [2100, 3000])
def test_rhs_of_a_species_wider_than_a_wave(ab, dev, n_rx):
    # H takes part in n_rx reactions: 64 lanes of 33 (47) entries, more than
    # kRhsSegment per lane; at 47 the lanes are too long to be held in
    # registers, so the per-cell kernel runs instead of the streaming one.
    # Z takes part in none, so its f is exactly zero
    from tests import tiny_nets
    net = tiny_nets.hub(n_rx)
    g = ab.Network.from_text(net.to_text())
    rng = np.random.default_rng(15)
    conds = [dict(T=T, n_H=1e4, A_V=2.0, zeta=1.3e-17, G0=1.0) for T in (10.0, 30.0, 100.0, 300.0, 1000.0)]
    x = np.exp(rng.uniform(np.log(1e-8), 0.0, (len(conds), net.n_species)))
    K = np.array([chem.rate_coefficients(net, **cd) for cd in conds])
    f = ab.rhs(g, t(K, dev), t(x, dev)).cpu().numpy()
    absnu = abs(chem.stoichiometry(net))
    z = net.species.index("Z")
    assert np.all(f[:, z] == 0.0)
    for c in range(len(conds)):
        ref = chem.Chemistry(net, K[c]).f(x[c])
        bound = 16 * EPS * (absnu @ chem.reaction_rates(net, K[c], x[c]))
        assert np.all(np.abs(f[c] - ref) <= bound + 1e-300)
        assert f[c, 0] < 0 and abs(f[c, 0] - ref[0]) <= bound[0]


@pytest.mark.parametrize("name,n", [("net200", 1100), ("net500", 1500)])
def test_rhs_batch_streams_cells(ab, dev, name, n):
    # more cells than resident workgroups, so each workgroup takes several in
    # turn (the next one's inputs loading while the current one's sums run):
    # sampled rows match the oracle, every row conserves the elements, and a
    # row equals the same cell evaluated alone, bit for bit
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    rng = np.random.default_rng(17)
    # the coefficients are any positive numbers to the right-hand side
    K = np.exp(rng.uniform(np.log(1e-14), np.log(1e-2), (n, net.n_reactions)))
    x = np.exp(rng.uniform(np.log(1e-20), 0.0, (n, net.n_species)))
    Kd = t(K, dev)
    f = ab.rhs(g, Kd, t(x, dev)).cpu().numpy()
    absnu = abs(chem.stoichiometry(net))
    sample = np.unique(np.concatenate([[0, 1, n - 1], rng.choice(n, 21, replace=False)]))
    for c in sample:
        ref = chem.Chemistry(net, K[c]).f(x[c])
        bound = 16 * EPS * (absnu @ chem.reaction_rates(net, K[c], x[c]))
        assert np.all(np.abs(f[c] - ref) <= bound + 1e-300), c
    W = net.conservation_matrix().astype(float)
    scale = np.array([absnu @ chem.reaction_rates(net, K[c], x[c]) for c in range(n)])
    assert np.all(np.abs(f @ W.T) <= 32 * EPS * (scale @ np.abs(W).T) + 1e-300)
    for c in sample[:4]:
        alone = ab.rhs(g, Kd[c:c + 1], t(x[c:c + 1], dev)).cpu().numpy()
        assert np.array_equal(alone[0], f[c]), c


@pytest.mark.parametrize("name", ["small", "net200", "net500"])
def test_newton_matrix_matches_oracle(ab, dev, name):
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    cells = synth.sample_cells(net, 5, seed=14)
    rng = np.random.default_rng(15)
    x = np.exp(rng.uniform(np.log(1e-20), 0.0, (cells.n, net.n_species)))
    K = np.array([chem.rate_coefficients(net, **cells.cell(c)) for c in range(cells.n)])
    cvec = np.exp(rng.uniform(np.log(1e2), np.log(1e13), cells.n))
    M = ab.newton_matrix(g, t(K, dev), t(x, dev), t(cvec, dev)).cpu().numpy()
    absnu = abs(chem.stoichiometry(net))
    for c in range(cells.n):
        ch = chem.Chemistry(net, K[c])
        ref = np.eye(net.n_species) - cvec[c] * ch.jac(x[c])
        absJ = (absnu @ abs(chem.rate_derivative(net, K[c], x[c]))).toarray()
        bound = 16 * EPS * (cvec[c] * absJ + np.abs(ref))
        assert np.all(np.abs(M[c] - ref) <= bound + 1e-300)


def _newton_like_matrices(n, batch, seed):
    """Diagonally heavy, badly scaled matrices like I - cJ, plus plain random ones."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(batch, n, n))
    for b in range(0, batch, 2):
        scale = np.exp(rng.uniform(-8, 8, n))
        A[b] = np.eye(n) + (A[b] * (rng.random((n, n)) < 0.2)) * scale[None, :]
    return A


@pytest.mark.parametrize("n", [1, 12, 37, 200, 500])
@pytest.mark.parametrize("prec", ["fp64", "fp32_lu"])
def test_lu_factor_backward_error(ab, dev, n, prec):
    import torch
    batch = 6
    A = _newton_like_matrices(n, batch, seed=n)
    LU, perm, info = ab.lu_factor(t(A, dev), precision=prec)
    LU, perm, info = LU.cpu().numpy(), perm.cpu().numpy(), info.cpu().numpy()
    u = EPS / 2 if prec == "fp64" else np.finfo(np.float32).eps / 2
    for b in range(batch):
        L = np.tril(LU[b], -1) + np.eye(n)
        U = np.triu(LU[b])
        assert sorted(perm[b]) == list(range(n))
        PA = A[b][perm[b]]
        err = np.abs(PA - L @ U).max() / np.abs(A[b]).max()
        assert err <= 30 * n * u, err
        assert info[b] == 0
        # threshold pivoting: a 16-column sub-panel keeps its diagonal pivots
        # while every multiplier is at most 4 in magnitude, else it is
        # factored with partial pivoting; either way |L| <= 4
        assert np.abs(L).max() <= 4.0 * (1 + 1e-6)
        if prec == "fp64":
            _, piv = sla.lu_factor(A[b])
            growth_ref = np.abs(np.triu(sla.lu_factor(A[b])[0])).max() / np.abs(A[b]).max()
            assert np.abs(U).max() / np.abs(A[b]).max() <= 16 * max(growth_ref, 1.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32_lu"])
def test_lu_threshold_pivoting_keeps_or_exchanges(ab, dev, prec):
    # An identity of order 40 with a 2 x 2 block at rows/columns 5, 6 whose
    # column 5 holds the diagonal entry d and 1 below it: partial pivoting
    # (LAPACK) exchanges rows 5 and 6 for d < 1; the threshold rule keeps the
    # diagonal while 1 / d <= 4 and exchanges them below that.
    n = 40
    A = np.eye(n)[None].repeat(3, 0)
    for b, d in enumerate((0.5, 0.25, 0.1)):
        A[b, 5, 5], A[b, 6, 5], A[b, 5, 6], A[b, 6, 6] = d, 1.0, 1.0, 1.0
    LU, perm, info = ab.lu_factor(t(A, dev), precision=prec)
    perm, LU = perm.cpu().numpy(), LU.cpu().numpy()
    ident = np.arange(n)
    swapped = ident.copy()
    swapped[[5, 6]] = [6, 5]
    assert np.array_equal(perm[0], ident) and np.array_equal(perm[1], ident)
    assert np.array_equal(perm[2], swapped)
    tenth = float(np.float32(0.1)) if prec == "fp32_lu" else 0.1
    assert LU[0, 6, 5] == 2.0 and LU[1, 6, 5] == 4.0 and LU[2, 6, 5] == tenth
    _, piv = sla.lu_factor(A[0])
    assert piv[5] == 6                  # LAPACK exchanges where the threshold rule does not


def test_lu_factor_reports_zero_pivot(ab, dev):
    A = np.eye(20)[None].repeat(2, 0)
    A[1, :, 7] = 0.0
    _, _, info = ab.lu_factor(t(A, dev))
    assert list(info.cpu().numpy()) == [0, 8]


@pytest.mark.parametrize("n", [1, 12, 37, 64, 200, 500, 512])
def test_lu_solve_matches_linalg(ab, dev, n):
    # orders below, at and one short of the 16-padded size (odd n: the
    # products stop one column into the identity padding)
    batch = 4
    A = _newton_like_matrices(n, batch, seed=100 + n)
    rng = np.random.default_rng(n)
    bvec = rng.normal(size=(batch, n))
    LU, perm, _ = ab.lu_factor(t(A, dev))
    z = ab.lu_solve(LU, perm, t(bvec, dev)).cpu().numpy()
    for b in range(batch):
        ref = np.linalg.solve(A[b], bvec[b])
        res = np.abs(A[b] @ z[b] - bvec[b]).max() / (np.abs(A[b]).max() * np.abs(z[b]).max())
        assert res <= 30 * n * EPS
        cond = np.linalg.cond(A[b])
        assert np.abs(z[b] - ref).max() <= 100 * n * EPS * cond * np.abs(ref).max()


@pytest.mark.parametrize("n", [200, 208, 500])
def test_lu_factor_is_deterministic(ab, dev, n):
    # repeated factorisations of one batch give the same bits: every LDS
    # region is written before it is read, also at orders that are not
    # multiples of the 64-wide block column (a staging buffer that shares the
    # panel's memory once raced with the panel's last read-back at order 208)
    import torch
    rng = np.random.default_rng(n)
    A = rng.normal(size=(256, n, n))
    A[::2] = np.eye(n) + 0.01 * A[::2]
    At = t(A, dev)
    ref = ab.lu_factor(At)
    for _ in range(3):
        again = ab.lu_factor(At)
        assert torch.equal(again[0], ref[0]) and torch.equal(again[1], ref[1])
