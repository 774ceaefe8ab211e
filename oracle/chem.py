"""Rate coefficients, mass-action right-hand side and Jacobian (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

State variable: fractional abundance x_i = n_i / n_H.  Dividing the paper's
rate equation for n_i (Sec. 2) by the constant n_H turns every two-body term
k n_a n_b into (k n_H) x_a x_b while one-body terms keep their coefficient, so
two-body coefficients are multiplied by n_H here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

TWO_BODY, COSMIC_RAY, PHOTO, CR_PHOTON = 0, 1, 2, 3


def rate_coefficients(net, T, n_H, A_V, zeta, G0) -> np.ndarray:
    """k_r for one cell.

    two-body  (Sec. 2, Kooij-Arrhenius): alpha (T/300)^beta exp(-gamma/T), times n_H
    cosmic ray (Sec. 2, direct ionisation): alpha zeta
    photo     (App. B.1): alpha G0 exp(-gamma A_V), G0 being the UV field F_UV
    cosmic-ray-induced photons (App. B.1): alpha (T/300)^beta E zeta / (1 - omega),
              E the efficiency (the gamma field), omega the network's dust albedo
    """
    k = np.empty(net.n_reactions)
    for r in range(net.n_reactions):
        a, b, g = net.alpha[r], net.beta[r], net.gamma[r]
        t = net.rtype[r]
        if t == TWO_BODY:
            k[r] = a * (T / 300.0) ** b * np.exp(-g / T) * n_H
        elif t == COSMIC_RAY:
            k[r] = a * zeta
        elif t == PHOTO:
            k[r] = a * G0 * np.exp(-g * A_V)
        elif t == CR_PHOTON:
            k[r] = a * (T / 300.0) ** b * g * zeta / (1.0 - net.albedo)
        else:
            raise ValueError(f"unknown reaction type {t}")
    return k


PHYS_PARAMS = ("T", "n_H", "A_V", "zeta", "G0")


def log_rate_derivatives(net, T, n_H, A_V, zeta, G0) -> np.ndarray:
    """d log k_r / d phi_j (R x 5) for phi = (T, n_H, A_V, zeta, G0), from the
    rate laws of rate_coefficients:

    two-body:   log k = log alpha + beta log(T/300) - gamma/T + log n_H
                -> d/dT = beta/T + gamma/T^2, d/dn_H = 1/n_H
    cosmic ray: log k = log alpha + log zeta -> d/dzeta = 1/zeta
    photo:      log k = log alpha + log G0 - gamma A_V
                -> d/dA_V = -gamma, d/dG0 = 1/G0
    CR photons: log k = log alpha + beta log(T/300) + log E + log zeta - log(1 - omega)
                -> d/dT = beta/T, d/dzeta = 1/zeta
    """
    D = np.zeros((net.n_reactions, 5))
    for r in range(net.n_reactions):
        b, g = net.beta[r], net.gamma[r]
        t = net.rtype[r]
        if t == TWO_BODY:
            D[r, 0] = b / T + g / T ** 2
            D[r, 1] = 1.0 / n_H
        elif t == COSMIC_RAY:
            D[r, 3] = 1.0 / zeta
        elif t == PHOTO:
            D[r, 2] = -g
            D[r, 4] = 1.0 / G0
        elif t == CR_PHOTON:
            D[r, 0] = b / T
            D[r, 3] = 1.0 / zeta
        else:
            raise ValueError(f"unknown reaction type {t}")
    return D


def rate_parameter_derivatives(net, T, n_H, A_V, zeta, G0) -> np.ndarray:
    """dk_r / dphi_j (R x 5) for phi = (T, n_H, A_V, zeta, G0), differentiating
    the rate laws of rate_coefficients term by term:

    two-body:   k = alpha (T/300)^beta exp(-gamma/T) n_H
                -> dk/dT = k (beta/T + gamma/T^2), dk/dn_H = alpha (T/300)^beta exp(-gamma/T)
    cosmic ray: k = alpha zeta -> dk/dzeta = alpha
    photo:      k = alpha G0 exp(-gamma A_V)
                -> dk/dA_V = -gamma k, dk/dG0 = alpha exp(-gamma A_V)
    CR photons: k = alpha (T/300)^beta E zeta / (1 - omega)
                -> dk/dT = k beta / T, dk/dzeta = alpha (T/300)^beta E / (1 - omega)

    Nothing is divided by zeta or G0, so the derivatives stay exact where a
    cell has zeta = 0 or G0 = 0 (those reactions then have k = 0)."""
    k = rate_coefficients(net, T, n_H, A_V, zeta, G0)
    D = np.zeros((net.n_reactions, 5))
    for r in range(net.n_reactions):
        a, b, g = net.alpha[r], net.beta[r], net.gamma[r]
        t = net.rtype[r]
        if t == TWO_BODY:
            D[r, 0] = k[r] * (b / T + g / T ** 2)
            D[r, 1] = a * (T / 300.0) ** b * np.exp(-g / T)
        elif t == COSMIC_RAY:
            D[r, 3] = a
        elif t == PHOTO:
            D[r, 2] = -g * k[r]
            D[r, 4] = a * np.exp(-g * A_V)
        elif t == CR_PHOTON:
            D[r, 0] = k[r] * b / T
            D[r, 3] = a * (T / 300.0) ** b * g / (1.0 - net.albedo)
        else:
            raise ValueError(f"unknown reaction type {t}")
    return D


def phys_gradient_from_rate_gradient(net, cell: dict, g_k) -> np.ndarray:
    """dL/dphi (5) of one cell from its dL/dk (R): sum_r dL/dk_r dk_r/dphi."""
    return rate_parameter_derivatives(net, **cell).T @ np.asarray(g_k, dtype=float)


def phys_gradient(net, cell: dict, g_log_alpha) -> np.ndarray:
    """dL/dphi (5) of one cell from its dL/dlog alpha (R).  The parameters enter
    the rate equations only through the coefficients k_r = alpha_r h_r(phi), so
    dL/dlog k_r = dL/dlog alpha_r and dL/dphi_j = sum_r dL/dlog k_r d log k_r / d phi_j."""
    return log_rate_derivatives(net, **cell).T @ np.asarray(g_log_alpha, dtype=float)


def stoichiometry(net) -> sp.csr_matrix:
    """nu (S x R): count of species i among products minus among reactants."""
    S, R = net.n_species, net.n_reactions
    nu = np.zeros((S, R))
    for r in range(R):
        for i in net.products[r]:
            if i >= 0:
                nu[i, r] += 1
        for i in net.reactants[r]:
            if i >= 0:
                nu[i, r] -= 1
    return sp.csr_matrix(nu)


def reaction_rates(net, k, x) -> np.ndarray:
    """rate_r = k_r times the product of its reactants' abundances (A + A gives x_A^2)."""
    rate = k.copy()
    for col in range(2):
        idx = net.reactants[:, col]
        has = idx >= 0
        rate[has] = rate[has] * x[idx[has]]
    return rate


def rate_derivative(net, k, x) -> sp.csr_matrix:
    """d rate_r / d x_j (R x S) for rates of mass-action form: k_r for one
    reactant, 2 k_r x_a for A + A, and k_r x_b (at column a), k_r x_a (at column
    b) for A + B.  The entries are built with whole-array operations; their
    values and order are those of a loop over reactions."""
    R = net.n_reactions
    a, b = net.reactants[:, 0], net.reactants[:, 1]
    one, same, pair = b < 0, (b >= 0) & (a == b), (b >= 0) & (a != b)
    rr = np.arange(R)
    # per reaction up to two entries: (r, a, v_a) and, for A + B, (r, b, v_b)
    va = np.where(one, k, np.where(same, 2.0 * k * x[np.where(same, a, 0)], k * x[np.where(pair, b, 0)]))
    vb = k * x[np.where(pair, a, 0)]
    rows = np.concatenate([rr, rr[pair]])
    cols = np.concatenate([a, b[pair]])
    vals = np.concatenate([va, vb[pair]])
    order = np.argsort(np.concatenate([2 * rr, 2 * rr[pair] + 1]), kind="stable")
    return sp.csr_matrix((vals[order], (rows[order], cols[order])), shape=(R, net.n_species))


class Chemistry:
    """f(x) = nu . rate(x) and J(x) = nu . d rate / dx for one cell's coefficients."""

    def __init__(self, net, k, nu=None):
        self.net = net
        # real coefficients in FP64 (or extended precision when given as
        # np.longdouble); complex ones are kept for complex-step derivatives
        k = np.asarray(k)
        self.k = k.astype(np.result_type(k.dtype, np.float64))
        self.nu = stoichiometry(net) if nu is None else nu

    def f(self, x) -> np.ndarray:
        return self.nu @ reaction_rates(self.net, self.k, x)

    def jac(self, x) -> np.ndarray:
        return (self.nu @ rate_derivative(self.net, self.k, x)).toarray()

    def df_dlogalpha(self, x) -> sp.csr_matrix:
        """d f / d log alpha_r = nu[:, r] rate_r (S x R), since k_r is linear in alpha_r."""
        return self.nu @ sp.diags(reaction_rates(self.net, self.k, x))


def cell_chemistry(net, cell: dict) -> Chemistry:
    return Chemistry(net, rate_coefficients(net, **cell))


class TrajectoryChemistry:
    """A cell whose physical conditions change along a trajectory: an expanding
    flow with phi_j(t) = phi_j(0) (1 + t / t_c)^(-p_j) for each of
    phi = (T, n_H, A_V, zeta, G0).  A wind moving out at constant speed has
    radius r = r0 (1 + t / t_c), density n_H ~ r^-2 and radial extinction
    A_V ~ r^-1 (p = 2 and 1); the paper's outflow study (App. A) integrates the
    chemistry along such trajectories.  t_c <= 0 keeps phi constant.  at(t) is
    the Chemistry of the rate coefficients at time t (paper Sec. 2 and
    App. B.1 rate laws at phi(t))."""

    def __init__(self, net, cell: dict, t_c: float, exponents):
        self.net = net
        self.cell = dict(cell)
        self.t_c = float(t_c)
        self.p = np.asarray(exponents, dtype=float)
        self.nu = stoichiometry(net)

    def phi(self, t: float) -> dict:
        if self.t_c <= 0.0:
            return dict(self.cell)
        s = 1.0 + t / self.t_c
        return {name: self.cell[name] * s ** (-pj) for name, pj in zip(PHYS_PARAMS, self.p)}

    def at(self, t: float) -> Chemistry:
        return Chemistry(self.net, rate_coefficients(self.net, **self.phi(t)), nu=self.nu)
