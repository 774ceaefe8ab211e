"""Seeded per-cell physical conditions, initial abundances and request streams.

A cell is one independent gas parcel: temperature T [K], hydrogen nuclei
density n_H [cm^-3], visual extinction A_V [mag], cosmic-ray ionisation rate
zeta [s^-1], UV field G0 [Habing], an initial fractional-abundance vector x0
(x_i = n_i / n_H) and an integration horizon t_end [s].
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .network import Network

YEAR_S = 3.15576e7          # Julian year in seconds
ZETA0 = 1.3e-17             # galactic cosmic-ray ionisation rate [s^-1] (paper Sec. 4)

# atomic initial abundances relative to H nuclei
_ATOMIC_SMALL = {"H": 1.0, "C": 1e-4, "O": 3e-4}
_ATOMIC_LARGE = {"H": 1.0, "He": 0.1, "C": 1e-4, "N": 5e-5, "O": 3e-4, "S": 1e-6}


@dataclasses.dataclass
class Cells:
    T: np.ndarray
    n_H: np.ndarray
    A_V: np.ndarray
    zeta: np.ndarray
    G0: np.ndarray
    x0: np.ndarray      # (C, S)
    t_end: np.ndarray   # (C,) seconds

    @property
    def n(self) -> int:
        return int(self.T.shape[0])

    def subset(self, idx) -> "Cells":
        idx = np.asarray(idx)
        return Cells(self.T[idx], self.n_H[idx], self.A_V[idx], self.zeta[idx],
                     self.G0[idx], self.x0[idx], self.t_end[idx])

    def cell(self, i: int) -> dict:
        return dict(T=float(self.T[i]), n_H=float(self.n_H[i]), A_V=float(self.A_V[i]),
                    zeta=float(self.zeta[i]), G0=float(self.G0[i]))

    @staticmethod
    def concat(parts) -> "Cells":
        return Cells(*[np.concatenate([getattr(p, f.name) for p in parts])
                       for f in dataclasses.fields(Cells)])


def initial_abundances(net: Network) -> np.ndarray:
    """Atomic neutral start: every element in its neutral atom, nothing else."""
    table = _ATOMIC_SMALL if net.n_species <= 12 else _ATOMIC_LARGE
    x0 = np.zeros(net.n_species)
    for name, v in table.items():
        x0[net.index(name)] = v
    return x0


def single_cell(net: Network, t_end_yr: float = 1e6) -> Cells:
    """The one-cell dense-cloud case: n_H 1e4, T 10 K, A_V 0, zeta = zeta0."""
    x0 = initial_abundances(net)[None, :]
    one = np.ones(1)
    return Cells(10.0 * one, 1e4 * one, 0.0 * one, ZETA0 * one, one.copy(), x0,
                 t_end_yr * YEAR_S * one)


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def sample_cells(net: Network, n: int, seed: int, t_end_yr=1e6) -> Cells:
    """n cells: n_H log-uniform 1e2..1e6, T log-uniform 10..300 K, A_V uniform
    0..20, zeta log-uniform 1e-17..1e-15, G0 = 1; t_end scalar or per cell [yr]."""
    rng = np.random.default_rng(seed)
    n_H = _loguniform(rng, 1e2, 1e6, n)
    T = _loguniform(rng, 10.0, 300.0, n)
    A_V = rng.uniform(0.0, 20.0, n)
    zeta = _loguniform(rng, 1e-17, 1e-15, n)
    G0 = np.ones(n)
    x0 = np.tile(initial_abundances(net), (n, 1))
    t_end = np.broadcast_to(np.asarray(t_end_yr, dtype=float) * YEAR_S, (n,)).copy()
    return Cells(T, n_H, A_V, zeta, G0, x0, t_end)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float    # arrival offset from stream start, wall-clock seconds
    cells: Cells


def request_stream(net: Network, n_requests: int, seed: int, rate_per_s: float,
                   max_cells: int = 1024, t_end_yr=(1e3, 1e7)) -> list:
    """Poisson arrivals at `rate_per_s`; each request holds floor(exp(U[0, ln(max+1))))
    cells (1..max_cells, log-uniform) sharing one t_end log-uniform in t_end_yr."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s) if rate_per_s > 0 else 0.0
        nc = int(np.floor(np.exp(rng.uniform(0.0, np.log(max_cells + 1)))))
        nc = max(1, min(max_cells, nc))
        t_end = float(np.exp(rng.uniform(np.log(t_end_yr[0]), np.log(t_end_yr[1]))))
        cells = sample_cells(net, nc, seed=int(rng.integers(2**31)), t_end_yr=t_end)
        out.append(Request(rid, t, cells))
    return out
