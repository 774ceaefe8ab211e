"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds reaction networks, per-cell physical conditions, initial
abundances and request streams.  It contains no part of the solver's
arithmetic (no rate laws, no right-hand side, no integrator): only integer
bookkeeping of element and charge totals and random draws.
"""
from .network import (  # noqa: F401
    ELEMENTS,
    Network,
    small_network,
    large_network,
    network_for_config,
    write_network,
    make_network,
    TWO_BODY,
    COSMIC_RAY,
    PHOTO,
    CR_PHOTON,
)
from .cells import (  # noqa: F401
    YEAR_S,
    ZETA0,
    Cells,
    single_cell,
    sample_cells,
    initial_abundances,
    request_stream,
)
