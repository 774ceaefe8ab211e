"""The entry point that allocates nothing, abdf_solve_noalloc (GPU).

Its results must equal those of abdf_solve on the same inputs (each cell's
arithmetic is the same; only the workspace and the launch stream differ), on
two calls in a row sharing the device's scratch array, the second with fewer
cells, with more cells than the scratch array holds slots (so that freed
slots are refilled), in FP64 and in the FP32-LU form.
"""
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


@pytest.mark.parametrize("name,n_first,n_second,precision", [
    ("net200", 130, 7, "fp64"),        # ~100 slots fit: the first call refills slots
    ("net500", 30, 3, "fp32_lu"),      # 24 slots fit
    ("small", 5, 1, "fp64"),
])
def test_noalloc_equals_solve_on_two_calls(ab, dev, name, n_first, n_second, precision):
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    for n, seed in ((n_first, 301), (n_second, 302)):
        cells = synth.sample_cells(net, n, seed=seed, t_end_yr=1e5)
        print(f"[noalloc] {name} {precision}: {n} cells", flush=True)
        xb, sb, stb = solve_cells(ab, g, cells, dev, precision=precision, lu_reuse=0.3)
        xn, sn, stn = solve_cells(ab, g, cells, dev, precision=precision, lu_reuse=0.3, noalloc=True)
        assert (sb == 0).all() and np.array_equal(sn, sb)
        assert np.array_equal(xn, xb), "abdf_solve_noalloc differs from abdf_solve"
        assert np.array_equal(stn["n_steps"], stb["n_steps"]) and np.array_equal(stn["n_lu"], stb["n_lu"])
    ref = bdf.solve(chem.cell_chemistry(net, cells.cell(0)), cells.x0[0], cells.t_end[0], 1e-6, 1e-20)
    assert rel_err_above(xn[0], ref.x) <= 1e-4


def test_noalloc_refusals(ab, dev):
    net = synth.network_for_config("small")
    cells = synth.sample_cells(net, 2, seed=303, t_end_yr=1e4)
    fresh = ab.Network.from_text(net.to_text())       # tables never uploaded
    with pytest.raises(ab.AbdfError) as e:
        solve_cells(ab, fresh, cells, dev, noalloc=True)
    assert e.value.code == 1 and "not on this device" in str(e.value)
    solve_cells(ab, fresh, cells, dev)                  # uploads them
    x, st, _ = solve_cells(ab, fresh, cells, dev, noalloc=True)
    assert (st == 0).all()
    with pytest.raises(ab.AbdfError) as e:
        solve_cells(ab, fresh, cells, dev, noalloc=True, hbm_budget_bytes=4096)
    assert e.value.code == 6 and "no-allocation" in str(e.value)
