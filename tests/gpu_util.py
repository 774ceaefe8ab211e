"""Shared helpers of the GPU tests (device tensors from seeded numpy inputs)."""
import numpy as np
import pytest


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    return torch.device("cuda:0")


def t(a, dev, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device=dev)


def solve_cells(ab, gnet, cells, dev, **kw):
    x, status, stats = ab.solve(gnet, t(cells.T, dev), t(cells.n_H, dev), t(cells.A_V, dev), t(cells.zeta, dev),
                                t(cells.G0, dev), t(cells.x0, dev), t(cells.t_end, dev), with_stats=True, **kw)
    return x.cpu().numpy(), status.cpu().numpy(), stats


def rel_err_above(x, ref, floor=1e-12):
    """max |x - ref| / ref over entries with ref > floor (abundance parity measure)."""
    m = ref > floor
    if not m.any():
        return 0.0
    return float(np.max(np.abs(x[m] - ref[m]) / ref[m]))
