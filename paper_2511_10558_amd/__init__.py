"""Python binding of the astrobdf C-ABI (include/astrobdf.h).

Every array argument is a torch tensor on the HIP device; this module only
checks shapes and dtypes, passes raw pointers and the current stream, and
raises on a non-OK status.  All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import CellStats, LibraryMissing, Options  # noqa: F401

PREC = {"fp64": 0, "fp32_lu": 1}
METHOD = {"bdf": 0, "esdirk5": 1}
CELL_STATUS = {0: "ok", 1: "step_too_small", 2: "max_steps", 3: "nonfinite", 4: "bad_input", 5: "tape_full"}
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_PARSE", 3: "E_NONCONSERVING", 4: "E_IO", 5: "E_DEVICE",
                6: "E_BUDGET", 7: "E_NOMEM", 8: "E_BUSY"}


class AbdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        msg = _lib.lib().abdf_last_error()
        raise AbdfError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="array"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Network:
    """A loaded, validated reaction network (host handle; tables reach the
    device on first use)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def from_text(cls, text: str) -> "Network":
        L = _lib.lib()
        h = ctypes.c_void_p()
        b = text.encode()
        _check(L.abdf_network_load_mem(b, len(b), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def from_file(cls, path) -> "Network":
        L = _lib.lib()
        h = ctypes.c_void_p()
        _check(L.abdf_network_load(str(path).encode(), ctypes.byref(h)))
        return cls(h)

    @property
    def handle(self):
        return self._h

    @property
    def n_species(self) -> int:
        return _lib.lib().abdf_network_num_species(self._h)

    @property
    def n_reactions(self) -> int:
        return _lib.lib().abdf_network_num_reactions(self._h)

    @property
    def n_elements(self) -> int:
        return _lib.lib().abdf_network_num_elements(self._h)

    def species_name(self, i: int):
        v = _lib.lib().abdf_network_species_name(self._h, i)
        return None if v is None else v.decode()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.lib().abdf_network_free(h)
            except Exception:
                pass
            self._h = None


def load_network(path_or_text) -> Network:
    s = str(path_or_text)
    if s.lstrip().startswith("astrobdf-network"):
        return Network.from_text(s)
    return Network.from_file(s)


def default_options() -> Options:
    o = Options()
    _lib.lib().abdf_options_default(ctypes.byref(o))
    return o


def make_options(rtol=1e-6, atol=1e-20, max_steps=100000, precision="fp64", check_every=8,
                 hbm_budget_bytes=0, newton_tol=0.0, lu_reuse=0.0, max_order=5, h0=0.0,
                 h_max=0.0, atol_species=None, phi_tc=None, phi_exp=None, method="bdf") -> Options:
    """abdf_options.  atol_species: an FP64 device tensor of one absolute
    tolerance per species (used in place of atol); phi_tc: an FP64 device
    tensor of one expansion time per cell (conditions phi_j(0) (1 + t/t_c)^-p_j,
    p = phi_exp, five exponents for T, n_H, A_V, zeta, G0).  method: "bdf" or
    "esdirk5" (ABDF_METHOD_*).  Tensors are kept referenced by the returned
    options."""
    o = default_options()
    o.rtol, o.atol, o.max_steps = rtol, atol, max_steps
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.check_every, o.hbm_budget_bytes, o.newton_tol = check_every, hbm_budget_bytes, newton_tol
    o.lu_reuse, o.max_order = lu_reuse, max_order
    o.h0, o.h_max = h0, h_max
    o.method = METHOD[method] if isinstance(method, str) else int(method)
    if atol_species is not None:
        torch = _torch()
        if atol_species.dtype != torch.float64 or atol_species.dim() != 1 or not atol_species.is_contiguous():
            raise ValueError("atol_species must be a contiguous 1-D float64 tensor")
        o.atol_species = ctypes.c_void_p(atol_species.data_ptr())
        o._atol_species = atol_species   # keeps the array alive with the options
    if phi_tc is not None:
        torch = _torch()
        if phi_tc.dtype != torch.float64 or phi_tc.dim() != 1 or not phi_tc.is_contiguous():
            raise ValueError("phi_tc must be a contiguous 1-D float64 tensor")
        o.phi_tc = ctypes.c_void_p(phi_tc.data_ptr())
        o._phi_tc = phi_tc
    if phi_exp is not None:
        if len(phi_exp) != 5:
            raise ValueError("phi_exp holds five exponents (T, n_H, A_V, zeta, G0)")
        for j, v in enumerate(phi_exp):
            o.phi_exp[j] = float(v)
    return o


_STATS_DTYPE = np.dtype([("n_steps", "<i4"), ("n_attempts", "<i4"), ("n_err_reject", "<i4"),
                         ("n_newton_fail", "<i4"), ("n_rhs", "<i4"), ("n_jac", "<i4"), ("n_lu", "<i4"),
                         ("order", "<i4"), ("h", "<f8"), ("t", "<f8"), ("n_lu_fp64", "<i4"),
                         ("reserved", "<i4")])


def stats_to_numpy(buf) -> np.ndarray:
    """Device byte tensor of abdf_cell_stats -> numpy structured array."""
    return buf.cpu().numpy().view(_STATS_DTYPE)


def solve(net: Network, T, n_H, A_V, zeta, G0, x0, t_end, *, options: Options | None = None,
          with_stats=False, noalloc=False, **opts):
    """Integrates every cell to its t_end.  Returns (x_out, status[, stats]).
    noalloc: through abdf_solve_noalloc, the entry point that allocates
    nothing on the device (the outputs here are still torch tensors)."""
    torch = _torch()
    C, S = x0.shape
    f64 = torch.float64
    args = [_ptr(v, f64, (C,), nm) for v, nm in
            ((T, "T"), (n_H, "n_H"), (A_V, "A_V"), (zeta, "zeta"), (G0, "G0"))]
    args.append(_ptr(x0, f64, (C, net.n_species), "x0"))
    args.append(_ptr(t_end, f64, (C,), "t_end"))
    o = options if options is not None else make_options(**opts)
    x_out = torch.empty_like(x0)
    status = torch.full((C,), -1, dtype=torch.int32, device=x0.device)
    st = None
    st_ptr = ctypes.c_void_p(None)
    if with_stats:
        st = torch.zeros((max(C, 1) * ctypes.sizeof(CellStats),), dtype=torch.uint8, device=x0.device)
        st_ptr = ctypes.c_void_p(st.data_ptr())
    entry = _lib.lib().abdf_solve_noalloc if noalloc else _lib.lib().abdf_solve
    _check(entry(net.handle, C, *args, ctypes.byref(o),
                 ctypes.c_void_p(x_out.data_ptr()), ctypes.c_void_p(status.data_ptr()), st_ptr, _stream()))
    if with_stats:
        return x_out, status, stats_to_numpy(st)[:C]
    return x_out, status


def _cell_args(net, T, n_H, A_V, zeta, G0, x0, t_end):
    torch = _torch()
    C = x0.shape[0]
    f64 = torch.float64
    args = [_ptr(v, f64, (C,), nm) for v, nm in
            ((T, "T"), (n_H, "n_H"), (A_V, "A_V"), (zeta, "zeta"), (G0, "G0"))]
    args.append(_ptr(x0, f64, (C, net.n_species), "x0"))
    args.append(_ptr(t_end, f64, (C,), "t_end"))
    return C, args


class Tape:
    """Step tape of a recording solve (abdf_solve_record); reverse sweeps with adjoint()."""

    def __init__(self, handle, net, n_cells, device):
        self._h, self._net, self.n_cells, self._dev = handle, net, n_cells, device

    @property
    def nbytes(self) -> int:
        return int(_lib.lib().abdf_tape_bytes(self._h))

    def adjoint(self, dL_dx, per_cell=False, x0_grad=False, phys_grad=False):
        """(dL/dlog alpha [R], dL/dlog alpha per cell [C, R] or None, dL/dx0 [C, S] or None,
        dL/d(T, n_H, A_V, zeta, G0) per cell [C, 5] or None)."""
        torch = _torch()
        C, S, R = self.n_cells, self._net.n_species, self._net.n_reactions
        g = torch.empty((R,), dtype=torch.float64, device=self._dev)
        gc = torch.empty((C, R), dtype=torch.float64, device=self._dev) if per_cell else None
        dx0 = torch.empty((C, S), dtype=torch.float64, device=self._dev) if x0_grad else None
        dphi = torch.empty((C, 5), dtype=torch.float64, device=self._dev) if phys_grad else None
        p = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else None)
        _check(_lib.lib().abdf_tape_adjoint(self._h, _ptr(dL_dx.contiguous(), torch.float64, (C, S), "dL_dx"),
                                            p(g), p(gc), p(dx0), p(dphi), _stream()))
        return g, gc, dx0, dphi

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.lib().abdf_tape_free(h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve_record(net: Network, T, n_H, A_V, zeta, G0, x0, t_end, *, alpha=None, max_tape_steps=0,
                 options: Options | None = None, with_stats=False, **opts):
    """Solve and record the step tape.  Returns (x_out, status, tape[, stats])."""
    torch = _torch()
    C, args = _cell_args(net, T, n_H, A_V, zeta, G0, x0, t_end)
    a = ctypes.c_void_p(None) if alpha is None else _ptr(alpha, torch.float64, (net.n_reactions,), "alpha")
    o = options if options is not None else make_options(**opts)
    x_out = torch.empty_like(x0)
    status = torch.full((C,), -1, dtype=torch.int32, device=x0.device)
    st = torch.zeros((max(C, 1) * ctypes.sizeof(CellStats),), dtype=torch.uint8, device=x0.device) \
        if with_stats else None
    h = ctypes.c_void_p()
    _check(_lib.lib().abdf_solve_record(net.handle, C, *args, a, ctypes.byref(o), int(max_tape_steps),
                                        ctypes.c_void_p(x_out.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                                        ctypes.c_void_p(st.data_ptr() if st is not None else None),
                                        ctypes.byref(h), _stream()))
    tape = Tape(h, net, C, x0.device)
    if with_stats:
        return x_out, status, tape, stats_to_numpy(st)[:C]
    return x_out, status, tape


def solve_adjoint(net: Network, T, n_H, A_V, zeta, G0, x0, t_end, dL_dx, *, alpha=None,
                  options: Options | None = None, per_cell=False, x0_grad=False, phys_grad=False, **opts):
    """One call: (x_out, status, dL/dlog alpha [R], per cell [C, R] or None, dL/dx0 or None,
    dL/d(T, n_H, A_V, zeta, G0) per cell [C, 5] or None)."""
    torch = _torch()
    C, args = _cell_args(net, T, n_H, A_V, zeta, G0, x0, t_end)
    S, R = net.n_species, net.n_reactions
    a = ctypes.c_void_p(None) if alpha is None else _ptr(alpha, torch.float64, (R,), "alpha")
    o = options if options is not None else make_options(**opts)
    x_out = torch.empty_like(x0)
    status = torch.full((C,), -1, dtype=torch.int32, device=x0.device)
    g = torch.empty((R,), dtype=torch.float64, device=x0.device)
    gc = torch.empty((C, R), dtype=torch.float64, device=x0.device) if per_cell else None
    dx0 = torch.empty((C, S), dtype=torch.float64, device=x0.device) if x0_grad else None
    dphi = torch.empty((C, 5), dtype=torch.float64, device=x0.device) if phys_grad else None
    p = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else None)
    _check(_lib.lib().abdf_solve_adjoint(net.handle, C, *args, a, ctypes.byref(o),
                                         _ptr(dL_dx.contiguous(), torch.float64, (C, S), "dL_dx"),
                                         p(x_out), p(status), p(g), p(gc), p(dx0), p(dphi), ctypes.c_void_p(None),
                                         _stream()))
    return x_out, status, g, gc, dx0, dphi


PHYS_PARAMS = ("T", "n_H", "A_V", "zeta", "G0")


def phys_gradient(net: Network, T, n_H, A_V, zeta, G0, dL_dlog_alpha_cell):
    """dL/dphi [C, 5] (columns T, n_H, A_V, zeta, G0) from the per-cell
    gradients with respect to log alpha [C, R] (abdf_phys_gradient).  Where a
    cell has zeta = 0 or G0 = 0 that column is not recoverable from log-alpha
    gradients; Tape.adjoint(..., phys_grad=True) is exact there."""
    torch = _torch()
    C = T.shape[0]
    args = [_ptr(v, torch.float64, (C,), nm) for v, nm in
            ((T, "T"), (n_H, "n_H"), (A_V, "A_V"), (zeta, "zeta"), (G0, "G0"))]
    g = _ptr(dL_dlog_alpha_cell.contiguous(), torch.float64, (C, net.n_reactions), "dL_dlog_alpha_cell")
    out = torch.empty((C, 5), dtype=torch.float64, device=T.device)
    _check(_lib.lib().abdf_phys_gradient(net.handle, C, *args, g, ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def _autograd_function():
    torch = _torch()

    class SolveFunction(torch.autograd.Function):
        """x(t_end) as a differentiable function of log alpha [R], x0 [C, S] and
        the cells' physical parameters T, n_H, A_V, zeta, G0 [C]; the backward
        pass is the discrete adjoint of the recorded solve.  Cells that did not
        reach t_end (status other than ok) have no gradient: backward raises."""

        @staticmethod
        def forward(ctx, log_alpha, x0, net, T, n_H, A_V, zeta, G0, t_end, options, max_tape_steps):
            alpha = torch.exp(log_alpha.detach()).contiguous()
            phys = [v.detach().contiguous() for v in (T, n_H, A_V, zeta, G0)]
            x, status, tape = solve_record(net, *phys, x0.detach().contiguous(), t_end,
                                           alpha=alpha, options=options, max_tape_steps=max_tape_steps)
            ctx.tape, ctx.net, ctx.phys = tape, net, phys
            ctx.failed = status.ne(0)
            ctx.mark_non_differentiable(status)
            return x, status

        @staticmethod
        def backward(ctx, gx, _gstatus):
            n_failed = int(ctx.failed.sum().item())
            if n_failed:
                first = int(torch.nonzero(ctx.failed)[0, 0].item())
                raise AbdfError(1, f"{n_failed} cell(s) did not reach t_end (first: cell {first}); the adjoint "
                                   "differentiates completed solves only")
            need_phys = any(ctx.needs_input_grad[3:8])
            g, _, dx0, gphi = ctx.tape.adjoint(gx.contiguous(), x0_grad=ctx.needs_input_grad[1],
                                               phys_grad=need_phys)
            gp = [None] * 5
            if need_phys:
                gp = [gphi[:, j].clone() if ctx.needs_input_grad[3 + j] else None for j in range(5)]
            return (g, dx0, None, *gp, None, None, None)

    return SolveFunction


_SOLVE_FN = None


def solve_diff(net: Network, T, n_H, A_V, zeta, G0, x0, t_end, log_alpha, *, max_tape_steps=0,
               options: Options | None = None, **opts):
    """Differentiable solve: (x_out, status); gradients flow to log_alpha [R],
    x0 [C, S] and the physical parameters T, n_H, A_V, zeta, G0 [C]."""
    global _SOLVE_FN
    if _SOLVE_FN is None:
        _SOLVE_FN = _autograd_function()
    o = options if options is not None else make_options(**opts)
    return _SOLVE_FN.apply(log_alpha, x0, net, T, n_H, A_V, zeta, G0, t_end, o, max_tape_steps)


def rates(net: Network, T, n_H, A_V, zeta, G0):
    torch = _torch()
    C = T.shape[0]
    args = [_ptr(v, torch.float64, (C,), nm) for v, nm in
            ((T, "T"), (n_H, "n_H"), (A_V, "A_V"), (zeta, "zeta"), (G0, "G0"))]
    k = torch.empty((C, net.n_reactions), dtype=torch.float64, device=T.device)
    _check(_lib.lib().abdf_rates(net.handle, C, *args, ctypes.c_void_p(k.data_ptr()), _stream()))
    return k


def rhs(net: Network, k, x):
    torch = _torch()
    C = x.shape[0]
    f = torch.empty_like(x)
    _check(_lib.lib().abdf_rhs(net.handle, C, _ptr(k, torch.float64, (C, net.n_reactions), "k"),
                               _ptr(x, torch.float64, (C, net.n_species), "x"),
                               ctypes.c_void_p(f.data_ptr()), _stream()))
    return f


def newton_matrix(net: Network, k, x, c):
    torch = _torch()
    C, S = x.shape
    M = torch.empty((C, S, S), dtype=torch.float64, device=x.device)
    _check(_lib.lib().abdf_newton_matrix(net.handle, C, _ptr(k, torch.float64, (C, net.n_reactions), "k"),
                                         _ptr(x, torch.float64, (C, S), "x"), _ptr(c, torch.float64, (C,), "c"),
                                         ctypes.c_void_p(M.data_ptr()), _stream()))
    return M


def lu_factor(A, precision="fp64"):
    """Batched P A = L U of A (B, n, n) FP64; returns (LU, perm, info)."""
    torch = _torch()
    B, n, n2 = A.shape
    if n != n2:
        raise ValueError("square matrices required")
    LU = A.clone()
    perm = torch.empty((B, n), dtype=torch.int32, device=A.device)
    info = torch.empty((B,), dtype=torch.int32, device=A.device)
    _check(_lib.lib().abdf_lu_factor(n, B, _ptr(LU, torch.float64, None, "A"), ctypes.c_void_p(perm.data_ptr()),
                                     ctypes.c_void_p(info.data_ptr()), PREC[precision], _stream()))
    return LU, perm, info


def lu_solve(LU, perm, b):
    torch = _torch()
    B, n, _ = LU.shape
    z = b.clone()
    _check(_lib.lib().abdf_lu_solve(n, B, _ptr(LU, torch.float64, None, "LU"), _ptr(perm, torch.int32, (B, n), "perm"),
                                    _ptr(z, torch.float64, (B, n), "b"), _stream()))
    return z


def profile_enable(on: bool = True):
    """Turns the library's per-kernel-family HIP-event timers on or off."""
    _lib.lib().abdf_profile_enable(1 if on else 0)


def profile_read(reset: bool = False) -> dict:
    """{family: (launches, total_ms)} accumulated by the kernel timers."""
    p = _lib.Profile()
    _lib.lib().abdf_profile_read(ctypes.byref(p), 1 if reset else 0)
    return {k: (int(p.launches[i]), float(p.ms[i])) for i, k in enumerate(_lib.PROFILE_KINDS)}


class Server:
    """Continuous-batching request server (abdf_server_*).  Inputs are host
    numpy arrays copied at submission; each request's outputs are host numpy
    arrays owned here until its completion is returned by poll()."""

    def __init__(self, net: Network, *, max_slots=0, max_queued_cells=0, options: Options | None = None, **opts):
        L = _lib.lib()
        so = _lib.ServerOptions()
        L.abdf_server_options_default(ctypes.byref(so))
        if options is not None:
            so.solve = options
        else:
            o = so.solve
            for k, v in opts.items():
                if k == "precision":
                    v = PREC[v] if isinstance(v, str) else int(v)
                if k == "atol_species" and v is not None:
                    o.atol_species = make_options(atol_species=v).atol_species   # read at creation
                    continue
                setattr(o, k, v)
        so.max_slots, so.max_queued_cells = max_slots, max_queued_cells
        self._net = net           # the network must outlive the server
        self._S = net.n_species
        h = ctypes.c_void_p()
        _check(L.abdf_server_create(net.handle, ctypes.byref(so), ctypes.byref(h)))
        self._h = h
        self._live = {}

    def submit(self, T, n_H, A_V, zeta, G0, x0, t_end, rtol=0.0, atol=-1.0) -> int:
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        T, n_H, A_V, zeta, G0, t_end = (f(v).reshape(-1) for v in (T, n_H, A_V, zeta, G0, t_end))
        x0 = f(x0)
        C = T.shape[0]
        if x0.shape != (C, self._S) or any(v.shape != (C,) for v in (n_H, A_V, zeta, G0, t_end)):
            raise ValueError("inconsistent request shapes")
        x_out = np.empty((C, self._S), dtype=np.float64)
        status = np.full((C,), -1, dtype=np.int32)
        stats = np.zeros((C,), dtype=_STATS_DTYPE)
        r = _lib.Request()
        r.n_cells = C
        for name, v in (("T", T), ("n_H", n_H), ("A_V", A_V), ("zeta", zeta), ("G0", G0), ("x0", x0),
                        ("t_end", t_end)):
            setattr(r, name, v.ctypes.data)
        r.rtol, r.atol = rtol, atol
        r.x_out, r.cell_status, r.stats = x_out.ctypes.data, status.ctypes.data, stats.ctypes.data
        rid = ctypes.c_uint64()
        _check(_lib.lib().abdf_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._live[rid.value] = (x_out, status, stats)
        return rid.value

    def poll(self, max_n=256, timeout_ms=0) -> list:
        """Completed requests: dicts with id, x, status, stats, t_submit,
        t_first_admit, t_done, cancelled."""
        buf = (_lib.Completion * max_n)()
        n = ctypes.c_int32()
        _check(_lib.lib().abdf_server_poll(self._h, buf, max_n, ctypes.byref(n), timeout_ms))
        out = []
        for i in range(n.value):
            c = buf[i]
            x, st, sts = self._live.pop(c.id, (None, None, None))
            out.append({"id": c.id, "x": x, "status": st, "stats": sts, "n_cells": c.n_cells,
                        "n_failed": c.n_failed, "cancelled": bool(c.cancelled), "t_submit": c.t_submit,
                        "t_first_admit": c.t_first_admit, "t_done": c.t_done})
        return out

    def cancel(self, rid: int):
        _check(_lib.lib().abdf_server_cancel(self._h, rid))

    def clock(self) -> float:
        return _lib.lib().abdf_server_clock(self._h)

    def info(self) -> dict:
        i = _lib.ServerInfo()
        _check(_lib.lib().abdf_server_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _lib.ServerInfo._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.lib().abdf_server_destroy(h)
        self._h = None
        self._live = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def selftest():
    _check(_lib.lib().abdf_selftest(_stream()))
