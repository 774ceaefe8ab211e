"""ctypes declarations of the C-ABI in include/astrobdf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libastrobdf.so")

c_double_p = ctypes.c_void_p
c_void_p = ctypes.c_void_p


class Options(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double),
        ("atol", ctypes.c_double),
        ("max_steps", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("max_order", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("newton_tol", ctypes.c_double),
        ("lu_reuse", ctypes.c_double),
        ("h0", ctypes.c_double),
        ("h_max", ctypes.c_double),
        ("atol_species", ctypes.c_void_p),
        ("phi_tc", ctypes.c_void_p),
        ("phi_exp", ctypes.c_double * 5),
        ("method", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class CellStats(ctypes.Structure):
    _fields_ = [
        ("n_steps", ctypes.c_int32),
        ("n_attempts", ctypes.c_int32),
        ("n_err_reject", ctypes.c_int32),
        ("n_newton_fail", ctypes.c_int32),
        ("n_rhs", ctypes.c_int32),
        ("n_jac", ctypes.c_int32),
        ("n_lu", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("t", ctypes.c_double),
        ("n_lu_fp64", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class ServerOptions(ctypes.Structure):
    _fields_ = [("solve", Options), ("max_slots", ctypes.c_int64), ("max_queued_cells", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64)] + [(n, c_void_p) for n in ("T", "n_H", "A_V", "zeta", "G0", "x0",
                                                                       "t_end")] + [
        ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
        ("x_out", c_void_p), ("cell_status", c_void_p), ("stats", c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("n_cells", ctypes.c_int64), ("n_failed", ctypes.c_int64),
                ("cancelled", ctypes.c_int32), ("reserved", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_first_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int64), ("occupied", ctypes.c_int64), ("queued_cells", ctypes.c_int64),
                ("completed_requests", ctypes.c_int64), ("completed_cells", ctypes.c_int64),
                ("busy_slot_seconds", ctypes.c_double), ("uptime", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 11), ("ms", ctypes.c_double * 11)]


PROFILE_KINDS = ("admit", "factor", "newton", "control", "harvest", "rhs", "adj_solve", "adj_step", "rhs_side",
                 "newton_side", "rhs_eval")

# name -> (restype, argtypes); mirrors include/astrobdf.h
SIGNATURES = {
    "abdf_options_default": (None, [ctypes.POINTER(Options)]),
    "abdf_last_error": (ctypes.c_char_p, []),
    "abdf_network_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(c_void_p)]),
    "abdf_network_load_mem": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(c_void_p)]),
    "abdf_network_free": (None, [c_void_p]),
    "abdf_network_num_species": (ctypes.c_int32, [c_void_p]),
    "abdf_network_num_reactions": (ctypes.c_int32, [c_void_p]),
    "abdf_network_num_elements": (ctypes.c_int32, [c_void_p]),
    "abdf_network_species_name": (ctypes.c_char_p, [c_void_p, ctypes.c_int32]),
    "abdf_solve": (ctypes.c_int, [c_void_p, ctypes.c_int64] + [c_void_p] * 7 +
                   [ctypes.POINTER(Options), c_void_p, c_void_p, c_void_p, c_void_p]),
    "abdf_solve_noalloc": (ctypes.c_int, [c_void_p, ctypes.c_int64] + [c_void_p] * 7 +
                           [ctypes.POINTER(Options), c_void_p, c_void_p, c_void_p, c_void_p]),
    "abdf_rates": (ctypes.c_int, [c_void_p, ctypes.c_int64] + [c_void_p] * 6 + [c_void_p]),
    "abdf_phys_gradient": (ctypes.c_int, [c_void_p, ctypes.c_int64] + [c_void_p] * 7 + [c_void_p]),
    "abdf_rhs": (ctypes.c_int, [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "abdf_newton_matrix": (ctypes.c_int, [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p]),
    "abdf_lu_factor": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, c_void_p, c_void_p, c_void_p,
                                      ctypes.c_int32, c_void_p]),
    "abdf_lu_solve": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "abdf_selftest": (ctypes.c_int, [c_void_p]),
    "abdf_profile_enable": (None, [ctypes.c_int32]),
    "abdf_solve_record": (ctypes.c_int, [c_void_p, ctypes.c_int64] + [c_void_p] * 8 +
                          [ctypes.POINTER(Options), ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                           ctypes.POINTER(c_void_p), c_void_p]),
    "abdf_tape_adjoint": (ctypes.c_int, [c_void_p] * 7),
    "abdf_tape_bytes": (ctypes.c_int64, [c_void_p]),
    "abdf_tape_free": (None, [c_void_p]),
    "abdf_solve_adjoint": (ctypes.c_int, [c_void_p, ctypes.c_int64] + [c_void_p] * 8 +
                           [ctypes.POINTER(Options)] + [c_void_p] * 9),
    "abdf_server_options_default": (None, [ctypes.POINTER(ServerOptions)]),
    "abdf_server_create": (ctypes.c_int, [c_void_p, ctypes.POINTER(ServerOptions), ctypes.POINTER(c_void_p)]),
    "abdf_server_submit": (ctypes.c_int, [c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "abdf_server_poll": (ctypes.c_int, [c_void_p, ctypes.POINTER(Completion), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "abdf_server_cancel": (ctypes.c_int, [c_void_p, ctypes.c_uint64]),
    "abdf_server_clock": (ctypes.c_double, [c_void_p]),
    "abdf_server_info_get": (ctypes.c_int, [c_void_p, ctypes.POINTER(ServerInfo)]),
    "abdf_server_destroy": (None, [c_void_p]),
    "abdf_profile_read": (None, [ctypes.POINTER(Profile), ctypes.c_int32]),
}

_LIB = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded library; raises LibraryMissing (never falls back) if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
        # this library binds to.  Loaded the other way round, torch would bring a
        # second runtime to which this library's device pointers are unknown.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB
