"""C-ABI surface on the CPU: the library loads, exports every declared symbol,
and validates network text without touching the GPU."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "astrobdf.h")

ab = pytest.importorskip("paper_2511_10558_amd")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abdf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("abdf_network_load", "abdf_solve", "abdf_rates", "abdf_rhs", "abdf_newton_matrix",
                 "abdf_lu_factor", "abdf_lu_solve", "abdf_last_error", "abdf_options_default"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = ab._lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) <= set(ab._lib.SIGNATURES)


def test_options_default_values():
    o = ab.default_options()
    assert o.rtol == 1e-6 and o.atol == 1e-20 and o.max_steps == 100000
    assert o.precision == 0 and o.check_every == 8 and o.hbm_budget_bytes == 0 and o.lu_reuse == 0.0
    assert o.max_order == 5 and o.h0 == 0.0 and o.h_max == 0.0
    assert o.phi_tc is None and list(o.phi_exp) == [0.0] * 5


@pytest.mark.parametrize("name", ["small", "net200", "net500"])
def test_generated_networks_load(name):
    net = synth.network_for_config(name)
    g = ab.Network.from_text(net.to_text())
    assert g.n_species == net.n_species
    assert g.n_reactions == net.n_reactions
    assert g.n_elements == len(synth.ELEMENTS)
    assert [g.species_name(i) for i in range(net.n_species)] == net.species
    assert g.species_name(-1) is None and g.species_name(net.n_species) is None


def test_cosmic_ray_photon_type_and_albedo_line():
    from tests import tiny_nets
    net = tiny_nets.four_types(albedo=0.6)
    text = net.to_text()
    assert "albedo 0.6" in text
    g = ab.Network.from_text(text)
    assert g.n_species == net.n_species and g.n_reactions == 10
    for bad in ("albedo 1.0", "albedo -0.1", "albedo x"):
        with pytest.raises(ab.AbdfError) as e:
            ab.Network.from_text(text.replace("albedo 0.6", bad))
        assert e.value.code == 2
    # networks without the line keep their text (and an albedo of 0)
    assert "albedo" not in synth.network_for_config("small").to_text()


def test_network_file_load_and_missing_file(tmp_path):
    net = synth.network_for_config("small")
    p = tmp_path / "n.txt"
    synth.write_network(net, p)
    assert ab.Network.from_file(p).n_species == 12
    with pytest.raises(ab.AbdfError) as e:
        ab.Network.from_file(tmp_path / "missing.txt")
    assert e.value.code == 4


def _mutate(text, line_prefix, new_line):
    lines = text.splitlines()
    for i, l in enumerate(lines):
        if l.startswith(line_prefix):
            lines[i] = new_line
            break
    return "\n".join(lines) + "\n"


def test_nonconserving_reaction_is_rejected_with_its_index():
    net = synth.network_for_config("small")
    text = net.to_text()
    start = text.splitlines().index("reactions 40") + 1
    line = text.splitlines()[start + 3].split()
    line[6] = str((int(line[6]) + 1) % 12)      # change the first product
    bad = _mutate(text, " ".join(text.splitlines()[start + 3].split()[:2]) + " ", " ".join(line))
    with pytest.raises(ab.AbdfError) as e:
        ab.Network.from_text(bad)
    assert e.value.code == 3
    assert "reaction 3" in str(e.value)


def _first_reaction(text, new_line):
    """Replaces the line of reaction 0."""
    lines = text.splitlines()
    i = next(k for k, l in enumerate(lines) if l.startswith("reactions ")) + 1
    assert lines[i].startswith("0 ")
    lines[i] = new_line
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("edit", [
    lambda t: t.replace("astrobdf-network 1", "astrobdf-network 2"),
    lambda t: t.replace("\nend\n", "\n"),
    lambda t: t.replace("species 12", "species 13"),
    lambda t: _first_reaction(t, "0 7 2 3 6 3 4 7 11 1e-10 0 0"),
    lambda t: _first_reaction(t, "0 0 2 3 99 2 4 7 -1 1e-10 0 0"),
    lambda t: _first_reaction(t, "0 0 2 3 6 2 4 7 -1 nan 0 0"),
])
def test_malformed_network_text_is_a_parse_error(edit):
    text = synth.network_for_config("small").to_text()
    bad = edit(text)
    assert bad != text
    with pytest.raises(ab.AbdfError) as e:
        ab.Network.from_text(bad)
    assert e.value.code in (2, 3)


def test_null_and_invalid_arguments_without_gpu():
    L = ab._lib.lib()
    h = ctypes.c_void_p()
    assert L.abdf_network_load(None, ctypes.byref(h)) == 1
    assert L.abdf_network_num_species(None) == -1
    g = ab.Network.from_text(synth.network_for_config("small").to_text())
    o = ab.make_options(rtol=0.0)
    rc = L.abdf_solve(g.handle, 1, *([None] * 7), ctypes.byref(o), None, None, None, None)
    assert rc == 1 and b"rtol" in L.abdf_last_error()
    o = ab.make_options(precision=7)
    assert L.abdf_solve(g.handle, 1, *([None] * 7), ctypes.byref(o), None, None, None, None) == 1
    for bad in (-0.1, 1.0, float("nan")):
        o = ab.make_options(lu_reuse=bad)
        assert L.abdf_solve(g.handle, 1, *([None] * 7), ctypes.byref(o), None, None, None, None) == 1
        assert b"lu_reuse" in L.abdf_last_error()
    for bad in (-1, 6):
        o = ab.make_options(max_order=bad)
        assert L.abdf_solve(g.handle, 1, *([None] * 7), ctypes.byref(o), None, None, None, None) == 1
        assert b"max_order" in L.abdf_last_error()
    for kw, word in ((dict(h0=-1.0), b"h0"), (dict(h_max=float("nan")), b"h_max"), (dict(h_max=-2.0), b"h_max")):
        o = ab.make_options(**kw)
        assert L.abdf_solve(g.handle, 1, *([None] * 7), ctypes.byref(o), None, None, None, None) == 1
        assert word in L.abdf_last_error()
    o = ab.make_options()
    host = (ctypes.c_double * 12)()
    o.atol_species = ctypes.cast(host, ctypes.c_void_p)
    assert L.abdf_solve(g.handle, 1, *([None] * 7), ctypes.byref(o), None, None, None, None) == 1
    assert b"atol_species" in L.abdf_last_error()
    o = ab.make_options(max_order=0)   # 0 stands for 5
    assert L.abdf_solve(g.handle, 0, *([None] * 7), ctypes.byref(o), None, None, None, None) == 0
    o = ab.make_options()
    assert L.abdf_solve(g.handle, 0, *([None] * 7), ctypes.byref(o), None, None, None, None) == 0
    assert L.abdf_solve(g.handle, -1, *([None] * 7), ctypes.byref(o), None, None, None, None) == 1
    assert L.abdf_lu_factor(0, 1, None, None, None, 0, None) == 1


def test_server_without_device_fails_cleanly():
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    with pytest.raises(ab.AbdfError) as e:
        ab.Server(g)
    assert e.value.code == 5


def test_server_options_defaults():
    import ctypes
    so = ab._lib.ServerOptions()
    ab._lib.lib().abdf_server_options_default(ctypes.byref(so))
    assert so.solve.rtol == 1e-6 and so.solve.check_every == 4
    assert so.max_slots == 0 and so.max_queued_cells == 0


def test_adjoint_entry_points_reject_null_arguments():
    L = ab._lib.lib()
    import ctypes
    net = synth.network_for_config("small")
    g = ab.Network.from_text(net.to_text())
    o = ab.default_options()
    nul = ctypes.c_void_p(None)
    # no tape pointer
    rc = L.abdf_solve_record(g.handle, 1, *([nul] * 8), ctypes.byref(o), 0, nul, nul, nul, None, nul)
    assert rc == 1
    assert L.abdf_tape_adjoint(nul, nul, nul, nul, nul, nul, nul) == 1
    assert L.abdf_tape_bytes(nul) == 0
    L.abdf_tape_free(nul)
    # host pointers are not device pointers
    tape = ctypes.c_void_p()
    x = (ctypes.c_double * 64)()
    rc = L.abdf_solve_record(g.handle, 1, *([ctypes.cast(x, ctypes.c_void_p)] * 8), ctypes.byref(o), 0,
                             nul, nul, nul, ctypes.byref(tape), nul)
    assert rc == 1 and not tape.value
    # physical-parameter gradient: null network, count out of range, host pointers; empty is fine
    hp = ctypes.cast(x, ctypes.c_void_p)
    assert L.abdf_phys_gradient(nul, 1, *([nul] * 7), nul) == 1
    assert L.abdf_phys_gradient(g.handle, -1, *([nul] * 7), nul) == 1
    assert L.abdf_phys_gradient(g.handle, 1, *([hp] * 7), nul) == 1
    assert L.abdf_phys_gradient(g.handle, 0, *([nul] * 7), nul) == 0


def test_method_option_checks_without_gpu():
    import ctypes
    L = ab._lib.lib()
    g = ab.Network.from_text(synth.network_for_config("small").to_text())
    none7 = [None] * 7
    assert ab.default_options().method == 0
    o = ab.make_options(method=7)
    assert L.abdf_solve(g.handle, 1, *none7, ctypes.byref(o), None, None, None, None) == 1
    assert b"unknown method" in L.abdf_last_error()
    # the ESDIRK method factors every attempt and takes constant conditions
    o = ab.make_options(method="esdirk5", lu_reuse=0.3)
    assert L.abdf_solve(g.handle, 1, *none7, ctypes.byref(o), None, None, None, None) == 1
    assert b"lu_reuse" in L.abdf_last_error()
    o = ab.make_options(method="esdirk5")
    host = (ctypes.c_double * 4)()
    o.phi_tc = ctypes.cast(host, ctypes.c_void_p)
    assert L.abdf_solve(g.handle, 1, *none7, ctypes.byref(o), None, None, None, None) == 1
    assert b"ESDIRK" in L.abdf_last_error()
    o = ab.make_options(method="esdirk5")
    assert L.abdf_solve(g.handle, 0, *none7, ctypes.byref(o), None, None, None, None) == 0
    # the server runs the BDF method
    so = ab._lib.ServerOptions()
    L.abdf_server_options_default(ctypes.byref(so))
    so.solve.method = 1
    srv = ctypes.c_void_p()
    assert L.abdf_server_create(g.handle, ctypes.byref(so), ctypes.byref(srv)) == 1
    assert b"BDF" in L.abdf_last_error() and not srv.value
