"""The ctypes mirrors of the C-ABI structs have the C compiler's layout: a
host-only C program built against include/astrobdf.h prints sizeof and every
member's offset, and the binding's structures must agree field by field."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "astrobdf.h")

_lib = pytest.importorskip("paper_2511_10558_amd._lib")

MIRRORS = {
    "abdf_options": _lib.Options,
    "abdf_cell_stats": _lib.CellStats,
    "abdf_server_options": _lib.ServerOptions,
    "abdf_request": _lib.Request,
    "abdf_completion": _lib.Completion,
    "abdf_server_info": _lib.ServerInfo,
    "abdf_profile": _lib.Profile,
}


def _members(struct):
    """Member names of a typedef'd struct in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct " + struct + r"\s*\{(.*?)\}\s*" + struct + ";", text, flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:   # "type a", "type *a, *b", "type a[N]": the declarators' names, in order
            for part in decl.split(","):
                names.append(re.search(r"(\w+)\s*(\[[^\]]*\])?\s*$", part.strip()).group(1))
    return names


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for s in MIRRORS:
        lines.append(f'    printf("{s} size %zu\\n", sizeof({s}));')
        for m in _members(s):
            lines.append(f'    printf("{s} {m} %zu\\n", offsetof({s}, {m}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    res = subprocess.run(["gcc", "-std=c11", str(src), "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    table = {}
    for line in out.splitlines():
        s, m, v = line.split()
        table[(s, m)] = int(v)
    return table


@pytest.mark.parametrize("struct", list(MIRRORS))
def test_ctypes_mirror_matches_c_layout(c_layout, struct):
    py = MIRRORS[struct]
    names = _members(struct)
    assert [f[0] for f in py._fields_] == names
    assert ctypes.sizeof(py) == c_layout[(struct, "size")]
    for m in names:
        assert getattr(py, m).offset == c_layout[(struct, m)], m
