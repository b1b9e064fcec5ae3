"""CPU checks of the C ABI: the library loads, exports every function include/eb.h declares,
and the host-only entry points validate their arguments (no device work is issued)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eb.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eb_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1905_07392_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1905_07392_amd import build
        build.build()
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.SIGNATURES) == set(names)


def test_workspace_query_and_validation(L):
    from paper_1905_07392_amd import api
    lib = L.lib()
    box = api.make_box((32, 32, 32), 1 / 32, wall_u=[[0, 0, -1]] * 6)
    body = api.make_body(kind=1, radius=0.2)
    n32 = api.eb_workspace_bytes(box, body)
    box64 = api.make_box((64, 64, 64), 1 / 64)
    n64 = api.eb_workspace_bytes(box64, body)
    assert n32 > 32 ** 3 * 8 * 50 and 7.0 < n64 / n32 < 9.0
    bad = api.make_box((31, 32, 32), 1 / 32)
    assert api.eb_workspace_bytes(bad, body) == 0
    assert "even" in lib.eb_last_error().decode()
    neg = api.make_box((32, 32, 32), -1.0)
    assert api.eb_workspace_bytes(neg, body) == 0
    # null pointers are rejected before any device call
    ctx = C.c_void_p()
    code = lib.eb_geometry_build(C.byref(box), C.byref(body), None, 0, C.byref(ctx), None)
    assert code == L.EB_EINVAL
    assert lib.eb_ctx_info(None, None, None, None) == L.EB_EINVAL
    assert lib.eb_rk2_step(None, None, None, 1e-3, None, None, None, None, None) == L.EB_EINVAL


def test_struct_layouts_match_header(L, tmp_path):
    # sizes and field offsets of the public structs as gcc lays them out from include/eb.h
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"eb_box": L.EbBox, "eb_body": L.EbBody, "eb_rheology": L.EbRheology,
               "eb_step_opts": L.EbStepOpts, "eb_step_stats": L.EbStepStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "eb.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, field, val = line.split()
        py = structs[cname]
        got = C.sizeof(py) if field == "sizeof" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)
