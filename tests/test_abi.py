"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its Python binding declares exactly those symbols.  No GPU work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uot.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(uot_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("uot_kernel_from_cost", "uot_sinkhorn", "uot_cost_from_points",
                     "uot_sinkhorn_workspace_size", "uot_status_string", "uot_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2412_11079_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libuot.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, f"symbols declared in uot.h but not exported: {missing}"


def test_binding_covers_exactly_the_header():
    from paper_2412_11079_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared_functions()


def test_struct_layouts_match_header(tmp_path):
    """Compile a C probe against uot.h and compare every field offset with ctypes."""
    import subprocess
    from paper_2412_11079_amd import _lib
    structs = {"uot_info": _lib.Info, "uot_problem": _lib.Problem, "uot_options": _lib.Options,
               "uot_outputs": _lib.Outputs, "uot_profile": _lib.Profile, "uot_batched_meta": _lib.BatchedMeta,
               "uot_eps_schedule": _lib.EpsSchedule}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "uot.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_status_strings_without_gpu():
    from paper_2412_11079_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libuot.so not built")
    L = _lib.lib()
    assert L.uot_status_string(0) == b"ok"
    assert L.uot_status_string(4) == b"workspace too small"
