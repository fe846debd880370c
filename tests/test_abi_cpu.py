"""The C-ABI library loads and exports every declared entry point; argument
validation that happens before any device call is checked here (no GPU)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swmi.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|int64_t|const char \*)\s*(sw_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["sw_db_open", "sw_db_search", "sw_db_topk", "sw_db_search_batch", "sw_db_close",
                 "sw_server_start", "sw_server_submit", "sw_server_wait", "sw_server_stop",
                 "sw_last_error"]:
        assert must in names


@pytest.fixture(scope="module")
def swmi():
    import paper_1404_4152_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.skip("libswmi.so not built")
    p.lib()
    return p


def test_library_exports_every_declared_symbol(swmi):
    L = swmi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(swmi.SIGNATURES)


def test_version(swmi):
    assert "gfx950" in swmi.sw_version()


@pytest.mark.parametrize("alphabet", [0, 33, -1])
def test_open_rejects_bad_alphabet(swmi, alphabet):
    with pytest.raises(swmi.SwError) as e:
        swmi.sw_db_open(np.zeros(4, np.uint8), np.array([0, 4]), alphabet)
    assert e.value.code == swmi.SW_EINVAL


def test_open_rejects_bad_codes(swmi):
    with pytest.raises(swmi.SwError) as e:
        swmi.sw_db_open(np.array([0, 1, 20, 3], np.uint8), np.array([0, 4]), 20)
    assert e.value.code == swmi.SW_EINVAL and "alphabet" in str(e.value)


def test_open_rejects_bad_offsets(swmi):
    with pytest.raises(swmi.SwError) as e:
        swmi.sw_db_open(np.zeros(4, np.uint8), np.array([0, 3, 2, 4]), 20)
    assert e.value.code == swmi.SW_EINVAL
    with pytest.raises(swmi.SwError):
        swmi.sw_db_open(np.zeros(4, np.uint8), np.array([1, 4]), 20)


def test_null_handle_calls(swmi):
    assert swmi.lib().sw_db_size(None) == -1
    swmi.lib().sw_db_close(None)          # ignored
    swmi.lib().sw_server_stop(None)       # ignored
    rc = swmi.lib().sw_db_set_opts(None, None)
    assert rc == swmi.SW_EINVAL


STRUCTS = ["sw_scoring", "sw_db_opts", "sw_search_opts", "sw_stats", "sw_server_opts", "sw_req_stats",
           "sw_alignment", "sw_index_opts", "sw_index_stats"]


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding passes across the boundary has the header's
    size and field offsets (a C program built against include/swmi.h prints
    them; the binding's ctypes layout must agree field by field)."""
    import ctypes
    import shutil
    import subprocess
    import paper_1404_4152_amd as p
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "swmi.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'    printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in getattr(p, name)._fields_:
            lines.append(f'    printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.split("\n") if l)
    for name in STRUCTS:
        cls = getattr(p, name)
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"
