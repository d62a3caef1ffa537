"""The C-ABI library loads and exports every symbol include/plc.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plc.h")
LIB = os.path.join(ROOT, "paper_1604_07515_amd", "libplc.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(plc_[a-z_]+)\s*\(", src)))


def test_header_declares_api():
    names = declared()
    for must in ("plc_init", "plc_destroy", "plc_graph_load", "plc_run", "plc_result_copy",
                 "plc_release", "plc_status_str"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libplc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libplc.so not built")
def test_binding_symbol_list_matches_header():
    import paper_1604_07515_amd as plc
    assert sorted(plc.SYMBOLS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libplc.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.plc_status_str.restype = ctypes.c_char_p
    assert lib.plc_status_str(0) == b"ok"
    assert lib.plc_status_str(-2) == b"arena exhausted"
    assert lib.plc_status_str(-99) == b"unknown status"


def test_product_package_does_not_touch_oracle():
    pkg = os.path.join(ROOT, "paper_1604_07515_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.c" not in text and "liboracle" not in text, f


STRUCTS = ("plc_options", "plc_query", "plc_graph_info", "plc_result_info", "plc_tune",
           "plc_kernel_time")


def _c_layout(tmp_path):
    """Size and field offsets of every plc.h struct, as a C compiler lays them out."""
    import shutil
    import subprocess
    import paper_1604_07515_amd as plc
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "plc.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (s, s))
        for f, _ in getattr(plc, s)._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (s, f, s, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of the C structs have the header's size and field offsets."""
    import paper_1604_07515_amd as plc
    c = _c_layout(tmp_path)
    for s in STRUCTS:
        cls = getattr(plc, s)
        assert c[(s, "size")] == ctypes.sizeof(cls), s
        for f, _ in cls._fields_:
            assert c[(s, f)] == getattr(cls, f).offset, (s, f)
