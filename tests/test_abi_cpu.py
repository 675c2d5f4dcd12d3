"""CPU checks of the C-ABI library: it builds, loads, and exports every entry
point include/sabr.h declares, and the Python structures have the C layout.
No GPU call is made here."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sabr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sabr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libsabr():
    from paper_2407_20713_amd import sabr
    if not os.path.exists(sabr.LIB_PATH):
        from paper_2407_20713_amd import build
        build.build()
    return sabr


def test_library_exports_every_declared_symbol(libsabr):
    names = declared_functions()
    assert len(names) >= 8
    out = subprocess.run(["nm", "-D", "--defined-only", libsabr.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (sabr_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(libsabr.EXPORTED)


def test_library_loads(libsabr):
    L = libsabr.lib()
    for n in declared_functions():
        assert hasattr(L, n)


def test_struct_layouts_match_header(libsabr):
    """sizeof and field offsets of every ABI struct, printed by a C program
    compiled against include/sabr.h, equal the ctypes mirrors."""
    import ctypes as C
    structs = {"sabr_market": libsabr.sabr_market, "sabr_problem": libsabr.sabr_problem,
               "sabr_objspec": libsabr.sabr_objspec, "sabr_sa": libsabr.sabr_sa, "sabr_mc": libsabr.sabr_mc,
               "sabr_result": libsabr.sabr_result, "sabr_request": libsabr.sabr_request}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sabr.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, fname, name, fname))
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[name + "." + fname]) == getattr(cls, fname).offset, (name, fname)


def test_product_path_has_no_cpu_fallback():
    """The binding refuses to run without the HIP library rather than
    computing anything itself, and never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2407_20713_amd", "sabr.py")).read()
    assert "oracle" not in src
    assert "raise ImportError" in src
    for fn in os.listdir(os.path.join(ROOT, "paper_2407_20713_amd")):
        if fn.endswith(".py"):
            assert "import oracle" not in open(os.path.join(ROOT, "paper_2407_20713_amd", fn)).read()
