"""Host-side checks of the C ABI: the library loads and exports every symbol
declared in include/hom.h; the ctypes structures match the header layout."""
import ctypes as ct
import os
import re

import pytest

from paper_2109_14403_amd import hom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hom.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hom_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hom.LIB_PATH):
        pytest.skip("libhom.so not built")
    return hom.library()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(hom.EXPORTS)


def test_default_options(lib):
    o = hom.Options()
    lib.hom_default_options(ct.byref(o))
    assert o.scheme == hom.SCHEME_NEWTON_CG and o.precision == hom.FP32
    assert o.tol == 1e-6 and o.use_graph == 1


STRUCTS = {"hom_grid": hom.Grid, "hom_law": hom.Law, "hom_options": hom.Options, "hom_macro_temp": hom.MacroTemp,
           "hom_result": hom.Result, "hom_load": hom.Load, "hom_tangent": hom.Tangent,
           "hom_dmn_train_opts": hom.DmnTrainOpts, "hom_dmn_result": hom.DmnResult}


def test_struct_layout(tmp_path):
    """Every ctypes structure has the size and field offsets that the C
    compiler gives the header's declaration."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hom.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        c, f, v = ln.split()
        got[(c, f)] = int(v)
    for cname, cls in STRUCTS.items():
        assert ct.sizeof(cls) == got[(cname, "size")], cname
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == got[(cname, fname)], (cname, fname)


def test_dmn_result_record_matches_the_struct():
    """DmnOnline.step hands the library a numpy record array of this dtype."""
    dt = hom.DMN_RESULT_DTYPE
    assert dt.itemsize == ct.sizeof(hom.DmnResult)
    for name, _ in hom.DmnResult._fields_:
        assert dt.fields[name][1] == getattr(hom.DmnResult, name).offset, name


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(hom, "_lib", None)
    with pytest.raises(hom.HomError):
        hom.library(str(tmp_path / "nope.so"))
