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


def test_struct_layout():
    # field offsets follow the C declaration order with natural alignment
    assert ct.sizeof(hom.Grid) == 40
    assert hom.Law.E.offset == 8
    assert ct.sizeof(hom.Law) == 8 + 6 * 8 + 8 + 32 * 8 + 10 * 8
    assert ct.sizeof(hom.Result) == 6 * 8 + 3 * 8 + 4 * 8 + 4 * 4 + 2 * 8


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(hom, "_lib", None)
    with pytest.raises(hom.HomError):
        hom.library(str(tmp_path / "nope.so"))
