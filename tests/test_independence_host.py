"""The product path and the oracle are independent: neither imports, includes
or links the other, and the product's binding fails loudly, rather than
falling back to anything on the host, when its library is missing."""
import glob
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PKG = os.path.join(ROOT, "paper_2403_05463_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _sources(folder, exts):
    out = []
    for ext in exts:
        out += glob.glob(os.path.join(folder, "**", "*" + ext), recursive=True)
    assert out, folder
    return out


def test_product_sources_never_name_the_oracle():
    bad = re.compile(r"\boracle\b\s*import|import\s+oracle\b|from\s+oracle\b|liboracle|hdg_oracle|\borc_[a-z]")
    for path in _sources(PKG, (".py", ".cpp", ".hip", ".h")):
        text = open(path).read()
        assert not bad.search(text), path


def test_oracle_sources_never_name_the_product():
    for path in _sources(ORACLE, (".c", ".h")):
        includes = re.findall(r'#include\s*[<"]([^>"]+)', open(path).read())
        assert all(i in ("hdg_oracle.h", "math.h", "stdio.h", "stdlib.h", "string.h", "omp.h", "stddef.h")
                   for i in includes), (path, includes)
    for path in _sources(ORACLE, (".py",)):
        text = open(path).read()
        assert "paper_2403_05463_amd" not in text and "libhdg" not in text, path


def test_library_does_not_link_the_oracle():
    from paper_2403_05463_amd import hdg
    if not os.path.exists(hdg.LIB_PATH):
        pytest.skip("libhdg.so not built")
    blob = open(hdg.LIB_PATH, "rb").read()
    assert b"liboracle" not in blob and b"orc_" not in blob


def test_binding_raises_when_the_library_is_missing(monkeypatch, tmp_path):
    from paper_2403_05463_amd import hdg
    monkeypatch.setattr(hdg, "_lib", None)
    monkeypatch.setattr(hdg, "LIB_PATH", str(tmp_path / "libhdg.so"))
    with pytest.raises(RuntimeError, match="missing"):
        hdg.lib()
