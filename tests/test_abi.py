"""CPU checks of the C-ABI library: it loads without a GPU and exports every declared symbol."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "kgdb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kgdb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    syms = declared_symbols()
    for f in ("kgdb_init_melt", "kgdb_md_steps", "kgdb_db_sweep", "kgdb_observables"):
        assert f in syms


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2109_11001_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libkgdb.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == declared_symbols()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2109_11001_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_params_struct_matches_header_fields():
    from paper_2109_11001_amd import _lib
    src = open(os.path.join(ROOT, "include", "kgdb.h")).read()
    body = src[src.index("typedef struct {"):src.index("} kgdb_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b([a-zA-Z_0-9]+)\s*[,;]", body)
    assert names == [f for f, _ in _lib.Params._fields_]


def test_network_size_agrees_everywhere():
    from oracle import oracle as o
    from paper_2109_11001_amd import _lib
    src = open(os.path.join(ROOT, "include", "kgdb.h")).read()
    n_hdr = int(re.search(r"#define KGDB_MLP_NPARAM (\d+)", src).group(1))
    assert n_hdr == _lib.MLP_NPARAM == o.NN_NPARAM == _lib.load().kgdb_mlp_nparam()
