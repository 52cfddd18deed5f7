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


def test_plain_c_program_calls_the_library(tmp_path):
    # the boundary is a C ABI: a C program built against include/kgdb.h links libkgdb.so and
    # calls a host-only entry point (the protocol's stage plan), compared with the oracle's
    import shutil
    import subprocess
    from oracle import protocol as op
    from paper_2109_11001_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "plan.c"
    src.write_text("""
#include <stdio.h>
#include "kgdb.h"
int main(void) {
  double n[12], taus[4];
  int64_t steps[12];
  int ns = kgdb_protocol_schedule(2.0, 400, 0.008, 46.3354, n, steps, taus);
  if (ns != 12) return 1;
  for (int i = 0; i < ns; ++i) printf("%g %lld\\n", n[i], (long long)steps[i]);
  return kgdb_protocol_schedule(-1.0, 400, 0.008, 46.3354, n, steps, taus) == KGDB_E_PARAM ? 0 : 2;
}
""")
    exe = tmp_path / "plan"
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-o", str(exe), str(src), "-I" + os.path.join(ROOT, "include"),
                           "-L" + libdir, "-lkgdb", "-Wl,-rpath," + libdir])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    n_ref, steps_ref = op.schedule(2.0, 400, 0.008)
    assert [float(v) for v in out[0::2]] == n_ref
    assert [int(v) for v in out[1::2]] == steps_ref
