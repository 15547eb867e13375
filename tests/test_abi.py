"""The C ABI library loads and exports every entry point include/lagp.h
declares; the Python struct mirrors the C layout.  CPU only (no compute)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lagp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lagp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    import paper_1409_0074_amd as lg

    if not os.path.exists(lg.LIB_PATH):
        from paper_1409_0074_amd import build

        build.build()
    return lg.LIB_PATH


def test_every_declared_symbol_is_exported(libpath):
    names = _declared()
    assert "lagp_predict" in names and "lagp_server_submit" in names
    L = ctypes.CDLL(libpath)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lagp_[a-z_]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_binding_names_match_header():
    import paper_1409_0074_amd as lg

    names = _declared()
    assert sorted(lg.EXPORTED) == names
    for n in names:
        assert callable(getattr(lg, n)), n


def test_params_struct_layout_matches_c():
    import paper_1409_0074_amd as lg

    prog = r"""
#include <stddef.h>
#include <stdio.h>
#include "lagp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lagp_params), offsetof(lagp_params, d),
         offsetof(lagp_params, g), offsetof(lagp_params, brent_maxit), offsetof(lagp_params, brent_tol),
         offsetof(lagp_params, scoring), sizeof(lagp_mle_params), offsetof(lagp_mle_params, dmin),
         offsetof(lagp_mle_params, tol));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "t.c")
        exe = os.path.join(td, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    P, Q = lg.lagp_params, lg.lagp_mle_params
    assert got == [ctypes.sizeof(P), P.d.offset, P.g.offset, P.brent_maxit.offset, P.brent_tol.offset,
                   P.scoring.offset, ctypes.sizeof(Q), Q.dmin.offset, Q.tol.offset]


def test_header_compiles_as_c_and_cxx():
    with tempfile.TemporaryDirectory() as td:
        for lang, comp in (("c", "gcc"), ("cpp", "g++")):
            f = os.path.join(td, f"h.{lang}")
            open(f, "w").write('#include "lagp.h"\nint main(void){return LAGP_OK;}\n')
            subprocess.run([comp, "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), f, "-o", f + ".out"],
                           check=True)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1409_0074_amd as lg

    monkeypatch.setattr(lg, "_lib", None)
    monkeypatch.setattr(lg, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        lg.lib()
