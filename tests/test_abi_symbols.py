"""The C-ABI library loads and exports every symbol include/mggpu.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mggpu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(\w+)\s*\(", src, flags=re.M)))


def _lib_path():
    from paper_2110_00328_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mg_ctx_create", "cic_assign", "mg_solve", "mg_force", "mg_solve_adjoint",
                 "mg_force_adjoint", "mg_solve_batched", "mg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing


def test_binding_covers_the_header_and_loads():
    from paper_2110_00328_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()
    L = ctypes.CDLL(_lib_path())
    for s in _declared():
        assert hasattr(L, s)
