"""The C-ABI library loads and exports every function include/ldg.h declares (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ldg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ldg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["ldg_mesh_create", "ldg_residual", "ldg_jvp", "ldg_gmres_solve", "ldg_newton_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2205_07824_amd", "libldg.so"))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2205_07824_amd import ldg
    assert sorted(ldg.EXPORTED) == [n for n in declared_functions() if n in ldg.EXPORTED]
    assert set(declared_functions()) == set(ldg.EXPORTED)
