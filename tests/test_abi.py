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


def header_enum(name):
    src = open(os.path.join(ROOT, "include", "ldg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef enum \{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    return {k: int(v) for k, v in re.findall(r"\b(LDG_[A-Z0-9_]+)\s*=\s*(\d+)", body)}


def test_binding_precision_constants_match_header():
    from paper_2205_07824_amd import ldg
    e = header_enum("ldg_precision")
    for py, c in (("FP64", "LDG_FP64"), ("FP32", "LDG_FP32"), ("BF16_MFMA", "LDG_BF16_MFMA"),
                  ("FP16_MFMA", "LDG_FP16_MFMA"), ("JVP_FD", "LDG_JVP_FD"), ("BF16", "LDG_BF16"), ("FP16", "LDG_FP16")):
        assert getattr(ldg, py) == e[c], (py, c)
    assert len(e) == 7
