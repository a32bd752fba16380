"""Host-side validation of ldg_mesh_create (runs before any device call; no GPU needed)."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2205_07824_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _create(nd, p, nq, vert, ev, period=None, ftag=None):
    from paper_2205_07824_amd import ldg
    L = ldg.lib()
    v = np.ascontiguousarray(vert, dtype=np.float64)
    e = np.ascontiguousarray(ev, dtype=np.int64)
    per = np.ascontiguousarray(np.zeros(nd) if period is None else period, dtype=np.float64)
    h = C.c_void_p()
    dp = C.POINTER(C.c_double)
    st = L.ldg_mesh_create(nd, p, nq, v.shape[0], v.ctypes.data_as(dp), e.shape[0],
                           e.ctypes.data_as(C.POINTER(C.c_int64)), per.ctypes.data_as(dp), None, C.byref(h))
    return st, L.ldg_last_error().decode()


def test_bad_dimensions_and_orders():
    box = I.box_mesh(2, 3)
    assert _create(4, 2, 3, box.vert, box.elem_vert)[0] == 1
    assert _create(2, 0, 1, box.vert, box.elem_vert)[0] == 1
    assert _create(2, 6, 7, box.vert, box.elem_vert)[0] == 1
    assert _create(2, 2, 2, box.vert, box.elem_vert)[0] == 1   # fewer quadrature points than nodes


def test_empty_mesh_rejected():
    box = I.box_mesh(2, 2)
    st, msg = _create(2, 1, 2, box.vert, box.elem_vert[:0])
    assert st == 1 and "sizes" in msg


def test_vertex_index_out_of_range():
    box = I.box_mesh(2, 2)
    ev = box.elem_vert.copy()
    ev[1, 2] = 999
    st, msg = _create(2, 1, 2, box.vert, ev)
    assert st == 1 and "range" in msg


def test_inverted_element_rejected():
    vert = np.array([[0, 0], [1, 0], [0, 1], [1, 1.0]])
    ev = np.array([[1, 0, 3, 2]])   # x-mirrored corner order: negative Jacobian
    st, msg = _create(2, 1, 2, vert, ev)
    assert st == 1 and "Jacobian" in msg


def test_inconsistent_face_orientation_unsupported():
    # element B is element A's right neighbour rotated by 180 degrees: the shared
    # face is +xi for both elements
    vert = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 0], [2, 1.0]])
    ev = np.array([[0, 1, 2, 3], [5, 3, 4, 1]])
    st, msg = _create(2, 1, 2, vert, ev)
    assert st == 2 and "orientation" in msg


def test_face_shared_by_three_elements():
    box = I.box_mesh(2, 2)
    ev = np.concatenate([box.elem_vert, box.elem_vert[:1]])
    st, msg = _create(2, 1, 2, box.vert, ev)
    assert st == 1


def test_periodic_direction_with_two_elements():
    box = I.box_mesh(2, 2, periodic=(True, True))
    st, msg = _create(2, 1, 2, box.vert, box.elem_vert, period=box.period)
    assert st == 1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_binding_rejects_host_and_missing_tensors():
    """The binding checks every tensor before its pointer crosses the ABI (no device needed for these)."""
    import torch
    from paper_2205_07824_amd import ldg
    with pytest.raises(ValueError, match="device"):
        ldg._ptr(torch.zeros(4, dtype=torch.float64), "v")
    with pytest.raises(ValueError, match="required"):
        ldg._ptr(None, "v", optional=False)
    assert ldg._ptr(None, "v") is None
    with pytest.raises(ValueError, match="device"):
        ldg.Time(a0=1.0, r1=torch.zeros(4, dtype=torch.float64)).c(4)
