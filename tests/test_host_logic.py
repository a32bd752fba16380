"""Host-side logic of the library's Python layer checked without a GPU."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("scheme", ["be", "dirk22", "dirk33", "dirk34"])
def test_library_dirk_stage_form_matches_stability_function(scheme):
    # the library's stage form (a0 = 1/(a_ii dt), r1 = u_n + sum_l c_il Y_l, u_{n+1} = u_n + sum_l e_l Y_l) on
    # u' = -lam u, where each stage equation a0 (U - r1) + lam U = 0 is solved exactly, against the resolvent
    # of the oracle's tableau: the transformation and the library's constants, checked without a GPU
    from paper_2205_07824_amd import timestep as TS
    lam, dt, un = 0.9, 0.37, 1.0
    A, b = TS.dirk_tableau(scheme)
    c, e = TS.dirk_stage_coefficients(A, b)
    Y = []
    for i in range(len(b)):
        a0 = 1.0 / (A[i][i] * dt)
        r1 = un + sum(c[i, l] * Y[l] for l in range(i))
        Y.append(a0 * r1 / (a0 + lam) - un)
    unew = un + sum(e[l] * Y[l] for l in range(len(b)))
    Ao, bo = O.dirk_tableau(scheme)
    z = -lam * dt
    Rz = 1.0 + z * bo @ np.linalg.solve(np.eye(len(bo)) - z * Ao, np.ones(len(bo)))
    assert abs(unew - Rz) < 1e-14
    assert np.abs(np.asarray(A) - Ao).max() < 1e-15 and np.abs(np.asarray(b) - bo).max() < 1e-15
