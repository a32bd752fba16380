"""The tangent at an exact kink of the Lax-Friedrichs flux (needs an MI355X).

The Taylor-Green state has w = 0 exactly, so on every z-face of an
axis-aligned mesh the normal velocity v.n is exactly zero and |v.n| sits at its
kink.  The mesh is moved off the state's symmetry planes (x, y, z = k pi/2):
a face on such a plane sees mirror-equal traces from its two sides, so the
wave speeds in max(lambda-, lambda+) would tie up to rounding, and the branch
would then depend on the last bit of two independent trace computations.  There J v is not a derivative but a one-sided directional derivative,
fixed by the tie convention (sign(0) = +1).  The oracle forms both one-sided
derivatives (the tie broken each way); the GPU result must equal one of them
to the FP64 bar, and the two must differ, so that the case really exercises
the kink.
"""
import numpy as np
import pytest

import oracle as O
from paper_2205_07824_amd import inputs as I
from tests import cases as CS
from tests.test_gpu_parity import L, build_gpu, rel  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_jvp_at_lax_friedrichs_kink_is_one_sided(L, prec):
    c = CS.c4_ns3d(n=3, p=3, shift=0.3)
    xn = c.om.points()[0]
    U = I.taylor_green(xn, mach=0.1).transpose(0, 2, 1).reshape(-1)
    assert np.all(U.reshape(c.om.E, 5, c.om.nn)[:, 3] == 0.0)   # w = 0 exactly
    c.u = U
    om = c.oracle_model()
    J_plus = c.om.jvp(om, c.u, c.v)
    with O.tie_break(-1):
        J_minus = c.om.jvp(om, c.u, c.v)
    gap = rel(J_plus, J_minus)
    print("one-sided JVPs differ by", gap, flush=True)
    assert gap > 1e-8
    m, md, t, dev = build_gpu(L, c)
    Jv = md.jvp(dev(c.u), dev(c.v), time=t, prec=L.FP64 if prec == "fp64" else L.FP32).cpu().numpy()
    e = min(rel(Jv, J_plus), rel(Jv, J_minus))
    print(prec, "GPU vs nearest one-sided JVP", rel(Jv, J_plus), rel(Jv, J_minus), flush=True)
    assert e < (1e-12 if prec == "fp64" else 1e-5)
    if prec == "fp64":
        # the library's convention is sign(0) = +1, the oracle's default
        assert rel(Jv, J_plus) < 1e-12
