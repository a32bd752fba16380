"""The Jacobian-vector product with q(u) cached (ldg_jvp_prepare / ldg_jvp_prepared), needs an MI355X.

With the cache filled for u, the product must be the oracle's J(u) v to the
precision bar (1e-12 FP64, 1e-5 FP32) and bitwise equal to ldg_jvp, which runs
the same kernels after forming q(u) itself.  A product whose q is not cached
for this u and precision is an error, not a silent use of a stale cache.
"""
import sys

import numpy as np
import pytest

from tests import cases as CS
from tests.test_gpu_parity import L, build_gpu, rel  # noqa: F401

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c5"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prepared_jvp_matches_oracle_and_jvp(L, name, prec):
    import torch
    c = CS.ALL[name]()
    _say("prepared jvp", name, prec)
    m, md, t, dev = build_gpu(L, c)
    P = L.FP64 if prec == "fp64" else L.FP32
    u, v = dev(c.u), dev(c.v)
    ref = c.om.jvp(c.oracle_model(), c.u, c.v)
    md.jvp_prepare(u, P)
    Jp = md.jvp_prepared(u, v, time=t, prec=P)
    Jp2 = md.jvp_prepared(u, 2.0 * v, time=t, prec=P)     # the cache serves any number of products
    Jd = md.jvp(u, v, time=t, prec=P)
    torch.cuda.synchronize()
    assert rel(Jp.cpu().numpy(), ref) < (1e-12 if prec == "fp64" else 1e-5)
    assert torch.equal(Jp, Jd)
    assert rel(Jp2.cpu().numpy(), 2.0 * ref) < (1e-12 if prec == "fp64" else 1e-5)


def test_prepared_jvp_needs_its_cache(L):
    c = CS.c4_ns3d(n=3, p=2)
    _say("prepared jvp cache checks")
    m, md, t, dev = build_gpu(L, c)
    u, v = dev(c.u), dev(c.v)
    with pytest.raises(L.LDGError) as ei:
        md.jvp_prepared(u, v, time=t)                       # never prepared
    assert ei.value.status == L.LDG_EINVAL
    md.jvp_prepare(u, L.FP64)
    with pytest.raises(L.LDGError):
        md.jvp_prepared(u, v, time=t, prec=L.FP32)           # prepared in FP64 only
    u2 = u.clone()
    with pytest.raises(L.LDGError):
        md.jvp_prepared(u2, v, time=t)                      # another state
    md.jvp(u2, v, time=t)                                   # ldg_jvp refills the FP64 cache for u2
    with pytest.raises(L.LDGError):
        md.jvp_prepared(u, v, time=t)
    md.jvp_prepared(u2, v, time=t)


def test_direction_traces_follow_the_direction(L):
    """The FP64 Navier-Stokes tangent reads face traces of the direction written by the gradient pass of the
    same product.  They are tied to the direction's buffer only until the next tangent of q: a product after
    the buffer's contents changed, after a product in another direction, and after a block-Jacobi build (whose
    probing products run on element subsets and in batches) must still be the oracle's J(u) v."""
    import torch
    c = CS.c4_ns3d(n=3, p=2, shift=0.3)
    _say("direction traces: c4 n=3 p=2")
    m, md, t, dev = build_gpu(L, c)
    om = c.oracle_model()
    u = dev(c.u)
    rng = np.random.default_rng(11)
    v1 = dev(rng.uniform(-1, 1, md.N))
    v2 = dev(rng.uniform(-1, 1, md.N))
    md.jvp_prepare(u, L.FP64)

    def check(v, what):
        J = md.jvp_prepared(u, v, time=t, prec=L.FP64)
        torch.cuda.synchronize()
        e = rel(J.cpu().numpy(), c.om.jvp(om, c.u, v.cpu().numpy()))
        _say(what, e)
        assert e < 1e-12

    check(v1, "v1")
    check(v2, "v2")
    v1.copy_(dev(rng.uniform(-1, 1, md.N)))          # same buffer, new contents
    check(v1, "v1 refilled")
    pc = L.BlockJacobi(md, u_lin=u, time=t, per_variable=True, prec=L.FP64)
    torch.cuda.synchronize()
    del pc
    md.jvp_prepare(u, L.FP64)
    check(v1, "v1 after a block build")
    J = md.jvp(u, v2, time=t, prec=L.FP64)            # forms the cache itself, same kernels
    torch.cuda.synchronize()
    assert rel(J.cpu().numpy(), c.om.jvp(om, c.u, v2.cpu().numpy())) < 1e-12
