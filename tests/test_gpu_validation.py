"""Wrong tensors are refused by the binding before any kernel sees them (needs an MI355X
only to create the device tensors and the model; nothing here launches a kernel with a bad buffer)."""
import numpy as np
import pytest

from tests import cases as CS
from tests.test_gpu_parity import L, build_gpu  # noqa: F401

pytestmark = pytest.mark.gpu


def test_operator_calls_check_dtype_and_length(L):
    import torch
    c = CS.c1_poisson2d()
    m, md, t, dev = build_gpu(L, c)
    u, v = dev(c.u), dev(c.v)
    with pytest.raises(ValueError, match="dtype"):
        md.jvp(u, v.float())
    with pytest.raises(ValueError, match="elements"):
        md.jvp(u, v[:-1].contiguous())
    with pytest.raises(ValueError, match="elements"):
        md.jvp(u, v, out=torch.empty(md.N + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="elements"):
        md.residual(u, q_out=torch.empty(md.N, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="r1"):
        md.residual(u, time=L.Time(a0=1.0, r1=dev(c.u[:-3]), c1=1.0))
    with pytest.raises(ValueError, match="contiguous"):
        md.jvp(u, torch.stack([v, v], 1)[:, 0])
    bj = L.BlockJacobi(md, dev(c.u))
    with pytest.raises(ValueError, match="elements"):
        bj.apply(v[:5].contiguous())
    with pytest.raises(ValueError, match="elements"):
        L.gmres(md, v[:-1].contiguous())
    # a correct call still works after the refusals
    Jv = md.jvp(u, v).cpu().numpy()
    assert np.isfinite(Jv).all()


def test_mlp_and_patch_calls_check_inputs(L):
    import torch
    c = CS.c5_convdiff2d(n=4)
    m, md, t, dev = build_gpu(L, c)
    net = L.MLP(20 * m.nn, 32, m.nn)
    X = torch.zeros((3, 20 * m.nn), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="dtype"):
        net.forward(X)
    with pytest.raises(ValueError, match="elements"):
        net.forward(torch.zeros((3, 20 * m.nn - 1), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="dtype"):
        net.train_step(X.float(), torch.zeros((3, m.nn), dtype=torch.float64, device="cuda"), 1e-3)
    r = dev(c.u)
    with pytest.raises(ValueError, match="indices"):
        L.gather_patches(md, r, elems=torch.tensor([0, m.E], dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError, match="dtype"):
        L.gather_patches(md, r, elems=torch.tensor([0, 1], dtype=torch.int64, device="cuda"))
    Xg, _, _ = L.gather_patches(md, r, elems=torch.tensor([0, m.E - 1], dtype=torch.int32, device="cuda"))
    assert Xg.shape == (2, 20 * m.nn)
