"""Products and solves with FP32 state (needs an MI355X).

ldg_jvp_state32 reads u and v in FP32 storage and computes in FP32: against the
oracle's FP64 product at the same (rounded) inputs it meets the FP32 bar, 1e-5.
The FP32-state Newton-GMRES (preconditioned vectors and linearization point in
FP32 inside the products; basis, Gram-Schmidt, Givens and the Newton residual in
FP64) reaches the root of the oracle's residual to 1e-8.
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
def test_jvp_state32_matches_oracle(L, name):
    import torch
    c = CS.ALL[name]()
    _say("state32 jvp", name)
    m, md, t, dev = build_gpu(L, c)
    u32 = torch.as_tensor(c.u, device="cuda").float()
    v32 = torch.as_tensor(c.v, device="cuda").float()
    ur, vr = u32.double().cpu().numpy(), v32.double().cpu().numpy()
    ref = c.om.jvp(c.oracle_model(), ur, vr)
    Jv = md.jvp_state32(u32, v32, time=t)
    J64 = md.jvp(dev(ur), dev(vr), time=t, prec=L.FP32)
    torch.cuda.synchronize()
    e = rel(Jv.cpu().numpy(), ref)
    _say("state32 vs oracle", e, "vs FP32 mode with FP64 inputs", rel(Jv.cpu().numpy(), J64.cpu().numpy()))
    assert e < 1e-5


def test_state32_needs_fp32_products(L):
    import torch
    c = CS.c2_poisson3d()
    m, md, t, dev = build_gpu(L, c)
    b = dev(c.v)
    with pytest.raises(L.LDGError) as ei:
        L.gmres(md, b, state32=True, jvp_prec=L.FP64)
    assert ei.value.status == L.LDG_EINVAL
    with pytest.raises(L.LDGError) as ei:
        L.gmres(md, b, state32=True, jvp_prec=L.FP32, orth=L.ORTH_MGS)
    assert ei.value.status == L.LDG_EUNSUPPORTED


def test_gmres_state32_reaches_fp64_solution(L):
    """The linear Poisson system to 1e-10 with FP32-state FGMRES + FP32 block-Jacobi: the true FP64 residual
    drives the restarts, so the solution matches the FP64 solve."""
    import torch
    c = CS.c2_poisson3d()
    m, md, t, dev = build_gpu(L, c)
    b = dev(c.v)
    pc = L.BlockJacobi(md, prec=L.FP32)
    x64, st64, s64 = L.gmres(md, b, pc=pc, restart=30, rtol=1e-11, maxit=3000, check=False)
    x32, st32, s32 = L.gmres(md, b, pc=pc, restart=30, rtol=1e-11, maxit=3000, jvp_prec=L.FP32, state32=True,
                             check=False)
    _say("fp64", st64["iters"], st64["res_true"] / st64["res0"], "state32", st32["iters"],
         st32["res_true"] / st32["res0"])
    assert s64 == L.LDG_OK and s32 == L.LDG_OK
    assert rel(x32.cpu().numpy(), x64.cpu().numpy()) < 1e-8


def test_newton_ns_state32_matches_oracle(L):
    """The Navier-Stokes BDF2 step of the Newton parity test, solved with FP32 state."""
    import scipy.sparse.linalg as spla
    c = CS.c4_ns3d(n=3, p=2, shift=0.3)
    _say("case c4 n=3 p=2 newton state32")
    om = c.oracle_model()
    lu = spla.splu(c.om.jacobian(om, c.u).tocsc())
    u_ref = c.u.copy()
    g0 = np.linalg.norm(c.om.residual(om, u_ref))
    for _ in range(40):
        g = c.om.residual(om, u_ref)
        if np.linalg.norm(g) <= 1e-13 * g0:
            break
        u_ref -= lu.solve(g)
    m, md, t, dev = build_gpu(L, c)
    u = dev(c.u.copy())
    pc = L.BlockJacobi(md, u_lin=u, time=t, per_variable=True, prec=L.FP32)
    u, st, status = L.newton(md, u, time=t, rtol=1e-12, eta=1e-5, maxit=20, bj_refresh=True, pc=pc, restart=50,
                             jvp_prec=L.FP32, state32=True)
    _say("newton ns state32 stats", st)
    assert status == L.LDG_OK
    assert rel(u.cpu().numpy(), u_ref) < 1e-8


@pytest.mark.parametrize("state32", [False, True])
def test_long_cycles_keep_converging(L, state32):
    """Long restart cycles of the delayed Gram-Schmidt variant, FP32 products: the pending vector is rescaled
    every step, so its magnitude does not grow by |J M| per step over the cycle (unscaled, the FP32-state
    Newton solve of the 32^3 Poisson workload with FP16 blocks diverged at restart 256).  Every cycle length
    converges to the FP64 true residual, and a longer cycle never needs more iterations."""
    import torch
    from paper_2205_07824_amd import inputs as I
    box = I.box_mesh(3, 32, perturb=0.05, seed=0)
    m = L.Mesh(box, 3)
    xn, xq, xb, _ = m.points()
    _, _, f = I.mms_expsin3d(xq)
    ub, _, _ = I.mms_expsin3d(xb)
    md = L.Model(m, L.MODEL_POISSON, 1, [1.0, 16.0 * 32, 0.0], src=f.reshape(m.E, 1, m.nqv),
                 bdata=ub.reshape(m.nbf, 1, m.nqf), bc_kind=(0,))
    b = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, md.N), device="cuda")
    pc = L.BlockJacobi(md, prec=L.FP16)
    its = []
    for rs in (128, 256, 512):
        x, st, status = L.gmres(md, b, pc=pc, restart=rs, rtol=1e-8, maxit=4000, jvp_prec=L.FP32, state32=state32,
                                check=False)
        _say("restart", rs, "state32", state32, "iters", st["iters"], "res", st["res_true"] / st["res0"])
        assert status == L.LDG_OK
        r = b - md.jvp(None, x)
        assert L.norm(r) <= 1.01e-8 * st["res0"]
        its.append(st["iters"])
    assert its[1] <= its[0] and its[2] <= its[1]
    u = torch.zeros(md.N, dtype=torch.float64, device="cuda")
    u, st, status = L.newton(md, u, rtol=1e-8, eta=1e-4, maxit=8, pc=pc, restart=256, lin_maxit=4000,
                             jvp_prec=L.FP32, state32=state32, check=False)
    _say("newton restart 256", st)
    assert status == L.LDG_OK and st["res_final"] <= 1.01e-8 * st["res0"]
