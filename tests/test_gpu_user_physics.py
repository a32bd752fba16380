"""Run-time compiled physics on the GPU (needs an MI355X).

* A user source re-stating the Euler equations against the built-in Euler
  model and the oracle: residual and JVP in FP64 and FP32, and one implicit step.
* A model the library does not have (nonlinear diffusion, kappa(u) =
  mu0 (1 + mu2 u^2)): at mu2 = 0 against the built-in Poisson operator; at
  mu2 > 0 discrete conservation on a periodic mesh (the fluxes are
  conservative and the basis sums to one) and its JVP against central
  differences of its own residual.
"""
import sys

import numpy as np
import pytest

from tests import cases as CS
from tests import user_physics as U
from paper_2205_07824_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2205_07824_amd import ldg
    assert torch.cuda.is_available()
    ldg.lib()
    return ldg


def dev(a):
    import torch
    return None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_user_euler_matches_builtin_and_oracle(L):
    c = CS.c3_euler2d(n=4, p=3)
    _say("case c3 user euler")
    m = L.Mesh(c.box, c.p, c.nq)
    built = L.Model(m, L.MODEL_EULER, 4, c.mu, bc_kind=c.bc_kind)
    user = L.Model(m, L.MODEL_USER, 4, c.mu, bc_kind=c.bc_kind, physics_source=U.EULER_2D, has_q=False)
    t = L.Time(a0=c.a0, r1=dev(c.r1), c1=c.c1, r2=dev(c.r2), c2=c.c2)
    u, v = dev(c.u), dev(c.v)
    om = c.oracle_model()
    G_ref, Jv_ref = c.om.residual(om, c.u), c.om.jvp(om, c.u, c.v)
    for prec, tol, same in ((L.FP64, 1e-12, 1e-13), (L.FP32, 1e-5, 1e-6)):
        Gu = user.residual(u, time=t, prec=prec).cpu().numpy()
        Ju = user.jvp(u, v, time=t, prec=prec).cpu().numpy()
        Gb = built.residual(u, time=t, prec=prec).cpu().numpy()
        Jb = built.jvp(u, v, time=t, prec=prec).cpu().numpy()
        _say("prec", prec, "user vs built-in", rel(Gu, Gb), rel(Ju, Jb), "user vs oracle", rel(Gu, G_ref),
             rel(Ju, Jv_ref))
        assert rel(Gu, Gb) < same and rel(Ju, Jb) < same
        assert rel(Gu, G_ref) < tol and rel(Ju, Jv_ref) < tol


def test_user_euler_implicit_step_matches_builtin(L):
    from paper_2205_07824_amd import timestep as TS
    c = CS.c3_euler2d(n=4, p=3)
    _say("case c3 user euler bdf steps")
    m = L.Mesh(c.box, c.p, c.nq)
    built = L.Model(m, L.MODEL_EULER, 4, c.mu, bc_kind=c.bc_kind)
    user = L.Model(m, L.MODEL_USER, 4, c.mu, bc_kind=c.bc_kind, physics_source=U.EULER_2D, has_q=False)
    kw = dict(restart=50, eta=1e-10, rtol=1e-12, newton_maxit=12)
    ub, sb = TS.bdf_steps(built, dev(c.u), 0.5, 2, **kw)
    uu, su = TS.bdf_steps(user, dev(c.u), 0.5, 2, **kw)
    assert all(s["converged"] for s in sb + su)
    assert rel(uu.cpu().numpy(), ub.cpu().numpy()) < 1e-10


def _diffusion(L, mu2, n=4, p=3):
    box = I.box_mesh(2, n, periodic=(True, True))
    m = L.Mesh(box, p)
    tau = (p + 1) ** 2 * n
    user = L.Model(m, L.MODEL_USER, 1, [1.0, tau, mu2], bc_kind=(0,), physics_source=U.NONLINEAR_DIFFUSION,
                   has_q=True)
    return m, user, tau


def test_user_diffusion_reduces_to_builtin_poisson(L):
    m, user, tau = _diffusion(L, 0.0)
    _say("user diffusion at mu2 = 0")
    built = L.Model(m, L.MODEL_POISSON, 1, [1.0, tau, 0.0], bc_kind=(0,))
    rng = np.random.default_rng(3)
    u, v = dev(rng.uniform(-1, 1, user.N)), dev(rng.uniform(-1, 1, user.N))
    assert rel(user.residual(u).cpu().numpy(), built.residual(u).cpu().numpy()) < 1e-13
    assert rel(user.jvp(u, v).cpu().numpy(), built.jvp(None, v).cpu().numpy()) < 1e-13


def test_user_diffusion_conservation_and_tangent(L):
    m, user, tau = _diffusion(L, 0.5)
    _say("user diffusion at mu2 = 0.5")
    rng = np.random.default_rng(4)
    u0, v0 = rng.uniform(-1, 1, user.N), rng.uniform(-1, 1, user.N)
    G = user.residual(dev(u0)).cpu().numpy()
    assert abs(G.sum()) < 1e-12 * np.abs(G).sum()
    Jv = user.jvp(dev(u0), dev(v0)).cpu().numpy()
    assert abs(Jv.sum()) < 1e-12 * np.abs(Jv).sum()
    eps = 1e-5
    Gp = user.residual(dev(u0 + eps * v0)).cpu().numpy()
    Gm = user.residual(dev(u0 - eps * v0)).cpu().numpy()
    fd = (Gp - Gm) / (2 * eps)
    _say("tangent vs central difference", rel(Jv, fd))
    assert rel(Jv, fd) < 1e-7
    # the nonlinearity is active: the tangent differs from the frozen-coefficient operator
    _, lin, _ = _diffusion(L, 0.0)
    assert rel(Jv, lin.jvp(dev(u0), dev(v0)).cpu().numpy()) > 1e-2
