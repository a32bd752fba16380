"""Run-time compiled physics on the GPU (needs an MI355X).

* A user source re-stating the Euler equations against the built-in Euler
  model and the oracle: residual and JVP in FP64 and FP32, and one implicit step.
* The shallow-water system as a user source (the paper's second convection
  workload, a Bickley jet) against the oracle's shallow-water model: residual
  and JVP in FP64 and FP32, and a DIRK(3,3) step.
* A model the library does not have (nonlinear diffusion, kappa(u) =
  mu0 (1 + mu2 u^2)): at mu2 = 0 against the built-in Poisson operator; at
  mu2 > 0 discrete conservation on a periodic mesh (the fluxes are
  conservative and the basis sums to one) and its JVP against central
  differences of its own residual.
* A boundary function in the source (Euler slip walls) against the oracle's slip wall.
* The wave model with the coupled displacement ODE (Eq. 1c): one ODE stage
  against its defining equation, and DIRK(3,3) steps against the oracle's.
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


def _jet_case(n=4, p=3, g=100.0, seed=3):
    import oracle as O
    L = 4.0 * np.pi
    box = I.box_mesh(2, n, lo=(-L / 2, -L / 2), hi=(L / 2, L / 2), periodic=(True, True))
    om = O.Mesh(box, p)
    xn, _, _, _ = om.points()
    U0 = I.bickley_jet(xn, seed=seed, eps=0.05).transpose(0, 2, 1).reshape(-1)
    rng = np.random.default_rng(seed)
    u = U0 + 0.02 * rng.uniform(-1, 1, U0.shape)   # generic (off the symmetric state)
    return box, om, U0, u, rng.uniform(-1, 1, U0.shape)


def test_user_shallow_water_matches_oracle(L):
    import oracle as O
    g, dt = 100.0, 0.05
    box, om, U0, u, v = _jet_case(g=g)
    _say("case shallow-water jet")
    m = L.Mesh(box, 3)
    md = L.Model(m, L.MODEL_USER, 3, [g], bc_kind=(0,), physics_source=U.SHALLOW_WATER_2D, has_q=False)
    r1 = U0.copy()
    t = L.Time(a0=1.0 / dt, r1=dev(r1), c1=1.0 / dt)
    omd = O.Model(O.MODEL_SHALLOW_WATER, 3, [g], a0=1.0 / dt, r=r1 / dt)
    G_ref, Jv_ref = om.residual(omd, u), om.jvp(omd, u, v)
    for prec, tol in ((L.FP64, 1e-12), (L.FP32, 1e-5)):
        G = md.residual(dev(u), time=t, prec=prec).cpu().numpy()
        Jv = md.jvp(dev(u), dev(v), time=t, prec=prec).cpu().numpy()
        _say("prec", prec, "residual", rel(G, G_ref), "jvp", rel(Jv, Jv_ref))
        assert rel(G, G_ref) < tol and rel(Jv, Jv_ref) < tol


def test_user_shallow_water_dirk_step_matches_oracle(L):
    import oracle as O
    from paper_2205_07824_amd import timestep as TS
    g, dt = 100.0, 0.05
    box, om, U0, u, v = _jet_case(g=g)
    _say("case shallow-water jet dirk33")
    m = L.Mesh(box, 3)
    md = L.Model(m, L.MODEL_USER, 3, [g], bc_kind=(0,), physics_source=U.SHALLOW_WATER_2D, has_q=False)
    A, b = O.dirk_tableau("dirk33")
    u_ref = O.dirk_step(om, O.Model(O.MODEL_SHALLOW_WATER, 3, [g]), U0.copy(), dt, A, b)
    ug, stats = TS.dirk_steps(md, dev(U0.copy()), dt, 1, scheme="dirk33", restart=50, eta=1e-10, rtol=1e-12,
                              newton_maxit=12)
    _say("dirk stats", stats)
    assert stats[0]["converged"]
    assert rel(ug.cpu().numpy(), u_ref) < 1e-8


def test_user_diffusion_with_aux_and_dirichlet_data_matches_builtin_poisson(L):
    """Boundary data and aux fields through a compiled model: at mu2 = 0 the user source is the built-in
    Poisson operator with kappa(x), a source and Dirichlet data (whose data terms the built-in linear model
    integrates separately)."""
    from tests.util import penalty
    n, p = 4, 3
    box = I.box_mesh(2, n)
    m = L.Mesh(box, p)
    xn, xq, xb, _ = m.points()
    _, _, f = I.mms_sin2d(xq)
    ub, _, _ = I.mms_sin2d(xb)
    kap = 1.0 + 0.5 * np.sin(3.0 * xn[..., 0]) * np.cos(2.0 * xn[..., 1])
    mu = [1.3, penalty(p, 1.0 / n), 0.0]
    args = dict(aux=kap[:, None, :], src=f.reshape(m.E, 1, m.nqv), bdata=ub.reshape(m.nbf, 1, m.nqf), bc_kind=(0,))
    built = L.Model(m, L.MODEL_POISSON, 1, mu, **args)
    user = L.Model(m, L.MODEL_USER, 1, mu, physics_source=U.NONLINEAR_DIFFUSION, has_q=True, **args)
    rng = np.random.default_rng(8)
    u, v = dev(rng.uniform(-1, 1, user.N)), dev(rng.uniform(-1, 1, user.N))
    eg = rel(user.residual(u).cpu().numpy(), built.residual(u).cpu().numpy())
    ej = rel(user.jvp(u, v).cpu().numpy(), built.jvp(None, v).cpu().numpy())
    _say("user vs built-in with data: residual", eg, "jvp", ej)
    assert eg < 1e-12 and ej < 1e-12


def test_user_wave_model_matches_oracle(L):
    """The paper's wave model (q_t + grad u = 0, u_t + div(c^2 q) = 0) as a compiled first-order system
    against the oracle's: residual and JVP in FP64 and FP32, and a DIRK(3,3) step of a plane wave."""
    import oracle as O
    from paper_2205_07824_amd import timestep as TS
    c2, n, p, dt = 2.0, 4, 3, 0.02
    box = I.box_mesh(2, n, periodic=(True, True), perturb=0.05, seed=2)
    om = O.Mesh(box, p)
    k = 2 * np.pi * np.array([1.0, 2.0])
    th = om.points()[0] @ k
    U0 = np.stack([-np.cos(th), -k[0] * np.cos(th), -k[1] * np.cos(th)], axis=1).reshape(-1)
    rng = np.random.default_rng(6)
    u, v = U0 + 0.1 * rng.uniform(-1, 1, U0.shape), rng.uniform(-1, 1, U0.shape)
    m = L.Mesh(box, p)
    md = L.Model(m, L.MODEL_USER, 3, [c2], bc_kind=(0,), physics_source=U.WAVE_2D, has_q=False)
    t = L.Time(a0=1.0 / dt, r1=dev(U0), c1=1.0 / dt)
    omd = O.Model(O.MODEL_WAVE, 3, [c2], a0=1.0 / dt, r=U0 / dt)
    G_ref, Jv_ref = om.residual(omd, u), om.jvp(omd, u, v)
    for prec, tol in ((L.FP64, 1e-12), (L.FP32, 1e-5)):
        G = md.residual(dev(u), time=t, prec=prec).cpu().numpy()
        Jv = md.jvp(dev(u), dev(v), time=t, prec=prec).cpu().numpy()
        _say("wave prec", prec, "residual", rel(G, G_ref), "jvp", rel(Jv, Jv_ref))
        assert rel(G, G_ref) < tol and rel(Jv, Jv_ref) < tol
    A, b = O.dirk_tableau("dirk33")
    u_ref = O.dirk_step(om, O.Model(O.MODEL_WAVE, 3, [c2]), U0.copy(), dt, A, b)
    ug, stats = TS.dirk_steps(md, dev(U0.copy()), dt, 1, scheme="dirk33", restart=50, eta=1e-10, rtol=1e-12,
                              newton_maxit=6)
    assert stats[0]["converged"]
    assert rel(ug.cpu().numpy(), u_ref) < 1e-8


def test_user_model_argument_errors(L):
    m = L.Mesh(I.box_mesh(2, 2), 2)
    # a physics source needs kind MODEL_USER, and MODEL_USER needs a source
    with pytest.raises(L.LDGError):
        L.Model(m, L.MODEL_EULER, 4, [1.4], physics_source=U.EULER_2D, has_q=False)
    with pytest.raises(L.LDGError):
        L.Model(m, L.MODEL_USER, 4, [1.4])
    # declared sizes that contradict the source, and a source that does not compile: the compiler's message
    with pytest.raises(L.LDGError) as e:
        L.Model(m, L.MODEL_USER, 5, [1.4], physics_source=U.EULER_2D, has_q=False)
    assert "differs" in str(e.value)
    with pytest.raises(L.LDGError) as e:
        L.Model(m, L.MODEL_USER, 1, [1.0], physics_source=U.BROKEN, has_q=True)
    assert "physics_source:6" in str(e.value)
    # more aux fields than the source's NAUX bound (the kernels hold NAUX values per point)
    aux = np.ones((m.E, 2, m.nn))
    with pytest.raises(L.LDGError) as e:
        L.Model(m, L.MODEL_USER, 4, [1.4], aux=aux, physics_source=U.EULER_2D, has_q=False)
    assert "NAUX" in str(e.value)
    # the library stays usable after the failures
    md = L.Model(m, L.MODEL_USER, 4, [1.4], physics_source=U.EULER_2D, has_q=False)
    assert md.N == 4 * 9 * 4


def test_ode_stage_matches_its_definition(L):
    """One implicit stage of the coupled ODE, alpha (a0 w - c1 r1 - c2 r2) + beta w = s_w(u), at every node,
    against the stage equation solved in numpy with the source's s_w = (u, mu1 q1 q2)."""
    import torch
    m = L.Mesh(I.box_mesh(2, 3, periodic=(True, True), perturb=0.05, seed=4), 3)
    md = L.Model(m, L.MODEL_USER, 3, [2.0, 0.5], bc_kind=(0,), physics_source=U.WAVE_2D_W, has_q=False)
    assert md.nw == 2
    E, nn = m.E, m.nn
    rng = np.random.default_rng(8)
    u = rng.uniform(-1, 1, (E, 3, nn))
    r1, r2 = rng.uniform(-1, 1, (E, 2, nn)), rng.uniform(-1, 1, (E, 2, nn))
    sw = np.stack([u[:, 0], 0.5 * u[:, 1] * u[:, 2]], axis=1)
    for alpha, beta, a0, c1, c2, with_r2 in ((1.3, 0.4, 1.7, 0.9, -0.3, True), (1.0, 0.0, 25.0, 25.0, 0.0, False),
                                             (0.0, 2.0, 5.0, 5.0, 0.0, False)):
        t = L.Time(a0=a0, r1=dev(r1.reshape(-1)), c1=c1, r2=dev(r2.reshape(-1)) if with_r2 else None, c2=c2)
        w = md.ode_stage(dev(u.reshape(-1)), t, alpha, beta).cpu().numpy().reshape(E, 2, nn)
        # residual of the stage equation, relative to its terms
        res = alpha * (a0 * w - c1 * r1 - (c2 * r2 if with_r2 else 0.0)) + beta * w - sw
        scale = np.abs(alpha * a0 * w).max() + np.abs(beta * w).max() + np.abs(sw).max()
        _say("ode stage", alpha, beta, np.abs(res).max() / scale)
        assert np.abs(res).max() < 1e-14 * scale
    # w may overwrite r1 in place
    r1d = dev(r1.reshape(-1))
    t = L.Time(a0=1.7, r1=r1d, c1=0.9)
    ref = md.ode_stage(dev(u.reshape(-1)), t, 1.3, 0.4).cpu().numpy()
    md.ode_stage(dev(u.reshape(-1)), t, 1.3, 0.4, out=r1d)
    torch.cuda.synchronize()
    assert np.array_equal(r1d.cpu().numpy(), ref)
    # a singular stage and a model without an ODE are errors
    with pytest.raises(L.LDGError):
        md.ode_stage(dev(u.reshape(-1)), L.Time(a0=2.0, r1=r1d, c1=2.0), 1.0, -2.0)
    md0 = L.Model(m, L.MODEL_USER, 3, [2.0], bc_kind=(0,), physics_source=U.WAVE_2D, has_q=False)
    assert md0.nw == 0
    with pytest.raises(L.LDGError):
        md0.ode_stage(dev(u.reshape(-1)), t, 1.0, 0.0)


def test_dirk_with_coupled_ode_matches_oracle(L):
    """The wave model with its displacement ODE (and a nonlinear second component) through two DIRK(3,3)
    steps against the oracle's DIRK step with the same ODE; and BDF1/BDF2 on a steady state, where the
    displacement grows exactly linearly."""
    import oracle as O
    import torch
    from paper_2205_07824_amd import timestep as TS
    c2, n, p, dt = 2.0, 4, 3, 0.02
    box = I.box_mesh(2, n, periodic=(True, True), perturb=0.05, seed=2)
    om = O.Mesh(box, p)
    k = 2 * np.pi * np.array([1.0, 2.0])
    th = om.points()[0] @ k
    U0 = np.stack([-np.cos(th), -k[0] * np.cos(th), -k[1] * np.cos(th)], axis=1).reshape(-1)
    m = L.Mesh(box, p)
    md = L.Model(m, L.MODEL_USER, 3, [c2, 0.5], bc_kind=(0,), physics_source=U.WAVE_2D_W, has_q=False)
    E, nn = m.E, m.nn
    w0 = np.random.default_rng(9).uniform(-1, 1, E * 2 * nn)

    def sw(X):
        X = X.reshape(E, 3, nn)
        return np.stack([X[:, 0], 0.5 * X[:, 1] * X[:, 2]], axis=1).reshape(-1)

    A, b = O.dirk_tableau("dirk33")
    for alpha, beta in ((1.0, 0.0), (2.0, 0.5)):
        u_ref, w_ref = U0.copy(), w0.copy()
        for _ in range(2):
            u_ref, w_ref = O.dirk_step(om, O.Model(O.MODEL_WAVE, 3, [c2]), u_ref, dt, A, b,
                                       ode=(sw, alpha, beta, w_ref))
        ode = TS.Ode(w=dev(w0.copy()), alpha=alpha, beta=beta)
        ug, stats = TS.dirk_steps(md, dev(U0.copy()), dt, 2, scheme="dirk33", restart=50, eta=1e-10, rtol=1e-12,
                                  newton_maxit=6, ode=ode)
        assert all(s["converged"] for s in stats)
        eu, ew = rel(ug.cpu().numpy(), u_ref), rel(ode.w.cpu().numpy(), w_ref)
        _say("dirk33 + ode", alpha, beta, "u", eu, "w", ew)
        assert eu < 1e-8 and ew < 1e-8
    # steady state: BDF1 then BDF2 give w_n = w_0 + n dt u0 exactly for alpha w' = u0 (beta = 0)
    us = np.broadcast_to(np.array([0.7, -0.3, 0.4])[None, :, None], (E, 3, nn)).reshape(-1).copy()
    ode = TS.Ode(w=dev(w0.copy()), alpha=2.0, beta=0.0)
    _, stats = TS.bdf_steps(md, dev(us), dt, 3, restart=20, eta=1e-10, rtol=1e-12, atol=1e-12, newton_maxit=4,
                            ode=ode)
    assert all(s["converged"] for s in stats)
    torch.cuda.synchronize()
    w = ode.w.cpu().numpy().reshape(E, 2, nn)
    w_exact = w0.reshape(E, 2, nn) + 3 * dt * np.stack([np.full((E, nn), 0.7), np.full((E, nn), 0.5 * -0.3 * 0.4)],
                                                      axis=1) / 2.0
    _say("bdf + ode steady", np.abs(w - w_exact).max())
    assert np.abs(w - w_exact).max() < 1e-12


def test_user_slip_wall_matches_oracle(L):
    """A boundary function in the physics source: Euler in a channel (periodic in x) whose walls (tags 2, 3)
    reverse the normal momentum, against the oracle's slip-wall boundary kind: residual and JVP in FP64 and
    FP32, with a time wrapper; and a uniform flow along the walls stays steady."""
    import oracle as O
    p = 3
    box = I.box_mesh(2, 4, periodic=(True, False), perturb=0.05, seed=5)
    om = O.Mesh(box, p)
    m = L.Mesh(box, p)
    md = L.Model(m, L.MODEL_USER, 4, [1.4], bc_kind=(0, 0, 0, 0), physics_source=U.EULER_2D_SLIP, has_q=False)
    rng = np.random.default_rng(11)
    E, nn = m.E, m.nn
    u = np.empty((E, 4, nn))
    u[:, 0] = 1.0 + 0.2 * rng.uniform(-1, 1, (E, nn))
    u[:, 1:3] = 0.3 * rng.uniform(-1, 1, (E, 2, nn))
    u[:, 3] = 2.5 + 0.2 * rng.uniform(-1, 1, (E, nn))
    u = u.reshape(-1)
    v = rng.uniform(-1, 1, u.size)
    r1 = u + 0.01 * rng.uniform(-1, 1, u.size)
    a0 = 4.0
    omd = O.Model(O.MODEL_EULER, 4, [1.4], bc_kind=(0, 0, O.BC_SLIP_WALL, O.BC_SLIP_WALL), a0=a0, r=a0 * r1)
    G_ref, Jv_ref = om.residual(omd, u), om.jvp(omd, u, v)
    t = L.Time(a0=a0, r1=dev(r1), c1=a0)
    for prec, tol in ((L.FP64, 1e-12), (L.FP32, 1e-5)):
        G = md.residual(dev(u), time=t, prec=prec).cpu().numpy()
        Jv = md.jvp(dev(u), dev(v), time=t, prec=prec).cpu().numpy()
        _say("slip wall prec", prec, "residual", rel(G, G_ref), "jvp", rel(Jv, Jv_ref))
        assert rel(G, G_ref) < tol and rel(Jv, Jv_ref) < tol
    state = np.array([1.2, 0.6, 0.0, 1.0 / 0.4 + 0.5 * 1.2 * 0.25])
    us = np.broadcast_to(state[None, :, None], (E, 4, nn)).reshape(-1).copy()
    G = md.residual(dev(us)).cpu().numpy()
    _say("slip wall channel flow residual", np.abs(G).max())
    assert np.abs(G).max() < 1e-12


def test_user_reaction_source_matches_builtin_poisson_and_oracle(L):
    """A state-dependent source s(u) = -lambda u (Eq. 1b) compiled at run time, with kappa(x), a data source and
    Dirichlet data: against the oracle's Poisson model with reaction lambda (residual and JVP, FP64 and FP32)
    and the built-in one."""
    import oracle as O
    from tests.util import penalty
    n, p, lam = 4, 3, 0.7
    box = I.box_mesh(2, n)
    om = O.Mesh(box, p)
    m = L.Mesh(box, p)
    xn, xq, xb, _ = om.points()
    _, _, f = I.mms_sin2d(xq)
    ub, _, _ = I.mms_sin2d(xb)
    kap = (1.0 + 0.5 * np.sin(3.0 * xn[..., 0]) * np.cos(2.0 * xn[..., 1]))[:, None, :]
    tau = penalty(p, 1.0 / n)
    data = dict(aux=kap, src=f.reshape(om.E, 1, om.nqv), bdata=ub.reshape(om.nbf, 1, om.nqf), bc_kind=(0,))
    built = L.Model(m, L.MODEL_POISSON, 1, [1.3, tau, lam], **data)
    user = L.Model(m, L.MODEL_USER, 1, [1.3, tau, 0.0, lam, 0.0], physics_source=U.REACTION_DIFFUSION, has_q=True,
                   **data)
    omd = O.Model(O.MODEL_POISSON, 1, [1.3, tau, lam], aux=kap, src=data["src"], bdata=data["bdata"], bc_kind=[0])
    rng = np.random.default_rng(12)
    u0, v0 = rng.uniform(-1, 1, user.N), rng.uniform(-1, 1, user.N)
    G_ref, J_ref = om.residual(omd, u0), om.jvp(omd, u0, v0)
    for prec, tol in ((L.FP64, 1e-12), (L.FP32, 1e-5)):
        G = user.residual(dev(u0), prec=prec).cpu().numpy()
        Jv = user.jvp(dev(u0), dev(v0), prec=prec).cpu().numpy()
        Gb = built.residual(dev(u0), prec=prec).cpu().numpy()
        _say("reaction source prec", prec, "vs oracle", rel(G, G_ref), rel(Jv, J_ref), "vs built-in", rel(G, Gb))
        assert rel(G, G_ref) < tol and rel(Jv, J_ref) < tol and rel(G, Gb) < tol
    # the source term alone: G(lambda) - G(0) = lambda M u, with M the oracle's mass matrix
    plain = L.Model(m, L.MODEL_USER, 1, [1.3, tau, 0.0, 0.0, 0.0], physics_source=U.REACTION_DIFFUSION,
                    has_q=True, **data)
    dG = user.residual(dev(u0)).cpu().numpy() - plain.residual(dev(u0)).cpu().numpy()
    Mu = lam * om.mass_apply(1, u0)
    _say("source term vs lambda M u", rel(dG, Mu))
    assert rel(dG, Mu) < 1e-11


def test_user_nonlinear_source_and_boundary_function_tangent(L):
    """A cubic source and a state-dependent boundary function on a q-dependent flux (outside state
    g + mu5 uL^2 on the x+ side, q+ = q-): the JVP against central differences of the residual, and with
    mu5 = 0 the boundary function reproduces the model without it."""
    from tests.util import penalty
    n, p = 4, 3
    box = I.box_mesh(2, n, perturb=0.04, seed=5)
    m = L.Mesh(box, p)
    rng = np.random.default_rng(13)
    data = dict(src=rng.uniform(-1, 1, (m.E, 1, m.nqv)), bdata=rng.uniform(-1, 1, (m.nbf, 1, m.nqf)),
                bc_kind=(0, 0, 0, 0))
    mu = [1.0, penalty(p, 1.0 / n), 0.3, 0.4, 0.5, 0.25]
    md = L.Model(m, L.MODEL_USER, 1, mu, physics_source=U.REACTION_DIFFUSION_BOU, has_q=True, **data)
    u0, v0 = rng.uniform(-1, 1, md.N), rng.uniform(-1, 1, md.N)
    Jv = md.jvp(dev(u0), dev(v0)).cpu().numpy()
    eps = 1e-5
    fd = (md.residual(dev(u0 + eps * v0)).cpu().numpy() - md.residual(dev(u0 - eps * v0)).cpu().numpy()) / (2 * eps)
    _say("source + boundary function: tangent vs central difference", rel(Jv, fd))
    assert rel(Jv, fd) < 1e-7
    mu0 = mu[:5] + [0.0]
    a = L.Model(m, L.MODEL_USER, 1, mu0, physics_source=U.REACTION_DIFFUSION_BOU, has_q=True, **data)
    b = L.Model(m, L.MODEL_USER, 1, mu0[:5], physics_source=U.REACTION_DIFFUSION, has_q=True, **data)
    assert rel(a.residual(dev(u0)).cpu().numpy(), b.residual(dev(u0)).cpu().numpy()) < 1e-14
    assert rel(a.jvp(dev(u0), dev(v0)).cpu().numpy(), b.jvp(dev(u0), dev(v0)).cpu().numpy()) < 1e-14
    # and with mu5 != 0 it changes the residual
    assert rel(md.residual(dev(u0)).cpu().numpy(), a.residual(dev(u0)).cpu().numpy()) > 1e-6
