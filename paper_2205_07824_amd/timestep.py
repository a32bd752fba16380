"""Implicit time stepping on the residual's time wrapper (Section 3.3 of the paper).

Every implicit stage solves G(u) = a0 M u - M (c1 r1 + c2 r2) + R(u) = 0 by
Newton-GMRES, with the block-Jacobi preconditioner rebuilt at every Newton
iterate.

* BDF: backward Euler for the first step (a0 = c1 = 1/dt, r1 = u_n), second-order
  backward differences after it (a0 = 3/(2 dt), r1 = u_n, c1 = 2/dt,
  r2 = u_{n-1}, c2 = -1/(2 dt)).
* DIRK (the paper's integrator family, Section 2): the stages U_i of
  M du/dt + R(u) = 0 satisfy M (U_i - u_n) = -dt sum_{j<=i} a_ij R(U_j).  With
  Y_l = U_l - u_n, the earlier stages' residuals are fixed by their values,
  R(U_j) = -(1/dt) sum_l (A^-1)_jl M Y_l, so stage i is the wrapper above with
  a0 = 1/(a_ii dt), r1 = u_n + sum_{l<i} c_il Y_l, c1 = a0, where
  c_il = sum_{l<=j<i} a_ij (A^-1)_jl; the step ends with
  u_{n+1} = u_n + sum_l (b^T A^-1)_l Y_l.  No inverse mass matrix is needed.
* The ODE coupled to the PDE (Eq. 1c), alpha dw/dt + beta w = s_w(u): its
  stages take the same form with the PDE's stage states, and each is one
  pointwise library call (w enters neither the flux nor the source).

Every numerical step is a library call; this module only sequences them and
records the per-step statistics.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import ldg


def euler_cfl_dt(U, nd, h, cfl, gamma=1.4):
    """dt = cfl * h / max(|v| + c) over the nodes of the conserved state U [E][nd+2][nn] (host array)."""
    U = np.asarray(U)
    rho = U[:, 0]
    mom = U[:, 1:1 + nd]
    E = U[:, 1 + nd]
    m2 = (mom ** 2).sum(axis=1)
    p = (gamma - 1.0) * (E - 0.5 * m2 / rho)
    speed = np.sqrt(m2) / rho + np.sqrt(gamma * p / rho)
    return cfl * h / float(speed.max())


@dataclasses.dataclass
class Ode:
    """State of the ODE coupled to the PDE (Eq. 1c), alpha dw/dt + beta w = s_w(u): w is a device vector
    [E][nw][nn] that the steppers advance in place."""
    w: torch.Tensor
    alpha: float = 1.0
    beta: float = 0.0


def bdf_steps(model, u0, dt, nsteps, restart=50, eta=1e-3, rtol=1e-8, jvp_prec=ldg.FP64, bj_prec=ldg.FP64,
              per_variable=False, newton_maxit=10, lin_maxit=5000, orth=ldg.ORTH_DCGS2, bj_refresh=1,
              log=None, atol=0.0, ode=None, state32=False, bj_every=1):
    """Advance u0 by nsteps implicit steps; returns (u, per-step statistics).  bj_refresh: 1 rebuilds the
    block-Jacobi preconditioner at every Newton iterate, 2 once per step (at its first iterate).  bj_every:
    steps between rebuilds; in between, a step keeps the blocks of the last rebuild (the first two steps, the
    BDF1 start and the first BDF2 step, whose time wrappers differ, always rebuild).  ode: the coupled ODE of
    the model (Ode), advanced with the same BDF formula from each step's solution.  state32: FP32 storage of
    the preconditioned Krylov vectors and of the linearization point in the products (jvp_prec must be
    FP32)."""
    u = u0.clone()
    u_prev = None
    w_prev = None
    stats = []
    pc = None
    for k in range(nsteps):
        un = u.clone()
        if k == 0:
            t = ldg.Time(a0=1.0 / dt, r1=un, c1=1.0 / dt)
        else:
            t = ldg.Time(a0=1.5 / dt, r1=un, c1=2.0 / dt, r2=u_prev, c2=-0.5 / dt)
        if pc is None:
            pc = ldg.BlockJacobi(model, u_lin=u, time=t, per_variable=per_variable, prec=bj_prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        refresh = bj_refresh if (k <= 1 or (k - 1) % bj_every == 0) else 0
        u, st, status = ldg.newton(model, u, time=t, rtol=rtol, atol=atol, eta=eta, maxit=newton_maxit,
                                   bj_refresh=refresh,
                                   bj_per_variable=per_variable, bj_prec=bj_prec, pc=pc, restart=restart,
                                   lin_maxit=lin_maxit, jvp_prec=jvp_prec, orth=orth, state32=state32,
                                   check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec = {"step": k + 1, "seconds": el, "converged": status == ldg.LDG_OK, "newton_iters": st["iters"],
               "blocks_rebuilt": refresh != 0,
               "gmres_iters": st["gmres_iters"], "res_ratio": st["res_final"] / max(st["res0"], 1e-300),
               "t_jvp": st["t_jvp"], "t_pc": st["t_pc"], "t_orth": st["t_orth"]}
        stats.append(rec)
        if log:
            log("step", rec)
        u_prev = un
        if status != ldg.LDG_OK:
            break
        if ode is not None:
            wn = ode.w.clone()
            tw = ldg.Time(a0=t.a0, r1=wn, c1=t.c1, r2=w_prev, c2=t.c2 if w_prev is not None else 0.0)
            model.ode_stage(u, tw, ode.alpha, ode.beta, out=ode.w)
            w_prev = wn
    return u, stats


def dirk_tableau(name):
    """Butcher matrix A and weights b of the singly diagonally implicit schemes: "be" implicit Euler;
    "dirk22" and "dirk33", Alexander's two- and three-stage L-stable schemes of orders 2 and 3 (the
    last row of A is b); "dirk34", the three-stage fourth-order A-stable scheme."""
    if name == "be":
        return [[1.0]], [1.0]
    if name == "dirk22":
        g = 1.0 - math.sqrt(0.5)
        return [[g, 0.0], [1.0 - g, g]], [1.0 - g, g]
    if name == "dirk33":
        # g: the root in (1/6, 1/2) of g^3 - 3 g^2 + (3/2) g - 1/6; with g = x + 1 the depressed cubic
        # x^3 + p x + q, p = -3/2, q = -2/3, whose three real roots have the trigonometric form below
        p, q = -1.5, -2.0 / 3.0
        amp = 2.0 * math.sqrt(-p / 3.0)
        th = math.acos(3.0 * q / (p * amp)) / 3.0
        g = 1.0 + amp * math.cos(th - 2.0 * math.pi / 3.0)
        b1 = -0.25 * (6.0 * g * g - 16.0 * g + 1.0)
        b2 = 0.25 * (6.0 * g * g - 20.0 * g + 5.0)
        return [[g, 0.0, 0.0], [0.5 * (1.0 + g) - g, g, 0.0], [b1, b2, g]], [b1, b2, g]
    if name == "dirk34":
        g = 0.5 + math.cos(math.pi / 18.0) / math.sqrt(3.0)
        d = 1.0 / (6.0 * (2.0 * g - 1.0) ** 2)
        return [[g, 0.0, 0.0], [0.5 - g, g, 0.0], [2.0 * g, 1.0 - 4.0 * g, g]], [d, 1.0 - 2.0 * d, d]
    raise ValueError(f"unknown DIRK scheme {name!r}")


def dirk_stage_coefficients(A, b):
    """For the stage form used by dirk_steps: c[i][l] (l < i), the weights of the earlier stage increments
    Y_l = U_l - u_n in stage i's right-hand side, and e = b^T A^-1, the weights of the step's final update."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    Ainv = np.linalg.inv(A)
    c = np.zeros((s, s))
    for i in range(s):
        for l in range(i):
            c[i, l] = sum(A[i, j] * Ainv[j, l] for j in range(l, i))
    return c, np.asarray(b, dtype=np.float64) @ Ainv


def dirk_steps(model, u0, dt, nsteps, scheme="dirk33", restart=50, eta=1e-3, rtol=1e-8, jvp_prec=ldg.FP64,
               bj_prec=ldg.FP64, per_variable=False, newton_maxit=10, lin_maxit=5000, orth=ldg.ORTH_DCGS2,
               bj_refresh=1, log=None, atol=0.0, ode=None):
    """Advance u0 by nsteps steps of a DIRK scheme (dirk_tableau); returns (u, per-step statistics).  Each
    stage starts Newton from the previous stage value and stops at ||G|| <= max(rtol ||G_0||, atol).  ode: the
    coupled ODE of the model (Ode); its stages take the same stage form, each from its PDE stage's state."""
    A, b = dirk_tableau(scheme)
    s = len(b)
    cst, e = dirk_stage_coefficients(A, b)
    u = u0.clone()
    stats = []
    pc = None
    for k in range(nsteps):
        un = u.clone()
        Y = []
        wn = ode.w.clone() if ode is not None else None
        Yw = []
        rec = {"step": k + 1, "seconds": 0.0, "converged": True, "newton_iters": 0, "gmres_iters": 0,
               "t_jvp": 0.0, "t_pc": 0.0, "t_orth": 0.0}
        U = un.clone()
        for i in range(s):
            a0 = 1.0 / (A[i][i] * dt)
            r1 = un.clone()
            for l in range(i):
                ldg.axpby(float(cst[i, l]), Y[l], 1.0, r1)
            t = ldg.Time(a0=a0, r1=r1, c1=a0)
            if pc is None:
                pc = ldg.BlockJacobi(model, u_lin=U, time=t, per_variable=per_variable, prec=bj_prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, st, status = ldg.newton(model, U, time=t, rtol=rtol, atol=atol, eta=eta, maxit=newton_maxit,
                                       bj_refresh=bj_refresh, bj_per_variable=per_variable, bj_prec=bj_prec, pc=pc,
                                       restart=restart, lin_maxit=lin_maxit, jvp_prec=jvp_prec, orth=orth,
                                       check=False)
            torch.cuda.synchronize()
            rec["seconds"] += time.perf_counter() - t0
            rec["newton_iters"] += st["iters"]
            rec["gmres_iters"] += st["gmres_iters"]
            for key in ("t_jvp", "t_pc", "t_orth"):
                rec[key] += st[key]
            if status != ldg.LDG_OK:
                rec["converged"] = False
                break
            Yi = U.clone()
            ldg.axpby(-1.0, un, 1.0, Yi)
            Y.append(Yi)
            if ode is not None:
                rw = wn.clone()
                for l in range(i):
                    ldg.axpby(float(cst[i, l]), Yw[l], 1.0, rw)
                Wi = model.ode_stage(U, ldg.Time(a0=a0, r1=rw, c1=a0), ode.alpha, ode.beta, out=rw)
                ldg.axpby(-1.0, wn, 1.0, Wi)
                Yw.append(Wi)
        if rec["converged"]:
            t0 = time.perf_counter()
            u = un.clone()
            for l in range(s):
                if e[l] != 0.0:
                    ldg.axpby(float(e[l]), Y[l], 1.0, u)
                    if ode is not None:
                        ldg.axpby(float(e[l]), Yw[l], 1.0, ode.w)
            torch.cuda.synchronize()
            rec["seconds"] += time.perf_counter() - t0
        stats.append(rec)
        if log:
            log("step", rec)
        if not rec["converged"]:
            break
    return u, stats
