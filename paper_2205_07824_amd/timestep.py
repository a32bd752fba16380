"""Implicit time stepping on the residual's time wrapper (Section 3.3 of the paper).

Each step solves G(u) = a0 M u - M (c1 r1 + c2 r2) + R(u) = 0 by Newton-GMRES:
backward Euler for the first step (a0 = c1 = 1/dt, r1 = u_n), second-order
backward differences after it (a0 = 3/(2 dt), r1 = u_n, c1 = 2/dt,
r2 = u_{n-1}, c2 = -1/(2 dt)).  The block-Jacobi preconditioner is rebuilt at
every Newton iterate.  Every numerical step is a library call; this module only
sequences them and records the per-step statistics.
"""
from __future__ import annotations

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


def bdf_steps(model, u0, dt, nsteps, restart=50, eta=1e-3, rtol=1e-8, jvp_prec=ldg.FP64, bj_prec=ldg.FP64,
              per_variable=False, newton_maxit=10, lin_maxit=5000, orth=ldg.ORTH_DCGS2, bj_refresh=1,
              log=None):
    """Advance u0 by nsteps implicit steps; returns (u, per-step statistics).  bj_refresh: 1 rebuilds the
    block-Jacobi preconditioner at every Newton iterate, 2 once per step (at its first iterate)."""
    u = u0.clone()
    u_prev = None
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
        u, st, status = ldg.newton(model, u, time=t, rtol=rtol, eta=eta, maxit=newton_maxit, bj_refresh=bj_refresh,
                                   bj_per_variable=per_variable, bj_prec=bj_prec, pc=pc, restart=restart,
                                   lin_maxit=lin_maxit, jvp_prec=jvp_prec, orth=orth, check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec = {"step": k + 1, "seconds": el, "converged": status == ldg.LDG_OK, "newton_iters": st["iters"],
               "gmres_iters": st["gmres_iters"], "res_ratio": st["res_final"] / max(st["res0"], 1e-300),
               "t_jvp": st["t_jvp"], "t_pc": st["t_pc"], "t_orth": st["t_orth"]}
        stats.append(rec)
        if log:
            log("step", rec)
        u_prev = un
        if status != ldg.LDG_OK:
            break
    return u, stats
