"""Learned element-patch preconditioner for the 2D convection-diffusion workload.

Pipeline (every numerical step is a library kernel; this module sequences calls):
  1. instances: -div(kappa grad u) + b.grad u = 1 on the unit square, u = 0 on
     the boundary, kappa log-normal (correlation length 0.1, unit variance), b a
     seeded divergence-free field with |b| <= A, A ~ LogUniform[1, 100];
  2. data: restarted FGMRES + block-Jacobi solves each instance to 1e-10; at
     every restart boundary k the pair (r_k = b - J x_k, e_k = x* - x_k) is
     turned into patch samples (features of r_k / s, target
     (e_k - B^-1 r_k) / s on the centre element: what block-Jacobi misses);
  3. training: Adam on the mean squared error, cosine learning-rate decay;
  4. use: z = B^-1 r + s N(patch(r) / s) as the right preconditioner of FGMRES,
     with block-Jacobi as the fallback.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import inputs as I
from . import ldg


def c5_instance(seed, n=128, p=3):
    box = I.box_mesh(2, n)
    m = ldg.Mesh(box, p)
    xn, xq, xb, _ = m.points()
    grf = I.GRF.sample(seed)
    bvel = I.DivFreeVelocity.sample(seed)
    aux = np.concatenate([np.exp(grf.log_kappa(xn))[:, None, :], bvel(xn).transpose(0, 2, 1)], axis=1)
    tau = (p + 1) ** 2 * n
    md = ldg.Model(m, ldg.MODEL_CONVDIFF, 1, [1.0, tau], aux=aux, src=np.ones((m.E, 1, m.nqv)),
                   bdata=np.zeros((m.nbf, 1, m.nqf)), bc_kind=(0,))
    zero = torch.zeros(md.N, dtype=torch.float64, device="cuda")
    b = -md.residual(zero)
    return {"seed": seed, "mesh": m, "model": md, "b": b, "A": bvel.A}


def solve_recording(inst, bj, restart=30, rtol=1e-10, max_cycles=60, ref_restart=128, ref_maxit=40000):
    """Iterates x_k at the restart boundaries of FGMRES(restart) + block-Jacobi
    (at most max_cycles cycles), and a reference solution x* from a
    large-restart solve to rtol (None if that does not converge either)."""
    md, b = inst["model"], inst["b"]
    x = torch.zeros_like(b)
    r0 = ldg.norm(b)
    tol = rtol * r0
    xs = []
    converged = False
    for _ in range(max_cycles):
        xs.append(x.clone())
        x, st, status = ldg.gmres(md, b, x=x, pc=bj, restart=restart, rtol=0.0, atol=tol, maxit=restart, check=False)
        if status == ldg.LDG_OK:
            converged = True
            break
    if not converged:
        x, st, status = ldg.gmres(md, b, x=x, pc=bj, restart=ref_restart, rtol=0.0, atol=tol, maxit=ref_maxit,
                                  check=False)
        if status != ldg.LDG_OK:
            return xs, None
    return xs, x


def make_samples(inst, bj, xs, xstar, per_pair=2048, rng=None):
    md, b = inst["model"], inst["b"]
    E = inst["mesh"].E
    Xs, Ys = [], []
    for xk in xs:
        r = b - md.jvp(None, xk)
        e = xstar - xk
        t = e - bj.apply(r)
        sel = rng.choice(E, size=min(per_pair, E), replace=False).astype(np.int32)
        elems = torch.as_tensor(sel, device="cuda")
        X, Y, _ = ldg.gather_patches(md, r, t, elems)
        Xs.append(X)
        Ys.append(Y)
    return Xs, Ys


def init_params(dims, seed):
    """Xavier-uniform weights, zero biases (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    i, w, o = dims
    out = []
    for (fo, fi) in ((w, i), (w, w), (o, w)):
        a = math.sqrt(6.0 / (fi + fo))
        out.append(rng.uniform(-a, a, (fo, fi)).astype(np.float32))
        out.append(np.zeros(fo, dtype=np.float32))
    return out


def train(net, X, Y, epochs=20, batch=8192, lr=1e-3, seed=0, log=None):
    n = X.shape[0]
    steps = max(1, epochs * (n // batch))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            lr_t = 0.5 * lr * (1 + math.cos(math.pi * step / steps))
            loss = net.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr_t)
            tot += loss
            cnt += 1
            step += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep} loss {hist[-1]:.4e}")
    return hist


def evaluate(inst, bj, pc, restart=30, rtol=1e-8, maxit=20000):
    md, b = inst["model"], inst["b"]
    res = {}
    for name, p in (("block_jacobi", bj), ("learned", pc)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, status = ldg.gmres(md, b, pc=p, restart=restart, rtol=rtol, maxit=maxit, check=False)
        torch.cuda.synchronize()
        res[name] = {"iters": st["iters"], "seconds": time.perf_counter() - t0, "ok": status == ldg.LDG_OK,
                     "fell_back": st["fell_back"], "res_true": st["res_true"], "res0": st["res0"]}
    return res
