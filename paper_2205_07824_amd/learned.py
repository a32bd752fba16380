"""Learned element-patch preconditioner for the 2D convection-diffusion workload.

Pipeline (the solver, the network's forward and backward passes and Adam run in
library kernels; this module draws seeded random vectors, rescales the training
targets by one constant, and sequences the calls):
  1. instances: -div(kappa grad u) + b.grad u = 1 on the unit square, u = 0 on
     the boundary, kappa log-normal (correlation length 0.1, unit variance), b a
     seeded divergence-free field with |b| <= A, A ~ LogUniform[1, 100];
  2. data: (residual, correction) pairs of the solver's own operator, J w = r:
     (a) seeded Gaussian y, the correction w = B^-1 y and its residual r = J w;
     (b) the steps of FGMRES with block-Jacobi, which records the input v_i of
     the preconditioner and J z_i for its output z_i = B^-1 v_i (so B z_i = v_i).
     Per sampled element K the sample is (features of r on the patch of K) / s
     -> (B w - r)_K / s, s = ||r on the patch||_2: the residual that the
     block-Jacobi step misses ((y - r) in (a), (v_i - J z_i) in (b));
  3. training: the network maps the coefficient features of the patch to a
     matrix A_K [nn][5 nn], and the loss is the mean squared error of A_K r / s
     against the target (ldg_mlp_train_step_bilinear); Adam, cosine learning-rate
     decay;
  4. use: z = B^-1 (r + A_K patch(r)) as the right preconditioner of flexible
     GMRES (ldg_precond_mlp, linear form), block-Jacobi as the fallback.

Why this form: the preconditioner is a fixed linear operator, as Krylov methods
assume, and the network's error enters the preconditioned residual through
B^-1 and J together (J B^-1 is close to the identity on each element), not
through J alone.  A network applied to the residual itself (the residual forms
of ldg_precond_mlp) gives a nonlinear, input-dependent map whose errors on the
Krylov vectors stall FGMRES.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import inputs as I
from . import ldg

_MESHES = {}


def c5_mesh(n=128, p=3):
    """The unit-square quad mesh of the workload (shared by all instances of one size)."""
    key = (n, p)
    if key not in _MESHES:
        m = ldg.Mesh(I.box_mesh(2, n), p)
        xn, _, _, _ = m.points()
        _MESHES[key] = (m, xn)
    return _MESHES[key]


def c5_instance(seed, n=128, p=3):
    m, xn = c5_mesh(n, p)
    grf = I.GRF.sample(seed)
    bvel = I.DivFreeVelocity.sample(seed)
    kappa = torch.exp(grf.log_kappa_on(xn, "cuda"))                                  # [E][nn]
    bv = torch.as_tensor(np.ascontiguousarray(bvel(xn).transpose(0, 2, 1)), dtype=torch.float64).cuda()
    aux = torch.cat([kappa[:, None, :], bv], dim=1).contiguous()                      # [E][3][nn]
    tau = (p + 1) ** 2 * n
    md = ldg.Model(m, ldg.MODEL_CONVDIFF, 1, [1.0, tau], aux=aux,
                   src=torch.ones((m.E, 1, m.nqv), dtype=torch.float64, device="cuda"),
                   bdata=torch.zeros((m.nbf, 1, m.nqf), dtype=torch.float64, device="cuda"), bc_kind=(0,))
    zero = torch.zeros(md.N, dtype=torch.float64, device="cuda")
    b = -md.residual(zero)
    return {"seed": seed, "mesh": m, "model": md, "b": b, "A": bvel.A}


def training_pairs(inst, bj, gen, nvec=2, per_vec=2048):
    """Samples from nvec seeded Gaussian vectors y: w = B^-1 y, r = J w, target y - r (= B w - r), on per_vec
    random elements each (patch features of r and the target, both divided by the patch scale s)."""
    md = inst["model"]
    E = inst["mesh"].E
    Xs, Ys = [], []
    for _ in range(nvec):
        y = torch.randn(md.N, dtype=torch.float64, device="cuda", generator=gen)
        r = md.jvp(None, bj.apply(y))
        t = y.clone()
        ldg.axpby(-1.0, r, 1.0, t)                     # t = y - r
        k = min(per_vec, E)
        elems = torch.randperm(E, device="cuda", generator=gen)[:k].to(torch.int32)
        X, Y, _ = ldg.gather_patches(md, r, t, elems)
        Xs.append(X)
        Ys.append(Y)
    return Xs, Ys


def solver_pairs(inst, bj, gen, steps=256, take=8, per_vec=1024, restart=128):
    """Samples from the steps of FGMRES(restart) + block-Jacobi solving the instance from x = 0: the solver
    records the preconditioner's input v_i and J z_i (ldg_gmres_opts.record_*); residual J z_i, target
    v_i - J z_i (= B z_i - J z_i).  `take` of the first `steps` steps, evenly spaced, per_vec elements each."""
    md, b = inst["model"], inst["b"]
    E = inst["mesh"].E
    V = torch.empty((steps, md.N), dtype=torch.float64, device="cuda")
    JZ = torch.empty_like(V)
    _, st, _ = ldg.gmres(md, b, pc=bj, restart=restart, rtol=0.0, maxit=steps, check=False, record=(V, JZ))
    done = min(int(st["iters"]), steps)
    Xs, Ys = [], []
    for i in np.unique(np.linspace(0, done - 1, take).round().astype(np.int64)):
        r = JZ[i]
        ldg.axpby(-1.0, r, 1.0, V[i])                 # V[i] := v_i - J z_i, the target
        k = min(per_vec, E)
        elems = torch.randperm(E, device="cuda", generator=gen)[:k].to(torch.int32)
        X, Y, _ = ldg.gather_patches(md, r, V[i], elems)
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
    """Adam with cosine learning-rate decay on the linear form's bilinear loss (ldg_mlp_train_step_bilinear)."""
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
            tot += net.train_step_bilinear(X[idx].contiguous(), Y[idx].contiguous(), lr_t)
            cnt += 1
            step += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep} loss {hist[-1]:.4e}")
    return hist


def fold_output_scale(net, c):
    """Multiply the last layer by c (a network trained on targets / c then predicts the targets)."""
    params, _ = net.get_params()
    params[4] = params[4] * np.float32(c)
    params[5] = params[5] * np.float32(c)
    net.set_params(params)


def training_set(seeds, n, p, gen, nvec, per_vec, solver_steps, solver_take, solver_per_vec, log=None):
    """Samples of every listed instance (training_pairs and solver_pairs)."""
    Xs, Ys = [], []
    t0 = time.perf_counter()
    for i, sd in enumerate(seeds):
        inst = c5_instance(sd, n=n, p=p)
        bj = ldg.BlockJacobi(inst["model"])
        if nvec:
            X, Y = training_pairs(inst, bj, gen, nvec=nvec, per_vec=per_vec)
            Xs += X
            Ys += Y
        if solver_take:
            X, Y = solver_pairs(inst, bj, gen, steps=solver_steps, take=solver_take, per_vec=solver_per_vec)
            Xs += X
            Ys += Y
        del bj, inst
        if log and (i + 1) % max(1, len(seeds) // 10) == 0:
            log(f"instances {i + 1}/{len(seeds)} ({time.perf_counter() - t0:.0f} s)")
    return torch.cat(Xs), torch.cat(Ys), time.perf_counter() - t0


def fit_network(train_seeds, n=128, p=3, nvec=2, per_vec=2048, solver_steps=256, solver_take=8,
                solver_per_vec=1024, width=256, epochs=30, batch=8192, lr=1e-3, seed=1, log=None):
    """Train the linear form's patch MLP (15 nn coefficient features -> nn x 5 nn map) on the pairs of the
    training instances; returns (net, info)."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    seeds = list(train_seeds)
    X, Y, t_data = training_set(seeds, n, p, gen, nvec, per_vec, solver_steps, solver_take, solver_per_vec,
                                log=log)
    c = float(torch.sqrt((Y.double() ** 2).mean()))       # one constant target scale, folded back afterwards
    Y /= c
    nn = Y.shape[1]
    dims = (15 * nn, width, 5 * nn * nn)
    net = ldg.MLP(*dims, bf16=True)
    net.set_params(init_params(dims, seed=seed))
    t1 = time.perf_counter()
    hist = train(net, X, Y, epochs=epochs, batch=min(batch, max(1, X.shape[0] // 4)), lr=lr, seed=seed, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    fold_output_scale(net, c)
    info = {"instances": len(seeds), "samples": int(X.shape[0]), "target_scale": c, "loss": hist,
            "data_seconds": round(t_data, 1), "train_seconds": round(t_train, 1), "n": n, "p": p, "nvec": nvec,
            "per_vec": per_vec, "solver_steps": solver_steps, "solver_take": solver_take,
            "solver_per_vec": solver_per_vec, "epochs": epochs, "lr": lr, "width": width, "dims": list(dims)}
    return net, info


def save_network(net, path, info):
    params, _ = net.get_params()
    np.savez(path, *params, dims=np.array(net.dims, dtype=np.int64), info=np.array(json.dumps(info)))


def load_network(path):
    """A network written by save_network, and its training record."""
    with np.load(path, allow_pickle=False) as f:
        dims = tuple(int(x) for x in f["dims"])
        params = [f[f"arr_{i}"] for i in range(6)]
        info = json.loads(str(f["info"]))
    net = ldg.MLP(*dims, bf16=True)
    net.set_params(params)
    return net, info


def evaluate(inst, net, restart=128, rtol=1e-8, maxit=20000, watch_window=0):
    """Time to rtol of FGMRES(restart) from x = 0 with block-Jacobi alone and with the learned composite
    (each time includes building its preconditioner); watch_window as in ldg_gmres_opts."""
    md, b = inst["model"], inst["b"]
    res = {}
    for name in ("block_jacobi", "learned"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bj = ldg.BlockJacobi(md)
        p = bj if name == "block_jacobi" else ldg.LearnedPrecond(md, net, bj, composite="linear")
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        x, st, status = ldg.gmres(md, b, pc=p, restart=restart, rtol=rtol, maxit=maxit, check=False,
                                  watch_window=watch_window)
        torch.cuda.synchronize()
        res[name] = {"iters": st["iters"], "seconds": round(time.perf_counter() - t0, 4),
                     "setup_seconds": round(t_setup, 4), "ok": status == ldg.LDG_OK, "fell_back": st["fell_back"],
                     "res_true": st["res_true"], "res0": st["res0"]}
        del p, bj
    return res


def summarize(rows):
    both = [r for r in rows if r["block_jacobi"]["ok"] and r["learned"]["ok"]]
    it = [r["learned"]["iters"] / r["block_jacobi"]["iters"] for r in both]
    tm = [r["learned"]["seconds"] / r["block_jacobi"]["seconds"] for r in both]
    return {"held_out": len(rows), "both_converged": len(both),
            "bj_only": sum(1 for r in rows if r["block_jacobi"]["ok"] and not r["learned"]["ok"]),
            "learned_only": sum(1 for r in rows if r["learned"]["ok"] and not r["block_jacobi"]["ok"]),
            "fell_back": sum(1 for r in rows if r["learned"]["fell_back"]),
            "iters_ratio_median": float(np.median(it)) if it else None,
            "time_ratio_median": float(np.median(tm)) if tm else None,
            "time_ratio_geomean": float(np.exp(np.mean(np.log(tm)))) if tm else None,
            "bj_seconds_total": round(sum(r["block_jacobi"]["seconds"] for r in both), 3),
            "learned_seconds_total": round(sum(r["learned"]["seconds"] for r in both), 3)}


def main(argv=None):
    ap = argparse.ArgumentParser(description="train the convection-diffusion patch network and evaluate it")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--train", type=int, default=2000, help="training instances (seeds 0..train-1)")
    ap.add_argument("--held-out", type=int, default=20, help="held-out instances (seeds 100000..)")
    ap.add_argument("--nvec", type=int, default=2)
    ap.add_argument("--per-vec", type=int, default=2048)
    ap.add_argument("--solver-steps", type=int, default=256)
    ap.add_argument("--solver-take", type=int, default=8)
    ap.add_argument("--solver-per-vec", type=int, default=1024)
    ap.add_argument("--watch-window", type=int, default=0)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--restart", type=int, default=128)
    ap.add_argument("--out", default=None, help="write the trained network here (.npz)")
    ap.add_argument("--record", default=None, help="write the training and held-out record here (.json)")
    ap.add_argument("--net", default=None, help="evaluate this network instead of training one")
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    if a.net:
        net, info = load_network(a.net)
    else:
        net, info = fit_network(range(a.train), n=a.n, p=a.p, nvec=a.nvec, per_vec=a.per_vec,
                                solver_steps=a.solver_steps, solver_take=a.solver_take,
                                solver_per_vec=a.solver_per_vec, epochs=a.epochs, lr=a.lr, log=log)
        info["command"] = "python -m paper_2205_07824_amd.learned " + " ".join(argv if argv is not None
                                                                                 else __import__("sys").argv[1:])
        log("trained", json.dumps({k: v for k, v in info.items() if k != "loss"}), "loss first/last",
            info["loss"][0], info["loss"][-1])
        if a.out:
            save_network(net, a.out, info)
    rows = []
    for sd in range(100000, 100000 + a.held_out):
        inst = c5_instance(sd, n=a.n, p=a.p)
        if not rows:   # the first solve of this basis size allocates the solver workspace: not timed
            bj = ldg.BlockJacobi(inst["model"])
            ldg.gmres(inst["model"], inst["b"], pc=bj, restart=a.restart, maxit=2, check=False)
            del bj
        r = evaluate(inst, net, restart=a.restart, watch_window=a.watch_window)
        r["seed"], r["A"] = sd, round(inst["A"], 3)
        log("held-out", json.dumps(r))
        rows.append(r)
        del inst
    summ = summarize(rows)
    log("summary", json.dumps(summ))
    if a.record:
        with open(a.record, "w") as f:
            json.dump({"training": info, "restart": a.restart, "held_out": rows, "summary": summ}, f, indent=1)


if __name__ == "__main__":
    main()
