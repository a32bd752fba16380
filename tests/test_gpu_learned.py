"""Learned preconditioner, end to end at a reduced size (needs an MI355X).

Train the element-patch MLP on solver-generated pairs from seeded
convection-diffusion instances, then solve held-out instances with FGMRES(30)
and record the iteration and time ratios against block-Jacobi alone.  What
must hold is asserted (training reduces the loss; every solve that reports
convergence passes the FP64 true-residual check); the gain is recorded.
"""
import json
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_learned_preconditioner_gain_on_held_out():
    import torch
    from paper_2205_07824_amd import ldg, learned as LP
    n, p = 32, 3
    train_seeds, test_seeds = range(0, 8), range(100000, 100004)
    rng = np.random.default_rng(0)
    Xs, Ys = [], []
    for sd in train_seeds:
        inst = LP.c5_instance(sd, n=n, p=p)
        bj = ldg.BlockJacobi(inst["model"])
        xs, xstar = LP.solve_recording(inst, bj, restart=30, rtol=1e-10)
        _say("instance", sd, "A", round(inst["A"], 2), "cycles", len(xs), "reference", xstar is not None)
        if xstar is None:
            continue
        X, Y = LP.make_samples(inst, bj, xs, xstar, per_pair=512, rng=rng)
        Xs += X
        Ys += Y
    X = torch.cat(Xs)
    Y = torch.cat(Ys)
    _say("samples", X.shape[0])
    net = ldg.MLP(X.shape[1], 256, Y.shape[1], bf16=True)
    net.set_params(LP.init_params((X.shape[1], 256, Y.shape[1]), seed=1))
    hist = LP.train(net, X, Y, epochs=30, batch=min(8192, X.shape[0] // 4), lr=1e-3, log=_say)
    assert np.isfinite(hist).all() and hist[-1] < hist[0]
    rows = []
    for sd in test_seeds:
        inst = LP.c5_instance(sd, n=n, p=p)
        bj = ldg.BlockJacobi(inst["model"])
        pc = ldg.LearnedPrecond(inst["model"], net, bj, composite=True)
        res = LP.evaluate(inst, bj, pc, restart=30, rtol=1e-8, maxit=6000)
        res["A"] = inst["A"]
        _say("held-out", sd, json.dumps(res))
        for k in ("block_jacobi", "learned"):
            if res[k]["ok"]:
                assert res[k]["res_true"] <= 1.01e-8 * res[k]["res0"]
        rows.append(res)
    both = [r for r in rows if r["block_jacobi"]["ok"] and r["learned"]["ok"]]
    ratios = [r["learned"]["iters"] / r["block_jacobi"]["iters"] for r in both]
    _say("converged with both:", len(both), "of", len(rows), "iteration ratios learned/BJ:", ratios,
         "learned-only converged:", sum(1 for r in rows if r["learned"]["ok"] and not r["block_jacobi"]["ok"]))
    _say("learned summary", json.dumps({"n": n, "p": p, "loss": hist, "held_out": rows}))
