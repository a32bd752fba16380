"""Learned preconditioner, end to end at a reduced size (needs an MI355X).

Train the element-patch MLP on solver-generated pairs from a few seeded
convection-diffusion instances, then solve held-out instances with FGMRES and
report the iteration and time ratio against block-Jacobi alone.  The true FP64
residual decides success.
"""
import json
import os
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
        X, Y = LP.make_samples(inst, bj, xs, xstar, per_pair=512, rng=rng)
        Xs += X
        Ys += Y
        _say("instance", sd, "A", round(inst["A"], 2), "cycles", len(xs))
    X = torch.cat(Xs)
    Y = torch.cat(Ys)
    _say("samples", X.shape[0])
    net = ldg.MLP(X.shape[1], 256, Y.shape[1], bf16=True)
    net.set_params(LP.init_params((X.shape[1], 256, Y.shape[1]), seed=1))
    hist = LP.train(net, X, Y, epochs=30, batch=min(8192, X.shape[0] // 4), lr=1e-3, log=_say)
    assert hist[-1] < hist[0]
    ratios = []
    for sd in test_seeds:
        inst = LP.c5_instance(sd, n=n, p=p)
        bj = ldg.BlockJacobi(inst["model"])
        pc = ldg.LearnedPrecond(inst["model"], net, bj, composite=True)
        res = LP.evaluate(inst, bj, pc, restart=30, rtol=1e-8)
        _say("held-out", sd, json.dumps(res))
        for v in res.values():
            assert v["ok"] and v["res_true"] <= 1.01e-8 * v["res0"]
        ratios.append(res["learned"]["iters"] / res["block_jacobi"]["iters"])
    _say("learned / block-Jacobi iteration ratio per held-out instance:", ratios, "mean", float(np.mean(ratios)))
    os.makedirs("gpurun_out", exist_ok=True)
    with open("gpurun_out/learned_small.json", "w") as f:
        json.dump({"n": n, "p": p, "train": list(train_seeds), "test": list(test_seeds), "loss": hist,
                   "iter_ratio": ratios}, f)
