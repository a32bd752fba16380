"""Learned-preconditioner kernels against the FP64 numpy oracle (needs an MI355X).

The FP32 GEMM path pins the indexing of every forward/backward product; the
MFMA bf16 path is checked to bf16 accuracy on the same weights and batch.
"""
import sys

import numpy as np
import pytest

import oracle as O
from tests import cases as CS

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
                 / max(np.linalg.norm(np.asarray(b, dtype=np.float64)), 1e-300))


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2205_07824_amd import ldg
    assert torch.cuda.is_available()
    ldg.lib()
    return ldg


def _params(rng, dims):
    i, w, o = dims
    shapes = [(w, i), (w,), (w, w), (w,), (o, w), (o,)]
    ps = []
    for s in shapes:
        fan = s[-1] if len(s) == 2 else s[0]
        ps.append(rng.uniform(-1, 1, s) * (1.0 / np.sqrt(fan)))
    return ps


@pytest.mark.parametrize("bf16,tol_f,tol_g", [(False, 1e-5, 1e-4), (True, 3e-2, 8e-2)])
@pytest.mark.parametrize("B", [300, 4099])
def test_mlp_forward_backward_vs_oracle(L, bf16, tol_f, tol_g, B):
    import torch
    _say("mlp bf16", bf16, "B", B)
    dims = (320, 256, 16)
    rng = np.random.default_rng(11)
    ps = _params(rng, dims)
    ps32 = [p.astype(np.float32) for p in ps]
    X = rng.normal(size=(B, dims[0])).astype(np.float32)
    T = rng.normal(size=(B, dims[2])).astype(np.float32)
    net = L.MLP(*dims, bf16=bf16)
    net.set_params(ps32)
    Xd, Td = torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda")
    Y = net.forward(Xd).cpu().numpy()
    pref = [p.astype(np.float64) for p in ps32]
    Yref, _ = O.mlp_forward(pref, X.astype(np.float64))
    ef = rel(Y, Yref)
    loss = net.train_step(Xd, Td, 0.0)
    lref, gref = O.mlp_loss_and_grad(pref, X.astype(np.float64), T.astype(np.float64))
    _, g = net.get_params()
    eg = [rel(a, b) for a, b in zip(g, gref)]
    _say("forward rel err", ef, "loss", loss, lref, "grad rel errs", eg)
    assert ef < tol_f
    assert abs(loss - lref) < tol_f * abs(lref) + 1e-7
    assert max(eg) < tol_g


def test_mlp_adam_step_vs_oracle(L):
    import torch
    dims = (40, 32, 8)
    rng = np.random.default_rng(12)
    ps32 = [p.astype(np.float32) for p in _params(rng, dims)]
    X = rng.normal(size=(77, 40)).astype(np.float32)
    T = rng.normal(size=(77, 8)).astype(np.float32)
    net = L.MLP(*dims, bf16=False)
    net.set_params(ps32)
    Xd, Td = torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda")
    pref = [p.astype(np.float64) for p in ps32]
    m = [np.zeros_like(p) for p in pref]
    v = [np.zeros_like(p) for p in pref]
    for t in range(1, 4):
        net.train_step(Xd, Td, 1e-2)
        _, gref = O.mlp_loss_and_grad(pref, X.astype(np.float64), T.astype(np.float64))
        pref = O.adam_step(pref, gref, m, v, t, 1e-2)
    p, _ = net.get_params()
    assert max(rel(a, b) for a, b in zip(p, pref)) < 1e-5


def test_patch_features(L):
    import torch
    c = CS.c5_convdiff2d(n=5, p=3)
    m = L.Mesh(c.box, c.p)
    md = L.Model(m, c.kind, c.ncu, c.mu, aux=c.aux, src=c.src, bdata=c.bdata, bc_kind=c.bc_kind)
    rng = np.random.default_rng(3)
    r = rng.uniform(-1, 1, m.E * m.nn)
    e = rng.uniform(-1, 1, m.E * m.nn)
    elems = torch.as_tensor(np.array([0, 7, 12, 24], dtype=np.int32), device="cuda")
    X, Y, S = L.gather_patches(md, torch.as_tensor(r, device="cuda"), torch.as_tensor(e, device="cuda"), elems,
                               want_scale=True)
    X, Y, S = X.cpu().numpy(), Y.cpu().numpy(), S.cpu().numpy()
    nb = c.om.neighbours()
    nn = m.nn
    R = r.reshape(m.E, nn)
    for row, K in enumerate([0, 7, 12, 24]):
        patch = [K] + [int(x) for x in nb[K]]
        rp = np.concatenate([R[k] if k >= 0 else np.zeros(nn) for k in patch])
        s = np.linalg.norm(rp) + 1e-300
        assert abs(S[row] - s) < 1e-12 * s
        assert np.abs(X[row, :5 * nn] - rp / s).max() < 1e-6
        lk = np.concatenate([np.log(c.aux[k, 0]) if k >= 0 else np.zeros(nn) for k in patch])
        assert np.abs(X[row, 5 * nn:10 * nn] - lk).max() < 1e-5
        bxy = 0.01 * np.concatenate([np.concatenate([c.aux[k, 1], c.aux[k, 2]]) if k >= 0 else np.zeros(2 * nn)
                                     for k in patch])
        assert np.abs(X[row, 10 * nn:] - bxy).max() < 1e-4 * (1 + np.abs(bxy).max())
        assert np.abs(Y[row] - e.reshape(m.E, nn)[K] / s).max() < 1e-6


def _c5_solver(L, n=16):
    import torch
    c = CS.c5_convdiff2d(n=n, p=3, seed=5)
    m = L.Mesh(c.box, c.p)
    md = L.Model(m, c.kind, c.ncu, c.mu, aux=c.aux, src=c.src, bdata=c.bdata, bc_kind=c.bc_kind)
    zero = torch.zeros(md.N, dtype=torch.float64, device="cuda")
    b = -md.residual(zero)
    return c, m, md, b


def test_zero_network_reproduces_block_jacobi(L):
    import torch
    c, m, md, b = _c5_solver(L)
    bj = L.BlockJacobi(md)
    net = L.MLP(20 * m.nn, 256, m.nn, bf16=True)
    net.set_params([np.zeros(s, dtype=np.float32) for s in net.shapes])
    pc = L.LearnedPrecond(md, net, bj, composite=True)
    x1, s1, st1 = L.gmres(md, b, pc=bj, restart=30, rtol=1e-8, maxit=3000)
    x2, s2, st2 = L.gmres(md, b, pc=pc, restart=30, rtol=1e-8, maxit=3000)
    _say("bj", s1["iters"], "zero-net composite", s2["iters"], "fell back", s2["fell_back"])
    assert st1 == st2 == L.LDG_OK
    assert s1["iters"] == s2["iters"]
    assert (x1 - x2).abs().max().item() == 0.0


def test_nan_network_falls_back_to_block_jacobi(L):
    c, m, md, b = _c5_solver(L)
    bj = L.BlockJacobi(md)
    net = L.MLP(20 * m.nn, 256, m.nn, bf16=True)
    net.set_params([np.full(s, np.nan, dtype=np.float32) for s in net.shapes])
    pc = L.LearnedPrecond(md, net, bj, composite=True)
    x, s, st = L.gmres(md, b, pc=pc, restart=30, rtol=1e-8, maxit=3000)
    _say("nan net", s)
    assert st == L.LDG_OK and s["fell_back"] == 1
    r = b - md.jvp(None, x)
    assert L.norm(r) <= 1.01e-8 * s["res0"]
