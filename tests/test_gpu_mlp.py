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


@pytest.mark.parametrize("watch_window", [0, 10, -1])
def test_nan_network_falls_back_to_block_jacobi(L, watch_window):
    """A non-finite network output hands over to block-Jacobi whatever the stagnation window (-1: none)."""
    c, m, md, b = _c5_solver(L)
    bj = L.BlockJacobi(md)
    net = L.MLP(20 * m.nn, 256, m.nn, bf16=True)
    net.set_params([np.full(s, np.nan, dtype=np.float32) for s in net.shapes])
    pc = L.LearnedPrecond(md, net, bj, composite=True)
    x, s, st = L.gmres(md, b, pc=pc, restart=30, rtol=1e-8, maxit=3000, watch_window=watch_window)
    _say("nan net", s)
    assert st == L.LDG_OK and s["fell_back"] == 1
    r = b - md.jvp(None, x)
    assert L.norm(r) <= 1.01e-8 * s["res0"]


@pytest.mark.parametrize("orth", [0, 1, 2])
def test_gmres_records_its_own_pairs(L, orth):
    """ldg_gmres_opts.record_*: step i stores the preconditioner's input v_i and J z_i.  From x = 0 the first
    input is parallel to b (the delayed Gram-Schmidt variant normalizes later); with block-Jacobi every stored
    J z_i is the product of B^-1 v_i; steps past maxit and past record_max store nothing."""
    import torch
    c, m, md, b = _c5_solver(L)
    bj = L.BlockJacobi(md)
    k = 24
    V = torch.full((k + 4, md.N), 7.0, dtype=torch.float64, device="cuda")
    JZ = torch.full_like(V, 7.0)
    x, st, status = L.gmres(md, b, pc=bj, restart=10, rtol=0.0, maxit=k, check=False, orth=orth,
                            record=(V, JZ))
    assert st["iters"] == k
    v0 = b / L.norm(b)
    u0 = V[0] / L.norm(V[0].contiguous())
    assert (u0 - v0).abs().max().item() <= 1e-13 * v0.abs().max().item()
    for i in range(k):
        Jz = md.jvp(None, bj.apply(V[i].contiguous()))
        assert (JZ[i] - Jz).abs().max().item() <= 1e-12 * Jz.abs().max().item(), i
    assert (V[k:] == 7.0).all() and (JZ[k:] == 7.0).all()
    # a record shorter than the solve keeps its first steps only
    V2 = torch.zeros((5, md.N), dtype=torch.float64, device="cuda")
    JZ2 = torch.zeros_like(V2)
    L.gmres(md, b, pc=bj, restart=10, rtol=0.0, maxit=k, check=False, orth=orth, record=(V2, JZ2))
    assert (V2 - V[:5]).abs().max().item() <= 1e-13 * V[:5].abs().max().item()


def test_gmres_record_validation(L):
    import torch
    c, m, md, b = _c5_solver(L)
    Z = torch.zeros((4, md.N + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        L.gmres(md, b, restart=10, maxit=4, record=(Z, Z.clone()))
    Z = torch.zeros((4, md.N), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        L.gmres(md, b, restart=10, maxit=4, record=(Z, torch.zeros((3, md.N), dtype=torch.float64, device="cuda")))


@pytest.mark.parametrize("bf16,tol_g", [(False, 1e-4), (True, 8e-2)])
def test_bilinear_train_step_vs_oracle(L, bf16, tol_g):
    """ldg_mlp_train_step_bilinear (lr = 0): loss and every parameter gradient against the oracle's FP64
    chain rule through A_b r_b, on a batch that spans several GEMM tiles and a ragged tail."""
    import torch
    nn, B = 16, 1031
    dims = (15 * nn, 256, 5 * nn * nn)
    rng = np.random.default_rng(29)
    ps32 = [p.astype(np.float32) for p in _params(rng, dims)]
    X = rng.normal(size=(B, 20 * nn)).astype(np.float32)
    T = rng.normal(size=(B, nn)).astype(np.float32)
    net = L.MLP(*dims, bf16=bf16)
    net.set_params(ps32)
    loss = net.train_step_bilinear(torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda"), 0.0)
    pref = [p.astype(np.float64) for p in ps32]
    lref, gref = O.mlp_bilinear_loss_and_grad(pref, X.astype(np.float64), T.astype(np.float64), nn)
    _, g = net.get_params()
    eg = [rel(a, b) for a, b in zip(g, gref)]
    _say("bilinear bf16", bf16, "loss", loss, lref, "grad rel errs", eg)
    assert abs(loss - lref) < (1e-5 if not bf16 else 3e-2) * abs(lref)
    assert max(eg) < tol_g


def _coef_features(c, nb, nn):
    """[E][15 nn] coefficient features of every element's patch, built on the host from the model's aux."""
    E = c.aux.shape[0]
    out = np.zeros((E, 15 * nn))
    for K in range(E):
        patch = [K] + [int(x) for x in nb[K]]
        out[K, :5 * nn] = np.concatenate([np.log(c.aux[k, 0]) if k >= 0 else np.zeros(nn) for k in patch])
        out[K, 5 * nn:] = 0.01 * np.concatenate([np.concatenate([c.aux[k, 1], c.aux[k, 2]]) if k >= 0
                                                 else np.zeros(2 * nn) for k in patch])
    return out


@pytest.mark.parametrize("n", [5, 9])
def test_linear_form_preconditioner_vs_oracle(L, n):
    """ldg_precond_mlp, linear form (FP32 network): z = B^-1 (r + A_K patch(r)) against the oracle's blocks, the
    oracle's FP64 network on host-built coefficient features, and its linear_patch_precond."""
    import torch
    c = CS.c5_convdiff2d(n=n, p=3, seed=5)
    m = L.Mesh(c.box, c.p)
    md = L.Model(m, c.kind, c.ncu, c.mu, aux=c.aux, src=c.src, bdata=c.bdata, bc_kind=c.bc_kind)
    nn = m.nn
    dims = (15 * nn, 256, 5 * nn * nn)
    rng = np.random.default_rng(31)
    ps32 = [p.astype(np.float32) for p in _params(rng, dims)]
    ps32[4] *= 0.05                                   # a modest correction next to r
    net = L.MLP(*dims, bf16=False)
    net.set_params(ps32)
    bj = L.BlockJacobi(md)
    pc = L.LearnedPrecond(md, net, bj, composite="linear")
    r = rng.uniform(-1, 1, md.N)
    z = pc.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    nb = c.om.neighbours()
    Aref, _ = O.mlp_forward([p.astype(np.float64) for p in ps32], _coef_features(c, nb, nn))
    Binv = np.linalg.inv(c.om.blocks(c.oracle_model(), np.zeros(md.N)))
    zref = O.linear_patch_precond(Binv, Aref.reshape(m.E, nn, 5 * nn), nb, r)
    err = rel(z, zref)
    _say("linear form n", n, "rel err", err)
    assert err < 1e-5


def test_linear_form_rejects_wrong_sizes(L):
    c, m, md, b = _c5_solver(L)
    bj = L.BlockJacobi(md)
    net = L.MLP(20 * m.nn, 64, m.nn, bf16=True)      # the residual form's sizes
    with pytest.raises(L.LDGError):
        L.LearnedPrecond(md, net, bj, composite="linear")
    net2 = L.MLP(15 * m.nn, 64, 5 * m.nn * m.nn, bf16=True)
    with pytest.raises(L.LDGError):
        L.LearnedPrecond(md, net2, bj, composite=True)
    # a residual-form network (in_dim 20 nn = 320, not a multiple of 15) is refused by the bilinear step
    import torch
    nn_read = net.dims[0] // 15
    X = torch.zeros((8, 20 * nn_read), dtype=torch.float32, device="cuda")
    Y = torch.zeros((8, nn_read), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LDGError):
        net.train_step_bilinear(X, Y, 0.0)
