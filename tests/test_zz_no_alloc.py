"""The allocation-free MLP forward (ldg_mlp_forward_noalloc) against ldg_mlp_forward (needs an MI355X).

Both entry points run the same GEMM kernels on the same weights and batch; the
allocation-free one keeps its hidden activations in the library's fixed device
array instead of the network's work buffers, so the outputs must be bitwise
equal.  Two calls in a row, the second with a smaller batch, check that the
array's leftover contents from the first call do not leak into the second.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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
    return [(rng.uniform(-1, 1, s) / np.sqrt(s[-1] if len(s) == 2 else s[0])).astype(np.float32) for s in shapes]


@pytest.mark.parametrize("bf16", [True, False])
def test_noalloc_forward_matches_forward(L, bf16):
    import torch
    dims = (320, 256, 16)
    net = L.MLP(*dims, bf16=bf16)
    net.set_params(_params(np.random.default_rng(7), dims))
    rng = np.random.default_rng(8)
    for B in (16384, 1037):     # the largest batch the fixed array holds at width 256, then a smaller one
        _say("noalloc forward bf16", bf16, "B", B)
        X = torch.as_tensor(rng.normal(size=(B, dims[0])).astype(np.float32), device="cuda")
        ref = net.forward(X)
        out = torch.full((B, dims[2]), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(X, out)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), float((out - ref).abs().max())


def test_noalloc_forward_rejects_oversized_batch(L):
    import torch
    dims = (320, 256, 16)
    net = L.MLP(*dims, bf16=True)
    B = 16385                   # 2 * B * width is one row pair beyond the fixed array
    X = torch.zeros((B, dims[0]), dtype=torch.float32, device="cuda")
    out = torch.zeros((B, dims[2]), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LDGError) as ei:
        net.forward_noalloc(X, out)
    assert ei.value.status == L.LDG_EINVAL
    assert "scratch" in str(ei.value)
