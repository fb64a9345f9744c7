"""The trace surrogate on the device (BF16 matrix-core GEMMs, FP32 accumulation) against the
CPU network oracle with the same parameters.

Tolerances follow from the arithmetic: both sides take the same BF16-rounded GEMM inputs in
the forward pass and sum in FP32 in different orders, so an intermediate value near a BF16
rounding boundary can round the other way (one BF16 step, 2^-8 relative); outputs and loss are
held to 2e-3 relative. The device also rounds the backward pass's GEMM inputs (the output
gradients) to BF16, which the oracle's autograd does not: gradients are held to 3e-2 relative
L2 per layer.
"""
import numpy as np
import pytest

from oracle.surrogate import SurrogateNet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1808_08645_amd.surrogate import Surrogate
    return Surrogate


def _inputs(B, nout, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (B, 16, 16, 16)).astype(np.float32)
    t = (0.5 * rng.standard_normal((B, nout))).astype(np.float32)
    return x, t


def test_layout_and_parameter_count(sur):
    print("[surrogate layout]", flush=True)
    s = sur(25600, 8, seed=3)
    L = s.layout()
    assert [l["cout"] for l in L] == [16, 32, 64, 256, 256, 64, 25600]
    assert 1.9e6 < s.num_params < 2.0e6
    p = s.get_params()
    assert np.all(p[L[0]["woff"] + 27 * 16:L[0]["woff"] + 32 * 16] == 0)  # padded rows
    assert np.all(p[L[6]["boff"]:] == 0)


@pytest.mark.parametrize("B,nout", [(1, 40), (5, 1000), (32, 25600)])
def test_forward_loss_and_gradient_match_oracle(sur, B, nout):
    import torch
    print(f"[surrogate parity] B={B} nout={nout}", flush=True)
    s = sur(nout, 32, seed=11)
    x, t = _inputs(B, nout, 12)
    p = s.get_params()
    net = SurrogateNet(s.layout(), nout)
    Jo, go, yo = net.loss_grad(p, x, t)
    y = s.forward(x).cpu().numpy()
    assert np.linalg.norm(y - yo) <= 2e-3 * np.linalg.norm(yo)
    J, g = s.loss_grad(x, t)
    assert abs(J - Jo) <= 2e-3 * Jo, (J, Jo)
    for l in s.layout():
        for a, b in ((l["woff"], l["boff"]), (l["boff"], l["boff"] + l["cout"])):
            d, r = g[a:b], go[a:b]
            assert np.linalg.norm(d - r) <= 3e-2 * np.linalg.norm(r) + 1e-12, (l, np.linalg.norm(d - r) / np.linalg.norm(r))
    torch.cuda.synchronize()


@pytest.mark.parametrize("B,nout", [(1, 40), (6, 2000)])
def test_input_gradient_matches_oracle(sur, B, nout):
    """dL/dx (the network as a differentiable stand-in for the solver) against the oracle's
    autograd; the device rounds the backward GEMM inputs to BF16, hence 3e-2 relative L2."""
    print(f"[surrogate input gradient] B={B} nout={nout}", flush=True)
    s = sur(nout, 8, seed=21)
    x, t = _inputs(B, nout, 22)
    net = SurrogateNet(s.layout(), nout)
    Jo, dxo = net.input_grad(s.get_params(), x, t)
    J, dx = s.input_grad(x, t)
    dx = dx.cpu().numpy()
    assert abs(J - Jo) <= 2e-3 * Jo, (J, Jo)
    assert dx.shape == dxo.shape
    assert np.linalg.norm(dx - dxo) <= 3e-2 * np.linalg.norm(dxo), np.linalg.norm(dx - dxo) / np.linalg.norm(dxo)


def test_set_params_roundtrip_and_training_reduces_the_loss(sur):
    print("[surrogate training]", flush=True)
    s = sur(300, 16, seed=5)
    p = s.get_params()
    s.set_params(p)
    assert np.array_equal(s.get_params(), p)
    x, t = _inputs(16, 300, 6)
    first = s.train_step(x, t, 1e-3)
    for _ in range(200):
        last = s.train_step(x, t, 1e-3)
    assert last < 0.05 * first, (first, last)
    assert not np.array_equal(s.get_params(), p)


def test_surrogate_error_paths(sur):
    import paper_1808_08645_amd as bb
    print("[surrogate errors]", flush=True)
    with pytest.raises(bb.BBWADGError):
        sur(100, 8, grid=8)
    with pytest.raises(bb.BBWADGError):
        sur(0, 8)
    s = sur(100, 4)
    x, t = _inputs(5, 100, 1)
    with pytest.raises(bb.BBWADGError):
        s.forward(x)  # batch above max_batch
    with pytest.raises(bb.BBWADGError):
        s.train_step(x[:2], t[:2], -1.0)
    bad = s.get_params()
    bad[7] = np.nan
    with pytest.raises(bb.BBWADGError):
        s.set_params(bad)
