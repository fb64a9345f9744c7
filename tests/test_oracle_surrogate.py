"""Pins of the surrogate network oracle (``oracle/surrogate.py``): the convolution layout
against a brute-force loop of its definition, the BF16 rounding against its definition (round
to nearest, ties to even), and the autograd gradient against float64 central differences."""
import numpy as np
import torch

from oracle.surrogate import SurrogateNet, bf16_round


def _layout(nout):
    """The documented parameter layout, built independently of the library."""
    L, off = [], 0
    for cin, cout in ((1, 16), (16, 32), (32, 64)):
        K = 27 * cin
        Kp = (K + 15) // 16 * 16
        L.append({"conv": True, "cin": cin, "cout": cout, "K": K, "Kp": Kp, "relu": True, "woff": off,
                  "boff": off + Kp * cout})
        off += Kp * cout + cout
    for i, (k, n) in enumerate(((512, 256), (256, 256), (256, 64), (64, nout))):
        L.append({"conv": False, "cin": k, "cout": n, "K": k, "Kp": k, "relu": i < 3, "woff": off, "boff": off + k * n})
        off += k * n + n
    return L, off


def test_bf16_rounding_is_nearest_even():
    x = torch.tensor([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5 + 2 ** -7 * 0.5, 3.0e38])
    want = []
    for v in x.tolist():
        # bf16 keeps 8 significant bits: round the significand to a multiple of 2^(e-7)
        e = np.floor(np.log2(abs(v)))
        q = 2.0 ** (e - 7)
        r = v / q
        lo = np.floor(r)
        frac = r - lo
        rr = lo + (1 if frac > 0.5 or (frac == 0.5 and lo % 2 == 1) else 0)
        want.append(rr * q)
    assert np.array_equal(bf16_round(x).numpy(), np.array(want, dtype=np.float32))


def test_convolution_layer_matches_its_definition():
    """Output voxel o, channel n = b_n + sum_{k,c} W[((kz*3+ky)*3+kx)*Cin + c][n] in(2o + k - 1, c)."""
    L, npar = _layout(8)
    rng = np.random.default_rng(1)
    p = rng.standard_normal(npar).astype(np.float32)
    net = SurrogateNet(L[:1], 8)
    x = rng.standard_normal((2, 16, 16, 16)).astype(np.float32)
    with torch.no_grad():
        y = net.forward(torch.tensor(p), torch.tensor(x), rounding=False)  # [2, 16, 8, 8, 8] after relu
    W = p[L[0]["woff"]:L[0]["woff"] + 32 * 16].reshape(32, 16)
    b = p[L[0]["boff"]:L[0]["boff"] + 16]
    for (bb, oz, oy, ox, n) in [(0, 0, 0, 0, 3), (1, 7, 2, 5, 15), (0, 3, 7, 7, 0), (1, 4, 4, 1, 9)]:
        s = b[n]
        for kz in range(3):
            for ky in range(3):
                for kx in range(3):
                    z, yy, xx = 2 * oz + kz - 1, 2 * oy + ky - 1, 2 * ox + kx - 1
                    if 0 <= z < 16 and 0 <= yy < 16 and 0 <= xx < 16:
                        s += W[(kz * 3 + ky) * 3 + kx, n] * x[bb, z, yy, xx]
        assert abs(float(y[bb, n, oz, oy, ox]) - max(s, 0.0)) < 1e-4


def test_gradient_matches_central_differences():
    """Without rounding, in float64: autograd against central differences on 14 parameters."""
    L, npar = _layout(5)
    rng = np.random.default_rng(2)
    p = (0.1 * rng.standard_normal(npar))
    x = rng.uniform(-1, 1, (2, 16, 16, 16))
    t = rng.standard_normal((2, 5))
    net = SurrogateNet(L, 5)
    J, g, _ = net.loss_grad(p, x, t, rounding=False, dtype=torch.float64)
    # in every layer, the weight and the bias with the largest gradient (all nonzero)
    nz = []
    for l in L:
        nz.append(l["woff"] + int(np.argmax(np.abs(g[l["woff"]:l["boff"]]))))
        nz.append(l["boff"] + int(np.argmax(np.abs(g[l["boff"]:l["boff"] + l["cout"]]))))
    assert all(abs(g[i]) > 1e-4 for i in nz)
    for i in nz:
        pp, pm = p.copy(), p.copy()
        pp[i] += 1e-6
        pm[i] -= 1e-6
        jp = net.loss_grad(pp, x, t, rounding=False, dtype=torch.float64)[0]
        jm = net.loss_grad(pm, x, t, rounding=False, dtype=torch.float64)[0]
        fd = (jp - jm) / 2e-6
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_input_gradient_matches_central_differences():
    """Without rounding, in float64: dL/dx by autograd against central differences at the
    input voxels with the largest gradient in each of two samples (and a few at random)."""
    L, npar = _layout(6)
    rng = np.random.default_rng(4)
    p = 0.1 * rng.standard_normal(npar)
    x = rng.uniform(-1, 1, (2, 16, 16, 16))
    t = rng.standard_normal((2, 6))
    net = SurrogateNet(L, 6)
    J, dx = net.input_grad(p, x, t, rounding=False, dtype=torch.float64)
    J2, _, _ = net.loss_grad(p, x, t, rounding=False, dtype=torch.float64)
    assert J == J2
    flat = dx.reshape(-1)
    picks = [int(np.argmax(np.abs(flat[:4096]))), 4096 + int(np.argmax(np.abs(flat[4096:])))]
    picks += [int(i) for i in rng.choice(8192, 4, replace=False)]
    for i in picks:
        xp, xm = x.copy().reshape(-1), x.copy().reshape(-1)
        xp[i] += 1e-6
        xm[i] -= 1e-6
        jp = net.loss_grad(p, xp.reshape(x.shape), t, rounding=False, dtype=torch.float64)[0]
        jm = net.loss_grad(p, xm.reshape(x.shape), t, rounding=False, dtype=torch.float64)[0]
        fd = (jp - jm) / 2e-6
        assert abs(fd - flat[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, flat[i])
    assert abs(flat[picks[0]]) > 1e-4
