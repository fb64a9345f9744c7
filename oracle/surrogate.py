"""The trace surrogate's network in plain PyTorch on the CPU (test infrastructure only).

Three 3x3x3 convolutions (stride 2, padding 1, ReLU) 1 -> 16 -> 32 -> 64 channels on a 16^3
grid, then dense layers 512 -> 256 -> 256 -> 64 (ReLU) -> nout, mean squared error loss; the
parameters are read from the library's flat vector with its documented layout (W[Kp][N]
row-major, convolution row ((kz*3 + ky)*3 + kx)*Cin + c, then the bias). The inputs of every
product (the input grid, the weights and each layer's output) are rounded to BF16 as the
library's matrix-core GEMMs take them; the products and sums are FP32. Gradients come from
torch autograd on this definition (without rounding the backward pass); the gradient with
respect to the input takes the input's BF16 rounding as the identity, as the library does.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def bf16_round(x: torch.Tensor) -> torch.Tensor:
    """Round FP32 to the nearest BF16 value (ties to even), returned as FP32."""
    return x.to(torch.bfloat16).to(torch.float32)


class SurrogateNet:
    def __init__(self, layout, nout: int):
        self.layout = layout
        self.nout = nout

    def weights(self, p: torch.Tensor):
        """Per layer (W, b): convolution W [Cout, Cin, 3, 3, 3], dense W [N, K]."""
        out = []
        for L in self.layout:
            N = L["cout"]
            W = p[L["woff"]:L["woff"] + L["Kp"] * N].reshape(L["Kp"], N)[:L["K"]]
            b = p[L["boff"]:L["boff"] + N]
            if L["conv"]:
                W = W.reshape(3, 3, 3, L["cin"], N).permute(4, 3, 0, 1, 2)  # [Cout, Cin, kz, ky, kx]
            else:
                W = W.t()
            out.append((W, b))
        return out

    def forward(self, p: torch.Tensor, x: torch.Tensor, rounding: bool = True):
        """x [B, 16, 16, 16] (z, y, x) -> [B, nout]."""
        rnd = bf16_round if rounding else (lambda t: t)
        h = rnd(x)[:, None]
        for (W, b), L in zip(self.weights(p), self.layout):
            W = rnd(W)
            if L["conv"]:
                h = F.conv3d(h, W, b, stride=2, padding=1)
            else:
                if h.dim() == 5:  # [B, C, z, y, x] -> the library's [B][voxel][C] order
                    h = h.permute(0, 2, 3, 4, 1).reshape(h.shape[0], -1)
                h = h @ W.t() + b
            if L["relu"]:
                h = torch.relu(h)
            if L is not self.layout[-1]:
                h = rnd(h)
        return h

    def loss_grad(self, p_np, x_np, t_np, rounding: bool = True, dtype=torch.float32):
        p = torch.tensor(np.asarray(p_np), dtype=dtype, requires_grad=True)
        x = torch.tensor(np.asarray(x_np), dtype=dtype)
        t = torch.tensor(np.asarray(t_np), dtype=dtype)
        y = self.forward(p, x, rounding)
        loss = torch.mean((y - t) ** 2)
        loss.backward()
        return float(loss.detach()), p.grad.detach().numpy(), y.detach().numpy()

    def input_grad(self, p_np, x_np, t_np, rounding: bool = True, dtype=torch.float32):
        """(loss, dL/dx) of the mean squared error by autograd."""
        p = torch.tensor(np.asarray(p_np), dtype=dtype)
        x = torch.tensor(np.asarray(x_np), dtype=dtype, requires_grad=True)
        t = torch.tensor(np.asarray(t_np), dtype=dtype)
        y = self.forward(p, x, rounding)
        loss = torch.mean((y - t) ** 2)
        loss.backward()
        return float(loss.detach()), x.grad.detach().numpy()
