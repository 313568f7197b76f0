"""FP64 CPU reference of the heating-rate denoiser network (plain PyTorch
CPU ops in float64 with autograd).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the HIP BF16
MFMA kernels (forward values and every gradient).  It follows the same
architecture as the GPU driver but is written independently with library
primitives (conv3d, avg_pool3d, nearest upsampling, concatenation):

  e0 = relu(conv3 x0); e1 = relu(conv3 pool e0); e2 = relu(conv3 pool e1)
  b = relu(conv3 pool e2); d2 = relu(conv3 [up b, e2]); d1 = relu(conv3
  [up d2, e1]); d0 = relu(conv3 [up d1, e0]); out = conv1 d0;
  pred = out[:2] + base; loss = mean (pred - target)^2.

Weights use the kernels' layout [Cout][k^3][Cin] (taps z-major, then y,
then x) and activations [D][H][W][C]; conversion to PyTorch's
[Cout][Cin][kz][ky][kx] / [1][C][D][H][W] happens here.  Parity pin:
torch.autograd.gradcheck against finite differences on a tiny network.
"""
from __future__ import annotations

from typing import Dict

import torch
import torch.nn.functional as F

ORDER = ("e0", "e1", "e2", "b", "d2", "d1", "d0", "head")


def to_torch_weight(w: torch.Tensor, ksize: int) -> torch.Tensor:
    cout, taps, cin = w.shape
    return w.reshape(cout, ksize, ksize, ksize, cin).permute(0, 4, 1, 2, 3).contiguous()


def conv(x, w, b, ksize):
    return F.conv3d(x, to_torch_weight(w, ksize), b, padding=ksize // 2)


def up(x):
    return x.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3).repeat_interleave(2, dim=4)


def forward(params: Dict[str, torch.Tensor], biases: Dict[str, torch.Tensor], feat: torch.Tensor,
            base: torch.Tensor):
    """feat [D][H][W][Cin], base [D][H][W][2] -> pred [D][H][W][2] (float64)."""
    x0 = feat.permute(3, 0, 1, 2).unsqueeze(0)
    r = torch.relu
    e0 = r(conv(x0, params["e0"], biases["e0"], 3))
    e1 = r(conv(F.avg_pool3d(e0, 2), params["e1"], biases["e1"], 3))
    e2 = r(conv(F.avg_pool3d(e1, 2), params["e2"], biases["e2"], 3))
    bb = r(conv(F.avg_pool3d(e2, 2), params["b"], biases["b"], 3))
    d2 = r(conv(torch.cat([up(bb), e2], 1), params["d2"], biases["d2"], 3))
    d1 = r(conv(torch.cat([up(d2), e1], 1), params["d1"], biases["d1"], 3))
    d0 = r(conv(torch.cat([up(d1), e0], 1), params["d0"], biases["d0"], 3))
    out = conv(d0, params["head"], biases["head"], 1)
    out = out[0].permute(1, 2, 3, 0)
    return out[..., :2] + base


def loss_and_grads(params, biases, feat, base, target):
    """Loss and its gradients with respect to every weight and bias (float64)."""
    p = {k: v.detach().double().clone().requires_grad_(True) for k, v in params.items()}
    b = {k: v.detach().double().clone().requires_grad_(True) for k, v in biases.items()}
    pred = forward(p, b, feat.double(), base.double())
    loss = ((pred - target.double()) ** 2).mean()
    loss.backward()
    return loss.item(), {k: v.grad for k, v in p.items()}, {k: v.grad for k, v in b.items()}, pred.detach()
