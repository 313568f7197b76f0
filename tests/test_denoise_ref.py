"""Pins of the FP64 denoiser reference (CPU): autograd gradients against
finite differences, and the tap / layout convention of the weights against
a direct sum."""
import torch

from oracle import denoise_ref as dr


def tiny_params(base=2, cin=3, seed=0):
    g = torch.Generator().manual_seed(seed)
    c0, c1, c2, c3 = base, 2 * base, 3 * base, 4 * base
    shapes = {"e0": (c0, 27, cin), "e1": (c1, 27, c0), "e2": (c2, 27, c1), "b": (c3, 27, c2),
              "d2": (c2, 27, c3 + c2), "d1": (c1, 27, c2 + c1), "d0": (c0, 27, c1 + c0), "head": (2, 1, c0)}
    p = {k: torch.randn(*s, generator=g, dtype=torch.float64) * 0.4 for k, s in shapes.items()}
    b = {k: torch.randn(s[0], generator=g, dtype=torch.float64) * 0.1 for k, s in shapes.items()}
    return p, b


def test_conv_tap_convention():
    """Weight tap t = (kz*3 + ky)*3 + kx multiplies input (z+kz-1, y+ky-1, x+kx-1)."""
    g = torch.Generator().manual_seed(1)
    D, H, W, cin, cout = 3, 4, 5, 2, 3
    x = torch.randn(D, H, W, cin, generator=g, dtype=torch.float64)
    w = torch.randn(cout, 27, cin, generator=g, dtype=torch.float64)
    y = dr.conv(x.permute(3, 0, 1, 2).unsqueeze(0), w, None, 3)[0].permute(1, 2, 3, 0)
    ref = torch.zeros(D, H, W, cout, dtype=torch.float64)
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                for t in range(27):
                    kz, ky, kx = t // 9, (t // 3) % 3, t % 3
                    zs, ys, xs = z + kz - 1, yy + ky - 1, xx + kx - 1
                    if 0 <= zs < D and 0 <= ys < H and 0 <= xs < W:
                        ref[z, yy, xx] += w[:, t, :] @ x[zs, ys, xs]
    assert torch.allclose(y, ref, atol=1e-12)


def test_reference_gradients_match_finite_differences():
    p, b = tiny_params()
    g = torch.Generator().manual_seed(2)
    feat = torch.randn(8, 8, 8, 3, generator=g, dtype=torch.float64)
    base = torch.randn(8, 8, 8, 2, generator=g, dtype=torch.float64)
    target = torch.randn(8, 8, 8, 2, generator=g, dtype=torch.float64)
    names = list(p)

    def f(*tensors):
        pp = dict(zip(names, tensors[:len(names)]))
        bb = dict(zip(names, tensors[len(names):]))
        pred = dr.forward(pp, bb, feat, base)
        return ((pred - target) ** 2).mean()

    inputs = tuple(v.clone().requires_grad_(True) for v in list(p.values()) + list(b.values()))
    assert torch.autograd.gradcheck(f, inputs, eps=1e-6, atol=1e-6, rtol=1e-4)
    loss, gw, gb, _ = dr.loss_and_grads(p, b, feat, base, target)
    assert loss > 0 and all(v is not None for v in gw.values())
