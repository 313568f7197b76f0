"""BF16 MFMA denoiser kernels against the FP64 CPU reference.

Convolution forward, data gradient (flipped kernel) and weight gradient are
compared on BF16-representable inputs, where the only differences are FP32
accumulation order (tight tolerance); the whole network (forward, every
gradient) is compared with a tolerance that allows for BF16 storage of the
activations between layers."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import torch.nn.functional as F  # noqa: E402

from oracle import denoise_ref as dr  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dn():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_2208_05247_amd import denoise
    denoise.load()
    return denoise


def bf(x):
    """Round a float tensor to BF16 and back (CPU float64)."""
    return x.to(torch.bfloat16).double()


def rel(a, b):
    return float((a - b).norm() / max(b.norm(), 1e-30))


@pytest.mark.parametrize("shape", [(3, 5, 37, 16, 32, 64, 3), (4, 4, 64, 32, 0, 32, 3), (2, 3, 20, 32, 0, 32, 1),
                                   (3, 18, 40, 32, 16, 32, 3), (5, 17, 33, 32, 0, 32, 3), (5, 11, 35, 32, 0, 64, 3)])
def test_conv_forward_and_gradients(dn, shape):
    D, H, W, c1, c2, cout, k = shape
    g = torch.Generator().manual_seed(7)
    cin = c1 + c2
    x = bf(torch.randn(D, H, W, cin, generator=g, dtype=torch.float64))
    w = bf(torch.randn(cout, k ** 3, cin, generator=g, dtype=torch.float64) * 0.2)
    b = torch.randn(cout, generator=g, dtype=torch.float64) * 0.1
    dev = lambda t, dt=torch.bfloat16: t.to(dt).cuda().contiguous()
    x1 = dev(x[..., :c1])
    x2 = dev(x[..., c1:]) if c2 else None
    yf = torch.empty(D, H, W, cout, dtype=torch.float32, device="cuda")
    y = torch.empty(D, H, W, cout, dtype=torch.bfloat16, device="cuda")
    dn.conv_fwd(x1, x2, dev(w), dev(b, torch.float32), True, cout, k, y1=y, yf=yf)
    xt = x.permute(3, 0, 1, 2).unsqueeze(0)
    ref = torch.relu(dr.conv(xt, w, b.float().double(), k))[0].permute(1, 2, 3, 0)
    assert rel(yf.double().cpu(), ref) < 1e-5
    assert torch.allclose(y.double().cpu(), bf(yf.double().cpu()))
    # data gradient = conv of dz with the flipped kernel; weight gradient
    dz = bf(torch.randn(D, H, W, cout, generator=g, dtype=torch.float64))
    xr = xt.clone().requires_grad_(True)
    wr = w.clone().requires_grad_(True)
    out = dr.conv(xr, wr, None, k)
    out.backward(dz.permute(3, 0, 1, 2).unsqueeze(0))
    gx = xr.grad[0].permute(1, 2, 3, 0)
    wt = torch.empty(cin, k ** 3, cout, dtype=torch.bfloat16, device="cuda")
    dn.flip(dev(w), cout, cin, k, wt)
    if cin % 32 == 0:
        dxf = torch.empty(D, H, W, cin, dtype=torch.float32, device="cuda")
        dn.conv_fwd(dev(dz), None, wt, None, False, cin, k, yf=dxf)
        assert rel(dxf.double().cpu(), gx) < 1e-5
    dw = torch.zeros(cout, k ** 3, cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    dn.conv_wgrad(x1, x2, dev(dz), cout, k, dw, db)
    assert rel(dw.double().cpu(), wr.grad) < 1e-5
    assert rel(db.double().cpu(), dz.sum(dim=(0, 1, 2))) < 1e-5
    # workspace variant: same result within rounding, bitwise reproducible
    ws = torch.empty(dn.wgrad_workspace_size(x1, x2, cout, k), dtype=torch.uint8, device="cuda")
    runs = []
    for _ in range(2):
        dw2 = torch.zeros_like(dw)
        db2 = torch.zeros_like(db)
        dn.conv_wgrad(x1, x2, dev(dz), cout, k, dw2, db2, workspace=ws)
        runs.append((dw2, db2))
    assert rel(runs[0][0].double().cpu(), wr.grad) < 1e-5
    assert rel(runs[0][1].double().cpu(), dz.sum(dim=(0, 1, 2))) < 1e-5
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])


def test_pool_and_upsample(dn):
    g = torch.Generator().manual_seed(3)
    x = bf(torch.randn(4, 6, 8, 16, generator=g, dtype=torch.float64))
    xd = x.to(torch.bfloat16).cuda()
    p = dn.pool2(xd).double().cpu()
    ref = F.avg_pool3d(x.permute(3, 0, 1, 2).unsqueeze(0), 2)[0].permute(1, 2, 3, 0)
    assert torch.allclose(p, bf(ref), atol=1e-2, rtol=1e-2)
    # exactly: FP32 sum of the 8 inputs in z, y, x order, times 1/8, rounded to BF16
    xf = x.float()
    s = torch.zeros(2, 3, 4, 16)
    for q in range(8):
        s = s + xf[(q >> 2)::2, ((q >> 1) & 1)::2, (q & 1)::2]
    assert torch.equal(p, (0.125 * s).to(torch.bfloat16).double())
    for c in (8, 24, 40):  # other multiples of 8 channels
        xc = torch.randn(2, 4, 6, c, generator=g).to(torch.bfloat16)
        sc = torch.zeros(1, 2, 3, c)
        for q in range(8):
            sc = sc + xc.float()[(q >> 2)::2, ((q >> 1) & 1)::2, (q & 1)::2]
        assert torch.equal(dn.pool2(xc.cuda()).cpu(), (0.125 * sc).to(torch.bfloat16))
    u = dn.up2(xd).double().cpu()
    assert torch.equal(u, dr.up(x.permute(3, 0, 1, 2).unsqueeze(0))[0].permute(1, 2, 3, 0))
    gu = dn.up2(dn.up2(xd), backward=True, out=torch.empty_like(xd)).double().cpu()
    assert torch.allclose(gu, bf(8 * x), rtol=1e-2)
    gp = dn.pool2(dn.pool2(xd), backward=True, out=torch.empty_like(xd)).double().cpu()
    assert torch.allclose(gp, bf(dr.up(ref.permute(3, 0, 1, 2).unsqueeze(0))[0].permute(1, 2, 3, 0) / 8),
                          atol=1e-2, rtol=2e-2)


def test_network_gradients_match_fp64_reference(dn):
    """One forward + backward of the full 4-level network (32 base channels)
    on a 16x16x16 field: loss, prediction and every weight / bias gradient
    against the FP64 autograd reference run with the same BF16 weights and
    inputs."""
    torch.manual_seed(0)
    net = dn.Denoiser(base=32, seed=3)
    # give the head real weights so every layer receives gradient
    g = torch.Generator().manual_seed(5)
    net.p["head"].copy_((torch.randn(net.p["head"].shape, generator=g) * 0.1).cuda())
    net.p["head"][2:] = 0
    net.pb["head"].copy_(net.p["head"].to(torch.bfloat16))
    for k in net.bias:
        net.bias[k].copy_((torch.randn(net.bias[k].shape, generator=g) * 0.05).cuda())
    D = H = W = 16
    hdir = torch.rand(D, H, W, generator=g).cuda() * 2
    hdif = torch.rand(D, H, W, generator=g).cuda()
    kext = torch.rand(D, H, W, generator=g).cuda() * 0.05
    feat, base = dn.features(hdir, hdif, kext, 0.1 * kext, 20.0, 1.0)
    target = (base + 0.3 * torch.randn(base.shape, generator=g).cuda()).contiguous()
    out = net.forward(feat, keep=True)
    pred, dout, loss = dn.mse(out, base, target, want_grad=True)
    net.backward(dout)
    params = {k: net.pb[k].double().cpu() for k in net.p}
    params["e0"] = params["e0"][:, :, :16]
    biases = {k: net.bias[k].double().cpu() for k in net.bias}
    rloss, gw, gb, rpred = dr.loss_and_grads(params, biases, feat.double().cpu(), base.double().cpu(),
                                             target.double().cpu())
    # measured on the MI355X: loss 3.0e-4 relative, predictions 1.2e-3, weight
    # gradients <= 1.7 % relative with cosine >= 0.99986, bias gradients
    # <= 1.5 % (e2 is the worst): the difference is the
    # BF16 storage of activations and gradients between layers
    say("loss gpu", loss.item(), "ref", rloss)
    assert abs(loss.item() - rloss) <= 1e-3 * rloss
    pe = rel(pred.double().cpu(), rpred)
    say("prediction rel err", round(pe, 6))
    assert pe < 5e-3
    for k in dr.ORDER:
        e = rel(net.g[k].double().cpu(), gw[k])
        cos = float((net.g[k].double().cpu() * gw[k]).sum() / (net.g[k].double().cpu().norm() * gw[k].norm()))
        eb = rel(net.gbias[k].double().cpu(), gb[k])
        say("grad", k, "rel err", round(e, 5), "cos", round(cos, 6), "bias rel err", round(eb, 5))
        assert e < 3e-2 and cos > 0.9995, k
        assert eb < 3e-2, (k, "bias", eb)


def test_training_reduces_loss(dn):
    """A few Adam steps on one denoising pair lower the loss."""
    g = torch.Generator().manual_seed(11)
    D = H = W = 32
    clean = torch.rand(D, H, W, generator=g) ** 4
    noisy_dir = (clean * (1 + 0.5 * torch.randn(D, H, W, generator=g))).clamp_min(0).cuda()
    noisy_dif = (clean * (1 + 0.5 * torch.randn(D, H, W, generator=g))).clamp_min(0).cuda()
    kext = clean.cuda() * 0.02
    net = dn.Denoiser(base=32, seed=1)
    s = dn.field_scale(noisy_dir, noisy_dif)
    feat, base = dn.features(noisy_dir, noisy_dif, kext, 0.1 * kext, 20.0, s)
    target = torch.stack([clean / s, clean / s], dim=-1).float().cuda().contiguous()
    losses = [dn.train_step(net, feat, base, target, 1e-3).item() for _ in range(30)]
    say("losses", losses[0], losses[-1])
    assert losses[-1] < 0.7 * losses[0]
    d1, d2 = dn.denoise(net, noisy_dir, noisy_dif, kext, 0.1 * kext, 20.0)
    assert d1.shape == noisy_dir.shape and torch.isfinite(d1).all() and (d1 >= 0).all()


def test_denoiser_gains_over_plain_tracing(dn):
    """Trained briefly on tracer-generated pairs (24 random cumulus scenes,
    64x64x64 cells of 25x25x20 m, 112 g-points), the network lowers the
    heating-rate RMS error of a held-out scene at equal photon counts; plain
    high-photon tracing (two independent halves) is the reference."""
    from paper_2208_05247_amd import experiment as ex
    net = dn.Denoiser(base=32, seed=0)
    losses, _ = ex.train(net, 24, 4, 64, 64, 25.0, 20.0, high=4096)
    assert np.mean(losses[-8:]) < np.mean(losses[:8])
    wl = ex.scene(123_456, 64, 64, 64, 25.0, 20.0, sza=50.0, az=30.0)
    tr = ex.Tracer(wl)
    a_dir, a_dif, _, _ = tr.heating(4096, seed=1)
    b_dir, b_dif, _, _ = tr.heating(4096, seed=2)
    ref_a, ref_b = a_dir + a_dif, b_dir + b_dif
    kext, kabs = tr.k_mean()
    for n in (256, 1024):
        hd, hf, _, _ = tr.heating(n, seed=10 + n)
        raw = ex.eps_against(hd + hf, ref_a, ref_b)
        od, of = dn.denoise(net, hd, hf, kext, kabs, 20.0)
        den = ex.eps_against(od + of, ref_a, ref_b)
        say("N", n, "eps raw", raw, "denoised", den)
        assert den < 0.7 * raw


@pytest.mark.parametrize("shape", [(4, 6, 10, 32, 16, 32), (2, 4, 18, 64, 32, 64), (3, 3, 5, 16, 0, 96)])
def test_fused_upsampling_equals_materialised(dn, shape):
    """A convolution that reads its first input nearest-upsampled on the fly
    equals the same convolution on the materialised 2x-upsampled input, bit
    for bit (same products, same order); partial tiles and a concatenated
    second input included."""
    d, h, w, c1, c2, cout = shape
    g = torch.Generator().manual_seed(17)
    x1 = torch.randn(d, h, w, c1, generator=g).to(torch.bfloat16).cuda()
    x2 = torch.randn(2 * d, 2 * h, 2 * w, c2, generator=g).to(torch.bfloat16).cuda() if c2 else None
    wt = (torch.randn(cout, 27, c1 + c2, generator=g) * 0.1).to(torch.bfloat16).cuda()
    bias = torch.randn(cout, generator=g).cuda()
    up = dn.up2(x1)
    ref = torch.empty(2 * d, 2 * h, 2 * w, cout, dtype=torch.float32, device="cuda")
    got = torch.empty_like(ref)
    dn.conv_fwd(up, x2, wt, bias, True, cout, 3, yf=ref)
    dn.conv_fwd(x1, x2, wt, bias, True, cout, 3, yf=got, up1=True)
    assert torch.equal(got, ref)


@pytest.mark.parametrize("shape", [(3, 18, 40, 32, 16, False, 2), (2, 9, 17, 32, 32, True, 2), (5, 16, 32, 16, 0, False, 32)])
def test_fused_head_equals_separate_layers(dn, shape):
    """The last 3x3x3 convolution (32 outputs, ReLU) and the 1x1x1 head in one
    launch equal the two launches with the BF16 activation stored in
    between, bit for bit; ragged tiles, odd depth, on-the-fly upsampling and
    every head channel included."""
    d, h, w, c1, c2, up, hcols = shape
    D, H, W = (2 * d, 2 * h, 2 * w) if up else (d, h, w)
    g = torch.Generator().manual_seed(29)
    x1 = torch.randn(d, h, w, c1, generator=g).to(torch.bfloat16).cuda()
    x2 = torch.randn(D, H, W, c2, generator=g).to(torch.bfloat16).cuda() if c2 else None
    wt = (torch.randn(32, 27, c1 + c2, generator=g) * 0.1).to(torch.bfloat16).cuda()
    bias = torch.randn(32, generator=g).cuda()
    hw = (torch.randn(32, 1, 32, generator=g) * 0.2).to(torch.bfloat16).cuda()
    hb = torch.randn(32, generator=g).cuda()
    act = torch.empty(D, H, W, 32, dtype=torch.bfloat16, device="cuda")
    dn.conv_fwd(x1, x2, wt, bias, True, 32, 3, y1=act, up1=up)
    ref = torch.empty(D, H, W, hcols, dtype=torch.float32, device="cuda")
    dn.conv_fwd(act, None, hw, hb, False, 32, 1, yf=ref, yf_cols=hcols)
    got = torch.full((D, H, W, hcols), float("nan"), dtype=torch.float32, device="cuda")
    dn.conv_fwd_head(x1, x2, wt, bias, True, hw, hb, got, up1=up)
    assert torch.equal(got, ref)


def test_inference_forward_equals_training_forward(dn):
    net = dn.Denoiser(base=32, seed=4)
    g = torch.Generator().manual_seed(2)
    feat = torch.randn(16, 16, 24, 16, generator=g).to(torch.bfloat16).cuda()
    a = net.forward(feat, keep=True)
    b = net.forward(feat, keep=False)
    assert b.shape[-1] == dn.NOUT
    assert torch.equal(a[..., :dn.NOUT].contiguous(), b)


def test_training_is_bitwise_reproducible(dn):
    """Two networks from the same seed trained on the same pairs end with
    bitwise-identical weights (every sum in the backward pass runs in a
    fixed order)."""
    g = torch.Generator().manual_seed(21)
    D = H = W = 16
    clean = torch.rand(D, H, W, generator=g) ** 4
    noisy = (clean * (1 + 0.5 * torch.randn(D, H, W, generator=g))).clamp_min(0).cuda()
    kext = clean.cuda() * 0.02
    s = dn.field_scale(noisy, noisy)
    feat, base = dn.features(noisy, noisy, kext, 0.1 * kext, 20.0, s)
    target = torch.stack([clean / s, clean / s], dim=-1).float().cuda().contiguous()
    nets = [dn.Denoiser(base=32, seed=5) for _ in range(2)]
    for net in nets:
        for _ in range(5):
            dn.train_step(net, feat, base, target, 1e-3)
    for k in nets[0].p:
        assert torch.equal(nets[0].p[k], nets[1].p[k]), k
        assert torch.equal(nets[0].bias[k], nets[1].bias[k]), k


def test_direct_feature_closed_form_and_translation(dn):
    """Direct-beam feature: in horizontally uniform layers it is the closed
    form (1 - f_d) exp(-tau_above / mu0) (1 - exp(-k dz / mu0)) k_a / k scale
    (tau_above: extinction of the levels above times dz); on the periodic
    grid, shifting the fields shifts the feature."""
    import math
    from paper_2208_05247_amd.synthetic import Grid
    nx, ny, nz, dz = 24, 20, 9, 20.0
    grid = Grid(nx, ny, nz, 25.0, 25.0, dz)
    g = torch.Generator().manual_seed(31)
    kz = torch.rand(nz, generator=g, dtype=torch.float64) * 0.02
    kz[4] = 0.0  # a level without extinction
    az = kz * torch.rand(nz, generator=g, dtype=torch.float64)
    ke = kz[:, None, None].expand(nz, ny, nx).float().contiguous().cuda()
    ka = az[:, None, None].expand(nz, ny, nx).float().contiguous().cuda()
    ls = (torch.rand(nz, generator=g, dtype=torch.float64) + 0.5).cuda()
    sza, fd = 50.0, 0.8
    out = dn.direct_feature(ke, ka, grid, sza, 33.0, fd, ls).double().cpu()
    mu0 = math.cos(math.radians(sza))
    ke64, ka64 = ke[:, 0, 0].double().cpu(), ka[:, 0, 0].double().cpu()
    for k in range(nz):
        above = float(ke64[k + 1:].sum()) * dz
        frac = (1 - math.exp(-float(ke64[k]) * dz / mu0)) * float(ka64[k] / ke64[k]) if ke64[k] > 0 else 0.0
        ref = fd * math.exp(-above / mu0) * frac * float(ls[k])
        assert torch.allclose(out[k], torch.full_like(out[k], ref), rtol=2e-5, atol=1e-12), k
    # a 3D field: translation equivariance on the periodic grid
    ke3 = (torch.rand(nz, ny, nx, generator=g) * 0.05).cuda()
    ka3 = ke3 * 0.01
    f = dn.direct_feature(ke3, ka3, grid, sza, 200.0, fd, ls)
    fs = dn.direct_feature(torch.roll(ke3, (3, 5), (1, 2)).contiguous(), torch.roll(ka3, (3, 5), (1, 2)).contiguous(),
                           grid, sza, 200.0, fd, ls)
    # equal up to the rounding of the interpolation weights (i + offset - floor)
    assert torch.allclose(torch.roll(f, (3, 5), (1, 2)), fs, rtol=1e-5, atol=0.0)
    assert (f > 0).all()


def test_field_scale_and_fused_output(dn):
    """rt3d_dn_field_scale against the FP64 means (and reproducible to the
    bit); rt3d_dn_residual_unfeature bitwise equal to features' base, the
    residual head (rt3d_dn_mse) and rt3d_dn_unfeature in turn."""
    g = torch.Generator().manual_seed(23)
    for shape in ((3, 5, 7), (16, 64, 96)):
        hd = (torch.rand(shape, generator=g) * 3.0).cuda()
        hf = (torch.rand(shape, generator=g) * 0.5).cuda()
        s = dn.field_scale(hd, hf)
        ref = (hd.double().mean().item() + hf.double().mean().item()) / 2.0
        assert abs(s - ref) <= 1e-12 * ref
        assert dn.field_scale(hd, hf) == s
        assert dn.field_scale(torch.zeros_like(hd), torch.zeros_like(hf)) == 1.0
        ke = torch.rand(shape, generator=g).cuda() * 0.01
        out = torch.randn(*shape, 4, generator=g).cuda()
        feat, base = dn.features(hd, hf, ke, 0.1 * ke, 20.0, s, cpad=4)
        pred, _, _ = dn.mse(out, base, None, want_grad=False)
        od_ref, of_ref = torch.empty_like(hd), torch.empty_like(hf)
        dn._check(dn.load().rt3d_dn_unfeature(dn._p(pred), float(s), hd.numel(), dn._p(od_ref), dn._p(of_ref),
                                              dn._s()), "unfeature")
        od, of = torch.empty_like(hd), torch.empty_like(hf)
        dn._check(dn.load().rt3d_dn_residual_unfeature(dn._p(out), 4, dn._p(hd), dn._p(hf), float(s), hd.numel(),
                                                       dn._p(od), dn._p(of), dn._s()), "residual_unfeature")
        assert torch.equal(od.view(torch.int32), od_ref.view(torch.int32))
        assert torch.equal(of.view(torch.int32), of_ref.view(torch.int32))
        assert (od_ref == 0).any() and (od_ref > 0).any()  # both sides of the clamp


def test_first_layer_with_pooling_is_bitwise(dn):
    """rt3d_dn_conv3d_fwd_pool: the packed first layer and its 2x2x2 pooling
    in one launch equal the two separate launches bit for bit, partial tiles
    in y and x included; shapes it does not take are refused."""
    g = torch.Generator().manual_seed(17)
    for D, H, W in ((4, 20, 36), (2, 16, 32), (6, 34, 66)):
        x = torch.randn(D, H, W, 4, generator=g).to(torch.bfloat16).cuda()
        w = (torch.randn(32, 27, 4, generator=g) * 0.2).to(torch.bfloat16).cuda()
        b = (torch.randn(32, generator=g) * 0.1).cuda()
        for relu in (True, False):
            y_ref = torch.empty(D, H, W, 32, dtype=torch.bfloat16, device="cuda")
            dn.conv_fwd(x, None, w, b, relu, 32, 3, y1=y_ref)
            p_ref = dn.pool2(y_ref)
            y = torch.full((D, H, W, 32), 7.0, dtype=torch.bfloat16, device="cuda")
            p = torch.full((D // 2, H // 2, W // 2, 32), 7.0, dtype=torch.bfloat16, device="cuda")
            dn.conv_fwd_pool(x, w, b, relu, y, p)
            assert torch.equal(y.view(torch.int16), y_ref.view(torch.int16)), (D, H, W, relu)
            assert torch.equal(p.view(torch.int16), p_ref.view(torch.int16)), (D, H, W, relu)
    x = torch.zeros(3, 16, 32, 4, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(Exception):
        dn.conv_fwd_pool(x, w, b, True, torch.empty(3, 16, 32, 32, dtype=torch.bfloat16, device="cuda"),
                         torch.empty(1, 8, 16, 32, dtype=torch.bfloat16, device="cuda"))


def test_packed_five_channel_first_layer(dn):
    """The packed first layer of the network with the direct-beam input (5
    inputs in 8 channels, 15 products per MFMA K-chunk) and its pooling
    against the unpacked 16-channel first layer and rt3d_dn_pool2 (equal up
    to the order of the products: within BF16 rounding), partial tiles
    included; the whole inference forward likewise."""
    g = torch.Generator().manual_seed(41)
    for D, H, W in ((4, 20, 36), (2, 16, 32)):
        x16 = torch.zeros(D, H, W, 16, dtype=torch.float64)
        x16[..., :5] = torch.randn(D, H, W, 5, generator=g, dtype=torch.float64)
        x16 = x16.to(torch.bfloat16).cuda()
        x8 = x16[..., :8].contiguous()
        w = (torch.randn(32, 27, 16, generator=g) * 0.2)
        w[:, :, 5:] = 0.0
        w = w.to(torch.bfloat16).cuda()
        b = (torch.randn(32, generator=g) * 0.1).cuda()
        y_ref = torch.empty(D, H, W, 32, dtype=torch.bfloat16, device="cuda")
        yf = torch.empty(D, H, W, 32, dtype=torch.float32, device="cuda")
        dn.conv_fwd(x16, None, w, b, True, 32, 3, y1=y_ref, yf=yf)
        p_ref = dn.pool2(y_ref)
        y = torch.empty_like(y_ref)
        p = torch.empty_like(p_ref)
        dn.conv_fwd_pool(x8, w, b, True, y, p)
        assert (y.float() - yf).abs().max().item() <= 8e-3 * yf.abs().max().item()
        assert (p.float() - p_ref.float()).abs().max().item() <= 8e-3 * p_ref.float().abs().max().item()
    net = dn.Denoiser(base=32, seed=7, n_in=5)
    hd = torch.rand(16, 16, 24, generator=g).cuda()
    hf = torch.rand(16, 16, 24, generator=g).cuda()
    ke = torch.rand(16, 16, 24, generator=g).cuda() * 0.02
    dirf = torch.rand(16, 16, 24, generator=g).cuda()
    f16, _ = dn.features(hd, hf, ke, 0.1 * ke, 20.0, 1.0, direct=dirf)
    f8, _ = dn.features(hd, hf, ke, 0.1 * ke, 20.0, 1.0, cpad=8, direct=dirf)
    assert torch.equal(f16[..., :8].contiguous(), f8) and f8[..., 4].abs().sum() > 0
    a = net.forward(f16)
    b8 = net.forward(f8)
    assert rel(b8.double().cpu(), a.double().cpu()) < 2e-2


def test_packed_first_layer(dn):
    """The first layer with 4 input channels (three x-taps per MFMA K-chunk)
    against the FP64 convolution, partial tiles included, and the inference
    forward from 4-channel features against the 16-channel one (same
    products, other summation order in the first layer)."""
    g = torch.Generator().manual_seed(9)
    for D, H, W in ((3, 20, 37), (2, 16, 32)):
        x = bf(torch.randn(D, H, W, 4, generator=g, dtype=torch.float64))
        w = bf(torch.randn(32, 27, 4, generator=g, dtype=torch.float64) * 0.2)
        b = torch.randn(32, generator=g, dtype=torch.float64) * 0.1
        yf = torch.empty(D, H, W, 32, dtype=torch.float32, device="cuda")
        y = torch.empty(D, H, W, 32, dtype=torch.bfloat16, device="cuda")
        dn.conv_fwd(x.to(torch.bfloat16).cuda(), None, w.to(torch.bfloat16).cuda(), b.float().cuda(), True, 32, 3,
                    y1=y, yf=yf)
        ref = torch.relu(dr.conv(x.permute(3, 0, 1, 2).unsqueeze(0), w, b.float().double(), 3))[0].permute(1, 2, 3, 0)
        assert rel(yf.double().cpu(), ref) < 1e-5
        assert torch.allclose(y.double().cpu(), bf(yf.double().cpu()))
    net = dn.Denoiser(base=32, seed=6)
    hd = torch.rand(16, 16, 24, generator=g).cuda()
    hf = torch.rand(16, 16, 24, generator=g).cuda()
    ke = torch.rand(16, 16, 24, generator=g).cuda() * 0.02
    f16, base = dn.features(hd, hf, ke, 0.1 * ke, 20.0, 1.0)
    f4, base4 = dn.features(hd, hf, ke, 0.1 * ke, 20.0, 1.0, cpad=4)
    assert torch.equal(f16[..., :4].contiguous(), f4) and torch.equal(base, base4)
    a = net.forward(f16)
    b4 = net.forward(f4)
    assert rel(b4.double().cpu(), a.double().cpu()) < 2e-2
