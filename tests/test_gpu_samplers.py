"""The tracer's own scattering samplers and direction turn on the GPU
(through rt3d_phase_sample / rt3d_turn, the device functions the tracing
kernel calls), against the FP64 oracle's samplers at the same uniforms and
against the moments the phase functions fix: Henyey-Greenstein Legendre
moments <P_l(mu)> = g^l, Rayleigh <mu> = 0 and <mu^2> = 2/5 (sec. 2.3,
phase-function paragraph).  Uniforms are stratified midpoints, so the
moments are quadratures with negligible error."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

pytestmark = pytest.mark.gpu
N = 1 << 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rt3d():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_2208_05247_amd import rt3d as lib
    lib.load()
    return lib


def strata():
    return ((np.arange(N) + 0.5) / N).astype(np.float32)


@pytest.mark.parametrize("g", [-1.0, -0.999, -0.9, -0.3, -0.05, -1e-4, 0.0, 1e-7, 1e-5, 1e-3, 0.0999, 0.1, 0.5,
                               0.85, 0.86, 0.99, 0.999, 1.0])
def test_hg_sampler(rt3d, g):
    xi = strata()
    dxi = torch.from_numpy(xi).cuda()
    gg = torch.full_like(dxi, np.float32(g))
    mu = rt3d.phase_sample("hg", dxi, gg).cpu().numpy().astype(np.float64)
    gf = float(np.float32(g))
    assert np.all(np.abs(mu) <= 1.0) and np.all(np.isfinite(mu))
    assert abs(mu.mean() - gf) < 1e-5, (mu.mean(), gf)
    assert abs((1.5 * mu * mu - 0.5).mean() - gf * gf) < 1e-5
    if abs(g) <= 0.99:
        # FP32 arithmetic error; it grows as 1 - |g| shrinks (backscatter
        # end of a strongly peaked phase function)
        ref = oracle.hg_cos(gf, xi.astype(np.float64))
        err = np.abs(mu - ref).max()
        assert err < (5e-6 if abs(g) <= 0.9 else 2e-5), err
        # monotone in xi (an inverse distribution function)
        assert np.all(np.diff(mu) >= -1e-6)


def test_hg_sampler_edges(rt3d):
    """xi = 0 and the largest uniform below 1 at the extremes of g."""
    xi = torch.tensor([0.0, 1.0 - 2.0 ** -24] * 4, dtype=torch.float32, device="cuda")
    g = torch.tensor([1.0, 1.0, -1.0, -1.0, 0.999, 0.999, 0.0, 0.0], dtype=torch.float32, device="cuda")
    mu = rt3d.phase_sample("hg", xi, g).cpu().numpy()
    assert mu[0] == 1.0 and mu[1] == 1.0 and mu[2] == -1.0 and mu[3] == -1.0
    assert mu[4] == pytest.approx(-1.0, abs=1e-3) and mu[5] == pytest.approx(1.0, abs=1e-6)
    assert mu[6] == -1.0 and mu[7] == pytest.approx(1.0, abs=1e-6)


def test_rayleigh_sampler(rt3d):
    xi = strata()
    mu = rt3d.phase_sample("rayleigh", torch.from_numpy(xi).cuda()).cpu().numpy().astype(np.float64)
    ref = oracle.rayleigh_cos(xi.astype(np.float64))
    assert np.abs(mu - ref).max() < 2e-6
    assert abs(mu.mean()) < 1e-6
    assert abs((mu * mu).mean() - 0.4) < 1e-6
    # the distribution: P(mu <= x) = (4 + 3x + x^3)/8 at the sample points
    x = np.linspace(-0.95, 0.95, 39)
    cdf = np.searchsorted(np.sort(mu), x) / N
    assert np.abs(cdf - (4 + 3 * x + x ** 3) / 8).max() < 2e-6


def test_turn(rt3d):
    """Unit length, d . d' = mu, and for uniform azimuths the mean turned
    direction is mu d (the azimuth is uniform about d), including exactly
    vertical directions (the kernel's fixed frame) and directions a few
    1e-3 to 1e-7 off vertical."""
    rng = np.random.default_rng(4)
    n = 1 << 16
    d = rng.standard_normal((n, 3))
    d[:16] = [0.0, 0.0, 1.0]
    d[16:32] = [0.0, 0.0, -1.0]
    d[32:48] = [1e-4, 0.0, -1.0]
    d[48:64] = [3e-3, 1e-3, -1.0]
    d[64:80] = [1e-7, 0.0, 1.0]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mu = rng.uniform(-1.0, 1.0, n)
    t = rng.uniform(0.0, 1.0, n)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    out = rt3d.turn(f(d), f(mu), f(t)).cpu().numpy().astype(np.float64)
    d32 = d.astype(np.float32).astype(np.float64)
    mu32 = mu.astype(np.float32).astype(np.float64)
    assert np.abs(np.linalg.norm(out, axis=1) - 1.0).max() < 2e-6
    assert np.abs((out * d32).sum(axis=1) - mu32).max() < 2e-5
    # azimuthal average for a few fixed (d, mu)
    m = 4096
    for dv, mv in (([0.3, -0.4, -0.866], 0.7), ([0.0, 0.0, 1.0], -0.2), ([0.6, 0.8, 0.0], 0.1),
                   ([0.0, 0.0, -1.0], 0.95)):
        dv = np.asarray(dv) / np.linalg.norm(dv)
        tt = (np.arange(m) + 0.5) / m
        o = rt3d.turn(f(np.tile(dv, (m, 1))), f(np.full(m, mv)), f(tt)).cpu().numpy().astype(np.float64)
        assert np.abs(o.mean(axis=0) - mv * dv).max() < 1e-5, (dv, mv, o.mean(axis=0))
