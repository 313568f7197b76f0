"""Pins of the FP64 two-stream column oracle (clear-sky TOD flux and diffuse
fraction, sec. 2.3 initialisation paragraph).

The oracle solves the two-point boundary-value problem by exact
matrix-exponential propagation through every (sub-)layer and one banded
linear system.  It is checked against a different algorithm for the same
equations (closed-form layer reflection/transmission combined with the
adding method, tests/two_stream_adding.py), closed forms for a pure
absorber, exact conservation for conservative scattering, the
single-scattering backscatter of a thin layer by quadrature of the phase
function, and exact Monte Carlo transport within the approximation's known
accuracy.  A dropped term, a wrong sign or a swapped coefficient fails one
of them."""
import numpy as np
import pytest

import two_stream_adding as adding
from oracle import two_stream as ts


def random_column(rng, n, tau_max=0.5):
    tau = rng.uniform(0.01, tau_max, n)
    ssa = rng.uniform(0.0, 1.0, n)
    g = rng.uniform(-0.5, 0.9, n)
    return tau, ssa, g


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mu0", [0.15, 0.5, 0.95])
@pytest.mark.parametrize("albedo", [0.0, 0.25, 1.0])
def test_matches_the_adding_method(seed, mu0, albedo):
    rng = np.random.default_rng(seed)
    tau, ssa, g = random_column(rng, 12, tau_max=0.5 if seed < 3 else 4.0)
    S, D, U = ts.column(tau, ssa, g, mu0, albedo, flux_toa=1361.0)
    S2, D2, U2 = adding.column(tau, ssa, g, mu0, albedo, flux_toa=1361.0)
    for a, b in ((S, S2), (D, D2), (U, U2)):
        assert np.allclose(a, b, rtol=1e-9, atol=1e-9 * 1361.0)


def test_conservative_and_rayleigh_layers_match_the_adding_method():
    """w = 1 (k = 0) and g = 0 gas layers, as in a clear sky."""
    tau = np.array([0.02, 0.05, 0.1, 0.3, 0.6])
    ssa = np.array([1.0, 1.0, 0.99, 1.0, 0.8])
    g = np.zeros(5)
    for mu0 in (0.3, 0.8):
        got = ts.column(tau, ssa, g, mu0, 0.2)
        ref = adding.column(tau, ssa, g, mu0, 0.2)
        for a, b in zip(got, ref):
            assert np.allclose(a, b, rtol=1e-9, atol=1e-12)


def test_thick_absorbing_layers_stay_accurate():
    """Optically thick absorbing layers (k tau up to 100) are cut into
    sub-layers; the result matches the adding method, whose closed forms
    are stable there."""
    tau = np.array([0.5, 50.0, 3.0, 20.0])
    ssa = np.array([0.3, 0.0, 0.9, 0.5])
    g = np.array([0.0, 0.0, 0.7, 0.2])
    for mu0 in (0.2, 0.9):
        got = ts.column(tau, ssa, g, mu0, 0.4)
        ref = adding.column(tau, ssa, g, mu0, 0.4)
        for a, b in zip(got, ref):
            assert np.allclose(a, b, rtol=1e-9, atol=1e-13)


def test_resonant_layer():
    """k mu0 = 1, where closed-form particular solutions are singular: the
    oracle needs no special case there; the adding method's mean of the two
    sides of the resonance (mu0 shifted by 1e-5 either way) is good to 1e-9."""
    ssa, g = 0.5, 0.0
    g1, g2, _, _ = ts.gammas(ssa, g, 0.5)
    k = float(np.sqrt((g1 - g2) * (g1 + g2)))
    for mu0 in (1.0 / k, 1.0 / k * (1 + 3e-4), 1.0 / k * (1 + 6e-6), 1.0 / k * (1 - 1e-7)):
        tau = np.array([0.3, 0.7])
        got = ts.column(tau, [ssa, ssa], [g, g], mu0, 0.3)
        ref = adding.column(tau, [ssa, ssa], [g, g], mu0, 0.3)
        for a, b in zip(got, ref):
            assert np.allclose(a, b, rtol=1e-9, atol=1e-12)
    # continuity across the resonance in the oracle itself
    m0 = 1.0 / k
    vals = [ts.column([0.3, 0.7], [ssa, ssa], [g, g], m0 * (1 + e), 0.3)[2][0] for e in (-1e-6, 0.0, 1e-6)]
    assert abs(vals[1] - 0.5 * (vals[0] + vals[2])) < 1e-10


def test_splitting_a_layer_changes_nothing():
    """The adding of two halves of a homogeneous layer reproduces the layer."""
    for ssa, g, tau in ((0.9, 0.7, 2.0), (1.0, 0.0, 5.0), (0.3, -0.2, 0.4), (0.999, 0.86, 20.0)):
        one = ts.column([tau], [ssa], [g], 0.6, 0.2)
        many = ts.column([tau / 8] * 8, [ssa] * 8, [g] * 8, 0.6, 0.2)
        for a, b in zip(one, many):
            assert np.allclose(a[[0, -1]], b[[0, -1]], rtol=1e-10, atol=1e-13)


def test_pure_absorber():
    """w = 0: the beam follows Beer-Lambert, no diffuse light goes down, the
    surface reflection leaves with the PIFM diffuse transmittance exp(-2 tau)
    per layer."""
    tau = np.array([0.1, 0.4, 1.3])
    mu0, alb = 0.4, 0.35
    S, D, U = ts.column(tau, np.zeros(3), np.zeros(3), mu0, alb)
    cum = np.concatenate([[0.0], np.cumsum(tau)])
    assert np.allclose(S, mu0 * np.exp(-cum / mu0), rtol=1e-14)
    assert np.all(D == 0.0)
    up_sfc = alb * S[-1]
    assert np.allclose(U, up_sfc * np.exp(-2.0 * (cum[-1] - cum)), rtol=1e-13)


def test_energy_conservation():
    """Conservative scattering over a black surface: reflected + everything
    reaching the surface = incoming; over a white surface all of it leaves
    the TOA.  With absorption: TOA net flux = column + surface absorption."""
    rng = np.random.default_rng(9)
    tau = rng.uniform(0.05, 2.0, 8)
    g = rng.uniform(0.0, 0.9, 8)
    for mu0 in (0.2, 0.7):
        S, D, U = ts.column(tau, np.ones(8), g, mu0, 0.0)
        assert U[0] + S[-1] + D[-1] == pytest.approx(mu0, rel=1e-12)
        S, D, U = ts.column(tau, np.ones(8), g, mu0, 1.0)
        assert U[0] == pytest.approx(mu0, rel=1e-10)
        ssa = rng.uniform(0.5, 1.0, 8)
        S, D, U = ts.column(tau, ssa, g, mu0, 0.3)
        net = S + D - U
        assert np.all(np.diff(net) <= 1e-14)  # absorbing layers only remove flux
        assert net[-1] == pytest.approx(0.7 * (S[-1] + D[-1]), rel=1e-12)


def test_top_of_domain_fraction():
    """Diffuse fraction at a level: zero above any scatterer, grows with the
    scattering optical depth above the level, and lies in [0, 1]."""
    tau = np.full(20, 0.05)
    ssa = np.ones(20)
    g = np.zeros(20)
    fr = [ts.top_of_domain(tau, ssa, g, 0.5, 0.2, lev)[1] for lev in range(0, 21, 4)]
    assert fr[0] == 0.0
    assert all(b > a for a, b in zip(fr, fr[1:]))
    assert all(0.0 <= f <= 1.0 for f in fr)


@pytest.mark.parametrize("g", [-0.4, 0.0, 0.5, 0.85])
@pytest.mark.parametrize("mu0", [0.1, 0.45, 0.9])
def test_thin_layer_backscatter_of_the_direct_beam(g, mu0):
    """For tau -> 0 a layer reflects w tau/mu0 times the fraction of singly
    scattered sunlight that goes up.  PIFM's gamma3 is that fraction for the
    phase function truncated after its first Legendre term, 1 + 3 g cos(Theta);
    here it is integrated over the sphere by quadrature (Gauss-Legendre in the
    scattered direction's vertical cosine, uniform in azimuth)."""
    x, wq = np.polynomial.legendre.leggauss(32)
    mu = 0.5 * (x + 1.0)          # upward hemisphere, mu in (0, 1)
    wm = 0.5 * wq
    phi = (np.arange(64) + 0.5) * (2 * np.pi / 64)
    s0 = np.sqrt(1 - mu0 * mu0)
    M, F = np.meshgrid(mu, phi, indexing="ij")
    cos_t = np.sqrt(1 - M * M) * np.cos(F) * s0 + M * (-mu0)  # incident (s0, 0, -mu0)
    p = 1.0 + 3.0 * g * cos_t
    up = float((p * wm[:, None]).sum() * (2 * np.pi / 64) / (4 * np.pi))
    tau, ssa = 1e-6, 0.8
    S, D, U = ts.column([tau], [ssa], [g], mu0, 0.0)
    rdir = U[0] / S[0]    # upward diffuse flux per unit direct flux, black surface
    assert rdir * mu0 / (ssa * tau) == pytest.approx(up, rel=1e-5)


def test_two_stream_is_close_to_exact_transport():
    """Gross-error check of the whole approximation against the Monte Carlo
    oracle (exact transport) in a plane-parallel slab (one periodic column)
    over a black surface: isotropic and moderately forward-scattering cloud
    layers, a thick g = 0.85 cloud and Rayleigh gas.  The direct beam is
    exact in both; PIFM's reflectance and diffuse transmittance are within
    6 % in these regimes (a wrong coefficient, e.g. mu0 dropped from gamma3
    or gamma3 and gamma4 swapped, is off by far more).  Not used: a
    moderately thick strongly forward-scattering layer (g = 0.85, tau = 2),
    where two-stream without delta scaling underestimates the reflectance
    by about a quarter."""
    import oracle
    from paper_2208_05247_amd import synthetic as syn
    grid = syn.Grid(1, 1, 10, 100.0, 100.0, 10.0)
    cases = ((1.0, 0.9, 0.0, True, 0.8), (2.0, 0.95, 0.5, True, 0.8), (10.0, 0.999, 0.85, True, 0.6),
             (0.3, 1.0, 0.0, False, 0.5), (0.1, 1.0, 0.0, False, 0.3))
    for tau, ssa, g, cloud, mu0 in cases:
        k = tau / 100.0
        f = syn.uniform_fields(grid, k, k if cloud else 0.0, ssa, g if cloud else 0.0, albedo=0.0)
        n = 1 << 18
        sza = float(np.degrees(np.arccos(mu0)))
        r = oracle.trace(f, sza, 0.0, n, 7, brick=(1, 1, 10))
        w = float(n) * 2 ** 31
        refl = float(r["toa_up"].sum()) / w
        t_dir = float(r["sfc_dir"].sum()) / w
        t_dif = float(r["sfc_dif"].sum()) / w
        S, D, U = ts.column([tau], [ssa], [g], mu0, 0.0)
        p = S[-1] / mu0
        assert t_dir == pytest.approx(p, abs=4 * np.sqrt(p * (1 - p) / n) + 1.0 / n)
        assert U[0] / mu0 == pytest.approx(refl, rel=0.06), (tau, ssa, g)
        assert D[-1] / mu0 == pytest.approx(t_dif, rel=0.06), (tau, ssa, g)
