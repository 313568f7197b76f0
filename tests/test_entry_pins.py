"""Pins of the scrambled-Sobol entry points of the oracle (sec. 2.3,
initialisation paragraph).

* dimension 1 is the base-2 radical inverse, recomputed here digit by digit
  with integer division;
* dimension 2 is the Sobol dimension of the polynomial x + 1, whose
  generator matrix is Pascal's triangle mod 2: digit r of the point is the
  parity of sum_c binom(c, r) i_c over the bits i_c of the index (Lucas'
  theorem: binom(c, r) is odd iff r & c == r);
* both, before and after scrambling, form (0, m, 2)-nets: every elementary
  box of area 2^-m holds exactly one of 2^m consecutive aligned points;
* the scramble is nested (points sharing their first d digits keep sharing
  them and keep differing at digit d when they did) and uniform over seeds;
* scrambled-Sobol estimates of a smooth integral converge far faster than
  independent points, and the traced entry positions keep every tally's
  expectation."""
import numpy as np
import pytest
from scipy import stats

import oracle


def radical_inverse_2(i: int) -> int:
    out, scale = 0, 1 << 31
    while i:
        i, digit = divmod(i, 2)
        out += digit * scale
        scale >>= 1
    return out


def pascal_mod2_point(i: int) -> int:
    out = 0
    for r in range(32):          # output digit r (0 = the 2^-1 place)
        parity = 0
        for c in range(32):      # index bit c (0 = lowest)
            if (i >> c) & 1 and (r & c) == r:
                parity ^= 1
        out |= parity << (31 - r)
    return out


def test_first_dimension_is_the_radical_inverse():
    idx = list(range(64)) + [2 ** 20 + 12345, 2 ** 31 + 7, 2 ** 32 - 1]
    a, _ = oracle.sobol_points(idx)
    assert [int(x) for x in a] == [radical_inverse_2(i) for i in idx]


def test_second_dimension_is_the_pascal_matrix_mod_2():
    rng = np.random.default_rng(1)
    idx = list(range(64)) + [int(x) for x in rng.integers(0, 2 ** 32, 200, dtype=np.uint64)]
    _, b = oracle.sobol_points(idx)
    assert [int(x) for x in b] == [pascal_mod2_point(i) for i in idx]
    # first points by hand: 0, 1/2, 3/4, 1/4, 5/8
    assert [int(x) / 2 ** 32 for x in b[:5]] == [0.0, 0.5, 0.75, 0.25, 0.625]


def is_net(x: np.ndarray, y: np.ndarray, m: int) -> bool:
    for a in range(m + 1):
        b = m - a
        cell = (x.astype(np.uint64) >> np.uint64(32 - a)) * np.uint64(1 << b) + \
            (y.astype(np.uint64) >> np.uint64(32 - b)) if a and b else \
            (x.astype(np.uint64) >> np.uint64(32 - a)) if a else (y.astype(np.uint64) >> np.uint64(32 - b))
        if np.bincount(cell.astype(np.int64), minlength=1 << m).max() != 1:
            return False
    return True


@pytest.mark.parametrize("m", [1, 4, 7, 10])
@pytest.mark.parametrize("block", [0, 3])
def test_nets_before_and_after_scrambling(m, block):
    idx = np.arange(block << m, (block + 1) << m, dtype=np.uint32)
    x, y = oracle.sobol_points(idx)
    assert is_net(x, y, m)
    for seed in (1, 0xdeadbeef):
        assert is_net(oracle.owen_scramble(x, seed), oracle.owen_scramble(y, seed ^ 0x5bd1e995), m)
    xy = oracle.sobol_entry(block << m, 1 << m, 77, 12345)
    assert is_net(xy[:, 0], xy[:, 1], m)
    # a non-net as a control: independent random points
    rng = np.random.default_rng(m)
    r = rng.integers(0, 2 ** 32, (2, 1 << m), dtype=np.uint64).astype(np.uint32)
    assert m < 2 or not is_net(r[0], r[1], m)


def test_scramble_is_nested():
    rng = np.random.default_rng(2)
    v = rng.integers(0, 2 ** 32, 4000, dtype=np.uint64).astype(np.uint32)
    w = rng.integers(0, 2 ** 32, 4000, dtype=np.uint64).astype(np.uint32)
    d = rng.integers(0, 32, 4000)
    # w shares the first d digits of v
    mask = np.array([(0xffffffff << (32 - k)) & 0xffffffff if k else 0 for k in d], dtype=np.uint64)
    w = ((v.astype(np.uint64) & mask) | (w.astype(np.uint64) & ~mask & 0xffffffff)).astype(np.uint32)
    for seed in (3, 99):
        a = oracle.owen_scramble(v, seed).astype(np.uint64)
        b = oracle.owen_scramble(w, seed).astype(np.uint64)
        assert np.all((a & mask) == (b & mask))
        bit = np.array([1 << (31 - k) for k in d], dtype=np.uint64)
        assert np.all(((a ^ b) & bit) == ((v.astype(np.uint64) ^ w.astype(np.uint64)) & bit))


def test_scramble_is_uniform_over_seeds():
    for v in (0, 0x80000000, 0x12345678):
        out = np.array([oracle.owen_scramble([v], s)[0] for s in range(4096)], dtype=np.uint64)
        counts = np.bincount((out >> np.uint64(28)).astype(np.int64), minlength=16)
        assert stats.chisquare(counts).pvalue > 1e-4
        # the second digit is independent of the first
        pair = ((out >> np.uint64(30)) & np.uint64(3)).astype(np.int64)
        assert stats.chisquare(np.bincount(pair, minlength=4)).pvalue > 1e-4


def test_scrambled_sobol_beats_independent_points_on_a_smooth_integral():
    """f(x, y) = exp(x) sin(pi y)^2 on the unit square: exact integral
    (e - 1) / 2.  With 1024 points the scrambled-Sobol RMSE over 64 columns
    (independent scrambles) is far below the N^-1/2 error of random points,
    and the estimate is unbiased."""
    f = lambda x, y: np.exp(x) * np.sin(np.pi * y) ** 2
    exact = (np.e - 1.0) / 2.0
    est = []
    for col in range(64):
        xy = (oracle.sobol_entry(0, 1024, col, 2024).astype(np.float64) + 0.5) / 2 ** 32
        est.append(f(xy[:, 0], xy[:, 1]).mean())
    est = np.array(est)
    rng = np.random.default_rng(5)
    mc = np.array([f(*rng.random((2, 1024))).mean() for _ in range(64)])
    rmse_q = np.sqrt(np.mean((est - exact) ** 2))
    rmse_mc = np.sqrt(np.mean((mc - exact) ** 2))
    assert rmse_q < 0.02 * rmse_mc
    assert abs(est.mean() - exact) < 5 * est.std(ddof=1) / 8 + 1e-12


def test_sobol_entry_keeps_beer_lambert_and_the_ledger():
    """Entry positions change where photons start inside their column, not
    the physics: clear-sky direct transmittance and the exact ledger hold."""
    from paper_2208_05247_amd import synthetic as syn
    grid = syn.Grid(8, 8, 16, 50.0, 50.0, 25.0)
    f = syn.uniform_fields(grid, 4e-4, 0.0, 0.0, 0.0, albedo=0.0)
    n = 1 << 16
    r = oracle.trace(f, 30.0, 20.0, n, 3, brick=(4, 4, 4), sobol_entry=True)
    t = float(r["sfc_dir"].sum()) / (n * 2.0 ** 31)
    p = np.exp(-4e-4 * 400.0 / np.cos(np.radians(30.0)))
    assert abs(t - p) < 4 * np.sqrt(p * (1 - p) / n)
    led = dict(zip(oracle.LEDGER, (int(x) for x in r["ledger"])))
    assert led["incoming"] + led["rr_gain"] == (led["toa"] + led["atm_dir"] + led["atm_dif"] + led["sfc"]
                                                + led["rr_loss"] + led["lost"])


def test_sobol_entry_lowers_column_noise_of_direct_irradiance():
    """Vacuum under a slanted sun: a photon lands 3.4 columns away from
    where it entered, so a surface column collects the parts of four entry
    columns its shifted outline covers, and its direct irradiance is the
    share of entry points in those parts.  With independent points that
    share is binomial (noise ~ N^-1/2); a scrambled (0, m, 2)-net miscounts
    such a rectangle by a few points (noise ~ N^-1): at 1024 photons per
    column the per-column noise is below a tenth of the independent points',
    and it falls more than 10x from 64 to 1024 photons per column.  Mean 1
    in every case (nothing is absorbed)."""
    from paper_2208_05247_amd import synthetic as syn
    grid = syn.Grid(16, 16, 4, 100.0, 100.0, 100.0)
    f = syn.uniform_fields(grid, 0.0, 0.0, 0.0, 0.0, albedo=0.0)
    sd = {}
    for per in (64, 1024):
        for sob in (False, True):
            vals = []
            for s in range(8):
                r = oracle.trace(f, 40.0, 35.0, 256 * per, 100 + s, brick=(4, 4, 4), sobol_entry=sob)
                vals.append(r["sfc_dir"].astype(np.float64) / (per * 2.0 ** 31))
            vals = np.array(vals)
            assert vals.mean() == pytest.approx(1.0, abs=1e-12)
            sd[per, sob] = vals.std(axis=0, ddof=1).mean()
    assert sd[1024, True] < 0.1 * sd[1024, False]
    assert sd[1024, True] < 0.1 * sd[64, True]
    assert sd[1024, False] > 0.18 * sd[64, False]  # N^-1/2: a factor 1/4


def test_scrambles_of_x_and_y_are_independent():
    """The first point (pass 0) of every column is (0, 0) before scrambling;
    after it, (x, y) over many columns must fill the square uniformly (the
    two coordinates take independent scrambles, else pass 0 would sit on the
    diagonal)."""
    pts = np.array([oracle.sobol_entry(0, 1, c, 31337)[0] for c in range(4096)], dtype=np.uint64)
    cell = (pts[:, 0] >> np.uint64(30)) * np.uint64(4) + (pts[:, 1] >> np.uint64(30))
    assert stats.chisquare(np.bincount(cell.astype(np.int64), minlength=16)).pvalue > 1e-4


@pytest.mark.parametrize("per,sza,az,seed", [(1, 37.0, 61.0, 5), (16, 52.0, 200.0, 6), (48, 20.0, 300.0, 7)])
def test_traced_entry_points_are_the_documented_ones(per, sza, az, seed):
    """In vacuum every photon flies straight from its entry point to the
    surface, so the direct surface irradiance of each column is the number
    of entry points whose shifted position lands in it.  Photon id enters
    column (id + o) mod ncol as its (id div ncol)-th photon, at the scrambled
    Sobol point of that pass (oracle.sobol_entry); predicting every landing
    column from that rule reproduces the traced tallies photon for photon."""
    from paper_2208_05247_amd import synthetic as syn
    nx, ny, nz, d = 8, 4, 2, 50.0
    grid = syn.Grid(nx, ny, nz, d, d, d)
    f = syn.uniform_fields(grid, 0.0, 0.0, 0.0, 0.0, albedo=0.0)
    ncol = nx * ny
    n = per * ncol + 3            # a ragged last pass
    r = oracle.trace(f, sza, az, n, seed, brick=(1, 1, 1), sobol_entry=True)
    o = int(oracle.philox4x32_10(np.array([[0, 0, 0xfffffffe, 0]], dtype=np.uint32), seed)[0, 0]) * ncol >> 32
    th, ph = np.radians(sza), np.radians(az)
    H = nz * d
    shift = (-np.sin(th) * np.sin(ph) / np.cos(th) * H, -np.sin(th) * np.cos(ph) / np.cos(th) * H)
    want = np.zeros((ny, nx), dtype=np.int64)
    for pid in range(n):
        col = (pid + o) % ncol
        ic, jc = col % nx, col // nx
        xy = oracle.sobol_entry(pid // ncol, 1, col, seed)[0].astype(np.float64)
        x = (ic + (xy[0] + 0.5) / 2 ** 32) * d + shift[0]
        y = (jc + (xy[1] + 0.5) / 2 ** 32) * d + shift[1]
        want[int(np.floor(y / d)) % ny, int(np.floor(x / d)) % nx] += 1
    got = r["sfc_dir"].astype(np.int64) // 2 ** 31
    assert np.array_equal(got, want)
