"""GPU parity of the HIP tracer against the FP64 CPU oracle, through the C ABI.

Integer results (Philox words, majorants, the energy ledger, reruns and
chunked runs) must agree bit for bit.  Monte Carlo tallies are compared
statistically: B independent sub-runs per side, per-cell batch means, and
|m_gpu - m_oracle| <= 4 sqrt(se_gpu^2 + se_oracle^2) in >= 99.9 % of the
dense cells; sparse cells are compared in column / layer aggregates.  The
global budget (sum of FP32 outputs vs the uint64 ledger) must hold to 1e-5
relative."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import reference_solutions as rs  # noqa: E402
from mc_stats import RunningBatches, batch_mean_se, compare_batches, compare_running  # noqa: E402
from paper_2208_05247_amd import synthetic as syn  # noqa: E402

pytestmark = pytest.mark.gpu
W1 = 2 ** 31
ARRAYS = ("abs_dir", "abs_dif", "sfc_dir", "sfc_dif", "sfc_abs", "toa_up")


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


def ledger_ok(h):
    L = [int(v) for v in h["ledger"]]
    inc, toa, adir, adif, sfc, gain, loss, lost = L
    assert inc + gain == toa + adir + adif + sfc + loss + lost
    assert adir == int(h["abs_dir"].sum(dtype=np.uint64))
    assert adif == int(h["abs_dif"].sum(dtype=np.uint64))
    assert sfc == int(h["sfc_abs"].sum(dtype=np.uint64))
    assert toa == int(h["toa_up"].sum(dtype=np.uint64))
    S = dict(zip(oracle.STATS, [int(v) for v in h["stats"]]))
    assert S["photons"] == S["escape"] + S["rr_kill"] + S["absorbed"] + S["capped"]
    assert inc == S["photons"] * W1


def gpu_batches(rt3d, df, sza, az, per, B, seed, brick, **kw):
    grid = df.grid
    outs = {k: [] for k in ARRAYS}
    for b in range(B):
        raw = rt3d.trace(df, sza, az, per, seed, brick=brick, photon_offset=b * per, **kw)
        fin = rt3d.finalize(grid, raw, per)
        for k in ARRAYS:
            outs[k].append(fin[k].double().cpu().numpy())
    return {k: np.stack(v) for k, v in outs.items()}


def oracle_batches(fields, sza, az, per, B, seed, brick, **kw):
    outs = {k: [] for k in ARRAYS}
    for b in range(B):
        raw = oracle.trace(fields, sza, az, per, seed, brick=brick, photon_offset=b * per, **kw)
        fin = oracle.finalize(raw, fields.grid, per)
        for k in ARRAYS:
            outs[k].append(fin[k])
    return {k: np.stack(v) for k, v in outs.items()}


def parity(g, o, min_frac=0.999, label=""):
    """4-SE rule on dense cells; sparse cells in column sums (3D) or in
    4x4 column blocks (2D)."""
    report = {}
    for k in ARRAYS:
        frac, n_dense, n_sparse, dense, z = compare_batches(g[k], o[k], n_se=4.0)
        report[k] = (frac, n_dense, n_sparse)
        assert frac >= min_frac, (label, k, frac, n_dense)
        if k.startswith("abs"):
            ga, oa = g[k].sum(axis=1), o[k].sum(axis=1)   # column totals
        else:
            B, ny, nx = g[k].shape
            ga = g[k].reshape(B, ny // 4, 4, nx // 4, 4).sum(axis=(2, 4)) if ny % 4 == 0 and nx % 4 == 0 else g[k]
            oa = o[k].reshape(B, ny // 4, 4, nx // 4, 4).sum(axis=(2, 4)) if ny % 4 == 0 and nx % 4 == 0 else o[k]
        frac2, n2, _, _, _ = compare_batches(ga, oa, n_se=4.0)
        assert frac2 >= 0.99, (label, k, "aggregate", frac2, n2)
    say(label, {k: (round(v[0], 5), v[1], v[2]) for k, v in report.items()})
    return report


# ---------------------------------------------------------------------------
# Bit-exact pieces
# ---------------------------------------------------------------------------

def test_philox_bit_exact(rt3d):
    rng = np.random.default_rng(0)
    n = 1 << 16
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:16] = 0
    ctr[16:32] = 0xFFFFFFFF
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        dev = torch.from_numpy(ctr.view(np.int32)).cuda()
        got = rt3d.philox4x32_10(dev, seed).cpu().numpy().view(np.uint32)
        ref = oracle.philox4x32_10(ctr, seed)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("brick", [(1, 1, 1), (4, 4, 4), (8, 4, 2), (32, 32, 64), (2, 8, 16)])
def test_majorant_bit_exact(rt3d, brick):
    for f in (syn.small_cumulus().fields, syn.random_fields(syn.Grid(32, 32, 64, 10, 10, 10), seed=5)):
        k = torch.from_numpy(f.k_ext).cuda()
        got = rt3d.majorant_build(f.grid, k, brick).cpu().numpy()
        assert np.array_equal(got, oracle.majorant(f.k_ext, brick))


# ---------------------------------------------------------------------------
# Exact invariants of the GPU path
# ---------------------------------------------------------------------------

def test_ledger_determinism_and_chunks(rt3d):
    wl = syn.small_cumulus()
    df = rt3d.DeviceFields.from_host(wl.fields)
    n = 1 << 18
    a = rt3d.to_host(rt3d.trace(df, wl.sza, wl.azimuth, n, 1, brick=wl.brick))
    ledger_ok(a)
    b = rt3d.to_host(rt3d.trace(df, wl.sza, wl.azimuth, n, 1, brick=wl.brick, grid_blocks=7))
    for k in ARRAYS + ("ledger", "stats"):
        assert np.array_equal(a[k], b[k]), k
    out = None
    for off, m in ((0, 1000), (1000, 70000), (71000, n - 71000)):
        out = rt3d.trace(df, wl.sza, wl.azimuth, m, 1, brick=wl.brick, photon_offset=off,
                         accumulate=out is not None, out=out)
    c = rt3d.to_host(out)
    for k in ARRAYS + ("ledger", "stats"):
        assert np.array_equal(a[k], c[k]), k
    say("stats", dict(zip(oracle.STATS, a["stats"].tolist())))


def test_vacuum_exact(rt3d):
    grid = syn.Grid(4, 3, 5, 100.0, 100.0, 40.0)
    f = syn.uniform_fields(grid, 0.0, albedo=0.3)
    df = rt3d.DeviceFields.from_host(f)
    n = grid.ncol * 50
    w_ref = int(np.rint(np.float64(np.float32(0.3)) * W1))
    for sza in (0.0, 35.0):
        h = rt3d.to_host(rt3d.trace(df, sza, 120.0, n, 5, brick=(2, 3, 5), rr_threshold=0.0))
        ledger_ok(h)
        assert int(h["sfc_dir"].sum()) == n * W1
        assert int(h["ledger"][1]) == n * w_ref
        if sza == 0.0:
            assert np.all(h["sfc_dir"] == 50 * W1)


def test_edge_cases(rt3d):
    wl = syn.small_cumulus()
    df = rt3d.DeviceFields.from_host(wl.fields)
    for n in (1, 63, 65, 1025, 3 * 1024 + 7):
        h = rt3d.to_host(rt3d.trace(df, 0.0, 0.0, n, 3, brick=(32, 32, 64)))
        ledger_ok(h)
        assert int(h["stats"][0]) == n
    # one-cell grid, diffuse entry, roulette off, whole-domain and unit bricks
    g1 = syn.Grid(1, 1, 1, 10.0, 10.0, 10.0)
    f1 = syn.uniform_fields(g1, 0.05, k_cld_z=0.03, ssa_z=0.7, g_z=0.5, albedo=0.6)
    d1 = rt3d.DeviceFields.from_host(f1)
    h = rt3d.to_host(rt3d.trace(d1, 89.0, 10.0, 5000, 9, brick=(1, 1, 1), diffuse_fraction=1.0,
                                rr_threshold=0.0))
    ledger_ok(h)
    assert int(h["sfc_dir"].sum()) == 0
    # iteration cap: weight goes to the LOST ledger entry
    h = rt3d.to_host(rt3d.trace(df, 30.0, 0.0, 5000, 1, brick=wl.brick, max_iters=5))
    ledger_ok(h)
    assert int(h["stats"][11]) > 0 and int(h["ledger"][7]) > 0


def test_validation_and_errors(rt3d):
    wl = syn.small_cumulus()
    f = wl.fields
    bad = syn.Fields(f.grid, f.k_ext.copy(), f.k_ext_cloud.copy(), f.ssa.copy(), f.g.copy(), f.albedo.copy())
    bad.ssa[3, 4, 5] = 1.5
    dbad = rt3d.DeviceFields.from_host(bad)
    with pytest.raises(rt3d.Rt3dError) as e:
        rt3d.trace(dbad, 30.0, 0.0, 100, 1, brick=wl.brick, validate=True)
    assert e.value.status == rt3d.EDOMAIN
    dgood = rt3d.DeviceFields.from_host(f)
    rt3d.trace(dgood, 30.0, 0.0, 100, 1, brick=wl.brick, validate=True)
    for kw in (dict(brick=(3, 4, 4)), dict(brick=(4, 4, 4), diffuse_fraction=2.0)):
        with pytest.raises(rt3d.Rt3dError) as e:
            rt3d.trace(dgood, 30.0, 0.0, 100, 1, **kw)
        assert e.value.status == rt3d.EINVAL
    with pytest.raises(rt3d.Rt3dError):
        rt3d.trace(dgood, 90.0, 0.0, 100, 1, brick=(4, 4, 4))
    with pytest.raises(rt3d.Rt3dError):
        rt3d.trace(dgood, 30.0, 0.0, 0, 1, brick=(4, 4, 4))


def test_finalize_budget(rt3d):
    """Sum of the FP32 outputs (in FP64) matches the exact ledger to 1e-5."""
    wl = syn.small_cumulus()
    df = rt3d.DeviceFields.from_host(wl.fields)
    n = 1 << 20
    raw = rt3d.trace(df, wl.sza, wl.azimuth, n, 1, brick=wl.brick)
    fin = rt3d.finalize(wl.fields.grid, raw, n)
    h = rt3d.to_host(raw)
    norm = wl.fields.grid.ncol / (n * W1)
    for k, li in (("abs_dir", 2), ("abs_dif", 3), ("sfc_abs", 4), ("toa_up", 1)):
        got = fin[k].double().sum().item()
        ref = int(h["ledger"][li]) * norm
        assert abs(got - ref) <= 1e-5 * abs(ref) + 1e-12, k
    ls = torch.linspace(1.0, 2.0, wl.fields.grid.nz, dtype=torch.float64, device="cuda")
    fin2 = rt3d.finalize(wl.fields.grid, raw, n, layer_scale=ls, flux_scale=3.0)
    assert torch.allclose(fin2["abs_dir"].double(), fin["abs_dir"].double() * ls[:, None, None], rtol=1e-6)
    assert torch.allclose(fin2["sfc_dir"], fin["sfc_dir"] * 3.0, rtol=1e-6)


# ---------------------------------------------------------------------------
# Same random stream, no scattering: near-identical photon paths
# ---------------------------------------------------------------------------

def test_same_stream_absorbing_medium(rt3d):
    """With omega = 0 nothing scatters, so with the same seed the GPU and the
    oracle follow the same photons through the same cells; only FP32 vs FP64
    rounding separates them."""
    grid = syn.Grid(16, 16, 32, 100.0, 100.0, 50.0)
    rng = np.random.default_rng(3)
    kc = syn.cloud_blobs(grid, rng, 3, 0.01, z_range=(500.0, 1200.0))
    f = syn.mix(grid, syn.gas_profile(grid, k0=1e-4), 0.0, kc, 0.0, 0.0, 0.4)
    df = rt3d.DeviceFields.from_host(f)
    n = 1 << 18
    g = rt3d.to_host(rt3d.trace(df, 40.0, 60.0, n, 77, brick=(4, 4, 8), rr_threshold=0.0))
    o = oracle.trace(f, 40.0, 60.0, n, 77, brick=(4, 4, 8), rr_threshold=0.0)
    ledger_ok(g)
    for k in ("abs_dir", "sfc_dir", "sfc_abs"):
        a, b = g[k].astype(np.float64), o[k].astype(np.float64)
        assert abs(a.sum() - b.sum()) <= 2e-5 * b.sum(), k
        # the same photons land in the same cells
        assert np.abs(a - b).sum() <= 2e-3 * b.sum(), k


# ---------------------------------------------------------------------------
# Statistical parity
# ---------------------------------------------------------------------------

def test_parity_small_cumulus(rt3d):
    """32x32x64 cumulus, SZA 30, 2^20 photons as 64 batches of 2^14."""
    wl = syn.small_cumulus()
    df = rt3d.DeviceFields.from_host(wl.fields)
    B, per = 64, (1 << 20) // 64
    say("parity small cumulus: gpu")
    g = gpu_batches(rt3d, df, wl.sza, wl.azimuth, per, B, 1, wl.brick)
    say("parity small cumulus: oracle")
    o = oracle_batches(wl.fields, wl.sza, wl.azimuth, per, B, 2, wl.brick)
    parity(g, o, label="cumulus_32x32x64")


@pytest.mark.parametrize("case", ["diffuse_entry", "no_roulette", "unit_bricks", "side_sun"])
def test_parity_variants(rt3d, case):
    wl = syn.small_cumulus()
    kw, sza, az, brick = {}, wl.sza, wl.azimuth, wl.brick
    if case == "diffuse_entry":
        kw = dict(diffuse_fraction=0.4)
    elif case == "no_roulette":
        kw = dict(rr_threshold=0.0)
    elif case == "unit_bricks":
        brick = (1, 1, 1)
    else:
        sza, az = 75.0, 228.1
    df = rt3d.DeviceFields.from_host(wl.fields)
    B, per = 64, 1 << 14
    g = gpu_batches(rt3d, df, sza, az, per, B, 11, brick, **kw)
    o = oracle_batches(wl.fields, sza, az, per, B, 12, brick, **kw)
    parity(g, o, label=case)


def test_closed_form_milne_on_gpu(rt3d):
    """Isotropic slab over a Lambertian surface against the Milne integral
    equation, on the GPU directly."""
    profile = [0.004, 0.006, 0.01, 0.005]
    grid = syn.Grid(1, 1, 4, 100.0, 100.0, 100.0)
    ke = np.array(profile)
    f = syn.uniform_fields(grid, ke, k_cld_z=ke, ssa_z=0.9, g_z=0.0, albedo=0.3)
    ref = rs.isotropic_slab(f.k_ext[:, 0, 0].astype(np.float64) * 100.0, float(f.ssa[0, 0, 0]),
                            np.cos(np.radians(30.0)), albedo=float(np.float32(0.3)))
    df = rt3d.DeviceFields.from_host(f)
    g = gpu_batches(rt3d, df, 30.0, 0.0, 1 << 16, 32, 5, (1, 1, 2))
    for k in ("sfc_dir", "sfc_dif", "sfc_abs", "toa_up"):
        m, s = batch_mean_se(g[k][:, 0, 0])
        assert abs(m - ref[k]) <= 4.5 * s + 1e-6, (k, m, ref[k], s)
    for k in ("abs_dir", "abs_dif"):
        m, s = batch_mean_se(g[k][:, :, 0, 0])
        assert np.all(np.abs(m - ref[k]) <= 4.5 * s + 1e-6), (k, m, ref[k], s)


def test_les_full_size_properties(rt3d):
    """The 256x256x128 LES-shaped cumulus at its full 2^26 photons, in the
    benchmark's launch configuration: exact ledger, bitwise rerun, direct
    irradiance of sampled columns against the oracle's deterministic line
    integrals, and layer / column-block aggregates against the oracle."""
    wl = syn.les_cumulus()
    f = wl.fields
    df = rt3d.DeviceFields.from_host(f)
    n = wl.photons
    say("les: full run")
    raw = rt3d.trace(df, wl.sza, wl.azimuth, n, 1, brick=wl.brick)
    h = rt3d.to_host(raw)
    ledger_ok(h)
    say("les stats", dict(zip(oracle.STATS, h["stats"].tolist())))
    h2 = rt3d.to_host(rt3d.trace(df, wl.sza, wl.azimuth, n, 1, brick=wl.brick))
    for k in ("abs_dir", "sfc_dir", "ledger", "stats"):
        assert np.array_equal(h[k], h2[k]), k
    # sampled columns: expected direct irradiance by line integrals
    per_col = n / f.grid.ncol
    sfc_dir = h["sfc_dir"].astype(np.float64) / (per_col * W1)
    rng = np.random.default_rng(0)
    cols = [(int(i), int(j)) for i, j in zip(rng.integers(0, 256, 48), rng.integers(0, 256, 48))]
    ref = oracle.direct_transmittance(f, wl.sza, wl.azimuth, cols, n=16)
    got = np.array([sfc_dir[j, i] for i, j in cols])
    # binomial-like noise of 1024 photons per column
    se = np.sqrt(np.maximum(ref * (1 - ref), 1e-4) / per_col)
    assert np.all(np.abs(got - ref) <= 5 * se + 1e-3), np.c_[got, ref, se]
    # aggregates against the oracle at 2^21 photons
    B = 64
    per = (1 << 21) // B
    say("les: oracle batches")
    o = oracle_batches(f, wl.sza, wl.azimuth, per, B, 9, wl.brick)
    say("les: gpu batches")
    g = gpu_batches(rt3d, df, wl.sza, wl.azimuth, per, B, 8, wl.brick)

    def agg(d):
        return {"abs_dir": d["abs_dir"].sum(axis=(2, 3)), "abs_dif": d["abs_dif"].sum(axis=(2, 3)),
                **{k: d[k].reshape(B, 16, 16, 16, 16).sum(axis=(2, 4)) for k in ARRAYS[2:]}}
    ga, oa = agg(g), agg(o)
    for k in ga:
        frac, n_dense, _, dense, z = compare_batches(ga[k], oa[k])
        say("les aggregate", k, frac, n_dense)
        assert frac >= 0.99 and np.all(np.abs(z[dense]) < 5.5), k


def test_parity_les_cumulus_per_cell(rt3d):
    """The 256x256x128 LES-shaped cumulus (8x8x8 bricks, SZA 45 deg) cell by
    cell: 2^25 photons per side as 64 batches of 2^19, the 4-SE rule in
    >= 99.9 % of the dense cells of every tally, sparse cells in column
    totals (3D) and 4x4 column blocks (2D)."""
    wl = syn.les_cumulus()
    f = wl.fields
    grid = f.grid
    df = rt3d.DeviceFields.from_host(f)
    B, per = 64, (1 << 25) // 64
    run = {side: {k: RunningBatches(grid.shape3 if k.startswith("abs") else grid.shape2) for k in ARRAYS}
           for side in ("gpu", "oracle")}
    agg = {side: {k: [] for k in ARRAYS} for side in ("gpu", "oracle")}

    def keep(side, fin):
        for k in ARRAYS:
            x = fin[k]
            run[side][k].add(x)
            agg[side][k].append(x.sum(axis=0) if k.startswith("abs") else
                                x.reshape(grid.ny // 4, 4, grid.nx // 4, 4).sum(axis=(1, 3)))

    out = rt3d.alloc_tallies(grid)
    ws = rt3d.alloc_workspace(rt3d.workspace_size(grid, rt3d.options(brick=wl.brick)))
    say("les per-cell parity: gpu")
    for b in range(B):
        raw = rt3d.trace(df, wl.sza, wl.azimuth, per, 31, brick=wl.brick, photon_offset=b * per, out=out,
                         workspace=ws)
        fin = rt3d.finalize(grid, raw, per)
        keep("gpu", {k: fin[k].double().cpu().numpy() for k in ARRAYS})
    say("les per-cell parity: oracle")
    for b in range(B):
        r = oracle.trace(f, wl.sza, wl.azimuth, per, 32, brick=wl.brick, photon_offset=b * per)
        keep("oracle", oracle.finalize(r, grid, per))
    for k in ARRAYS:
        frac, n_dense, n_sparse, dense, z = compare_running(run["gpu"][k], run["oracle"][k])
        say("les per-cell", k, round(frac, 5), n_dense, n_sparse)
        assert frac >= 0.999 and np.all(np.abs(z[dense]) < 8.0), k
        frac2, n2, _, dense2, z2 = compare_batches(np.stack(agg["gpu"][k]), np.stack(agg["oracle"][k]))
        assert frac2 >= 0.99 and np.all(np.abs(z2[dense2]) < 8.0), (k, "aggregate", frac2, n2)
