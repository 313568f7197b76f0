"""Throughput benchmark of the MI355X photon tracer.

Headline step = one pass of the whole hot path over the largest workload:
1024 x 1024 x 128 cells of 25 x 25 x 20 m (cumulus field of ~800 Gaussian
blobs), 112 shortwave g-points traced in ONE persistent launch
(rt3d_trace_batched: tally clearing, packing, per-g-point majorants,
tracing) and rt3d_finalize (heating rates), 2^30 photons split over the
g-points in proportion to the two-stream flux entering the top of the
domain (per-g-point diffuse fractions), sun at 60 deg zenith, surface
albedo U[0.1, 0.3] per column.  Inputs are resident in HBM before timing
starts.  Prints one JSON line; secondary legs (the 256x256x128 LES-shaped
single g-point field, the 512x512x96 batched field, the memory-access
ceiling, the two-stream column, denoiser inference, the time to a 5 %
heating-rate error, the CPU oracle) are fields of the same line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon events/s + time to 5% heating-rate RMS, plain vs batched+denoised"
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
HEADLINE = dict(seed=99_999, nx=1024, nz=128, dx=25.0, dz=20.0, sza=60.0, az=0.0, photons=1 << 30)
HEADLINE_NAME = "batched_cumulus_1024x1024x128_112g"
# acceleration cell of the headline launch: the least Monte Carlo cost
# (kernel time x heating-tally variance, from two seeds at the full 2^30
# photons) of a same-box sweep; relative cost 8x8x8 1.000, 8x8x16 1.005,
# 4x8x8 1.014, 16x16x16 1.017, 8x8x4 1.028, 16x16x8 1.028, 4x4x8 1.051,
# 4x4x4 1.119.  Finer cells trace a photon faster (4x4x8 1472 ms against
# 1557 ms) but deposit absorption at fewer tentative collisions
HEADLINE_BRICK = (8, 8, 8)
# entry tile of the photon schedule for the headline launch (order only, the
# tallies are bitwise those of any other tile): the fastest of a same-box
# sweep, 128x128 1651 ms against 1667 ms for the automatic 128x256 and
# 1861 ms for one whole-domain tile
HEADLINE_TILE = (128, 128)
TTR_REFERENCE_PER_COLUMN = 1 << 17


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic HBM bytes per event of the tracing kernel (random gathers and
# tally read-modify-writes at the method's granularity; majorants are not
# counted):
#   tentative collision: 8 B (k_ext, ssa) + 8 B heating-tally update
#   real scattering:     + 4 B (k_ext_cloud); cloud scattering: + 4 B (g)
#   surface hit:         4 B albedo + 8 B irradiance + 8 B absorbed tally
#   escape:              8 B TOD tally
def algorithmic_bytes(stats) -> float:
    s = {k: float(v) for k, v in stats.items()}
    return (16.0 * s["collisions"] + 4.0 * (s["scat_gas"] + s["scat_cloud"]) + 4.0 * s["scat_cloud"]
            + 20.0 * s["surface"] + 8.0 * s["escape"])


def source_hash(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


TRACER_SOURCES = ("paper_2208_05247_amd/csrc/rt3d.hip",)


def profile_fields(name: str) -> dict:
    """Indented 'key: value' lines of a committed profile summary."""
    prof = os.path.join(ROOT, "profiles", name)
    fields = {}
    if not os.path.exists(prof):
        return fields
    for line in open(prof):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    return fields


def measured_traffic(profile: str, workload: str):
    """HBM bytes per launch of the tracing kernel from the committed
    rocprofv3 PMC summary (FETCH_SIZE and WRITE_SIZE, each scaled by its
    calibration factor), if it was taken on this exact kernel source and
    workload; else None."""
    f = profile_fields(profile)
    if f.get("source_sha256_16") != source_hash(TRACER_SOURCES) or f.get("workload") != workload:
        return None
    try:
        return float(f["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def headline_key(brick, tile) -> str:
    """Workload key of the headline's committed counter summary: the
    workload, acceleration cell and schedule tile the counters were taken
    with."""
    return f"{HEADLINE_NAME}, brick {brick[0]}x{brick[1]}x{brick[2]}, schedule tile {tile[0]}x{tile[1]}"


def parse_brick(text: str):
    """--brick: one edge (cubic) or bx,by,bz; empty: the headline's."""
    if not text:
        return HEADLINE_BRICK
    v = tuple(int(x) for x in text.split(","))
    return v * 3 if len(v) == 1 else v


CELL_SWEEP = [(8, 8, 8), (4, 4, 8), (8, 8, 4), (4, 8, 8), (8, 8, 16), (16, 16, 8), (4, 4, 4), (16, 16, 16)]


def cell_sweep(tr, counts) -> list:
    """The headline's photons per acceleration cell: kernel ms and the
    variance of the heating tallies from two seeds (summed squared
    difference, halved); cost = ms x variance relative to the first cell
    (time to a given error is proportional to it)."""
    import torch
    from paper_2208_05247_amd import autotune, rt3d
    wl = tr.wl
    rows, ref = [], None
    for b in CELL_SWEEP:
        ws = rt3d.alloc_workspace(rt3d.workspace_size_batched(tr.grid, tr.m.n_gpoints, rt3d.options(brick=b)))
        kms, heat = [], []
        for seed in (1, 2):
            raw = rt3d.trace_batched(tr.dm, wl.sza, wl.azimuth, counts, seed, brick=b, out=tr.out, workspace=ws,
                                     timed=True, gpoint_diffuse=tr.fd, tile=tr.tile)
            kms.append(rt3d.last_trace_ms())
            heat.append(raw["abs_dir"].double() + raw["abs_dif"].double())
        noise = autotune._noise(heat[0], heat[1])
        mean_sq = float((0.25 * (heat[0] + heat[1]) ** 2).sum())
        st = dict(zip(rt3d.STATS, raw["stats"].cpu().tolist()))
        ms = min(kms)
        ref = ms * noise if ref is None else ref
        rows.append({"brick": list(b), "kernel_ms": kms, "relative_variance": noise / mean_sq,
                     "cost_relative": ms * noise / ref, "events_per_photon": st["collisions"] / st["photons"]})
        log(json.dumps(rows[-1]))
        del ws, heat
        torch.cuda.empty_cache()
    return rows


def headline_scene():
    from paper_2208_05247_amd import experiment as ex
    h = HEADLINE
    return ex.scene(h["seed"], h["nx"], h["nx"], h["nz"], h["dx"], h["dz"], sza=h["sza"], az=h["az"],
                    photons=h["photons"])


def tracer_roofline(stats_tot: dict, launches: int, mean_kms: float, traffic) -> dict:
    bytes_per_launch = algorithmic_bytes(stats_tot) / launches
    achieved = bytes_per_launch / (mean_kms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_GBps": None if traffic is None else traffic / (mean_kms * 1e-3) / 1e9,
            "traffic_frac": None if traffic is None else traffic / (mean_kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kernel": "trace_kernel", "bytes_per_launch": bytes_per_launch}


def headline(tr, counts, steps: int, warmup: int) -> dict:
    """Batched launch + finalize on the largest workload, K timed steps."""
    import torch
    from paper_2208_05247_amd import rt3d
    wl = tr.wl
    total = int(counts.sum())

    def step(seed):
        raw = rt3d.trace_batched(tr.dm, wl.sza, wl.azimuth, counts, seed, brick=tr.brick, out=tr.out,
                                 workspace=tr.ws, timed=True, gpoint_diffuse=tr.fd, tile=tr.tile)
        kms = rt3d.last_trace_ms()
        rt3d.finalize(tr.grid, raw, total, layer_scale=tr.ls)
        return kms, raw["stats"].clone()

    for w in range(warmup):
        step(1000 + w)
    torch.cuda.synchronize()
    kms, stats = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        a, b = step(k + 1)
        kms.append(a)
        stats.append(b)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = {n: 0 for n in rt3d.STATS}
    for st in stats:
        for n, v in zip(rt3d.STATS, st.cpu().tolist()):
            tot[n] += v
    return {"wall": wall, "kernel_ms": kms, "stats": tot}


def les_measurement(steps: int) -> dict:
    """The 256x256x128 LES-shaped single g-point field (2^26 photons, 8^3
    bricks, SZA 45 deg): trace + finalize per step."""
    import torch
    from paper_2208_05247_amd import rt3d
    from paper_2208_05247_amd import synthetic as syn
    wl = syn.les_cumulus()
    grid = wl.fields.grid
    df = rt3d.DeviceFields.from_host(wl.fields, "cuda")
    out = rt3d.alloc_tallies(grid)
    ws = rt3d.alloc_workspace(rt3d.workspace_size(grid, rt3d.options(brick=wl.brick)))

    def step(seed):
        raw = rt3d.trace(df, wl.sza, wl.azimuth, wl.photons, seed, brick=wl.brick, out=out, workspace=ws, timed=True)
        kms = rt3d.last_trace_ms()
        rt3d.finalize(grid, raw, wl.photons)
        return kms, raw["stats"].clone()

    step(999)
    torch.cuda.synchronize()
    kms, stats = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        a, b = step(k + 1)
        kms.append(a)
        stats.append(b)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = {n: 0 for n in rt3d.STATS}
    for st in stats:
        for n, v in zip(rt3d.STATS, st.cpu().tolist()):
            tot[n] += v
    ev = tot["collisions"] + tot["surface"]
    mean_kms = sum(kms) / len(kms)
    traffic = measured_traffic("trace_kernel_les_cumulus_256x256x128.md", wl.name)
    return {"workload": wl.name, "grid": [grid.nx, grid.ny, grid.nz], "photons": wl.photons,
            "brick": list(wl.brick), "photon_events_per_s": ev / wall, "photons_per_s": tot["photons"] / wall,
            "events_per_photon": ev / tot["photons"], "ms_per_step": wall * 1e3 / steps, "trace_kernel_ms": mean_kms,
            "roofline": tracer_roofline(tot, steps, mean_kms, traffic)}


def batched_measurement(steps: int) -> dict:
    """112 g-points over a 512x512x96 cumulus field, 2^28 photons (multinomial
    over Dirichlet(1) flux weights) in ONE persistent launch, against the
    same g-points traced one launch each."""
    import torch
    from paper_2208_05247_amd import rt3d
    from paper_2208_05247_amd import synthetic as syn

    wl = syn.batched_cumulus()
    m = wl.medium
    dm = rt3d.DeviceBatchedMedium.from_host(m)
    out = rt3d.alloc_tallies(m.grid)
    opt = rt3d.options(brick=wl.brick)
    ws = rt3d.alloc_workspace(rt3d.workspace_size_batched(m.grid, m.n_gpoints, opt))
    total = int(wl.photons.sum())
    rt3d.trace_batched(dm, wl.sza, wl.azimuth, wl.photons, 999, brick=wl.brick, out=out, workspace=ws)
    torch.cuda.synchronize()
    kms, evs = [], 0
    t0 = time.perf_counter()
    for k in range(steps):
        raw = rt3d.trace_batched(dm, wl.sza, wl.azimuth, wl.photons, 1 + 1000 * k, brick=wl.brick, out=out,
                                 workspace=ws, timed=True)
        kms.append(rt3d.last_trace_ms())
        rt3d.finalize(m.grid, raw, total)
        st = raw["stats"].cpu().tolist()
        evs += st[rt3d.STATS.index("collisions")] + st[rt3d.STATS.index("surface")]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # the paper's way: every g-point traced independently, one launch each
    dsingles = [rt3d.DeviceBatchedMedium(m.grid, dm.k_gas[n:n + 1].contiguous(), dm.ssa_gas[n:n + 1].contiguous(),
                                         dm.k_cloud, dm.ssa_cloud, dm.g_cloud, dm.albedo)
                for n in range(m.n_gpoints)]
    ws1 = rt3d.alloc_workspace(rt3d.workspace_size_batched(m.grid, 1, opt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(m.n_gpoints):
        if int(wl.photons[n]) == 0:
            continue
        rt3d.trace_batched(dsingles[n], wl.sza, wl.azimuth, [int(wl.photons[n])], 1 + n, brick=wl.brick,
                           out=out, workspace=ws1, accumulate=n > 0)
    torch.cuda.synchronize()
    sep = time.perf_counter() - t0
    return {"workload": wl.name, "grid": [m.grid.nx, m.grid.ny, m.grid.nz], "g_points": m.n_gpoints,
            "photons": total, "brick": list(wl.brick), "ms_per_launch": wall * 1e3,
            "trace_kernel_ms": sum(kms) / len(kms), "photon_events_per_s": evs / (wall * steps),
            "photons_per_s": total / wall, "separate_launches_ms": sep * 1e3,
            "speedup_vs_separate_launches": sep / wall}


def two_stream_measurement(reps: int = 20) -> dict:
    """Kernel time of the clear-sky two-stream TOD column for 112 g-points
    (32 layers above the domain + the 96 levels of the batched field)."""
    import torch
    from paper_2208_05247_amd import rt3d
    from paper_2208_05247_amd import synthetic as syn

    wl = syn.batched_cumulus()
    tau, ssa, g = syn.clear_sky_columns(wl.medium, n_above=32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    t, w, a = dev(tau), dev(ssa), dev(g)
    alb = dev(np.full(tau.shape[0], 0.2))
    mu0 = float(np.cos(np.radians(wl.sza)))
    rt3d.two_stream(t, w, a, alb, mu0, 32)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        o = rt3d.two_stream(t, w, a, alb, mu0, 32)
    e1.record()
    torch.cuda.synchronize()
    fd = o["tod_diffuse_fraction"].cpu().numpy()
    return {"columns": int(tau.shape[0]), "layers": int(tau.shape[1]), "ms_per_call": e0.elapsed_time(e1) / reps,
            "diffuse_fraction_range": [float(fd.min()), float(fd.max())]}


def denoiser_flops(net, D, H, W) -> float:
    from paper_2208_05247_amd import denoise as dn
    flops = 0.0
    for L in net.layers:
        level = {"e0": 0, "e1": 1, "e2": 2, "b": 3, "d2": 2, "d1": 1, "d0": 0, "head": 0}[L.name]
        cin = net.n_in if L.name == "e0" else L.c1 + L.c2
        cout = dn.NOUT if L.name == "head" else L.cout
        flops += 2.0 * L.ksize ** 3 * cin * cout * (D * H * W) / 8 ** level
    return flops


def denoiser_measurement(reps: int = 3) -> dict:
    """Inference time of the denoiser on the 1024x1024x128 evaluation grid
    (random weights; time does not depend on them) and its MFMA roofline:
    algorithmic FLOPs of the network as defined (first layer: its 4 real
    input channels; head: its 2 real outputs) over the wall time of one
    inference (features, every convolution, pooling, residual head)."""
    import torch
    from paper_2208_05247_amd import denoise as dn
    from paper_2208_05247_amd import experiment as ex
    from paper_2208_05247_amd.synthetic import Grid

    D, H, W = 128, 1024, 1024
    n_in = ex.committed_denoiser_inputs()
    net = dn.Denoiser(base=32, seed=0, n_in=n_in)
    g = torch.Generator(device="cuda").manual_seed(1)
    hd = torch.rand(D, H, W, device="cuda", generator=g)
    hf = torch.rand(D, H, W, device="cuda", generator=g)
    ke = torch.rand(D, H, W, device="cuda", generator=g) * 0.01
    ka = 0.1 * ke
    grid = Grid(W, H, D, 25.0, 25.0, 20.0)
    direct = {"grid": grid, "sza": 60.0, "azimuth": 0.0, "direct_fraction": 0.88,
              "layer_scale": ex.layer_scale(grid)} if n_in == 5 else None
    flops = denoiser_flops(net, D, H, W)
    dn.denoise(net, hd, hf, ke, ka, 20.0, direct=direct)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dn.denoise(net, hd, hf, ke, ka, 20.0, direct=direct)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    achieved = flops / (ms * 1e-3) / 1e12
    return {"grid": [D, H, W], "inputs": n_in, "parameters": net.n_params(), "ms_per_inference": ms,
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "flops_per_call": flops}}


def access_ceiling(ncell: int, collisions_per_launch: float, atomics_per_16: int, kernel_ms=None,
                   chains=(1, 2, 4)) -> dict:
    """What the memory system delivers for the tracer's access pattern on a
    footprint of ncell 16-byte records and 2 x ncell uint64 tallies
    (rt3d_probe_gathers): as many dependent random gathers as the tracer
    makes tentative collisions per launch, atomics_per_16 of every 16
    followed by a random 64-bit atomic add, with 1, 2 and 4 independent
    chains per lane; and once without the atomics.  The tracer's collision
    rate as a fraction of the one-chain ceiling (when kernel_ms is given)."""
    import torch
    from paper_2208_05247_amd import probe
    g = torch.Generator(device="cuda").manual_seed(3)
    rec = torch.rand((ncell, 4), generator=g, device="cuda", dtype=torch.float32)
    tally = torch.zeros(2 * ncell, dtype=torch.int64, device="cuda")
    lanes = probe.lanes(0)
    probe.gathers(rec, tally, 16, 1, atomics_per_16, seed=1)
    torch.cuda.synchronize()
    rates = {}
    for a16 in (atomics_per_16, 0):
        for c in chains:
            events = max(1, int(round(collisions_per_launch / lanes / c)))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            probe.gathers(rec, tally, events, c, a16, seed=2 + c)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rates[f"{'with_atomics' if a16 else 'gathers_only'}_chains{c}"] = \
                {"ms": ms, "gathers_per_s": lanes * events * c / (ms * 1e-3)}
    del rec, tally
    torch.cuda.empty_cache()
    res = {"lanes": lanes, "atomics_per_16": atomics_per_16, "records_bytes": ncell * 16,
           "tally_bytes": 2 * ncell * 8, "rates": rates}
    if kernel_ms:
        tracer = collisions_per_launch / (kernel_ms * 1e-3)
        ceil1 = rates[f"with_atomics_chains1"]["gathers_per_s"]
        res.update({"tracer_collisions_per_s": tracer, "frac_of_one_chain_ceiling": tracer / ceil1})
    return res


def time_to_5pct(tr, ref_per_col: int) -> dict:
    """Plain vs batched+denoised time to a 5 % heating-rate RMS error on the
    headline scene, run here: the committed denoiser weights (trained by
    `python -m paper_2208_05247_amd.experiment`, sha256-checked), a
    reference of ref_per_col photons per column (two independent halves,
    its own noise variance removed), the plain convergence sweep and the
    denoised sweep (experiment.evaluate)."""
    from paper_2208_05247_amd import experiment as ex
    net, info = ex.load_committed_denoiser()
    t0 = time.perf_counter()
    res = ex.evaluate(net, tr.wl, ref_per_col, tracer=tr)
    res["evaluation_wall_s"] = time.perf_counter() - t0
    res["weights"] = info
    return res


def cpu_baseline(tr, counts, gpu_events_per_photon: float, target_s: float = 20.0) -> dict:
    """The FP64 C oracle on a bounded sample of the headline workload, on
    every host core: photons of a few g-points drawn with probability
    proportional to their photon shares (each g-point traced on its full
    1024x1024x128 fields with its own diffuse fraction).  A call on these
    fields has a fixed cost (zeroed 2 GiB tallies, the majorant pass) that
    would dominate a short sample, so each g-point is traced twice, with a
    short and a long run, and the rate is the marginal one between them:
    (events of the long run - events of the short run) / (time difference).
    The long runs are sized to about target_s of CPU time in total."""
    import oracle
    threads = os.cpu_count() or 1
    m = tr.m
    rng = np.random.default_rng(12345)
    shares = counts.astype(np.float64) / counts.sum()
    picks = sorted(set(int(x) for x in rng.choice(m.n_gpoints, size=3, replace=False, p=shares)))
    fdh = tr.fd.cpu().numpy() if tr.fd is not None else np.zeros(m.n_gpoints, np.float32)
    fields = {n: m.fields_of(n) for n in picks}

    def run(n, photons, seed):
        t = time.perf_counter()
        r = oracle.trace(fields[n], tr.wl.sza, tr.wl.azimuth, photons, seed, brick=tr.brick,
                         diffuse_fraction=float(fdh[n]), nthreads=threads)
        dt = time.perf_counter() - t
        st = dict(zip(oracle.STATS, r["stats"].tolist()))
        return dt, st["collisions"] + st["surface"]

    n0, n1 = 1 << 16, 1 << 18
    short, per_photon = {}, 0.0
    for n in picks:
        t0, _ = run(n, n0, 5 + n)
        t1, e1 = run(n, n1, 77 + n)
        short[n] = (t1, e1)
        per_photon += max(t1 - t0, 1e-6) / (n1 - n0)
    per = n1
    while per < (1 << 24) and per_photon * 2 * per < target_s:
        per *= 2
    ev, ph, dt, wall = 0, 0, 0.0, 0.0
    for n in picks:
        t2, e2 = run(n, per, 77 + n)
        ev += e2 - short[n][1]
        ph += per - n1
        dt += t2 - short[n][0]
        wall += t2
    return {"value": ev / dt, "unit": "photon events/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"g-points {picks} of the {HEADLINE_NAME} workload (drawn by photon share; full fields, "
                      f"two-stream diffuse fractions; FP64 C oracle, {threads} threads): marginal rate between "
                      f"runs of {n1} and {per} photons per g-point ({wall:.1f} s for the long runs, "
                      f"{dt:.1f} s marginal), {ev / max(ph, 1):.1f} events/photon against "
                      f"{gpu_events_per_photon:.1f} for the GPU's whole g-point mix",
            "photons_per_s": ph / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="only the headline (and cpu baseline)")
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-5 %% evaluation")
    ap.add_argument("--ttr-reference", type=int, default=TTR_REFERENCE_PER_COLUMN,
                    help="photons per column of the time-to-5 %% reference")
    ap.add_argument("--brick", default="", help="acceleration cell of the headline: one edge or bx,by,bz "
                                               "(default: the headline's)")
    ap.add_argument("--budget-s", type=float, default=540.0,
                    help="wall-clock budget of the whole run: optional legs that would not fit are skipped "
                         "(and say so) so that the JSON line is always printed")
    ap.add_argument("--inference-only", action="store_true",
                    help="only time denoiser inference on the 1024x1024x128 grid (prints its JSON)")
    ap.add_argument("--probe-only", action="store_true",
                    help="only run the memory-access ceiling probe on the headline footprint (prints its JSON)")
    ap.add_argument("--les-only", action="store_true", help="only the 256x256x128 single g-point leg")
    ap.add_argument("--cell-sweep", action="store_true",
                    help="only the headline's photons per acceleration cell: kernel time, tally variance and "
                         "their product (prints its JSON)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run one plain device copy of this many bytes (for HBM counter scaling)")
    ap.add_argument("--calibrate-gathers", type=int, default=0,
                    help="only run the probe's random 16-byte gathers (no atomics) on this many bytes of "
                         "records: one gather per 128-byte line, then the same with the line's other half "
                         "gathered too (for the counters' fetch granularity)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the tracer is single-GPU (photons or g-points would be "
              "sharded across GPUs with one all-reduce of the tallies; not built here)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy}), flush=True)
        return
    if args.calibrate_gathers:
        import torch
        from paper_2208_05247_amd import probe
        n = args.calibrate_gathers // 16 // 8 * 8
        rec = torch.ones((n, 4), dtype=torch.float32, device="cuda")
        tally = torch.zeros(8, dtype=torch.int64, device="cuda")
        res = {"records_bytes": n * 16, "lanes": probe.lanes(0), "events": 64}
        for pair in (False, True):
            probe.gathers(rec, tally, 64, 1, 0, line_pair=pair, seed=3)
            torch.cuda.synchronize()
        res["gathers_per_call"] = probe.lanes(0) * 64
        print(json.dumps(res), flush=True)
        return
    if args.inference_only:
        print(json.dumps({"denoiser_inference": denoiser_measurement()}), flush=True)
        return
    if args.les_only:
        print(json.dumps({"les": les_measurement(max(1, args.steps))}), flush=True)
        return

    import torch
    from paper_2208_05247_amd import experiment as ex
    from paper_2208_05247_amd import rt3d

    log("headline scene ...")
    wl = headline_scene()
    brick = parse_brick(args.brick)
    tr = ex.Tracer(wl, brick=brick, tile=HEADLINE_TILE if brick == HEADLINE_BRICK else (0, 0))
    counts = ex.multinomial_counts(tr.shares, HEADLINE["photons"], 5)
    if args.probe_only:
        print(json.dumps({"access_ceiling": access_ceiling(tr.grid.ncell, 5.0e10, 11)}), flush=True)
        return
    if args.cell_sweep:
        print(json.dumps({"cell_sweep": cell_sweep(tr, counts)}), flush=True)
        return
    log("headline steps ...")
    hl = headline(tr, counts, args.steps, args.warmup)
    tot = hl["stats"]
    events = tot["collisions"] + tot["surface"]
    mean_kms = sum(hl["kernel_ms"]) / len(hl["kernel_ms"])
    traffic = measured_traffic("trace_kernel_batched_cumulus_1024x1024x128.md", headline_key(brick, tr.tile))
    g = tr.grid
    res = {
        "metric": METRIC,
        "value": events / hl["wall"],
        "unit": "photon events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hl["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": HEADLINE_NAME, "grid": [g.nx, g.ny, g.nz], "cell_m": [g.dx, g.dy, g.dz],
                   "g_points": int(tr.m.n_gpoints), "photons_per_step": int(counts.sum()),
                   "photons_per_column": int(counts.sum()) // g.ncol, "sza_deg": wl.sza,
                   "albedo": "U[0.1, 0.3] per column", "entry": "two-stream flux at the domain top",
                   "brick": list(brick), "schedule_tile": list(tr.tile), "parallelism": "single GPU"},
        "photons_per_s": tot["photons"] / hl["wall"],
        "events_per_photon": events / max(1, tot["photons"]),
        "trace_kernel_ms": mean_kms,
        "roofline": tracer_roofline(tot, args.steps, mean_kms, traffic),
        "paper_context": "A100 40GiB: ~1.9e8 photons/s derived from 90 s for 112 g-points x 256 "
                         "photons/column on 768x768 columns (different fields)",
    }
    log(f"headline: {res['value']:.3e} events/s, kernel {mean_kms:.1f} ms")
    left = lambda: args.budget_s - (time.perf_counter() - T_START)
    ms_per_photon = mean_kms / max(1, tot["photons"] // args.steps)
    if not args.no_ttr:
        # reference + plain sweep (16..4096 per column) + denoised sweep (64..1024), in headline-kernel time
        need = 1e-3 * ms_per_photon * g.ncol * (args.ttr_reference + 5456 + 6016) * 1.15 + 30.0
        if left() > need + 60.0:
            log(f"time to 5 % (about {need:.0f} s) ...")
            res["time_to_5pct_heating_rms"] = time_to_5pct(tr, args.ttr_reference)
        else:
            res["time_to_5pct_heating_rms"] = {"skipped": f"needs ~{need:.0f} s, {left():.0f} s of the "
                                                          f"{args.budget_s:.0f} s budget left"}
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(tr, counts, res["events_per_photon"],
                                           target_s=float(np.clip(left() - 120.0, 5.0, 20.0)))
    if not args.no_secondary and left() > 60.0:
        log("access ceiling ...")
        merged = float(np.clip(ACCESS_ATOMICS_PER_16, 0, 16))
        res["access_ceiling"] = access_ceiling(g.ncell, tot["collisions"] / args.steps, int(merged), mean_kms,
                                               chains=(1, 2))
    del tr
    torch.cuda.empty_cache()
    if not args.no_secondary:
        if left() > 90.0:
            log("secondary legs ...")
            res["les"] = les_measurement(max(1, min(args.steps, 5)))
            res["batched_512x512x96"] = batched_measurement(max(1, min(args.steps, 3)))
            res["two_stream_tod"] = two_stream_measurement()
            res["denoiser_inference"] = denoiser_measurement()
        else:
            res["secondary"] = {"skipped": f"{left():.0f} s of the {args.budget_s:.0f} s budget left"}
    res["bench_wall_s"] = time.perf_counter() - T_START
    print(json.dumps(res), flush=True)


# Tally atomics per 16 tentative collisions in the access probe: the merged
# deposits per tentative collision of the tracer (31.2 per 44.4 on the
# 256x256x128 field, ~11/16).
ACCESS_ATOMICS_PER_16 = 11


if __name__ == "__main__":
    main()
