"""Throughput benchmark of the MI355X photon tracer.

One step = one pass of the whole hot path over one batch of synthetic input:
rt3d_trace (tally clearing, majorant build, persistent tracing kernel) and
rt3d_finalize (normalisation) for 2^26 photons through the 256x256x128
LES-shaped cumulus field (50 x 50 x 25 m cells, 200 Gaussian cloud blobs,
SZA 45 deg, 8x8x8 acceleration-grid cells).  Inputs are resident in HBM
before timing starts.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon events/s + time to 5% heating-rate RMS, plain vs batched+denoised"
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense

# Algorithmic HBM bytes per event of the tracing kernel (random gathers and
# tally read-modify-writes at the method's granularity; majorants live in
# LDS/L1 and are not counted):
#   tentative collision: 8 B (k_ext, ssa) + 8 B heating-tally update
#   real scattering:     + 4 B (k_ext_cloud); cloud scattering: + 4 B (g)
#   surface hit:         4 B albedo + 8 B irradiance + 8 B absorbed tally
#   escape:              8 B TOD tally
def algorithmic_bytes(stats) -> float:
    s = {k: float(v) for k, v in stats.items()}
    return (16.0 * s["collisions"] + 4.0 * (s["scat_gas"] + s["scat_cloud"]) + 4.0 * s["scat_cloud"]
            + 20.0 * s["surface"] + 8.0 * s["escape"])


def measured_traffic(brick, photons):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it
    was taken on this exact kernel source and workload; else None."""
    import hashlib
    src = os.path.join(ROOT, "paper_2208_05247_amd", "csrc", "rt3d.hip")
    prof = os.path.join(ROOT, "profiles", "trace_kernel_les_cumulus_256x256x128.md")
    if tuple(brick) != (8, 8, 8) or photons != 1 << 26 or not os.path.exists(prof):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    fields = {}
    for line in open(prof):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256_16") != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


TTR_SOURCES = ("paper_2208_05247_amd/csrc/rt3d.hip", "paper_2208_05247_amd/csrc/denoise.hip",
               "paper_2208_05247_amd/denoise.py", "paper_2208_05247_amd/experiment.py")


def sources_hash(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def time_to_5pct():
    """Plain vs batched+denoised time to a 5 % heating-rate RMS error, from
    the committed summary of `python -m paper_2208_05247_amd.experiment`
    (minutes of training and tracing, too long for the default bench run);
    None unless it was measured with the current sources."""
    prof = os.path.join(ROOT, "profiles", "time_to_5pct_batched_cumulus_1024x1024x128.md")
    if not os.path.exists(prof):
        return None
    txt = open(prof).read()
    if "    sources_sha256_16: " + sources_hash(TTR_SOURCES) not in txt or "```json" not in txt:
        return None
    return json.loads(txt.split("```json", 1)[1].split("```", 1)[0])


def cpu_baseline(wl, target_s: float = 20.0) -> dict:
    import oracle
    threads = min(16, os.cpu_count() or 1)
    # probe twice (the first call also pays for converting the fields), then
    # size the sample so that it takes about target_s
    n = 1 << 19
    for _ in range(2):
        t0 = time.perf_counter()
        oracle.trace(wl.fields, wl.sza, wl.azimuth, n, 123, brick=wl.brick, nthreads=threads)
        dt = time.perf_counter() - t0
    n2 = n
    while n2 < wl.photons and dt * (n2 * 2) / n < target_s:
        n2 *= 2
    t0 = time.perf_counter()
    r = oracle.trace(wl.fields, wl.sza, wl.azimuth, n2, 123, brick=wl.brick, nthreads=threads)
    dt = time.perf_counter() - t0
    st = dict(zip(oracle.STATS, r["stats"].tolist()))
    ev = st["collisions"] + st["surface"]
    return {"value": ev / dt, "unit": "photon events/s", "cores": threads, "kind": "oracle",
            "sample": f"{n2} photons of the same 256x256x128 cumulus workload (FP64 C oracle, "
                      f"{threads} threads, {dt:.1f} s, {ev / n2:.1f} events/photon)",
            "photons_per_s": n2 / dt}


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
    singles = [syn.BatchedMedium(m.grid, m.k_gas[n:n + 1], m.ssa_gas[n:n + 1], m.k_cloud, m.ssa_cloud,
                                 m.g_cloud, m.albedo, m.weights[n:n + 1]) for n in range(m.n_gpoints)]
    dsingles = [rt3d.DeviceBatchedMedium(m.grid, dm.k_gas[n:n + 1].contiguous(), dm.ssa_gas[n:n + 1].contiguous(),
                                         dm.k_cloud, dm.ssa_cloud, dm.g_cloud, dm.albedo)
                for n in range(m.n_gpoints)]
    del singles
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


def entry_measurement(reps: int = 4) -> dict:
    """Scrambled-Sobol against independent entry positions at equal photon
    counts on the benchmark field: relative RMS error (the reference's own
    noise removed, reference = two independent halves of 1024 photons per
    column each) of the direct and diffuse surface irradiance and of the
    absorbed power per cell, at 16, 64 and 256 photons per column (RMS of
    `reps` seeds)."""
    import torch
    from paper_2208_05247_amd import rt3d
    from paper_2208_05247_amd import synthetic as syn
    from paper_2208_05247_amd.experiment import eps_against

    wl = syn.les_cumulus()
    grid = wl.fields.grid
    df = rt3d.DeviceFields.from_host(wl.fields)
    out = rt3d.alloc_tallies(grid)
    ws = rt3d.alloc_workspace(rt3d.workspace_size(grid, rt3d.options(brick=wl.brick)))

    def run(photons, seed, sob):
        raw = rt3d.trace(df, wl.sza, wl.azimuth, photons, seed, brick=wl.brick, out=out, workspace=ws,
                         sobol_entry=sob)
        fin = rt3d.finalize(grid, raw, photons)
        return {"sfc_dir": fin["sfc_dir"].double(), "sfc_dif": fin["sfc_dif"].double(),
                "absorbed": (fin["abs_dir"].double() + fin["abs_dif"].double())}

    ncol = grid.nx * grid.ny
    ref_a = run(1024 * ncol, 90001, False)
    ref_b = run(1024 * ncol, 90002, False)
    res = {"workload": "les_cumulus_256x256x128", "reference_photons_per_column": 2048, "seeds": reps}
    for per in (16, 64, 256):
        row = {}
        for sob in (False, True):
            acc = {k: 0.0 for k in ref_a}
            for r in range(reps):
                h = run(per * ncol, 1000 * per + r, sob)
                for k in acc:
                    acc[k] += eps_against(h[k], ref_a[k], ref_b[k]) ** 2 / reps
            row["sobol" if sob else "independent"] = {k: v ** 0.5 for k, v in acc.items()}
        row["error_ratio"] = {k: row["sobol"][k] / row["independent"][k] for k in ref_a}
        res[str(per)] = row
    torch.cuda.synchronize()
    return res


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


def denoiser_measurement(reps: int = 3) -> dict:
    """Inference time of the denoiser on the 1024x1024x128 evaluation grid
    (random weights; time does not depend on them) and its MFMA roofline:
    algorithmic FLOPs of the network as defined (first layer: its 4 real
    input channels; head: its 2 real outputs) over the wall time of one
    inference (features, every convolution, pooling, residual head)."""
    import torch
    from paper_2208_05247_amd import denoise as dn

    D, H, W = 128, 1024, 1024
    net = dn.Denoiser(base=32, seed=0)
    g = torch.Generator(device="cuda").manual_seed(1)
    hd = torch.rand(D, H, W, device="cuda", generator=g)
    hf = torch.rand(D, H, W, device="cuda", generator=g)
    ke = torch.rand(D, H, W, device="cuda", generator=g) * 0.01
    flops = 0.0
    for L in net.layers:
        level = {"e0": 0, "e1": 1, "e2": 2, "b": 3, "d2": 2, "d1": 1, "d0": 0, "head": 0}[L.name]
        cin = 4 if L.name == "e0" else L.c1 + L.c2
        cout = dn.NOUT if L.name == "head" else L.cout
        flops += 2.0 * L.ksize ** 3 * cin * cout * (D * H * W) / 8 ** level
    dn.denoise(net, hd, hf, ke, 0.1 * ke, 20.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dn.denoise(net, hd, hf, ke, 0.1 * ke, 20.0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    achieved = flops / (ms * 1e-3) / 1e12
    return {"grid": [D, H, W], "parameters": net.n_params(), "ms_per_inference": ms,
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "flops_per_call": flops}}


# Merged tally atomics per tentative collision of the tracer on the benchmark
# field: 31.2 per photon against 44.4 tentative collisions (0.70 ~ 11/16).
ACCESS_ATOMICS_PER_16 = 11


def access_ceiling(ncell: int, collisions_per_launch: float, kernel_ms=None, reps: int = 2) -> dict:
    """What the memory system delivers for the tracer's access pattern on
    the benchmark's footprint (ncell 16-byte records, 2 x ncell uint64
    tallies): rt3d_access_probe with as many dependent random gathers as the
    tracer makes tentative collisions per launch, 11 of 16 followed by a
    random 64-bit atomic add, and once without the atomics; the tracer's
    collision rate as a fraction of that ceiling (when kernel_ms is given)."""
    import torch
    from paper_2208_05247_amd import rt3d
    g = torch.Generator(device="cuda").manual_seed(3)
    rec = torch.rand((ncell, 4), generator=g, device="cuda", dtype=torch.float32)
    tally = torch.zeros(2 * ncell, dtype=torch.int64, device="cuda")
    lanes = int(rt3d.load().rt3d_access_probe_lanes(0))
    events = max(1, int(round(collisions_per_launch / lanes)))
    rt3d.access_probe(rec, tally, 64, ACCESS_ATOMICS_PER_16, seed=1)
    torch.cuda.synchronize()
    rates = {}
    for name, a16 in (("with_atomics", ACCESS_ATOMICS_PER_16), ("gathers_only", 0)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for r in range(reps):
            rt3d.access_probe(rec, tally, events, a16, seed=r + 2)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rates[name] = (ms, lanes * events / (ms * 1e-3))
    res = {"lanes": lanes, "gathers_per_lane": events, "atomics_per_16": ACCESS_ATOMICS_PER_16,
           "records_bytes": ncell * 16, "tally_bytes": 2 * ncell * 8,
           "probe_ms": rates["with_atomics"][0], "ceiling_gathers_per_s": rates["with_atomics"][1],
           "gathers_only_per_s": rates["gathers_only"][1]}
    if kernel_ms:
        tracer = collisions_per_launch / (kernel_ms * 1e-3)
        res.update({"tracer_collisions_per_s": tracer, "frac_of_ceiling": tracer / rates["with_atomics"][1]})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=int, default=1 << 26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lds-majorant", type=int, default=0)
    ap.add_argument("--no-merge", action="store_true", help="one tally atomic per deposit")
    ap.add_argument("--sobol-entry", action="store_true", help="scrambled Sobol entry positions")
    ap.add_argument("--refill-lanes", type=int, default=0, help="idle lanes before a wave refills (0 = 16)")
    ap.add_argument("--max-walk", type=int, default=0, help="brick crossings per loop iteration (0 = automatic)")
    ap.add_argument("--inference-only", action="store_true",
                    help="only time denoiser inference on the 1024x1024x128 grid (prints its JSON)")
    ap.add_argument("--access-probe", action="store_true",
                    help="only run the memory-access ceiling probe on the benchmark's footprint (prints its JSON)")
    ap.add_argument("--brick", type=int, default=8)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched g-point measurement")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run one plain device copy of this many bytes (for HBM counter scaling)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy}), flush=True)
        return
    if args.inference_only:
        print(json.dumps({"denoiser_inference": denoiser_measurement()}), flush=True)
        return
    if args.access_probe:
        # the benchmark launch's 2^26 photons x 44.4 events, its 256x256x128 cells
        print(json.dumps({"access_ceiling": access_ceiling(256 * 256 * 128, 44.4 * (1 << 26))}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the tracer is single-GPU (photons or g-points would be "
              "sharded across GPUs with one all-reduce of the tallies; not built here)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_05247_amd import rt3d
    from paper_2208_05247_amd import synthetic as syn

    wl = syn.les_cumulus(photons=args.photons, brick=(args.brick,) * 3)
    grid = wl.fields.grid
    df = rt3d.DeviceFields.from_host(wl.fields, "cuda")
    out = rt3d.alloc_tallies(grid)
    opt = rt3d.options(brick=wl.brick)
    ws = rt3d.alloc_workspace(rt3d.workspace_size(grid, opt))

    def step(seed):
        raw = rt3d.trace(df, wl.sza, wl.azimuth, wl.photons, seed, brick=wl.brick, out=out, workspace=ws,
                         timed=True, lds_majorant=args.lds_majorant, merge=not args.no_merge,
                         sobol_entry=args.sobol_entry, refill_lanes=args.refill_lanes, max_walk=args.max_walk)
        kms = rt3d.last_trace_ms()
        fin = rt3d.finalize(grid, raw, wl.photons)
        return kms, raw["stats"].clone(), fin

    for w in range(args.warmup):
        step(1000 + w)
    torch.cuda.synchronize()
    kernel_ms, stats = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        kms, st, _ = step(k + 1)
        kernel_ms.append(kms)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    tot = {n: 0 for n in rt3d.STATS}
    for st in stats:
        for n, v in zip(rt3d.STATS, st.cpu().tolist()):
            tot[n] += v
    events = tot["collisions"] + tot["surface"]
    ms_per_step = wall * 1e3 / args.steps
    mean_kms = sum(kernel_ms) / len(kernel_ms)
    bytes_per_launch = algorithmic_bytes(tot) / args.steps
    achieved = bytes_per_launch / (mean_kms * 1e-3) / 1e9
    traffic = measured_traffic(wl.brick, wl.photons) \
        if (args.lds_majorant, args.no_merge, args.sobol_entry, args.refill_lanes, args.max_walk) == (0, False, False, 0, 0) \
        else None
    res = {
        "metric": METRIC,
        "value": events / wall,
        "unit": "photon events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [grid.nx, grid.ny, grid.nz],
                   "cell_m": [grid.dx, grid.dy, grid.dz], "photons_per_step": wl.photons,
                   "photons_per_column": wl.photons // grid.ncol, "sza_deg": wl.sza,
                   "brick": list(wl.brick), "parallelism": "single GPU"},
        "photons_per_s": tot["photons"] / wall,
        "events_per_photon": events / max(1, tot["photons"]),
        "trace_kernel_ms": mean_kms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_GBps": None if traffic is None else traffic / (mean_kms * 1e-3) / 1e9,
                     "kernel": "trace_kernel",
                     "bytes_per_launch": bytes_per_launch},
        "paper_context": "A100 40GiB: ~1.9e8 photons/s derived from 90 s for 112 g-points x 256 "
                         "photons/column on 768x768 columns (different fields)",
    }
    if not args.no_batched:
        res["access_ceiling"] = access_ceiling(grid.ncell, tot["collisions"] / args.steps, mean_kms)
        res["batched"] = batched_measurement(max(1, min(args.steps, 3)))
        res["sobol_entry"] = entry_measurement()
        res["two_stream_tod"] = two_stream_measurement()
        res["denoiser_inference"] = denoiser_measurement()
    res["time_to_5pct_heating_rms"] = time_to_5pct()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
