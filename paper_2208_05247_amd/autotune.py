"""Autotuner for the tracer's launch options.

Picks the acceleration-grid cell ("brick") shape, the crossings a lane makes
per loop iteration, the persistent grid size, the photon-id pool a wave takes
per refill, how many idle lanes a wave waits for before it starts new photons,
the tally mode (merging a lane's deposits, wave-aggregated atomics), for
batched launches the cloud-cell mask, and the entry tile of the photon
schedule from short
calibration runs (the tile matters only when the sample holds full passes
over the columns, i.e. at least as many photons per g-point as columns).
Every candidate traces the same photons through the same fields, so the
choice never changes the estimator's expectation.  All options but the
acceleration cell only reorder work (the uint64 tallies are bitwise the
same), and their objective is tracing-kernel time (HIP events around the
kernel).  The acceleration cell also changes the variance: every tentative
collision, null ones included, deposits absorbed weight, so a looser
majorant costs more events per photon but samples the absorption more
often.  Its objective is therefore the Monte Carlo cost, kernel time times
the variance of the heating tallies (their summed squared difference between
two runs with different seeds, halved): the time to a given error is
proportional to it (error ~ N^-1/2, time ~ N, sec. 3.2).  Measured on the
1024x1024x128 field: 4x4x8 cells trace a photon 6 % faster than 8x8x8 but
with 9 % more variance (5 % more cost).

Results are cached in a JSON file keyed by device, library build, grid,
sun geometry and a fingerprint of the fields.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os
from typing import Callable, List, Optional

import numpy as np
import torch

from . import rt3d

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rt3d", "autotune.json")

BRICKS = [(4, 4, 4), (8, 8, 8), (16, 16, 16), (8, 8, 4), (8, 8, 16), (4, 4, 8), (16, 16, 8), (16, 16, 4)]
WALKS = [0, 1, 2, 4, 8]
POOLS = [64, 256, 1024]
REFILLS = [1, 4, 8, 16, 32]
TILES = [(16, 16), (32, 32), (128, 128), (256, 256), "domain"]  # automatic: 64 x 64 (largest divisor <= 64)


@dataclasses.dataclass
class TuneResult:
    options: dict                      # keyword arguments for rt3d.trace / trace_batched
    ms_per_photon: float               # calibration kernel time per photon (ms)
    table: List[dict]                  # every candidate measured
    cached: bool = False


def _divides(grid, b) -> bool:
    return grid.nx % b[0] == 0 and grid.ny % b[1] == 0 and grid.nz % b[2] == 0


def _fingerprint(arrays, extra) -> str:
    h = hashlib.sha256()
    for a in arrays:
        v = a.detach().reshape(-1)
        step = max(1, v.numel() // 4096)
        h.update(v[::step].float().cpu().numpy().tobytes())
    h.update(json.dumps(extra, sort_keys=True).encode())
    return h.hexdigest()[:16]


def _lib_hash() -> str:
    with open(rt3d.LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _noise(h0: torch.Tensor, h1: torch.Tensor) -> float:
    """Summed variance of one run's heating tallies from two independent
    runs: sum over cells of (h0 - h1)^2 / 2."""
    return float(((h0 - h1) ** 2).sum()) / 2.0


def _search(run: Callable[..., float], heat: Callable[[], torch.Tensor], grid, sample: int, bricks=None,
            walks=None, pools=None, grid_mults=(1,), try_merge=True, refills=None, tiles=None,
            try_cell_mask=False):
    """Staged coordinate search; run(opts, k) traces `sample` photons with
    seed offset k and returns the kernel ms, heat() the heating tallies of
    the last run (FP64, abs_dir + abs_dif)."""
    table = []

    def row(opts, **v):
        table.append({**{k: (list(x) if isinstance(x, tuple) else x) for k, x in opts.items()}, **v})

    def measure(opts):
        ms = min(run(opts, 0) for _ in range(2))
        row(opts, kernel_ms=ms, ms_per_photon=ms / sample)
        return ms

    def cost(opts):
        """Kernel ms x tally variance (two seeds)."""
        ms0 = run(opts, 0)
        h0 = heat()
        ms1 = run(opts, 1)
        ms = min(ms0, ms1)
        noise = _noise(h0, heat())
        del h0
        row(opts, kernel_ms=ms, ms_per_photon=ms / sample, tally_variance=noise, cost=ms * noise)
        return ms, ms * noise

    best = {"brick": (8, 8, 8) if _divides(grid, (8, 8, 8)) else (1, 1, 1)}
    best_cost = best_ms = float("inf")
    for b in (bricks or BRICKS):
        if not _divides(grid, b):
            continue
        ms, c = cost({"brick": b})
        if c < best_cost:
            best_cost, best_ms, best = c, ms, {"brick": b}
    for wk in (walks or WALKS):
        if wk == 0:
            continue
        o = {**best, "max_walk": wk}
        ms = measure(o)
        if ms < best_ms:
            best_ms, best = ms, o
    for pool in (pools or POOLS):
        if pool == 256:
            continue
        o = {**best, "pool_photons": pool}
        ms = measure(o)
        if ms < best_ms:
            best_ms, best = ms, o
    for rf in (refills or REFILLS):
        if rf == 16:
            continue
        o = {**best, "refill_lanes": rf}
        ms = measure(o)
        if ms < best_ms:
            best_ms, best = ms, o
    ncu = torch.cuda.get_device_properties(0).multi_processor_count if grid_mults else 0
    for m in grid_mults:   # persistent workgroups per CU below full occupancy
        o = {**best, "grid_blocks": int(ncu * m)}
        ms = measure(o)
        if ms < best_ms:
            best_ms, best = ms, o
    if try_merge:
        for o in ({**best, "merge": False}, {**best, "wave_aggregate": True}):
            ms = measure(o)
            if ms < best_ms:
                best_ms, best = ms, o
    if try_cell_mask:  # batched only: skip the record gather in cloud-free cells
        o = {**best, "cell_mask": True}
        ms = measure(o)
        if ms < best_ms:
            best_ms, best = ms, o
    for t in (tiles or TILES):
        t = (grid.nx, grid.ny) if t == "domain" else t
        if grid.nx % t[0] or grid.ny % t[1]:
            continue
        o = {**best, "tile": tuple(t)}
        ms = measure(o)
        if ms < best_ms:
            best_ms, best = ms, o
    return best, best_ms, table


def tune_trace(df: "rt3d.DeviceFields", sza: float, azimuth: float, sample: int = 1 << 22, seed: int = 77,
               cache_path: Optional[str] = DEFAULT_CACHE, force: bool = False, **search_kw) -> TuneResult:
    """Tune rt3d.trace for these fields and sun; returns the best options."""
    key = "|".join([torch.cuda.get_device_name(0), _lib_hash(), "trace",
                    f"{df.grid.nx}x{df.grid.ny}x{df.grid.nz}",
                    _fingerprint([df.k_ext, df.ssa, df.k_ext_cloud], {"sza": sza, "az": azimuth, "n": sample})])
    cache = _load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        c = cache[key]
        return TuneResult(_opts_from_json(c["options"]), c["ms_per_photon"], c["table"], cached=True)
    out = rt3d.alloc_tallies(df.grid)

    def run(opts, k=0):
        rt3d.trace(df, sza, azimuth, sample, seed + k, out=out, timed=True, **opts)
        return rt3d.last_trace_ms()

    def heat():
        return out["abs_dir"].double() + out["abs_dif"].double()

    search_kw.setdefault("grid_mults", (1,))
    best, best_ms, table = _search(run, heat, df.grid, sample, **search_kw)
    res = TuneResult(best, best_ms / sample, table)
    if cache_path:
        cache[key] = {"options": _opts_to_json(best), "ms_per_photon": res.ms_per_photon, "table": table}
        _store_cache(cache_path, cache)
    return res


def tune_batched(dm: "rt3d.DeviceBatchedMedium", sza: float, azimuth: float, photons, sample: int = 1 << 22,
                 seed: int = 77, cache_path: Optional[str] = DEFAULT_CACHE, force: bool = False,
                 **search_kw) -> TuneResult:
    """Tune rt3d.trace_batched: the calibration uses the g-points' photon
    shares scaled down to `sample` photons in total."""
    counts = np.asarray(photons, dtype=np.float64)
    share = np.floor(counts / counts.sum() * sample).astype(np.uint64)
    share[np.argmax(counts)] += np.uint64(sample - int(share.sum()))
    key = "|".join([torch.cuda.get_device_name(0), _lib_hash(), "batched",
                    f"{dm.grid.nx}x{dm.grid.ny}x{dm.grid.nz}x{dm.n_gpoints}",
                    _fingerprint([dm.k_gas, dm.k_cloud, dm.ssa_gas],
                                 {"sza": sza, "az": azimuth, "n": sample, "share": share.tolist()})])
    cache = _load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        c = cache[key]
        return TuneResult(_opts_from_json(c["options"]), c["ms_per_photon"], c["table"], cached=True)
    out = rt3d.alloc_tallies(dm.grid)

    def run(opts, k=0):
        rt3d.trace_batched(dm, sza, azimuth, share, seed + k, out=out, timed=True, **opts)
        return rt3d.last_trace_ms()

    def heat():
        return out["abs_dir"].double() + out["abs_dif"].double()

    search_kw.setdefault("grid_mults", (3, 4))
    search_kw.setdefault("try_cell_mask", True)
    best, best_ms, table = _search(run, heat, dm.grid, sample, **search_kw)
    res = TuneResult(best, best_ms / sample, table)
    if cache_path:
        cache[key] = {"options": _opts_to_json(best), "ms_per_photon": res.ms_per_photon, "table": table}
        _store_cache(cache_path, cache)
    return res


def _opts_to_json(o: dict) -> dict:
    return {k: (list(v) if isinstance(v, tuple) else v) for k, v in o.items()}


def _opts_from_json(o: dict) -> dict:
    return {k: (tuple(v) if isinstance(v, list) else v) for k, v in o.items()}
