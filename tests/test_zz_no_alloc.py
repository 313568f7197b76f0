"""rt3d_trace_noalloc: rt3d_trace with the library's static device scratch
as its workspace, for callers that cannot allocate.

On the GPU its raw uint64 tallies, ledger and counters must equal those of
rt3d_trace (caller workspace) bit for bit, on two calls in a row whose
second has a smaller grid (the scratch still holds the first call's
contents).  On the CPU: the host-side rejections (a grid whose workspace
exceeds the scratch, the timing flag) return before any HIP call."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2208_05247_amd import rt3d as r  # noqa: E402
from paper_2208_05247_amd import synthetic as syn  # noqa: E402

KEYS = r.TALLY3 + r.TALLY2 + ("ledger", "stats")


def _raw_call(grid, flags=0):
    lib = r.load()
    opt = r.options(brick=(8, 8, 8), flags=flags)
    gs = r.grid_struct(grid)
    return lib.rt3d_trace_noalloc(ctypes.byref(gs), None, None, 30.0, 0.0, 1 << 10, 1, ctypes.byref(opt), None,
                                  None)


def test_noalloc_rejects_oversize_grid_on_host():
    # 256 x 256 x 128 cells: 128 MiB of packed records, beyond the 32 MiB scratch
    grid = syn.Grid(256, 256, 128, 50.0, 50.0, 25.0)
    assert r.workspace_size(grid, r.options(brick=(8, 8, 8))) > r.NOALLOC_SCRATCH_BYTES
    assert _raw_call(grid) == r.ETOOBIG
    assert "32" in r.load().rt3d_last_device_error().decode() or "scratch" in \
        r.load().rt3d_last_device_error().decode()


def test_noalloc_rejects_timing_flag_on_host():
    grid = syn.Grid(32, 32, 64, 100.0, 100.0, 50.0)
    assert _raw_call(grid, flags=r.FLAG_TIME) == r.EINVAL


@pytest.mark.gpu
def test_noalloc_matches_trace_bitwise_twice():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    big = syn.small_cumulus()
    small_grid = syn.Grid(16, 8, 24, 100.0, 100.0, 50.0)
    small = syn.random_fields(small_grid, seed=5, k_max=0.01, albedo_range=(0.1, 0.4))
    cases = [(big.fields, big.sza, big.azimuth, 1 << 18, 11, big.brick, 0.0),
             (small, 50.0, 120.0, 1 << 16, 12, (4, 4, 4), 0.3)]
    for fields, sza, az, photons, seed, brick, fd in cases:
        print(f"noalloc case: grid {fields.grid.shape3}, {photons} photons, seed {seed}", flush=True)
        df = r.DeviceFields.from_host(fields, "cuda")
        ref = r.trace(df, sza, az, photons, seed, brick=brick, diffuse_fraction=fd)
        got = r.trace_noalloc(df, sza, az, photons, seed, r.alloc_tallies(fields.grid), brick=brick,
                              diffuse_fraction=fd)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(got[k], ref[k]), k
        led = [int(v) for v in r.as_uint64(got["ledger"])]
        assert led[0] == photons * 2 ** 31
        assert led[0] + led[5] == sum(led[1:5]) + led[6] + led[7]
