"""The photon schedule of the work queue (rt3d_schedule_slots, evaluated on
the host by the same decode the tracing kernel runs per refill).  The
schedule only reorders: every (g-point, photon id) pair of a call is handed
out exactly once and enters the column the sampling contract gives it,
(id + o_n) mod (nx*ny) (sec. 2.3, rays start at the top of the domain), so
results cannot depend on it.  Checked by enumeration on small grids, plus
the locality it is for: consecutive slots of the full passes stay inside one
entry tile."""
import numpy as np
import pytest

from paper_2208_05247_amd import rt3d
from paper_2208_05247_amd.synthetic import Grid


def grid(nx, ny):
    return Grid(nx, ny, 4, 10.0, 10.0, 10.0)


def schedule(nx, ny, counts, offs, tile=(0, 0), photon_offset=0):
    opt = rt3d.options(brick=(1, 1, 1), tile=tile, photon_offset=photon_offset)
    return rt3d.schedule_slots(grid(nx, ny), counts, offs, opt)


def check_bijection(nx, ny, counts, offs, tile=(0, 0), photon_offset=0):
    gp, ids, cols = schedule(nx, ny, counts, offs, tile, photon_offset)
    counts = np.asarray(counts, np.int64)
    assert len(gp) == counts.sum()
    # every (g-point, id) pair of the call exactly once
    expected = np.concatenate([np.stack([np.full(c, n), photon_offset + np.arange(c)], axis=1)
                               for n, c in enumerate(counts) if c] or [np.zeros((0, 2), np.int64)])
    got = np.stack([gp.astype(np.int64), ids.astype(np.int64)], axis=1)
    assert np.array_equal(np.unique(got, axis=0), np.unique(expected, axis=0))
    assert len(np.unique(got, axis=0)) == len(got)
    # the column the sampling contract assigns to that id
    ncol = nx * ny
    o = np.asarray(offs, np.int64)[gp]
    assert np.array_equal(cols.astype(np.int64), (ids.astype(np.int64) + o) % ncol)
    return gp, ids, cols


@pytest.mark.parametrize("tile", [(0, 0), (4, 3), (2, 2), (8, 6), (1, 1), (8, 1)])
def test_bijection_uneven_counts(tile):
    # g-points with full passes and a remainder, none, fewer photons than columns
    check_bijection(8, 6, [100, 0, 3, 49, 48, 96], [5, 0, 47, 1, 0, 20], tile)


def test_bijection_random_shapes():
    rng = np.random.default_rng(2208)
    for _ in range(40):
        nx, ny = int(rng.integers(1, 24)), int(rng.integers(1, 24))
        ngp = int(rng.integers(1, 9))
        counts = rng.integers(0, 5 * nx * ny, ngp)
        counts[int(rng.integers(ngp))] += 1
        offs = rng.integers(0, nx * ny, ngp)
        tx = [d for d in range(1, nx + 1) if nx % d == 0]
        ty = [d for d in range(1, ny + 1) if ny % d == 0]
        check_bijection(nx, ny, counts, offs, (int(rng.choice(tx)), int(rng.choice(ty))),
                        int(rng.integers(0, 1 << 40)))


def test_full_passes_are_tile_major():
    """Slots of the full passes: all photons entering tile 0 (of every
    g-point and pass) come first, then tile 1, ...; the left-over photons
    follow in order of k."""
    nx, ny, tx, ty = 16, 12, 4, 3
    counts = [5 * nx * ny + 17, 2 * nx * ny, 40]
    offs = [7, 100, 191]
    gp, ids, cols = check_bijection(nx, ny, counts, offs, (tx, ty))
    full = sum((c // (nx * ny)) * nx * ny for c in counts)
    per_tile = full // ((nx // tx) * (ny // ty))
    tile_of = (cols % nx) // tx + (cols // nx) // ty * (nx // tx)
    expected_tile = np.arange(full) // per_tile
    assert np.array_equal(tile_of[:full], expected_tile)
    # left-over photons: g-point by g-point, ids ascending
    rest_gp, rest_id = gp[full:], ids[full:].astype(np.int64)
    assert np.all(np.diff(rest_gp) >= 0)
    for n in np.unique(rest_gp):
        r = rest_id[rest_gp == n]
        assert np.array_equal(r, np.arange(r[0], r[0] + len(r)))


def tile_of_first_slots(nx, ny, nz, **opt):
    """Entry tile (x, y extent) of the first tile's slots: two full passes of
    one g-point, so the first tile's columns are the first cols until the
    first column repeats."""
    g = Grid(nx, ny, nz, 10.0, 10.0, 10.0)
    _, _, cols = rt3d.schedule_slots(g, [2 * nx * ny], [0], rt3d.options(brick=(1, 1, 1), **opt))
    t = int(np.argmax(cols[1:] == cols[0])) + 1
    xs, ys = cols[:t] % nx, cols[:t] // nx
    return int(xs.max() - xs.min() + 1), int(ys.max() - ys.min() + 1)


def test_automatic_tile_shape():
    """About 128 MiB of records + tallies (nz * 32 B per column) per tile,
    close to square, edges dividing the grid; the whole domain when it holds
    less; a given edge keeps the other automatic."""
    assert tile_of_first_slots(1024, 1024, 128) == (128, 256)    # 32768 columns
    assert tile_of_first_slots(512, 512, 96) == (128, 256)       # 43690 -> 128 x 256
    assert tile_of_first_slots(1000, 1000, 100) == (200, 200)    # 41943 -> divisors of 1000
    assert tile_of_first_slots(96, 10, 16384) == (24, 10)        # 256 columns, y is all of ny: widen x
    assert tile_of_first_slots(32, 32, 64) == (32, 32)           # whole domain holds less
    assert tile_of_first_slots(1024, 1024, 128, tile=(64, 0)) == (64, 512)
    assert tile_of_first_slots(1024, 1024, 128, tile=(0, 32)) == (1024, 32)
    assert tile_of_first_slots(1024, 1024, 128, tile=(16, 8)) == (16, 8)


def test_schedule_argument_checks():
    g = grid(8, 6)
    counts = np.array([10, 5], np.uint64)
    offs = np.array([0, 3], np.uint64)
    with pytest.raises(rt3d.Rt3dError):
        rt3d.schedule_slots(g, counts, offs, rt3d.options(brick=(1, 1, 1), tile=(3, 3)))  # 3 does not divide 8
    with pytest.raises(rt3d.Rt3dError):
        rt3d.schedule_slots(g, counts, offs, rt3d.options(brick=(1, 1, 1), tile=(-1, 0)))
    with pytest.raises(rt3d.Rt3dError):
        rt3d.schedule_slots(g, counts, np.array([0, 48], np.uint64), rt3d.options(brick=(1, 1, 1)))
    with pytest.raises(rt3d.Rt3dError):
        rt3d.schedule_slots(g, counts, offs, rt3d.options(brick=(1, 1, 1)), first_slot=10, n=6)
    gp, ids, cols = rt3d.schedule_slots(g, counts, offs, rt3d.options(brick=(1, 1, 1)), first_slot=15, n=0)
    assert len(gp) == 0
