"""The autotuner's search logic on the host, with a synthetic tracer: the
acceleration-cell stage minimises kernel time times tally variance (the Monte
Carlo cost, time to a given error ~ time per photon x variance per photon),
the stages that only reorder work minimise time."""
import torch

from paper_2208_05247_amd import autotune
from paper_2208_05247_amd.synthetic import Grid

GRID = Grid(16, 16, 16, 10.0, 10.0, 10.0)
TRUTH = torch.linspace(1.0, 2.0, 16 ** 3, dtype=torch.float64)


def fake_tracer(ms, sd):
    """ms[brick] kernel time, sd[brick] per-cell standard deviation; any
    other option leaves both unchanged except `pool_photons` 1024, which is
    faster."""
    state = {}

    def run(opts, k=0):
        state.update(opts=dict(opts), k=k)
        t = ms[opts["brick"]]
        return t * (0.9 if opts.get("pool_photons") == 1024 else 1.0)

    def heat():
        g = torch.Generator().manual_seed(1000 + state["k"])
        return TRUTH + sd[state["opts"]["brick"]] * torch.randn(TRUTH.shape, generator=g, dtype=torch.float64)

    return run, heat


def search(ms, sd):
    run, heat = fake_tracer(ms, sd)
    return autotune._search(run, heat, GRID, 1 << 20, bricks=list(ms), walks=[0], pools=[256, 1024],
                            grid_mults=(), try_merge=False, refills=[16], tiles=[(16, 16)])


def test_cell_stage_weighs_variance():
    # 4x4x4 is 10 % faster per photon but 30 % noisier (sd): cost 0.9 x 1.69 > 1.0
    best, best_ms, table = search({(4, 4, 4): 0.9, (8, 8, 8): 1.0}, {(4, 4, 4): 1.3, (8, 8, 8): 1.0})
    assert best["brick"] == (8, 8, 8) and best["pool_photons"] == 1024
    rows = {tuple(r["brick"]): r for r in table if "cost" in r}
    n = TRUTH.numel()
    for b, s in ((4, 4, 4), 1.3), ((8, 8, 8), 1.0):
        assert abs(rows[b]["tally_variance"] / (n * s * s) - 1.0) < 0.05
    # the same speed-up at equal noise wins
    best, _, _ = search({(4, 4, 4): 0.9, (8, 8, 8): 1.0}, {(4, 4, 4): 1.0, (8, 8, 8): 1.0})
    assert best["brick"] == (4, 4, 4)


def test_noise_of_identical_runs_is_zero():
    assert autotune._noise(TRUTH, TRUTH.clone()) == 0.0
