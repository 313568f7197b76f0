"""rt3d_probe_gathers, the memory-access ceiling the benchmark sets the tracer
against: its dependent gather chains and its atomics are replayed on the host
(numpy, same hash, same FP32 additions) lane by lane, bit for bit, so the
probe is known to do exactly the gathers and atomics it claims."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

C1 = np.uint64(0xbf58476d1ce4e5b9)
C2 = np.uint64(0x94d049bb133111eb)


def mix64(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * C1
        z = (z ^ (z >> np.uint64(27))) * C2
    return z ^ (z >> np.uint64(31))


def replay(rec, n_tally, lanes, events, a16, seed, chains=1, pair=False):
    n = np.uint64(rec.shape[0])
    lane = np.arange(lanes, dtype=np.uint64)
    h = [mix64(np.uint64(seed) ^ mix64(lane * np.uint64(chains) + np.uint64(c + 1))) for c in range(chains)]
    acc = np.zeros(lanes, dtype=np.float32)
    tally = np.zeros(n_tally, dtype=np.int64)
    lo = np.uint64(0xffffffff)
    for e in range(events):
        rows = [((h[c] & lo) * n) >> np.uint64(32) for c in range(chains)]
        for c in range(chains):
            v = rec[rows[c]]
            acc = acc + (v[:, 0] + v[:, 3])
            if pair:
                acc = acc + rec[rows[c] ^ np.uint64(4)][:, 1]
            key = (v[:, 0].view(np.uint32).astype(np.uint64) << np.uint64(32)) | \
                v[:, 1].view(np.uint32).astype(np.uint64)
            h[c] = mix64(h[c] ^ key ^ np.uint64(e))
            if e % 16 < a16:
                np.add.at(tally, ((h[c] >> np.uint64(32)) * np.uint64(n_tally)) >> np.uint64(32), 1)
    return acc, tally


@pytest.fixture(scope="module")
def probe():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_2208_05247_amd import probe as lib
    lib.load()
    return lib


@pytest.mark.parametrize("n_rec,n_tally,events,a16,seed,chains,pair",
                         [(1000, 777, 37, 11, 5, 1, False), (4096, 65536, 20, 16, 9, 1, False),
                          (3, 1, 17, 0, 2, 1, False), (1000, 777, 21, 11, 5, 2, False),
                          (4096, 333, 19, 7, 3, 4, False), (1024, 100, 18, 11, 4, 3, True),
                          (2048, 4096, 9, 0, 6, 1, True)])
def test_probe_replayed_bit_for_bit(probe, n_rec, n_tally, events, a16, seed, chains, pair):
    g = np.random.default_rng(seed)
    rec = g.random((n_rec, 4), dtype=np.float32)
    tally = torch.zeros(n_tally, dtype=torch.int64, device="cuda")
    recd = torch.from_numpy(rec).cuda()
    assert recd.data_ptr() % 128 == 0
    sink = probe.gathers(recd, tally, events, chains, a16, line_pair=pair, grid_blocks=2, seed=seed)
    torch.cuda.synchronize()
    acc, cnt = replay(rec, n_tally, 2048, events, a16, seed, chains, pair)
    assert np.array_equal(sink.cpu().numpy().view(np.uint32), acc.view(np.uint32))
    assert np.array_equal(tally.cpu().numpy(), cnt)
    assert int(cnt.sum()) == 2048 * chains * sum(1 for e in range(events) if e % 16 < a16)


def test_probe_rejects_a_short_sink(probe):
    rec = torch.zeros((16, 4), dtype=torch.float32, device="cuda")
    tally = torch.zeros(16, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1023, dtype=torch.float32, device="cuda")
    import ctypes
    st = probe.load().rt3d_probe_gathers(ctypes.c_void_p(rec.data_ptr()), 16, ctypes.c_void_p(tally.data_ptr()), 16,
                                         4, 1, 11, 0, 1, 1, ctypes.c_void_p(sink.data_ptr()), 1023, None)
    assert st == 1
