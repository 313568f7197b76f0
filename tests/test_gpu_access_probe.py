"""rt3d_access_probe, the memory-access ceiling the benchmark sets the tracer
against: its dependent gather chain and its atomics are replayed on the host
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


def replay(rec, n_tally, lanes, events, a16, seed):
    n = np.uint64(rec.shape[0])
    lane = np.arange(lanes, dtype=np.uint64)
    h = mix64(np.uint64(seed) ^ mix64(lane + np.uint64(1)))
    acc = np.zeros(lanes, dtype=np.float32)
    tally = np.zeros(n_tally, dtype=np.int64)
    lo = np.uint64(0xffffffff)
    for e in range(events):
        c = rec[((h & lo) * n) >> np.uint64(32)]
        acc = acc + (c[:, 0] + c[:, 3])
        key = (c[:, 0].view(np.uint32).astype(np.uint64) << np.uint64(32)) | c[:, 1].view(np.uint32).astype(np.uint64)
        h = mix64(h ^ key ^ np.uint64(e))
        if e % 16 < a16:
            np.add.at(tally, ((h >> np.uint64(32)) * np.uint64(n_tally)) >> np.uint64(32), 1)
    return acc, tally


@pytest.fixture(scope="module")
def rt3d():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_2208_05247_amd import rt3d as lib
    lib.load()
    return lib


@pytest.mark.parametrize("n_rec,n_tally,events,a16,seed", [(1000, 777, 37, 11, 5), (4096, 65536, 20, 16, 9),
                                                           (3, 1, 17, 0, 2)])
def test_access_probe_replayed_bit_for_bit(rt3d, n_rec, n_tally, events, a16, seed):
    g = np.random.default_rng(seed)
    rec = g.random((n_rec, 4), dtype=np.float32)
    tally = torch.zeros(n_tally, dtype=torch.int64, device="cuda")
    sink = rt3d.access_probe(torch.from_numpy(rec).cuda(), tally, events, a16, grid_blocks=2, seed=seed)
    torch.cuda.synchronize()
    acc, cnt = replay(rec, n_tally, 2048, events, a16, seed)
    assert np.array_equal(sink.cpu().numpy().view(np.uint32), acc.view(np.uint32))
    assert np.array_equal(tally.cpu().numpy(), cnt)
    assert int(cnt.sum()) == 2048 * sum(1 for e in range(events) if e % 16 < a16)


def test_access_probe_rejects_a_short_sink(rt3d):
    rec = torch.zeros((16, 4), dtype=torch.float32, device="cuda")
    tally = torch.zeros(16, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1023, dtype=torch.float32, device="cuda")
    import ctypes
    st = rt3d.load().rt3d_access_probe(ctypes.c_void_p(rec.data_ptr()), 16, ctypes.c_void_p(tally.data_ptr()), 16,
                                       4, 11, 1, 1, ctypes.c_void_p(sink.data_ptr()), 1023, None)
    assert st == rt3d.EINVAL
