"""The batch statistics used by the parity tests: the running (one batch at a
time) form equals the stacked form, and a cell that one side fills in every
batch while the other never does is tested, and fails, rather than being set
aside as sparse."""
import numpy as np

from mc_stats import RunningBatches, compare_batches, compare_running


def test_running_equals_stacked():
    rng = np.random.default_rng(0)
    B = 64
    a = rng.gamma(2.0, 1.0, (B, 30, 7)) * (rng.random((B, 30, 7)) < 0.7)
    b = rng.gamma(2.0, 1.0, (B, 30, 7)) * (rng.random((B, 30, 7)) < 0.3)
    ra, rb = RunningBatches(a.shape[1:]), RunningBatches(b.shape[1:])
    for i in range(B):
        ra.add(a[i])
        rb.add(b[i])
    f1, n1, s1, d1, z1 = compare_batches(a, b)
    f2, n2, s2, d2, z2 = compare_running(ra, rb)
    assert (f1, n1, s1) == (f2, n2, s2)
    assert np.array_equal(d1, d2)
    assert np.allclose(z1, z2, rtol=1e-9, atol=1e-12)


def test_one_sided_cell_is_dense_and_fails():
    rng = np.random.default_rng(1)
    B = 64
    a = rng.gamma(2.0, 1.0, (B, 10))
    b = a[::-1].copy()
    b[:, 3] = 0.0          # one side never deposits here
    frac, n_dense, n_sparse, dense, z = compare_batches(a, b)
    assert dense[3] and abs(z[3]) > 4.0
    assert n_dense == 10 and frac == 0.9
