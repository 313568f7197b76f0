"""Batch statistics for comparing Monte Carlo tallies.

Each side runs B independent sub-runs; per quantity the batch mean m and its
standard error s = sd / sqrt(B) are formed, and two estimates agree when
|m1 - m2| <= n_se * sqrt(s1^2 + s2^2).  With B >= 32 batches the t
distribution puts about 2e-4 probability beyond 4 standard errors, so the
bar "at least 99.9 % of cells agree within 4 SE" fails by chance only
rarely.  Quantities with fewer than B/2 non-zero batches on both sides are
too sparse for the batch-mean rule and are compared in aggregates instead.
"""
from __future__ import annotations

import numpy as np


def batch_mean_se(batches: np.ndarray):
    b = np.asarray(batches, dtype=np.float64)
    B = b.shape[0]
    m = b.mean(axis=0)
    s = b.std(axis=0, ddof=1) / np.sqrt(B)
    return m, s


def agree(m, s, exact, n_se=4.0, floor=0.0):
    """|m - exact| <= n_se * s (+ floor) elementwise."""
    return np.abs(np.asarray(m) - exact) <= n_se * np.asarray(s) + floor


def compare_batches(b1: np.ndarray, b2: np.ndarray, n_se: float = 4.0):
    """Per-element comparison of two batch stacks [B, ...].

    Returns (pass_fraction over dense elements, n_dense, n_sparse,
    mask_dense, z-scores)."""
    b1 = np.asarray(b1, dtype=np.float64)
    b2 = np.asarray(b2, dtype=np.float64)
    B1, B2 = b1.shape[0], b2.shape[0]
    m1, s1 = batch_mean_se(b1)
    m2, s2 = batch_mean_se(b2)
    nz1 = (b1 != 0).sum(axis=0)
    nz2 = (b2 != 0).sum(axis=0)
    both_zero = (nz1 == 0) & (nz2 == 0)
    # dense when EITHER side is non-zero in at least half of its batches, so
    # a cell one side always fills and the other never does is tested (and
    # fails) by the batch-mean rule instead of being set aside as sparse
    dense = (nz1 >= B1 / 2) | (nz2 >= B2 / 2)
    se = np.sqrt(s1 * s1 + s2 * s2)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(se > 0, (m1 - m2) / se, np.where(m1 == m2, 0.0, np.inf))
    ok = np.abs(z) <= n_se
    n_dense = int(dense.sum())
    frac = float(ok[dense].mean()) if n_dense else 1.0
    return frac, n_dense, int((~dense & ~both_zero).sum()), dense, z


class RunningBatches:
    """Per-element batch statistics accumulated one batch at a time (for
    grids too large to keep every batch): count, sum, sum of squares and
    the number of non-zero batches, in FP64."""

    def __init__(self, shape):
        self.B = 0
        self.s1 = np.zeros(shape, dtype=np.float64)
        self.s2 = np.zeros(shape, dtype=np.float64)
        self.nz = np.zeros(shape, dtype=np.int32)

    def add(self, x):
        x = np.asarray(x, dtype=np.float64)
        self.B += 1
        self.s1 += x
        self.s2 += x * x
        self.nz += x != 0

    def mean_se(self):
        B = self.B
        m = self.s1 / B
        var = np.maximum(self.s2 - B * m * m, 0.0) / (B - 1)
        return m, np.sqrt(var / B)


def compare_running(r1: RunningBatches, r2: RunningBatches, n_se: float = 4.0):
    """compare_batches for two RunningBatches: (pass fraction over dense
    elements, n_dense, n_sparse, mask_dense, z-scores)."""
    m1, s1 = r1.mean_se()
    m2, s2 = r2.mean_se()
    both_zero = (r1.nz == 0) & (r2.nz == 0)
    dense = (r1.nz >= r1.B / 2) | (r2.nz >= r2.B / 2)
    se = np.sqrt(s1 * s1 + s2 * s2)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(se > 0, (m1 - m2) / se, np.where(m1 == m2, 0.0, np.inf))
    ok = np.abs(z) <= n_se
    n_dense = int(dense.sum())
    frac = float(ok[dense].mean()) if n_dense else 1.0
    return frac, n_dense, int((~dense & ~both_zero).sum()), dense, z
