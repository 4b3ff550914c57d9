"""Randomized receiver selection (host logic, no GPU): one receiver from each
contiguous subset, seeded and reproducible, new draws per selection, and the
reuse schedule."""
import numpy as np
import pytest

import synth
from paper_2512_16642_amd import randomized as rz


def test_subsets_partition_the_receivers():
    for nr, k in [(273, 100), (450, 100), (200, 100), (16, 4), (7, 7), (10, 1)]:
        parts = rz.subsets(nr, k)
        assert len(parts) == k
        assert parts[0][0] == 0 and parts[-1][1] == nr
        sizes = [b - a for a, b in parts]
        assert max(sizes) - min(sizes) <= 1 and min(sizes) >= 1
        assert all(parts[i][1] == parts[i + 1][0] for i in range(k - 1))


def test_one_receiver_per_subset_and_reproducible():
    nr, k = 273, 100
    sel = rz.select(nr, k, seed=7, draw=3)
    assert len(sel) == k and np.all(np.diff(sel) > 0)
    for (a, b), r in zip(rz.subsets(nr, k), sel):
        assert a <= r < b
    np.testing.assert_array_equal(sel, rz.select(nr, k, seed=7, draw=3))
    assert not np.array_equal(sel, rz.select(nr, k, seed=7, draw=4))
    assert not np.array_equal(sel, rz.select(nr, k, seed=8, draw=3))


def test_draws_cover_every_receiver_uniformly():
    # every receiver of a 3-receiver subset is drawn with probability 1/3
    nr, k, n = 30, 10, 3000
    counts = np.zeros(nr)
    for d in range(n):
        counts[rz.select(nr, k, seed=1, draw=d)] += 1
    assert counts.min() > 0
    np.testing.assert_allclose(counts / n, 1.0 / 3.0, atol=0.035)


def test_reuse_schedule():
    s = synth.tiny()
    h = rz.RandomizedHessian(s, n_subsets=4, reuse=5, seed=2)
    sels = [tuple(h.selection(it)) for it in range(15)]
    assert len(set(sels[0:5])) == 1 and len(set(sels[5:10])) == 1
    assert sels[0] != sels[5] or sels[5] != sels[10]
    sub = h.subset_spec(np.array(sels[0]))
    assert sub.nr == 4 and sub.rec_ix == tuple(s.rec_ix[i] for i in sels[0])


def test_bad_arguments():
    with pytest.raises(ValueError):
        rz.subsets(5, 6)
    with pytest.raises(ValueError):
        rz.RandomizedHessian(synth.tiny(), 4, reuse=0)
