"""Pins of the oracle's merged time grid (oracle/merge.py) against what
fixes it independently: a worked example with ties (tests/golden/
merge_ties.txt), a two-pointer merge written out step by step, and Python's
stable sort with an explicit key."""
import os

import numpy as np
import pytest

from oracle.merge import merge_ranks, merge_times

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "merge_ties.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        rows[k] = v
    return rows


def test_worked_example_with_ties():
    g = _golden()
    tr = np.array(g["t_train"], float)
    te = np.array(g["t_test"], float)
    y = np.arange(1, tr.size + 1, dtype=np.float64) * 10.0
    t, ym, mask, pos = merge_times(tr, y, te)
    np.testing.assert_array_equal(t, np.array(g["t"], float))
    np.testing.assert_array_equal(pos, np.array(g["test_pos"], int))
    for k, s in enumerate(g["src"]):
        if s[0] == "r":
            assert mask[k] == 1 and ym[k] == y[int(s[1:])]
        else:
            assert mask[k] == 0 and ym[k] == 0.0


def _two_pointer(tr, te):
    """Stable merge by walking both sequences (training first at ties)."""
    out, i, j = [], 0, 0
    while i < len(tr) or j < len(te):
        if j == len(te) or (i < len(tr) and tr[i] <= te[j]):
            out.append(("r", i))
            i += 1
        else:
            out.append(("s", j))
            j += 1
    return out


@pytest.mark.parametrize("seed", range(6))
def test_ranks_match_two_pointer_and_stable_sort(seed):
    rng = np.random.default_rng(seed)
    n, m = rng.integers(0, 60, 2)
    # a coarse grid makes ties frequent, within and across the sequences
    tr = np.sort(rng.integers(0, 12, n)).astype(float)
    te = np.sort(rng.integers(0, 12, m)).astype(float)
    pr, pt = merge_ranks(tr, te)
    walk = _two_pointer(tr, te)
    for k, (s, idx) in enumerate(walk):
        assert (pr[idx] if s == "r" else pt[idx]) == k
    # stable sort of the union by (time, training before test, index)
    key = sorted([(tr[i], 0, i) for i in range(n)] + [(te[j], 1, j) for j in range(m)])
    for k, (_, s, idx) in enumerate(key):
        assert (pr[idx] if s == 0 else pt[idx]) == k


def test_properties_and_degenerate_cases():
    rng = np.random.default_rng(7)
    tr = np.sort(rng.uniform(0, 1, 500))
    te = np.sort(rng.uniform(0, 1, 300))
    mk = (rng.uniform(size=500) > 0.3).astype(np.uint8)
    t, y, mask, pos = merge_times(tr, np.ones(500, np.float32), te, mk)
    assert np.all(np.diff(t) >= 0)
    np.testing.assert_array_equal(t[pos], te)
    assert mask.sum() == mk.sum() and y.dtype == np.float32 and y.sum() == 500
    # empty sides, and all times equal (training block first)
    t, y, mask, pos = merge_times(np.zeros(0), None, te)
    assert y is None and np.all(mask == 0) and np.array_equal(pos, np.arange(300))
    t, y, mask, pos = merge_times(tr, None, np.zeros(0))
    assert np.all(mask == 1) and pos.size == 0 and np.array_equal(t, tr)
    t, y, mask, pos = merge_times(np.zeros(4), None, np.zeros(3))
    np.testing.assert_array_equal(mask, [1, 1, 1, 1, 0, 0, 0])
    np.testing.assert_array_equal(pos, [4, 5, 6])


def test_split_and_merge_back_reproduces_a_grid():
    """Splitting a sorted grid without ties into its observed and missing
    steps and merging them back gives the grid."""
    rng = np.random.default_rng(3)
    t0 = np.cumsum(rng.lognormal(np.log(0.01), 1.0, 4000))
    m0 = (rng.uniform(size=4000) >= 0.2).astype(np.uint8)
    t, _, mask, pos = merge_times(t0[m0 == 1], None, t0[m0 == 0])
    np.testing.assert_array_equal(t, t0)
    np.testing.assert_array_equal(mask, m0)
    np.testing.assert_array_equal(pos, np.flatnonzero(m0 == 0))
