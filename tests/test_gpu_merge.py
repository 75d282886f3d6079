"""GPU merge of test times into the training grid (pssgp_merge_times)
against the oracle's rank definition (oracle/merge.py): bit-exact times,
masks, values and positions, at sizes spanning many 2048-output tiles with
ragged tails, with heavy ties, empty sides, all-equal times, and the full
rbf6_lognormal grid split into its observed and missing steps and merged
back."""
import numpy as np
import pytest

import workloads as W
from oracle.merge import merge_times as oracle_merge

pytestmark = pytest.mark.gpu


def _P():
    import paper_2102_09964_amd as P
    return P


def _check(tr, te, y, mk, dtype):
    P = _P()
    t, yo, mask, pos = P.merge_times(tr, y, te, mask_train=mk, dtype=dtype)
    t0, y0, m0, p0 = oracle_merge(tr, y, te, mk)
    np.testing.assert_array_equal(t.cpu().numpy(), t0)
    np.testing.assert_array_equal(mask.cpu().numpy(), m0)
    np.testing.assert_array_equal(pos.cpu().numpy(), p0)
    if y is None:
        assert yo is None
    else:
        np.testing.assert_array_equal(yo.cpu().numpy(), y0)


SIZES = [(0, 0), (0, 5), (5, 0), (1, 1), (2047, 1), (2048, 0), (1, 2048), (3000, 5001), (20000, 7)]


@pytest.mark.parametrize("n,m", SIZES)
@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_merge_vs_oracle(n, m, dtype):
    rng = np.random.default_rng(n * 7919 + m)
    tr = np.sort(rng.uniform(0, 10, n))
    te = np.sort(rng.uniform(0, 10, m))
    y = rng.normal(size=n).astype(np.float32 if dtype == "float32" else np.float64)
    mk = (rng.uniform(size=n) > 0.25).astype(np.uint8)
    print("merge", n, m, dtype, flush=True)
    _check(tr, te, y, mk, dtype)
    _check(tr, te, None, None, dtype)


@pytest.mark.parametrize("seed", range(3))
def test_merge_heavy_ties(seed):
    """Times on a coarse integer grid: long runs of equal times inside and
    across the sequences, crossing tile boundaries."""
    rng = np.random.default_rng(100 + seed)
    n, m = 9000 + 1000 * seed, 7000 - 1500 * seed
    tr = np.sort(rng.integers(0, 40, n)).astype(float)
    te = np.sort(rng.integers(0, 40, m)).astype(float)
    y = rng.normal(size=n).astype(np.float32)
    _check(tr, te, y, None, "float32")


def test_merge_all_equal_times():
    tr, te = np.full(3000, 2.5), np.full(2500, 2.5)
    _check(tr, te, np.arange(3000, dtype=np.float32), None, "float32")


def test_merge_full_size_split_and_merge_back():
    """rbf6_lognormal (2^22 steps, 20% missing): merging the missing steps
    back into the observed ones gives the original grid, bit for bit."""
    P = _P()
    w = W.rbf6_lognormal()
    obs = w["mask"] == 1
    tr, te = w["t"][obs], w["t"][~obs]
    y = w["y"][obs].astype(np.float32)
    t, yo, mask, pos = P.merge_times(tr, y, te, dtype="float32")
    np.testing.assert_array_equal(t.cpu().numpy(), w["t"])
    np.testing.assert_array_equal(mask.cpu().numpy(), w["mask"])
    np.testing.assert_array_equal(pos.cpu().numpy(), np.flatnonzero(~obs))
    yh = yo.cpu().numpy()
    np.testing.assert_array_equal(yh[obs], y)
    assert np.all(yh[~obs] == 0)
