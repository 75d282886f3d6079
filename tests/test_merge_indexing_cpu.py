"""CPU emulation of the index arithmetic of the merge kernel
(csrc/merge.hip) at small tile sizes: for sorted inputs it reproduces the
oracle's merge; for unsorted inputs (whose order the library leaves
unspecified) every read and write stays inside its buffer and every output
position is written exactly once per tile. This backs the bounds argument
of the kernel without running unsorted inputs on a device."""
import numpy as np
import pytest

from oracle.merge import merge_ranks


def _split(A, B, d, lanes=32):
    """The kernel's split search for one half wave of `lanes` probes."""
    na, nb = len(A), len(B)
    lo, hi = max(0, d - nb), min(d, na)
    while lo < hi:
        step = 1
        while step * (lanes - 1) < hi - lo:
            step <<= 1
        base = lo & ~(step - 1)
        votes = []
        for sub in range(lanes):
            p = base + sub * step
            if p < lo:
                votes.append(True)
            elif p < hi:
                assert 0 <= p < na and 0 <= d - 1 - p < nb
                votes.append(bool(A[p] <= B[d - 1 - p]))
            else:
                votes.append(False)
        c = sum(votes)
        assert c == 0 or base + (c - 1) * step < hi
        nhi = base + c * step
        nlo = max(lo, base + (c - 1) * step + 1) if c > 0 else lo
        assert lo <= nlo <= min(hi, nhi) and (min(hi, nhi) - nlo) < (hi - lo)
        lo, hi = nlo, min(hi, nhi)
    return lo


def _emulate(A, B, threads, vt, lanes):
    na, nb = len(A), len(B)
    total, nv = na + nb, threads * vt
    out = [None] * total
    for blk in range((total + nv - 1) // nv):
        d0, d1 = blk * nv, min(blk * nv + nv, total)
        i0, i1 = _split(A, B, d0, lanes), _split(A, B, d1, lanes)
        i1 = min(max(i1, i0), i0 + (d1 - d0))
        j0, cnt = d0 - i0, d1 - d0
        na_t = i1 - i0
        nb_t = cnt - na_t
        assert 0 <= i0 <= i1 <= na and 0 <= j0 and j0 + nb_t <= nb
        s_t = [A[i0 + e] if e < na_t else B[j0 + e - na_t] for e in range(cnt)]
        src = [None] * cnt
        for tid in range(threads):
            dd = tid * vt
            if dd >= cnt:
                continue
            lo, hi = max(0, dd - nb_t), min(dd, na_t)
            while lo < hi:
                mid = (lo + hi) >> 1
                assert 0 <= mid < na_t and 0 <= dd - 1 - mid < nb_t
                if s_t[mid] <= s_t[na_t + dd - 1 - mid]:
                    lo = mid + 1
                else:
                    hi = mid
            ia, ib = lo, dd - lo
            for r in range(min(vt, cnt - dd)):
                assert ia < na_t or ib < nb_t
                take_a = ib >= nb_t or (ia < na_t and s_t[ia] <= s_t[na_t + ib])
                assert src[dd + r] is None
                src[dd + r] = ("a", ia) if take_a else ("b", ib)
                ia, ib = (ia + 1, ib) if take_a else (ia, ib + 1)
        for e in range(cnt):
            s, k = src[e]
            assert out[d0 + e] is None
            out[d0 + e] = (s, (i0 + k) if s == "a" else (j0 + k))
    return out


@pytest.mark.parametrize("seed", range(8))
def test_emulation_matches_oracle_on_sorted_inputs(seed):
    rng = np.random.default_rng(seed)
    n, m = rng.integers(0, 90, 2)
    A = np.sort(rng.integers(0, 15, n)).astype(float)
    B = np.sort(rng.integers(0, 15, m)).astype(float)
    out = _emulate(A, B, threads=4, vt=3, lanes=4)
    pa, pb = merge_ranks(A, B)
    for k, (s, i) in enumerate(out):
        assert (pa[i] if s == "a" else pb[i]) == k


@pytest.mark.parametrize("seed", range(8))
def test_emulation_stays_in_bounds_on_unsorted_inputs(seed):
    rng = np.random.default_rng(50 + seed)
    n, m = rng.integers(0, 90, 2)
    A = rng.uniform(0, 1, n)
    B = rng.uniform(0, 1, m)
    if seed % 2 and n:
        A[rng.integers(0, n, 3)] = np.nan
    _emulate(A, B, threads=4, vt=3, lanes=4)


def test_split_search_at_kernel_width():
    """The 32-probe search gives the rank definition's split on a large
    sorted input (every diagonal of a coarse sample)."""
    rng = np.random.default_rng(9)
    A = np.sort(rng.integers(0, 5000, 20000)).astype(float)
    B = np.sort(rng.integers(0, 5000, 7000)).astype(float)
    pa, _ = merge_ranks(A, B)
    for d in list(range(0, 27001, 997)) + [27000]:
        assert _split(A, B, d, 32) == int(np.sum(pa < d))
