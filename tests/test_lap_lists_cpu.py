"""The candidate-list rule of the device assignment's sequential bids,
restated on the CPU and checked against full scans (no GPU, no library).

A scan of row i splits the columns over 1024 threads (thread t takes the
column quads t, t + 1024, ...; the n mod 4 tail columns go to threads 0,
1, ...) grouped in 16 waves of 64. Each thread keeps its best value (lowest
column among equals) and its second value; each wave keeps the K best of
its threads' maxima as candidates and the largest value outside them
(tw): the other threads' maxima and every thread's second value. The bound
is T = max over waves of tw. Later, with prices only risen, a bid that
reads the candidates alone takes their best (v1, j1) and second value v2;
it is accepted when v1 > T and v2 >= T. Accepted bids must equal a full
scan's (v1, j1, v2) exactly, whatever the price rises; the check runs on
integer scores with many ties."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

NT, WAVE = 1024, 64


def _threads(n):
    c4 = n // 4
    j = np.arange(n)
    return np.where(j < 4 * c4, (j // 4) % NT, (j - 4 * c4) % NT)


def _full(V):
    v1 = V.max()
    j1 = int(np.flatnonzero(V == v1)[0])
    rest = np.delete(V, j1)
    return v1, j1, (rest.max() if rest.size else None)


def _lists(V, K):
    n = V.shape[0]
    thr = _threads(n)
    cand, T = [], None
    for w in range(NT // WAVE):
        lanes = []
        for t in range(w * WAVE, (w + 1) * WAVE):
            cols = np.flatnonzero(thr == t)
            if cols.size == 0:
                continue
            vals = V[cols]
            b = int(np.argmax(vals))          # first maximum: the lowest column
            second = np.delete(vals, b).max() if cols.size > 1 else None
            lanes.append((vals[b], int(cols[b]), second))
        lanes.sort(key=lambda e: (-e[0], e[1]))
        cand += [e[1] for e in lanes[:K]]
        outside = [e[0] for e in lanes[K:]] + [e[2] for e in lanes if e[2] is not None]
        if outside:
            T = max(outside) if T is None else max(T, max(outside))
    return np.array(cand), T


@settings(max_examples=30, deadline=None)
@given(seed=st.integers(0, 10_000), n=st.integers(2, 3000), K=st.sampled_from([2, 4]),
       levels=st.sampled_from([3, 50, 10**6]))
def test_accepted_list_bids_equal_full_scans(seed, n, K, levels):
    rng = np.random.default_rng(seed)
    c = rng.integers(0, levels, n).astype(np.int64) * (n + 1)
    price = rng.integers(0, levels, n).astype(np.int64)
    cand, T = _lists(c - price, K)
    accepted = 0
    for _ in range(20):
        # prices only rise: a few objects by random amounts, ties included
        k = rng.integers(1, max(2, n // 10))
        idx = rng.choice(n, k, replace=False)
        price[idx] += rng.integers(0, 3 * (n + 1), k)
        V = c - price
        vals = V[cand]
        order = np.lexsort((cand, -vals))
        v1, j1 = vals[order[0]], int(cand[order[0]])
        v2 = vals[order[1]] if cand.size > 1 else None
        if T is None:
            # every column is a candidate
            assert (v1, j1, v2) == _full(V)
            accepted += 1
        elif v2 is not None and v1 > T and v2 >= T:
            assert (v1, j1, v2) == _full(V)
            accepted += 1
    # the bound never lets a column outside the list beat it
    outside = np.setdiff1d(np.arange(n), cand)
    if outside.size and T is not None:
        assert (c - price)[outside].max() <= T


def test_bound_covers_every_column_outside_the_list():
    rng = np.random.default_rng(7)
    for n in (5, 64, 1000, 4099, 10000):
        V = rng.integers(0, 1000, n).astype(np.int64)
        cand, T = _lists(V, 4)
        assert len(set(cand.tolist())) == cand.size
        outside = np.setdiff1d(np.arange(n), cand)
        if outside.size:
            assert V[outside].max() <= T
        # the list holds the row's best column (lowest among equals)
        assert _full(V)[1] in set(cand.tolist())
