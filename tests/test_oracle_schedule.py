"""Pins of the oracle's memory schedules (which offsets m, with which multiplicity c,
enter the history sum at step k): eqs. (21), (22) and Def. 3.1-3.2 / Prop. 3.1 /
eq. (24) of Sec. 3.2.  Checked against hand-derived worked lists (tests/golden)
and against brute-force enumerations written from the definitions."""
import os

import numpy as np
import pytest

import oracle
from paper_1004_5128_amd import workloads as W


def load_worked(golden_dir):
    cases = []
    with open(os.path.join(golden_dir, "adaptive_schedules.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, terms = line.split(":", 1)
            rule, a, k = head.split()
            ms, cs = [], []
            for t in terms.split():
                m, c = t.split(":")
                ms.append(int(m))
                cs.append(float(c))
            cases.append((rule, int(a), int(k), ms, cs))
    return cases


def test_worked_schedules(golden_dir):
    cases = load_worked(golden_dir)
    assert len(cases) >= 9
    for rule, a, k, ms, cs in cases:
        gm, gc = oracle.schedule(W.memory("adaptive", a=a, rule=rule), k)
        assert gm.tolist() == ms, (rule, a, k)
        assert gc.tolist() == cs, (rule, a, k)


def brute_partition(a, k):
    """Region by region: the points of (a^(i-1), min(a^i,k)] split into consecutive groups
    of 2i-1; a whole group is represented by its middle point, a short last group point by
    point."""
    terms = [(m, 1) for m in range(0, min(a, k) + 1)]
    lo, i = a, 2
    while lo < k:
        hi = min(a ** i, k)
        pts = list(range(lo + 1, hi + 1))
        d = 2 * i - 1
        groups = [pts[s:s + d] for s in range(0, len(pts), d)]
        for g in groups:
            if len(g) == d:
                terms.append((g[d // 2], d))
            else:
                terms.extend((m, 1) for m in g)
        lo, i = a ** i, i + 1
    return terms


def brute_literal(a, k):
    """Prop. 3.1 read literally: medians a^(i-1) + (2i-1) eta - i + 1 for eta = 1, 2, ...
    inside I_i = [a^(i-1)+i, a^i]; in the interval holding k only medians whose
    increment (median +- (i-1)) ends by k; then the tail up to k."""
    terms = [(m, 1) for m in range(0, min(a, k) + 1)]
    if k <= a:
        return terms
    end = a
    i = 2
    while True:
        meds = []
        eta = 1
        while True:
            m = a ** (i - 1) + (2 * i - 1) * eta - i + 1
            if m > a ** i:
                break
            meds.append(m)
            eta += 1
        last = k <= a ** i
        if last:
            meds = [m for m in meds if m + i - 1 <= k]
        terms.extend((m, 2 * i - 1) for m in meds)
        if meds:
            end = meds[-1] + i - 1
        if last:
            terms.extend((p, 1) for p in range(end + 1, k + 1))
            return terms
        i += 1


@pytest.mark.parametrize("a", [2, 3, 4, 5, 7, 10])
def test_partition_matches_brute_force(a):
    for k in list(range(0, 400)) + [999, 1000, 1001, 4097, 20000]:
        ms, cs = oracle.schedule(W.memory("adaptive", a=a), k)
        assert list(zip(ms.tolist(), cs.astype(int).tolist())) == brute_partition(a, k), (a, k)


@pytest.mark.parametrize("a", [2, 3, 4, 5, 7, 10])
def test_literal_matches_brute_force(a):
    for k in list(range(0, 400)) + [999, 1000, 1001, 4097, 20000]:
        ms, cs = oracle.schedule(W.memory("adaptive", a=a, rule="literal"), k)
        assert list(zip(ms.tolist(), cs.astype(int).tolist())) == brute_literal(a, k), (a, k)


@pytest.mark.parametrize("a", [2, 3, 4, 10])
def test_partition_covers_every_offset_once(a):
    # Each sample stands for the (c-1)/2 points on either side of it; under the partition
    # reading those increments tile 0..k exactly, so the history keeps "contributions from
    # the entire past" (abstract, Sec. 3.2) and sum(c) = k + 1.
    for k in (0, 1, 5, 17, 64, 100, 333, 2048, 20000):
        ms, cs = oracle.schedule(W.memory("adaptive", a=a), k)
        cover = np.zeros(k + 1, int)
        for m, c in zip(ms, cs.astype(int)):
            h = (c - 1) // 2
            cover[m - h:m + h + 1] += 1
        assert np.all(cover == 1)
        assert np.all(np.diff(ms) > 0)


def test_literal_overlaps_and_gaps_are_possible():
    # The literal reading double counts some offsets: a = 2, k = 12 counts offset 5 twice.
    ms, cs = oracle.schedule(W.memory("adaptive", a=2, rule="literal"), 12)
    assert cs.sum() == 14


@pytest.mark.parametrize("k", [0, 1, 7, 100, 1234])
def test_degenerate_schedules_equal_full(k):
    fm, fc = oracle.schedule(W.memory("full"), k)
    assert fm.tolist() == list(range(k + 1)) and np.all(fc == 1)
    for mem in (W.memory("short", L=k), W.memory("short", L=k + 10 ** 6),
                W.memory("adaptive", a=max(k, 2)), W.memory("adaptive", a=3, rule="unit_stride"),
                W.memory("adaptive", a=2, rule="unit_stride")):
        ms, cs = oracle.schedule(mem, k)
        assert np.array_equal(ms, fm) and np.array_equal(cs, fc), mem


def test_short_window():
    ms, cs = oracle.schedule(W.memory("short", L=1000), 20000)
    assert ms.tolist() == list(range(1001)) and np.all(cs == 1)
    ms, cs = oracle.schedule(W.memory("short", L=0), 50)
    assert ms.tolist() == [0] and cs.tolist() == [1.0]


def test_adaptive_term_counts_are_logarithmic():
    # Sampled terms grow like sum_i a^(i-1)(a-1)/(2i-1): far fewer than k + 1.
    for a in (2, 4, 10):
        n20k = len(oracle.schedule(W.memory("adaptive", a=a), 20000)[0])
        assert n20k < 20001 / 5
