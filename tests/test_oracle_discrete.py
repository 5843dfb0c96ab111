"""Pins of the oracle's permutations and samples (Section 3.2).

Fisher-Yates must give every permutation of n elements with probability 1/n!;
Floyd's algorithm and reservoir sampling must give every k-subset with
probability 1/C(n, k).  Tested by chi-square over all outcomes of small cases
(enumerated), plus validity and inclusion frequencies on larger ones.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import Stream


def _chi2_uniform(counts, total):
    k = len(counts)
    exp = total / k
    chi = sum((c - exp) ** 2 / exp for c in counts)
    return stats.chi2.sf(chi, k - 1)


@pytest.mark.parametrize("n", [3, 4])
def test_permutations_uniform_over_all_orders(n):
    s = Stream.seeded("pcg64", 31)
    idx = {p: i for i, p in enumerate(itertools.permutations(range(n)))}
    counts = [0] * len(idx)
    T = 24000 * len(idx) // 6
    for _ in range(T):
        counts[idx[tuple(int(v) for v in s.permutation(n))]] += 1
    assert _chi2_uniform(counts, T) > 1e-4


def test_permutation_validity_and_positions():
    s = Stream.seeded("philox4x32", 32)
    n, T = 50, 4000
    pos0 = np.zeros(n)
    for _ in range(T):
        p = s.permutation(n)
        assert sorted(p.tolist()) == list(range(n))
        pos0[p[0]] += 1
    # element at position 0 uniform over the n values
    assert stats.chisquare(pos0).pvalue > 1e-4
    assert s.permutation(1).tolist() == [0]


@pytest.mark.parametrize("n,k", [(5, 2), (6, 3), (5, 4), (6, 5)])
def test_samples_uniform_over_all_subsets(n, k):
    """(5, 2) and (6, 3) use Floyd's algorithm, (5, 4) and (6, 5) the
    reservoir."""
    s = Stream.seeded("x256++", 33 + n + k)
    idx = {c: i for i, c in enumerate(itertools.combinations(range(n), k))}
    counts = [0] * len(idx)
    T = 3000 * len(idx)
    for _ in range(T):
        smp = s.sample(n, k)
        assert len(set(smp.tolist())) == k and smp.max() < n
        counts[idx[tuple(sorted(int(v) for v in smp))]] += 1
    assert _chi2_uniform(counts, T) > 1e-4


@pytest.mark.parametrize("n,k", [(1000, 10), (1000, 500), (1000, 501), (1000, 990)])
def test_sample_inclusion_frequencies(n, k):
    s = Stream.seeded("sfc64", 34)
    T = 400
    inc = np.zeros(n)
    for _ in range(T):
        smp = s.sample(n, k)
        assert len(np.unique(smp)) == k
        inc[smp] += 1
    p = k / n
    assert inc.sum() == T * k
    # each element included with probability k/n (binomial counts)
    assert np.abs(inc - T * p).max() < 6 * math.sqrt(T * p * (1 - p)) + 1
    assert stats.chisquare(inc).pvalue > 1e-5
