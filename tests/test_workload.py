"""Seeded input generators (shared by the oracle and the HIP path): string
enumeration and sampling properties, on the CPU."""
import math
from itertools import combinations

import numpy as np
import pytest

import workload as wl


def enumerate_plain(norb, n):
    out = np.array([sum(1 << p for p in c) for c in combinations(range(norb), n)],
                   dtype=np.uint64)
    out.sort()
    return out


@pytest.mark.parametrize("norb,n", [(1, 0), (1, 1), (6, 0), (6, 6), (8, 4), (12, 5), (12, 11),
                                    (16, 8), (20, 3), (64, 1), (64, 3), (64, 61), (64, 63),
                                    (64, 64), (40, 38)])
def test_all_strings_matches_itertools(norb, n):
    assert np.array_equal(wl.all_strings(norb, n), enumerate_plain(norb, n))


@pytest.mark.parametrize("norb,n,count,seed", [(16, 8, 2000, 1), (26, 7, 500, 2), (64, 61, 200, 3),
                                               (64, 3, 300, 4), (40, 20, 2100, 5), (12, 6, 924, 6)])
def test_sample_strings_properties(norb, n, count, seed):
    s = wl.sample_strings(norb, n, count, seed)
    assert s.size == min(count, math.comb(norb, n))
    assert np.all(s[1:] > s[:-1])                                       # sorted, unique
    assert all(bin(int(x)).count("1") == n for x in s)
    assert all(int(x) >> norb == 0 for x in s) or norb == 64
    assert int((1 << n) - 1) in set(s.tolist())                          # Aufbau included
    assert np.array_equal(s, wl.sample_strings(norb, n, count, seed))   # seeded


def test_sampling_prefers_low_levels():
    """Probability decays with the excitation level: per string, level-1 strings
    are drawn more often than level-3 ones (weight ratio exp(1.4) ~ 4; drawing
    without replacement saturates the likeliest strings, so the observed ratio is
    lower)."""
    norb, n = 16, 8
    s = wl.sample_strings(norb, n, 300, 11)
    lv = wl._level(s, n)
    frac = [np.mean(lv == k) / (math.comb(n, k) * math.comb(norb - n, k)) for k in (1, 3)]
    assert frac[0] > 2 * frac[1]


def test_string_sets_nested_across_sizes():
    """Where all C(norb, n) strings can be enumerated (weighted sampling keys),
    the same seed draws smaller string sets as subsets of larger ones: the
    successive-solve benchmark grows a sel26 basis this way.  (The rejection
    regime for larger spaces draws in batches sized by the count, so it makes
    no such promise.)"""
    for norb, n, sizes in ((26, 7, (600, 900, 1500)), (16, 8, (300, 700, 2000))):
        sets = [wl.sample_strings(norb, n, k, 3001) for k in sizes]
        for small, big in zip(sets, sets[1:]):
            assert np.isin(small, big).all()
    a = wl.make_config("sel26", nstr=6000).alpha
    b = wl.make_config("sel26", nstr=8000).alpha
    assert np.isin(a, b).all()


def test_sample_configurations_counts_and_repeats():
    s = wl.sample_configurations(12, 5, 4, 2000, 3)
    assert s.shape == (2000, 2) and s.dtype == np.uint64
    pa = np.array([bin(int(v)).count("1") for v in s[:, 0]])
    pb = np.array([bin(int(v)).count("1") for v in s[:, 1]])
    assert np.all(pa == 5) and np.all(pb == 4) and int(s.max()) < (1 << 12)
    assert np.array_equal(s, wl.sample_configurations(12, 5, 4, 2000, 3))
    # a measurement record repeats configurations
    keys = np.unique(s[:, 0] * np.uint64(1 << 12) + s[:, 1])
    assert keys.size < 2000
