"""Pins of the oracle's parameter generator (SEM of Section 2.2, SRFT of 2.1)."""
import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_known_answers():
    with open(os.path.join(GOLDEN, "splitmix64_kat.json")) as f:
        kat = json.load(f)
    for case in kat["cases"]:
        got = rng.splitmix64_sequence(case["seed"], len(case["outputs"]))
        assert got == [int(x, 16) for x in case["outputs"]]


@pytest.mark.parametrize("seed", [1, 7, 2**63 + 5])
def test_hash_uniform_and_signs_balanced(seed):
    n, s = 65536, 64
    h, sgn = rng.sem_hash(seed, n, s)
    assert h.min() >= 0 and h.max() < s
    counts = np.bincount(h, minlength=s)
    assert stats.chisquare(counts).pvalue > 1e-4
    assert set(np.unique(sgn)) == {-1, 1}
    # +-1 balance: |sum| within 5 standard deviations of a fair coin
    assert abs(int(sgn.sum())) < 5 * np.sqrt(n)
    # sign independent of bucket: both signs present in every bucket
    for b in range(s):
        assert set(np.unique(sgn[h == b])) == {-1, 1}


def test_srft_signs_balanced():
    d = rng.srft_signs(3, 4096)
    assert set(np.unique(d)) == {-1, 1}
    assert abs(int(d.sum())) < 5 * np.sqrt(4096)


@pytest.mark.parametrize("s,l", [(2, 2), (16, 5), (256, 30), (4096, 520)])
def test_selection_distinct_in_range(s, l):
    sel = rng.srft_select(11, s, l)
    assert sel.shape == (l,)
    assert len(set(sel.tolist())) == l
    assert sel.min() >= 0 and sel.max() < s


def test_selection_uniform_first_draw():
    s = 16
    first = [rng.srft_select(seed, s, 3)[0] for seed in range(3200)]
    counts = np.bincount(first, minlength=s)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_full_selection_is_permutation():
    sel = rng.srft_select(5, 64, 64)
    assert sorted(sel.tolist()) == list(range(64))


def test_streams_differ_and_seeds_differ():
    h1, _ = rng.sem_hash(1, 512, 256)
    h2, _ = rng.sem_hash(2, 512, 256)
    assert np.mean(h1 == h2) < 0.05


@pytest.mark.parametrize("seed", [0, 3, 2**64 - 7])
def test_streams_are_the_published_generator(seed):
    """The stream key K_t is the t-th output of SplitMix64 started at the
    seed, and draw i of stream t is output i + 1 of SplitMix64 started at K_t:
    both through the sequence that the published known answers pin."""
    seq = rng.splitmix64_sequence(seed, 6)
    for t in range(1, 7):
        key = rng.stream_key(seed, t)
        assert key == seq[t - 1]
        assert [rng.draw(key, i) for i in range(40)] == rng.splitmix64_sequence(key, 40)


@pytest.mark.parametrize("bad", [0, 1, 3, 12])
def test_bad_width_rejected(bad):
    with pytest.raises(ValueError):
        rng.sem_hash(1, 8, bad)
