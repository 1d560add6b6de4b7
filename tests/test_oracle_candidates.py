"""Pins of the candidate-enumeration oracle (oracle/candidates.py): closed
form counts, the defining properties of the brute-force list (lexicographic,
unique, no immediate repeat), agreement of the two oracle routines, and
agreement with the independent NumPy host generator of the workloads."""
import numpy as np
import pytest

from oracle import candidates as cand
from paper_2510_16172_amd import scenes


@pytest.mark.parametrize("no_repeat", [True, False])
def test_counts_closed_form(no_repeat):
    for K in range(1, 7):
        for n in range(1, 5):
            want = K * (K - 1) ** (n - 1) if no_repeat else K ** n
            assert cand.sequences(K, n, no_repeat) == want
    assert cand.total(64, 313, 1, 2) == 6_270_016
    assert cand.total(3, 5, 2, 3, False) == 3 * (25 + 125)


@pytest.mark.parametrize("P,K,omin,omax,no_repeat",
                         [(2, 4, 1, 3, True), (3, 3, 2, 4, False), (1, 1, 1, 3, True),
                          (2, 2, 1, 4, True)])
def test_brute_force_properties(P, K, omin, omax, no_repeat):
    c = cand.candidates(P, K, omin, omax, no_repeat)
    assert len(c) == cand.total(P, K, omin, omax, no_repeat)
    keys = [(len(s), p, s) for p, s in c]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    for p, s in c:
        assert 0 <= p < P and omin <= len(s) <= omax and all(0 <= k < K for k in s)
        if no_repeat:
            assert all(s[j] != s[j + 1] for j in range(len(s) - 1))
    if not no_repeat:
        assert sum(1 for _, s in c if len(s) == omax) == P * K ** omax


@pytest.mark.parametrize("P,K,omin,omax,no_repeat",
                         [(2, 4, 1, 3, True), (3, 3, 2, 4, False), (2, 5, 3, 3, True)])
def test_unrank_matches_brute_force(P, K, omin, omax, no_repeat):
    c = cand.candidates(P, K, omin, omax, no_repeat)
    for r, want in enumerate(c):
        assert cand.unrank(r, P, K, omin, omax, no_repeat) == want
    with pytest.raises(IndexError):
        cand.unrank(len(c), P, K, omin, omax, no_repeat)


def test_matches_host_generator():
    """The NumPy generator of the exhaustive workloads (repeat / tile /
    filter) lists the same candidates in the same order."""
    K, P = 5, 3
    sc = scenes.Batch(np.zeros((9, K), np.float32), np.zeros((3, 2 * P), np.float32),
                      np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8),
                      np.zeros((3, 0), np.int32), 1.0, {"n_pairs": P})
    b = scenes.canyon_all_paths(sc, n_max=3)
    c = cand.candidates(P, K, 1, 3)
    assert b.N == len(c)
    for i, (p, s) in enumerate(c):
        assert b.src[i] == 2 * p and b.dst[i] == 2 * p + 1 and b.order[i] == len(s)
        assert tuple(b.ids[: len(s), i]) == s and np.all(b.ids[len(s):, i] == -1)


def test_unrank_extremes_large():
    """First and last candidates of each order at the canyon's size, worked
    by hand: the smallest sequence alternates 0, 1; the largest 312, 311."""
    P, K = 64, 313
    first = 0
    for n in range(1, 7):
        per = P * K * (K - 1) ** (n - 1)
        assert cand.unrank(first, P, K, 1, 6) == (0, tuple((0, 1) * 3)[:n])
        assert cand.unrank(first + per - 1, P, K, 1, 6) == (P - 1, tuple((312, 311) * 3)[:n])
        # second candidate of the order: the last object moves up by one,
        # skipping its predecessor
        if n >= 2:
            want = list((0, 1) * 3)[:n]
            want[-1] += 1
            if want[-1] == want[-2]:
                want[-1] += 1
            assert cand.unrank(first + 1, P, K, 1, 6) == (0, tuple(want))
        first += per
    assert first == cand.total(P, K, 1, 6)
