"""Candidate enumeration oracle: TEST INFRASTRUCTURE ONLY.

Sec. III (problem statement): the candidates with n interactions are all the
ordered sequences of n objects, for n = 1..n_max, per TX/RX pair. Reading
taken here: candidates are ordered by order n, then by pair, then by the
object sequence in lexicographic order; with ``no_repeat`` a sequence never
names the same object twice in a row (a reflection or diffraction on the
object just left is degenerate).

Two plain implementations, written from that definition and from nothing
else:
  * ``candidates`` lists them by brute force (every n-tuple in
    lexicographic order, filtered), for small K;
  * ``unrank`` finds the candidate of a given rank by counting: at each
    position it walks the allowed objects in increasing order and skips
    whole blocks of completions, whose size ``completions`` counts by
    recursion over the remaining positions (memoised), for any K.
Only ``tests/`` may import this module.
"""
from __future__ import annotations

import functools
import itertools


def _allowed(seq, no_repeat: bool) -> bool:
    return not no_repeat or all(seq[j] != seq[j + 1] for j in range(len(seq) - 1))


def candidates(P: int, K: int, order_min: int, order_max: int,
               no_repeat: bool = True) -> list[tuple[int, tuple[int, ...]]]:
    """Every candidate (pair, objects) in rank order, by brute force."""
    out = []
    for n in range(order_min, order_max + 1):
        seqs = [s for s in itertools.product(range(K), repeat=n) if _allowed(s, no_repeat)]
        for p in range(P):
            out.extend((p, s) for s in seqs)
    return out


@functools.lru_cache(maxsize=None)
def completions(K: int, remaining: int, no_repeat: bool) -> int:
    """Number of ways to continue a sequence by `remaining` more objects
    (each position: every object, except the previous one with no_repeat)."""
    if remaining == 0:
        return 1
    choices = K - 1 if no_repeat else K
    return sum(completions(K, remaining - 1, no_repeat) for _ in range(choices))


def sequences(K: int, n: int, no_repeat: bool = True) -> int:
    """Number of allowed sequences of n objects (the first one is free)."""
    return sum(completions(K, n - 1, no_repeat) for _ in range(K))


def total(P: int, K: int, order_min: int, order_max: int, no_repeat: bool = True) -> int:
    return sum(P * sequences(K, n, no_repeat) for n in range(order_min, order_max + 1))


def unrank(rank: int, P: int, K: int, order_min: int, order_max: int,
           no_repeat: bool = True) -> tuple[int, tuple[int, ...]]:
    """The candidate of the given rank (0-based), by counting."""
    if rank < 0:
        raise IndexError(rank)
    for n in range(order_min, order_max + 1):
        per_pair = sequences(K, n, no_repeat)
        if rank < P * per_pair:
            pair, r = divmod(rank, per_pair) if per_pair else (0, 0)
            seq: list[int] = []
            for pos in range(n):
                block = completions(K, n - pos - 1, no_repeat)
                for v in range(K):
                    if no_repeat and seq and v == seq[-1]:
                        continue
                    if r < block:
                        seq.append(v)
                        break
                    r -= block
            return pair, tuple(seq)
        rank -= P * per_pair
    raise IndexError("rank beyond the last candidate")
