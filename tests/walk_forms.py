"""Replica-walk reference forms used by the tests (Sec. 2.3 round trips).

Independent of the oracle's online bookkeeping: a closed form for the
all-accepted exchange pass and an offline rescan of one slot's recorded
temperatures.
"""
from __future__ import annotations

import numpy as np


def expected_rotation(NT: int, P: int):
    """All exchanges accepted: the ascending pass moves the configuration at
    the lowest temperature to the highest and every other one down by one, so
    slot j of a set sits at temperature (j - m) mod NT after pass m and every
    round trip lasts exactly NT passes.  Returns the per-slot labels and trip
    beginnings and the round-trip bins [32][3] of one replica set after P
    passes."""
    lab = np.zeros(NT, np.int32)
    beg = np.zeros(NT, np.uint32)
    bins = np.zeros((32, 3), np.uint64)
    for j in range(NT):
        first = j if j >= 1 else NT  # first pass at the lowest temperature
        if P < first:
            continue
        m = first + NT
        while m <= P:  # every later arrival at the lowest ends a trip of NT
            bins[m.bit_length() - 1] += np.array([1, NT, NT * NT], np.uint64)
            m += NT
        beg[j] = first + ((P - first) // NT) * NT
        lab[j] = 1 if (j - P) % NT == 0 else 2  # the pass after a cold visit is hot
    return lab, beg, bins


def rescan(history, NT: int):
    """Round trips from one slot's temperatures after passes 1..P: a trip
    starts at the first arrival at the lowest temperature and at every arrival
    there that follows a visit to the highest since the previous start.
    Returns (label, begin of the current trip, bins [32][3])."""
    starts = []
    hot_since = False
    for m, k in enumerate(history, start=1):
        if k == NT - 1 and starts:
            hot_since = True
        if k == 0 and (not starts or hot_since):
            starts.append(m)
            hot_since = False
    bins = np.zeros((32, 3), np.uint64)
    for a, b in zip(starts[:-1], starts[1:]):
        n = b - a
        bins[b.bit_length() - 1] += np.array([1, n, n * n], np.uint64)
    if not starts:
        return 0, 0, bins
    return (2 if hot_since else 1), starts[-1], bins
