"""Pins of the oracle's PCRD rate allocation (Taubman 2000, as used by the
JPEG2000 base layer to meet the ratio r of Algorithm 1's enc_base)."""
import itertools

import numpy as np
import pytest


def _rand_tables(rng, nblk, maxp):
    npass = rng.integers(0, maxp + 1, nblk)
    stride = maxp + 1
    R = np.zeros((nblk, stride), np.int32)
    D = np.zeros((nblk, stride), np.int64)
    for b in range(nblk):
        r = 0
        d = 0
        for k in range(1, npass[b] + 1):
            r += int(rng.integers(0, 40))
            d += int(rng.integers(0, 2000)) if rng.random() < 0.85 else 0
            R[b, k] = max(r, 1)
            D[b, k] = d
    return npass, R, D


def _points(npass, R, D, b):
    return [(int(R[b, k]), int(D[b, k])) for k in range(npass[b] + 1)]


@pytest.mark.parametrize("seed", range(60))
def test_pcrd_lagrangian_optimal_bruteforce(ref, seed):
    """Among all combinations of pass counts with total length at most what
    the allocation used, none has more distortion reduction; and the budget
    is respected."""
    rng = np.random.default_rng(seed)
    nblk = int(rng.integers(1, 4))
    npass, R, D = _rand_tables(rng, nblk, 4)
    budget = int(rng.integers(0, 150))
    kb, used = ref.pcrd(npass, R, D, budget)
    assert used <= budget
    assert used == sum(int(R[b, kb[b]]) for b in range(nblk))
    dsel = sum(int(D[b, kb[b]]) for b in range(nblk))
    for combo in itertools.product(*[range(npass[b] + 1) for b in range(nblk)]):
        r = sum(int(R[b, k]) for b, k in enumerate(combo))
        d = sum(int(D[b, k]) for b, k in enumerate(combo))
        if r <= used:
            assert d <= dsel, (combo, r, d, used, dsel)


def test_pcrd_everything_fits(ref):
    rng = np.random.default_rng(5)
    npass, R, D = _rand_tables(rng, 6, 7)
    kb, used = ref.pcrd(npass, R, D, 10 ** 9)
    # every block ends at its last distortion-increasing hull point
    for b in range(6):
        if npass[b]:
            best = max(range(npass[b] + 1), key=lambda k: (D[b, k], -k))
            assert D[b, kb[b]] == D[b, best]


def test_pcrd_zero_budget(ref):
    rng = np.random.default_rng(6)
    npass, R, D = _rand_tables(rng, 5, 6)
    kb, used = ref.pcrd(npass, R, D, 0)
    assert used == 0 and (kb == 0).all()


def test_pcrd_long_codewords_ineligible(ref):
    npass = np.array([2])
    R = np.array([[0, 100, 70000]], np.int32)
    D = np.array([[0, 10, 10 ** 9]], np.int64)
    kb, used = ref.pcrd(npass, R, D, 10 ** 9)
    assert kb[0] == 1 and used == 100
