"""Pins of the oracle's SPIHT residual coder (Said & Pearlman 1996, the
residual layer of the paper's Method section)."""
import numpy as np
import pytest


def _field(rng, ny, nx, p=0.3, dens=0.5):
    q = ((rng.geometric(p, size=(ny, nx)) - 1) * (rng.random((ny, nx)) < dens)).astype(np.uint32)
    neg = rng.integers(0, 2, size=(ny, nx)).astype(np.uint8)
    return q, neg


@pytest.mark.parametrize("shape,L,T", [((8, 8), 3, 1), ((6, 6), 2, 1), ((13, 7), 2, 2), ((1, 1), 0, 1),
                                        ((1, 17), 0, 3), ((2, 2), 1, 1), ((91, 180), 5, 2), ((45, 46), 4, 1),
                                        ((33, 66), 5, 2), ((70, 6), 2, 3), ((70, 130), 6, 1), ((6, 6), 2, 2),
                                        ((45, 90), 5, 1)])
def test_all_planes_lossless(ref, shape, L, T):
    rng = np.random.default_rng(sum(shape) * 7 + L)
    L = ref.levels_eff(*shape, L)
    q, neg = _field(rng, *shape)
    sec = ref.spiht_encode(q, neg, L, T, 0)
    rc, m, ng = ref.spiht_decode(sec, *shape, L, T, 0)
    assert rc == 0
    assert (m == q).all()
    assert ((ng == neg) | (q == 0)).all()


@pytest.mark.parametrize("seed", range(12))
def test_truncation_closed_form(ref, seed):
    """Decoding planes n_max..n_s recovers q with the bits below n_s
    cleared (zero where q < 2^n_s), for every n_s."""
    rng = np.random.default_rng(seed)
    ny, nx = int(rng.integers(2, 60)), int(rng.integers(2, 60))
    L = ref.levels_eff(ny, nx, int(rng.integers(1, 6)))
    T = int(rng.integers(1, 4))
    q, neg = _field(rng, ny, nx, p=float(rng.uniform(0.05, 0.5)))
    nmax = int(q.max()).bit_length() - 1
    for ns in range(0, nmax + 2):
        sec = ref.spiht_encode(q, neg, L, T, ns)
        rc, m, _ = ref.spiht_decode(sec, ny, nx, L, T, ns)
        assert rc == 0
        assert (m == np.where(q >= (1 << ns), (q >> ns) << ns, 0)).all()


def _tiles(sec, ntiles):
    ent = np.frombuffer(sec[: 4 * ntiles], "<u4")
    lens = ent & 0x3FFFFFF
    offs = 4 * ntiles + np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    return ent, [sec[int(o): int(o) + int(l)] for o, l in zip(offs, lens)]


def test_embedded_prefix_per_tile(ref):
    """Each tile's code at plane n_s is a bit prefix of its code at n_s-1."""
    rng = np.random.default_rng(11)
    ny, nx, L, T = 40, 56, 3, 2
    q, neg = _field(rng, ny, nx, p=0.1)
    hL, wL = ny, nx
    for _ in range(L):
        hL, wL = (hL + 1) // 2, (wL + 1) // 2
    nt = -(-hL // T) * -(-wL // T)
    nmax = int(q.max()).bit_length() - 1
    prev = None
    for ns in range(nmax, -1, -1):
        ent, tiles = _tiles(ref.spiht_encode(q, neg, L, T, ns), nt)
        if prev is not None:
            for a, b in zip(prev, tiles):
                if len(a):
                    bits_a = np.unpackbits(np.frombuffer(a, np.uint8))
                    bits_b = np.unpackbits(np.frombuffer(b, np.uint8))
                    # the shorter code's bits (before its zero padding) are a prefix
                    nz = len(bits_a)
                    assert (bits_b[: nz][bits_a == 1] == 1).all()
                    assert len(b) >= len(a)
        prev = tiles


def test_tiles_independent(ref):
    """Changing coefficients of one tile's trees leaves other tiles' codes unchanged."""
    rng = np.random.default_rng(12)
    ny, nx, L, T = 64, 64, 3, 2
    q, neg = _field(rng, ny, nx)
    nt = 4 * 4
    _, t1 = _tiles(ref.spiht_encode(q, neg, L, T, 0), nt)
    q2 = q.copy()
    q2[:2, :2] += 5                  # LL roots of tile 0
    q2[40:48, 0:8] += 3              # a level-1 LH region under tile (1, 0)... rows 32+8.. of LH1
    _, t2 = _tiles(ref.spiht_encode(q2, neg, L, T, 0), nt)
    changed = [i for i in range(nt) if t1[i] != t2[i]]
    assert 0 in changed and len(changed) <= 2


def test_sorting_cost_of_empty_tiles(ref):
    q = np.zeros((32, 32), np.uint32)
    sec = ref.spiht_encode(q, np.zeros_like(q, dtype=np.uint8), 3, 2, 0)
    assert len(sec) == 4 * 4 and set(sec) == {0}
