"""Pins of the oracle's byte-granular residual truncation (Algorithm 1's
second binary search over a byte position of one embedded SPIHT code).

The tiles' codes form one embedded sequence ordered like a single SPIHT
code (plane by plane; in a plane the sorting passes of every tile, then the
refinement passes of every tile).  Pins, at every bit position of the last
plane's span:
  * what the decoder knows is q itself: known bits equal q's bits, bits
    below the lowest known plane are zero, signs of significant
    coefficients are q's (a sign or refinement bit past the cut would break
    these);
  * knowledge only grows with the cut: significant coefficients stay
    significant and their lowest known plane never rises;
  * the cut at the end of the span decodes like the plane-end truncation.
And at the compressor level, on small fields whose every byte candidate is
decoded and checked here (brute force): the stream meets the bound, is not
longer than the plane-end stream, and its cut is the one the bisection
over the brute-force feasibility table selects."""
import numpy as np
import pytest

from paper_2510_22265_amd import synth


def _field(rng, ny, nx, p=0.3, dens=0.6):
    q = ((rng.geometric(p, size=(ny, nx)) - 1) * (rng.random((ny, nx)) < dens)).astype(np.uint32)
    neg = rng.integers(0, 2, size=(ny, nx)).astype(np.uint8)
    return q, neg


@pytest.mark.parametrize("shape,L,T,seed", [((8, 8), 3, 1, 0), ((8, 8), 3, 1, 1), ((16, 24), 3, 1, 2),
                                             ((13, 7), 2, 2, 3), ((20, 20), 2, 1, 4), ((9, 30), 3, 1, 5)])
def test_cut_decoder_semantics_at_every_bit(ref, shape, L, T, seed):
    rng = np.random.default_rng(4000 + seed)
    ny, nx = shape
    L = ref.levels_eff(ny, nx, L)
    q, neg = _field(rng, ny, nx, p=float(rng.uniform(0.1, 0.4)))
    nmax = int(q.max()).bit_length() - 1
    checked = 0
    for ns in range(0, nmax + 1):
        _, (lo, hi) = ref.spiht_encode_cut(q, neg, L, T, ns, 0)
        assert 0 <= lo < hi
        prev = None
        for t in range(lo + 1, hi + 1):
            sec, _ = ref.spiht_encode_cut(q, neg, L, T, ns, t)
            rc, m, ng, pk = ref.spiht_decode_cut(sec, ny, nx, L, T, ns)
            assert rc == 0
            sig = m > 0
            sh = pk.astype(np.uint32)
            # known bits are q's; nothing below the lowest known plane
            assert ((m >> sh) == (q >> sh))[sig].all()
            assert ((m & ((np.uint32(1) << sh) - 1)) == 0)[sig].all()
            assert (ng == neg)[sig].all()
            assert (pk[sig] >= ns).all()
            # every plane above n_s is fully known
            full = q >= (1 << (ns + 1))
            assert (sig | ~full).all() and (pk[full] <= ns + 1).all()
            if prev is not None:
                psig, ppk = prev
                assert (sig | ~psig).all()
                assert (pk[psig] <= ppk[psig]).all()
            prev = (sig, pk)
            checked += 1
        # the end of the span is the plane-end truncation at n_s
        rc, m_p, _ = ref.spiht_decode(ref.spiht_encode(q, neg, L, T, ns), ny, nx, L, T, ns)
        assert rc == 0 and (prev[0] == (m_p > 0)).all() and (m == m_p).all()
        assert (pk[m_p > 0] == ns).all()
    assert checked > 0


def _recon(ref, stream, tr, x, q_r, neg_r, t, hi):
    """Decode of the stream whose residual is cut at position t: FP32
    midpoint dequantisation, inverse DWT, base added, denormalised."""
    ny, nx = x.shape
    L, er, ns = tr["L"], tr["e_r"], tr["n_s"]
    sec, _ = ref.spiht_encode_cut(q_r, neg_r, L, 1, ns, t)
    rc, m, ng, pk = ref.spiht_decode_cut(sec, ny, nx, L, 1, ns)
    assert rc == 0
    v = ((2 * m.astype(np.int64) + (np.int64(1) << pk.astype(np.int64))).astype(np.float32)
         * np.float32(2.0 ** (er - 1)))
    c = np.where(m > 0, np.where(ng == 1, -v, v), np.float32(0)).astype(np.float32)
    r = ref.dwt(c, L, inverse=True)
    hdr = np.frombuffer(stream[:48], np.uint8)
    xmin = hdr[16:20].view(np.float32)[0]
    range_f = hdr[20:24].view(np.float32)[0]
    a = tr["abase"] + r
    a = a + np.float32(0.5)
    a = a * range_f
    return xmin + a, sec


@pytest.mark.parametrize("var,shape,eps,level", [("u", (8, 8), 0.01, 0), ("v", (8, 8), 0.02, 1),
                                                  ("t", (16, 16), 0.005, 2), ("u", (16, 24), 0.01, 3),
                                                  ("q", (12, 20), 0.002, 4), ("v", (24, 24), 0.01, 5)])
def test_byte_search_brute_force(ref, var, shape, eps, level):
    x = synth.field(var, *shape, cfg=6, level=level)
    ny, nx = shape
    rng_ = float(x.max()) - float(x.min())
    s_plane, tr_p = ref.compress(x, eps, trace=True)
    s, tr = ref.compress(x, eps, trace=True, trunc=1)
    y = ref.decompress(s, ny, nx)
    assert np.abs(x.astype(np.float64) - y.astype(np.float64)).max() <= eps * rng_
    assert len(s) <= len(s_plane) + 8
    if tr["resid_bytes"] == 0:
        assert s == s_plane
        return
    assert (tr["n_s"], tr["e_r"], tr["n_max"]) == (tr_p["n_s"], tr_p["e_r"], tr_p["n_max"])
    assert s[34] & 1
    er = tr["e_r"]
    c = tr["cres"]
    q_r = np.minimum(np.floor(np.abs(c.astype(np.float64)) * 2.0 ** (-er)), (1 << 23) - 1).astype(np.uint32)
    neg_r = (c < 0).astype(np.uint8)
    _, (lo, hi) = ref.spiht_encode_cut(q_r, neg_r, tr["L"], 1, tr["n_s"], 0)
    blo, bhi = lo // 8, (hi + 7) // 8
    feas = {}
    for b in range(blo + 1, bhi + 1):
        t = min(8 * b, hi)
        xh, _ = _recon(ref, s, tr, x, q_r, neg_r, t, hi)
        feas[b] = bool(np.abs(x.astype(np.float64) - xh.astype(np.float64)).max() <= eps * rng_)
    assert feas[bhi]                                 # the end of plane n_s meets the bound
    while bhi - blo > 1:
        mid = (blo + bhi) // 2
        if feas[mid]:
            bhi = mid
        else:
            blo = mid
    _, sec = _recon(ref, s, tr, x, q_r, neg_r, min(8 * bhi, hi), hi)
    assert s[48 + tr["base_bytes"]:] == sec
    # where feasibility is monotone in b the search found the first feasible byte
    bs = sorted(feas)
    if all(feas[a] <= feas[b] for a, b in zip(bs, bs[1:])):
        assert bhi == min(b for b in bs if feas[b])
