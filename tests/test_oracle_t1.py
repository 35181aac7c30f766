"""Pins of the oracle's MQ coder (T.800 Annex C) and EBCOT tier-1 block
coder (T.800 Annex D)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "t800_contexts.txt")


def _match(spec, val):
    if spec in ("x", "-"):
        return True
    if spec.startswith(">="):
        return val >= int(spec[2:])
    return val == int(spec)


def test_zc_table_matches_t800(ref):
    rows = [l.split() for l in open(GOLDEN) if l.startswith("zc ")]
    cls_of = {0: "LLLH", 2: "LLLH", 1: "HL", 3: "HH"}
    for orient in range(4):
        for h in range(3):
            for v in range(3):
                for d in range(5):
                    got = ref.zc_ctx(orient, h, v, d)
                    cl = cls_of[orient]
                    hv = h + v
                    exp = None
                    for _, c, H, V, D, ctx in rows:
                        if c != cl:
                            continue
                        hval = hv if cl == "HH" else h
                        if _match(H, hval) and _match(V, v) and _match(D, d):
                            exp = int(ctx)
                            break
                    assert got == exp, (orient, h, v, d)


def test_sc_table_matches_t800(ref):
    for line in open(GOLDEN):
        if line.startswith("sc "):
            _, hc, vc, ctx, xr = line.split()
            assert ref.sc_ctx(int(hc), int(vc)) == (int(ctx), int(xr))


@pytest.mark.parametrize("seed", range(6))
def test_mq_roundtrip(ref, seed):
    rng = np.random.default_rng(seed)
    n = 20000 if seed else 100000
    cx = rng.integers(0, 19, n).astype(np.uint8)
    p = rng.uniform(0.001, 0.999, 19)
    bits = (rng.random(n) < p[cx]).astype(np.uint8)
    s = ref.mq_encode(cx, bits)
    assert (ref.mq_decode(s, cx) == bits).all()


@pytest.mark.parametrize("p", [0.02, 0.1, 0.3, 0.5])
def test_mq_rate_near_entropy(ref, p):
    """A single adaptive context on iid Bernoulli(p) codes within a few
    percent of the binary entropy."""
    rng = np.random.default_rng(7)
    n = 200000
    bits = (rng.random(n) < p).astype(np.uint8)
    cx = np.ones(n, np.uint8)               # context 1 starts at state 0
    s = ref.mq_encode(cx, bits)
    H = -(p * np.log2(p) + (1 - p) * np.log2(1 - p))
    assert len(s) * 8 <= n * H * 1.06 + 64
    assert len(s) * 8 >= n * H * 0.97


def test_mq_uniform_context_costs_one_bit(ref):
    rng = np.random.default_rng(8)
    n = 80000
    bits = rng.integers(0, 2, n).astype(np.uint8)
    s = ref.mq_encode(np.full(n, 18, np.uint8), bits)
    assert abs(len(s) * 8 - n) <= 0.01 * n + 32


def _block(rng, h, w):
    dens = rng.uniform(0.05, 1.0)
    q = (rng.geometric(rng.uniform(0.05, 0.9), size=(h, w)) - 1) * (rng.random((h, w)) < dens)
    if rng.random() < 0.3:
        q = q << int(rng.integers(0, 12))
    q = np.minimum(q, (1 << 23) - 1).astype(np.uint32)
    neg = rng.integers(0, 2, size=(h, w)).astype(np.uint8)
    return q, neg


def _e2(q, m, pk):
    q = q.astype(np.int64)
    m = m.astype(np.int64)
    e = np.where(m > 0, 2 * q + 1 - (2 * m + (np.int64(1) << pk.astype(np.int64))), 2 * q + 1)
    return e * e


@pytest.mark.parametrize("seed", range(40))
def test_t1_block_properties(ref, seed):
    rng = np.random.default_rng(100 + seed)
    h, w = [(32, 32), (4, 4), (1, 1), (3, 17), (32, 7), (5, 32), (64, 64), (13, 9)][seed % 8]
    orient = seed % 4
    q, neg = _block(rng, h, w)
    cw, R, D = ref.t1_encode(q, neg, orient)
    P = int(q.max()).bit_length()
    n = len(R) - 1
    assert n == (3 * P - 2 if P else 0)
    # all passes: lossless magnitudes and signs
    m, ng, pk = ref.t1_decode(cw, h, w, orient, P, n)
    assert (m == q).all() and ((ng == neg) | (q == 0)).all()
    assert R[0] == 0 and D[0] == 0
    ks = range(n + 1) if n <= 25 else sorted(set(rng.integers(0, n + 1, 12)) | {0, 1, n})
    for k in ks:
        cwk, _, _ = ref.t1_encode(q, neg, orient, keep=k)
        assert len(cwk) == R[k]                    # flushed length = R_k
        mk, ngk, pkk = ref.t1_decode(cwk, h, w, orient, P, k)
        sig = mk > 0
        sh = pkk.astype(np.uint32)
        # known bits are q's bits at and above the lowest known plane
        assert ((mk >> sh) == (q >> sh))[sig].all()
        assert ((mk & ((np.uint32(1) << sh) - 1)) == 0)[sig].all()
        # the bits known after k passes follow the pass order: plane p is
        # fully known once its cleanup pass (index 3(P-1-p)) is kept
        p_full = P - 1 - k // 3 if k % 3 == 1 else P - 1 - (k + 2) // 3 + 1 if k else P
        if k and k % 3 == 1:
            assert (mk == ((q >> np.uint32(p_full)) << np.uint32(p_full)) * (q >= (1 << p_full))).all()
        # distortion bookkeeping: D_k = sum of error-square reductions
        red = (_e2(q, np.zeros_like(q), pkk) - _e2(q, mk, pkk))[q > 0].sum()
        assert red == D[k]
        # prefix: the full codeword decoded for k passes agrees
        mf, nf, pf = ref.t1_decode(cw, h, w, orient, P, k)
        assert (mf == mk).all() and (pf[sig] == pkk[sig]).all()


def test_t1_empty_block(ref):
    q = np.zeros((32, 32), np.uint32)
    cw, R, D = ref.t1_encode(q, np.zeros_like(q, dtype=np.uint8), 0)
    assert cw == b"" and list(R) == [0] and list(D) == [0]


def test_t1_single_coefficient(ref):
    q = np.zeros((8, 8), np.uint32)
    q[3, 5] = 1
    neg = np.zeros((8, 8), np.uint8)
    neg[3, 5] = 1
    cw, R, D = ref.t1_encode(q, neg, 3)
    assert len(R) == 2 and D[1] == 9 - 0   # e^2: (2*1+1)^2 -> (3 - 3)^2
    m, ng, pk = ref.t1_decode(cw, 8, 8, 3, 1, 1)
    assert m[3, 5] == 1 and ng[3, 5] == 1 and m.sum() == 1


MQ_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "t800_mq_table.txt")
T88_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "t88_mq_test_sequence.txt")


def _mq_golden():
    rows = []
    for line in open(MQ_GOLDEN):
        if line.strip() and not line.startswith("#"):
            i, qe, nmps, nlps, sw = line.split()
            rows.append((int(i), int(qe, 16), int(nmps), int(nlps), int(sw)))
    return rows


def test_mq_table_matches_t800(ref):
    """The oracle's probability table equals T.800 Table C.2 entry by entry."""
    gold = _mq_golden()
    assert [r[0] for r in gold] == list(range(47))
    assert ref.mq_table() == [r[1:] for r in gold]


def test_mq_table_structure(ref):
    """Properties of the state machine that any mistyped entry is likely to
    break: the MPS switches only in the three 'fast attack' states 0, 6 and
    14; state 46 is the non-adapting uniform state; every MPS chain ends in
    the self-looping state 45; an MPS never raises Qe and an LPS never lowers
    it outside the switching states."""
    t = ref.mq_table()
    assert [i for i, r in enumerate(t) if r[3]] == [0, 6, 14]
    assert t[46] == (0x5601, 46, 46, 0)
    for s in range(46):
        seen, k = set(), s
        while k != t[k][1]:
            assert k not in seen
            seen.add(k)
            assert t[t[k][1]][0] <= t[k][0]
            k = t[k][1]
        assert k == 45
        if not t[s][3]:
            assert t[t[s][2]][0] >= t[s][0]
    assert all(r[0] & 1 for r in t)          # every Qe in the table is odd


def test_mq_matches_t88_test_sequence(ref):
    """The standard's test sequence of the MQ coder (T.88 Annex H.2): one
    context from state 0, MPS 0 (tier-1 context 1 starts there).  The
    oracle's codeword equals the standard's encoded bytes up to its final
    0xFF (T.800's FLUSH drops a trailing 0xFF; T.88 ends the sequence with
    the 0xFF 0xAC marker), and decoding the standard's bytes gives the input."""
    kv = dict(l.split() for l in open(T88_GOLDEN) if l.strip() and not l.startswith("#"))
    bits = np.unpackbits(np.frombuffer(bytes.fromhex(kv["input"]), np.uint8))
    enc = bytes.fromhex(kv["encoded"])
    cx = np.ones(bits.size, np.uint8)
    assert bits.size == 256 and enc[-2:] == b"\xff\xac"
    assert ref.mq_encode(cx, bits) == enc[:-2]
    assert (ref.mq_decode(enc, cx) == bits).all()


@pytest.mark.parametrize("seed", range(6))
def test_mq_decision_counters(ref, seed):
    """The work counters (measurement only): decoding every pass of a block
    makes exactly the decisions its encoder made, one block each; the
    cleanup pass of the top plane codes every sample at least through its
    run-length or zero-coding decision (one per 4-row column at least)."""
    rng = np.random.default_rng(900 + seed)
    h, w = [(32, 32), (16, 64), (7, 13), (64, 64), (5, 4), (32, 8)][seed]
    q, neg = _block(rng, h, w)
    ref.mq_counts(reset=True)
    cw, R, D = ref.t1_encode(q, neg, seed % 4)
    P = int(q.max()).bit_length()
    m, ng, pk = ref.t1_decode(cw, h, w, seed % 4, P, len(R) - 1)
    c = ref.mq_counts(reset=True)
    if P == 0:      # an all-zero block codes nothing
        assert c == {k: 0 for k in c}
        return
    assert c["enc_blocks"] == 1 and c["dec_blocks"] == 1
    assert c["enc"] == c["dec"] == c["enc_max_block"] == c["dec_max_block"]
    assert c["enc"] >= w * ((h + 3) // 4)
    assert ref.mq_counts() == {k: 0 for k in c}


@pytest.mark.parametrize("seed", range(16))
def test_t1_bypass_block_properties(ref, seed):
    """The arithmetic-coding bypass (T.800 D.6): every pass kept is lossless;
    each truncated codeword has the length R_k and decodes to q's known bits;
    distortion reductions are those of the arithmetic-coded block (the coding
    of a decision does not change what it tells); the first ten passes give
    the same bytes as without the bypass."""
    rng = np.random.default_rng(700 + seed)
    h, w = [(32, 32), (64, 64), (16, 32), (13, 9), (32, 7), (4, 64), (1, 1), (32, 32)][seed % 8]
    orient = seed % 4
    q, neg = _block(rng, h, w)
    if seed % 3 == 0:
        q = np.minimum(q << np.uint32(10), (1 << 23) - 1).astype(np.uint32)   # many planes: raw passes present
    cw, R, D = ref.t1_encode(q, neg, orient, bypass=1)
    cw0, R0, D0 = ref.t1_encode(q, neg, orient, bypass=0)
    P = int(q.max()).bit_length()
    n = len(R) - 1
    assert n == len(R0) - 1 == (3 * P - 2 if P else 0)
    assert (D == D0).all()
    m, ng, pk = ref.t1_decode(cw, h, w, orient, P, n, bypass=1)
    assert (m == q).all() and ((ng == neg) | (q == 0)).all()
    ks = range(n + 1) if n <= 30 else sorted(set(rng.integers(0, n + 1, 14)) | {0, 1, 10, 11, 12, 13, n})
    for k in ks:
        cwk, _, _ = ref.t1_encode(q, neg, orient, keep=k, bypass=1)
        assert len(cwk) == R[k]
        if k <= 10:
            cwk0, _, _ = ref.t1_encode(q, neg, orient, keep=k, bypass=0)
            assert cwk == cwk0
        mk, ngk, pkk = ref.t1_decode(cwk, h, w, orient, P, k, bypass=1)
        mk0, _, pkk0 = ref.t1_decode(ref.t1_encode(q, neg, orient, keep=k)[0], h, w, orient, P, k)
        assert (mk == mk0).all() and (pkk[mk > 0] == pkk0[mk > 0]).all()
        sig = mk > 0
        assert ((ngk == neg) | ~sig).all()


@pytest.mark.parametrize("seed", range(6))
def test_t1_bypass_raw_refinement_bits(ref, seed):
    """The raw bits of the first bypassed refinement pass (pass 12: plane
    P - 5) are bit P - 5 of every sample significant before that plane, in
    the stripe scan order (stripes of four rows, columns left to right, rows
    top to bottom), read from the end of the codeword kept after 12 passes."""
    rng = np.random.default_rng(7100 + seed)
    h, w = [(32, 32), (16, 16), (9, 13), (64, 32), (32, 5), (8, 64)][seed]
    q, neg = _block(rng, h, w)
    q = np.maximum(q, 1).astype(np.uint32) << np.uint32(14)
    q = np.minimum(q, (1 << 23) - 1).astype(np.uint32)
    P = int(q.max()).bit_length()
    assert 3 * P - 2 >= 12
    rb = ref.t1_rawbits(q, neg, seed % 4)
    cw, R, _ = ref.t1_encode(q, neg, seed % 4, keep=12, bypass=1)
    rby = cw[0] | (cw[1] << 8)
    assert rby == (rb[12] + 7) // 8
    raw = np.unpackbits(np.frombuffer(cw[len(cw) - rby:], np.uint8))
    got = raw[rb[11]: rb[12]]
    p = P - 5
    want = []
    for y0 in range(0, h, 4):
        for x in range(w):
            for y in range(y0, min(y0 + 4, h)):
                if q[y, x] >> (p + 1):
                    want.append((int(q[y, x]) >> p) & 1)
    assert got.tolist() == want


def _sig_delta(q, p):
    e0 = 2 * q + 1
    m = (q >> p) << p
    e1 = e0 - (2 * m + (1 << p))
    return e0 * e0 - e1 * e1


def _ref_delta(q, p):
    e = 2 * q + 1
    a = e - (2 * ((q >> (p + 1)) << (p + 1)) + (1 << (p + 1)))
    b = e - (2 * ((q >> p) << p) + (1 << p))
    return a * a - b * b


@pytest.mark.parametrize("seed", range(12))
def test_t1_distortion_closed_form(ref, seed):
    """The per-pass distortion reductions in closed form (what the GPU's
    distortion kernel computes after the coders): a sample with top bit ps
    becomes significant in pass 1 when ps = P - 1, else in the
    significance-propagation (pass 3(P-2-ps)+2) or cleanup (+4) pass of
    plane ps, and is refined in pass 3(P-2-p)+3 of every plane p < ps; D_k
    is the sum of those reductions up to pass k.  The significance pass of
    every sample is read from the oracle's decoder (first k at which it
    decodes significant), and the sums equal the oracle encoder's D."""
    rng = np.random.default_rng(300 + seed)
    h, w = [(32, 32), (4, 4), (3, 17), (16, 16), (13, 9), (8, 32)][seed % 6]
    q, neg = _block(rng, h, w)
    cw, R, D = ref.t1_encode(q, neg, seed % 4)
    P = int(q.max()).bit_length()
    n = len(R) - 1
    if P == 0:
        return
    sigk = np.zeros((h, w), np.int64)
    for k in range(n, 0, -1):                 # first pass after which a sample is significant
        mk, _, _ = ref.t1_decode(cw, h, w, seed % 4, P, k)
        sigk[mk > 0] = k
    dk = np.zeros(n + 1, np.int64)
    for (y, x), qv in np.ndenumerate(q):
        qv = int(qv)
        if not qv:
            continue
        ps = qv.bit_length() - 1
        k = int(sigk[y, x])
        if ps == P - 1:
            assert k == 1
        else:
            assert k in (3 * (P - 2 - ps) + 2, 3 * (P - 2 - ps) + 4)
        dk[k] += _sig_delta(qv, ps)
        for p in range(ps):
            dk[3 * (P - 2 - p) + 3] += _ref_delta(qv, p)
    assert (np.cumsum(dk) == D).all()
