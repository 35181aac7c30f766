"""Algorithm 1's base-ratio feedback search (q-quantile of the base error)
in the oracle.

Pins: every decoded sample meets the bound for every q; with q = 1 the base
alone meets it (no residual section); the fallback of Algorithm 1 makes the
stream for q < 1 never longer than the base-only stream (q = 1); and the
sequence of ratios the oracle evaluates, and the ratios it keeps, equal an
independent transcription of Algorithm 1's loops (halving while q_A < q,
doubling while q_A > q, bisection to 1e-3 keeping the largest ratio with
q_A >= q) driven by the q_A values the oracle measured, with the two guards
the algorithm leaves open: halving stops once every codable pass is kept,
doubling once the budget is zero."""
import math

import numpy as np
import pytest

from paper_2510_22265_amd import synth

FIELDS = [("t", (64, 96), 0.01, 1), ("u", (91, 180), 0.001, 2), ("q", (64, 96), 0.05, 3), ("v", (48, 130), 0.01, 4),
          ("u", (33, 47), 0.02, 5)]
QS = [1 - 1e-5, 0.99, 0.5, 1.0]


def _field(var, shape, cfg):
    return synth.field(var, *shape, cfg=cfg, level=1)


def _alg1(q, r0, ev):
    """Algorithm 1's ratio loops; ev(r) -> (q_A, every segment fitted, budget)."""
    seq = []

    def E(r):
        seq.append(r)
        return ev(r)

    qa0, fitted, bud0 = E(r0)
    r_low = r_high = r_f = r0
    q_f = qa = qa0
    guard = fitted
    while qa < q and not guard:
        r_low = r_low / 2.0
        qa, fitted, _ = E(r_low)
        r_f, q_f, guard = r_low, qa, fitted
    qa = qa0
    zero = bud0 == 0
    while qa > q and not zero:
        r_high = r_high * 2.0
        qa, _, bud = E(r_high)
        zero = bud == 0
    while r_high - r_low > 1e-3:
        r_mid = (r_low + r_high) / 2.0
        qa, _, _ = E(r_mid)
        if qa < q:
            r_high = r_mid
        else:
            r_low, r_f, q_f = r_mid, r_mid, qa
    return r_f, q_f, seq


@pytest.mark.parametrize("var,shape,eps,cfg", FIELDS)
@pytest.mark.parametrize("q", QS)
def test_search_follows_algorithm_1(ref, var, shape, eps, cfg, q):
    x = _field(var, shape, cfg)
    _, log = ref.compress_logged(x, eps, q)
    measured = {}
    for r, qa, fitted, bud in log:
        if not math.isnan(qa):
            measured.setdefault(r, (qa, fitted, bud))

    def ev(r):
        assert r in measured, f"the transcription evaluates r = {r}, the oracle did not"
        return measured[r]

    r_q, _, seq_q = _alg1(q, 30.0, ev)
    seqs = list(seq_q)
    r_only = None
    if q < 1.0:
        r1, q1, seq_1 = _alg1(1.0, 30.0, ev)
        seqs += seq_1
        if q1 >= 1.0:
            r_only = r1
    logged = [r for r, _, _, _ in log]
    assert logged[: len(seqs)] == seqs
    # then the base at the kept ratio, and possibly the base-only fallback
    assert logged[len(seqs)] == r_q
    rest = logged[len(seqs) + 1:]
    assert rest in ([], [r_only])
    assert all(math.isnan(qa) for _, qa, _, _ in log[len(seqs):])


@pytest.mark.parametrize("var,shape,eps,cfg", FIELDS)
def test_bound_fallback_and_base_only(ref, var, shape, eps, cfg):
    x = _field(var, shape, cfg)
    rng_ = float(x.max()) - float(x.min())
    sizes = {}
    for q in QS + [0.0]:
        s, tr = ref.compress(x, eps, q=q, trace=True)
        y = ref.decompress(s, *shape)
        assert np.abs(x.astype(np.float64) - y.astype(np.float64)).max() <= eps * rng_
        sizes[q] = len(s)
        if q == 1.0:
            assert tr["resid_bytes"] == 0          # the base alone meets the bound
    for q in QS:
        assert sizes[q] <= sizes[1.0]              # never worse than base-only (Algorithm 1's fallback)


def test_q_out_of_range_is_refused(ref):
    x = _field("t", (16, 16), 1)
    for q in (-0.1, 1.5, float("nan")):
        rc, _, _ = ref.compress_rc(x, 0.01, q=q)
        assert rc == ref.EINVAL


@pytest.mark.parametrize("var,cfg", [("t", 1), ("u", 2), ("q", 3)])
def test_base_quality_counts_errors_not_exceeding_eps(ref, var, cfg):
    """q_A of enc_base is the proportion of samples whose base-layer error
    does not exceed eps (Algorithm 1; inclusive, as the bound itself).  The
    base reconstruction at r0 comes from a trace of the fixed-ratio run; the
    bound is then set to one of the errors that reconstruction makes (in the
    same power-of-two bracket, so the base quantiser is unchanged), where
    the inclusive and the strict count differ.  The q_A the search logs for
    r0 must equal the inclusive count made here from the definition."""
    x = _field(var, (64, 96), cfg)
    xmin = np.float32(x.min())
    rng_d = float(x.max()) - float(x.min())
    range_f = np.float32(rng_d)
    _, tr = ref.compress(x, 0.01, trace=True)               # base at r0 = 30
    xh = xmin + ((tr["abase"] + np.float32(0.5)) * range_f)  # decoder arithmetic, FP32
    err = np.abs(x.astype(np.float64) - xh.astype(np.float64))
    lo, hi = 2.0 ** -7 * rng_d, 2.0 ** -6 * rng_d           # floor(log2 0.01) = -7
    cand = np.unique(err[(err >= lo) & (err < hi)])
    assert cand.size, "no base error in the bracket of the 1% bound"
    eps = float(cand[cand.size // 2])
    _, log = ref.compress_logged(x, eps, 0.5, bound_mode=1)
    r, qa, _, _ = log[0]
    assert r == 30.0
    incl = np.count_nonzero(err <= eps) / err.size
    strict = np.count_nonzero(err < eps) / err.size
    assert incl != strict
    assert qa == incl


ABL_QS = [1 - 1e-3, 1 - 1e-4, 1 - 1e-5, 1 - 1e-6]


@pytest.mark.parametrize("eps", [0.001, 0.01, 0.1])
def test_q_ablation_relative_cr_at_least_one(ref, eps):
    """Ablation Study: over q in [1 - 1e-3, 1] and range-relative bounds 0.1%
    to 10%, the compression ratio relative to q = 1 (base layer alone) is at
    least 1 for every field, because Algorithm 1 falls back to the base-only
    stream whenever it is the smaller; every stream meets the bound."""
    rels = []
    for k, (var, shape) in enumerate([("t", (45, 90)), ("u", (64, 96)), ("v", (48, 80)), ("q", (40, 72))]):
        x = synth.field(var, *shape, cfg=2, level=k)
        rng_ = float(x.max()) - float(x.min())
        base_only = len(ref.compress(x, eps, q=1.0))
        for q in ABL_QS:
            s = ref.compress(x, eps, q=q)
            y = ref.decompress(s, *shape)
            assert np.abs(x.astype(np.float64) - y.astype(np.float64)).max() <= eps * rng_
            rels.append(base_only / len(s))
    assert min(rels) >= 1.0
