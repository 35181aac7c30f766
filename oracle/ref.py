"""ctypes binding of the C oracle (``oracle/ebcc_oracle.c``).

Test infrastructure only: a plain, slow, single-threaded CPU implementation
of the EBCC compressor (arXiv 2510.22265, Method section and Algorithm 1)
that the GPU library is checked against.  It shares no code with the GPU path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebcc_oracle.so")
SRC_PATH = os.path.join(_HERE, "ebcc_oracle.c")

OK, EINVAL, ENOSPC, ECORRUPT, ENOMEM = 0, -1, -2, -3, -4
MODE_CONST, MODE_RAW, MODE_CODED = 0, 1, 2
HDR_BYTES = 48


def build(force=True):
    """Compile the oracle with the host C compiler (FP contraction off)."""
    import subprocess
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-ffp-contract=off", "-fno-fast-math",
                           "-shared", "-fPIC", "-o", tmp, SRC_PATH, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.ebcc_ref_compress_trace.argtypes = [P, C.c_size_t, C.c_size_t, C.c_double, C.c_int, C.c_double,
                                              C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                              P, C.c_size_t, C.POINTER(C.c_size_t), P]
        L.ebcc_ref_spiht_encode_cut.argtypes = [P, P, C.c_long, C.c_long, C.c_int, C.c_int, C.c_int, C.c_long, P,
                                                C.c_long, P]
        L.ebcc_ref_spiht_encode_cut.restype = C.c_long
        L.ebcc_ref_spiht_decode_cut.argtypes = [P, C.c_long, C.c_long, C.c_long, C.c_int, C.c_int, C.c_int, P, P, P]
        L.ebcc_ref_base_budget.argtypes = [C.c_long, C.c_long, C.c_double]
        L.ebcc_ref_base_budget.restype = C.c_long
        L.ebcc_ref_alg1_log.argtypes = [P, P, P, P, C.c_int]
        L.ebcc_ref_decompress.argtypes = [P, C.c_size_t, P, C.c_size_t, C.c_size_t]
        L.ebcc_ref_compress_bound.argtypes = [C.c_size_t, C.c_size_t]
        L.ebcc_ref_compress_bound.restype = C.c_size_t
        L.ebcc_ref_stream_info.argtypes = [P, C.c_size_t, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                           C.POINTER(C.c_int)]
        L.ebcc_ref_band_norm.argtypes = [C.c_int, C.c_int]
        L.ebcc_ref_band_norm.restype = C.c_double
        L.ebcc_ref_band_log2_gain.argtypes = [C.c_int, C.c_int]
        L.ebcc_ref_levels.argtypes = [C.c_long, C.c_long, C.c_int]
        L.ebcc_ref_dwt_f32.argtypes = [P, C.c_long, C.c_long, C.c_int, C.c_int]
        L.ebcc_ref_dwt_f64.argtypes = [P, C.c_long, C.c_long, C.c_int, C.c_int]
        L.ebcc_ref_mq_encode.argtypes = [P, P, C.c_long, P, C.c_long]
        L.ebcc_ref_mq_encode.restype = C.c_long
        L.ebcc_ref_mq_decode.argtypes = [P, C.c_long, P, C.c_long, P]
        L.ebcc_ref_zc_ctx.argtypes = [C.c_int] * 4
        L.ebcc_ref_sc_ctx.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.ebcc_ref_t1_encode.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, C.c_long,
                                         C.POINTER(C.c_long)]
        L.ebcc_ref_t1_decode.argtypes = [P, C.c_long, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, P,
                                         P]
        L.ebcc_ref_t1_rawbits.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P]
        L.ebcc_ref_pcrd.argtypes = [C.c_int, P, P, P, C.c_int, C.c_long, P]
        L.ebcc_ref_pcrd.restype = C.c_long
        L.ebcc_ref_spiht_encode.argtypes = [P, P, C.c_long, C.c_long, C.c_int, C.c_int, C.c_int, P, C.c_long]
        L.ebcc_ref_spiht_encode.restype = C.c_long
        L.ebcc_ref_spiht_decode.argtypes = [P, C.c_long, C.c_long, C.c_long, C.c_int, C.c_int, C.c_int, P, P]
        L.ebcc_ref_checksum.argtypes = [P, C.c_long]
        L.ebcc_ref_checksum.restype = C.c_uint32
        L.ebcc_ref_mq_table.argtypes = [C.c_int] + [C.POINTER(C.c_int)] * 4
        L.ebcc_ref_mq_counts.argtypes = [P, C.c_int]
        L.ebcc_ref_quant.argtypes = [C.c_float, C.c_int]
        L.ebcc_ref_quant.restype = C.c_uint32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Trace(C.Structure):
    _fields_ = [("coef", C.c_void_p), ("abase", C.c_void_p), ("cres", C.c_void_p),
                ("kb", C.c_void_p), ("pb", C.c_void_p), ("info", C.c_void_p)]


def n_blocks(ny, nx, levels=5, cbl2w=5, cbl2h=5):
    """Code-block count of the base layer (band-by-band tiling)."""
    L = lib().ebcc_ref_levels(ny, nx, levels)
    h, w = [ny], [nx]
    for _ in range(L):
        h.append((h[-1] + 1) // 2)
        w.append((w[-1] + 1) // 2)
    cw, ch = 1 << cbl2w, 1 << cbl2h
    cnt = lambda H, W: (-(-H // ch)) * (-(-W // cw)) if H > 0 and W > 0 else 0
    n = cnt(h[L], w[L])
    for l in range(L, 0, -1):
        n += cnt(h[l], w[l - 1] - w[l]) + cnt(h[l - 1] - h[l], w[l]) + cnt(h[l - 1] - h[l], w[l - 1] - w[l])
    return n


def compress(x, err_bound, bound_mode=0, base_ratio=30.0, levels=5, cbl2w=5, cbl2h=5, tile=1, trace=False, q=0.0,
             trunc=0, bypass=0):
    """Compress a 2-D float32 field.  Returns bytes (and a dict of
    intermediate results when ``trace`` is true).  trunc=1 cuts the residual
    at a byte position instead of a bit-plane end; bypass=1 sends the
    significance-propagation and refinement passes below the fourth
    bit-plane as raw bits."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    ny, nx = x.shape
    L = lib()
    cap = L.ebcc_ref_compress_bound(ny, nx)
    out = np.zeros(cap, dtype=np.uint8)
    n = C.c_size_t(0)
    tr = None
    bufs = {}
    if trace:
        nb = n_blocks(ny, nx, levels, cbl2w, cbl2h)
        bufs = dict(coef=np.zeros((ny, nx), np.float32), abase=np.zeros((ny, nx), np.float32),
                    cres=np.zeros((ny, nx), np.float32), kb=np.zeros(nb, np.uint8), pb=np.zeros(nb, np.uint8),
                    info=np.zeros(11, np.int32))
        tr = Trace(*[_p(bufs[k]).value for k in ("coef", "abase", "cres", "kb", "pb", "info")])
    rc = L.ebcc_ref_compress_trace(_p(x), ny, nx, float(err_bound), int(bound_mode), float(base_ratio), float(q),
                                   int(levels), int(cbl2w), int(cbl2h), int(tile), int(trunc), int(bypass), _p(out),
                                   cap, C.byref(n), C.byref(tr) if tr is not None else None)
    if rc != OK:
        raise RuntimeError(f"ebcc_ref_compress failed: {rc}")
    s = out[: n.value].tobytes()
    if trace:
        info = bufs["info"]
        bufs["mode"], bufs["L"], bufs["e0"], bufs["e_r"], bufs["n_max"], bufs["n_s"] = [int(v) for v in info[:6]]
        bufs["nblocks"], bufs["ntiles"], bufs["base_bytes"], bufs["resid_bytes"], bufs["checks"] = \
            [int(v) for v in info[6:11]]
        return s, bufs
    return s


def compress_rc(x, err_bound, bound_mode=0, base_ratio=30.0, levels=5, cbl2w=5, cbl2h=5, tile=1, cap=None, q=0.0,
                trunc=0, bypass=0):
    """Raw status-code form for error-path tests: returns (rc, bytes or None, out_len)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    ny, nx = x.shape if x.ndim == 2 else (x.size, 1)
    L = lib()
    if cap is None:
        cap = L.ebcc_ref_compress_bound(max(ny, 1), max(nx, 1))
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    n = C.c_size_t(0)
    rc = L.ebcc_ref_compress_trace(_p(x), ny, nx, float(err_bound), int(bound_mode), float(base_ratio), float(q),
                                   int(levels), int(cbl2w), int(cbl2h), int(tile), int(trunc), int(bypass), _p(out),
                                   cap, C.byref(n), None)
    return rc, (out[: n.value].tobytes() if rc == OK else None), n.value


def compress_logged(x, err_bound, q, base_ratio=30.0, cap=4096, **kw):
    """Compress with the enc_base log on: returns (stream, list of
    (ratio, q_A or nan, every segment fitted, budget)) in evaluation order."""
    L = lib()
    r = np.zeros(cap); qa = np.zeros(cap); af = np.zeros(cap, np.int32); bud = np.zeros(cap, np.int64)
    L.ebcc_ref_alg1_log(_p(r), _p(qa), _p(af), _p(bud), cap)
    try:
        s = compress(x, err_bound, base_ratio=base_ratio, q=q, **kw)
    finally:
        n = L.ebcc_ref_alg1_log(None, None, None, None, 0)
    n = min(n, cap)
    return s, [(float(r[i]), float(qa[i]), bool(af[i]), int(bud[i])) for i in range(n)]


def decompress(stream, ny, nx):
    buf = np.frombuffer(bytes(stream), dtype=np.uint8).copy()
    out = np.zeros((ny, nx), dtype=np.float32)
    rc = lib().ebcc_ref_decompress(_p(buf), buf.size, _p(out), ny, nx)
    if rc != OK:
        raise RuntimeError(f"ebcc_ref_decompress failed: {rc}")
    return out


def decompress_rc(stream, ny, nx):
    buf = np.frombuffer(bytes(stream), dtype=np.uint8).copy()
    out = np.zeros((max(ny, 1), max(nx, 1)), dtype=np.float32)
    return lib().ebcc_ref_decompress(_p(buf), buf.size, _p(out), ny, nx)


def stream_info(stream):
    buf = np.frombuffer(bytes(stream), dtype=np.uint8).copy()
    ny, nx, mode = C.c_size_t(), C.c_size_t(), C.c_int()
    rc = lib().ebcc_ref_stream_info(_p(buf), buf.size, C.byref(ny), C.byref(nx), C.byref(mode))
    if rc != OK:
        raise RuntimeError(f"bad stream: {rc}")
    return ny.value, nx.value, mode.value


def levels_eff(ny, nx, L):
    return lib().ebcc_ref_levels(ny, nx, L)


def dwt(a, levels, inverse=False, f64=False):
    """2-D multi-level 9/7 lifting DWT (Mallat layout), FP32 or FP64."""
    dt = np.float64 if f64 else np.float32
    a = np.ascontiguousarray(a, dtype=dt).copy()
    ny, nx = a.shape
    fn = lib().ebcc_ref_dwt_f64 if f64 else lib().ebcc_ref_dwt_f32
    fn(_p(a), ny, nx, int(levels), int(bool(inverse)))
    return a


def band_norm(level, orient):
    return lib().ebcc_ref_band_norm(level, orient)


def band_log2_gain(level, orient):
    return lib().ebcc_ref_band_log2_gain(level, orient)


def zc_ctx(orient, h, v, d):
    return lib().ebcc_ref_zc_ctx(orient, h, v, d)


def sc_ctx(hc, vc):
    x = C.c_int(0)
    c = lib().ebcc_ref_sc_ctx(hc, vc, C.byref(x))
    return c, x.value


def mq_encode(cx, bits):
    cx = np.ascontiguousarray(cx, np.uint8)
    bits = np.ascontiguousarray(bits, np.uint8)
    cap = 2 * cx.size + 16
    out = np.zeros(cap, np.uint8)
    n = lib().ebcc_ref_mq_encode(_p(cx), _p(bits), cx.size, _p(out), cap)
    assert n >= 0
    return out[:n].tobytes()


def mq_decode(stream, cx):
    cx = np.ascontiguousarray(cx, np.uint8)
    buf = np.frombuffer(bytes(stream) + b"\0", np.uint8).copy()
    bits = np.zeros(cx.size, np.uint8)
    lib().ebcc_ref_mq_decode(_p(buf), len(stream), _p(cx), cx.size, _p(bits))
    return bits


def t1_encode(q, neg, orient, keep=-1, bypass=0):
    """Encode one code-block (q: magnitudes h x w, neg: sign flags).
    Returns (codeword terminated after `keep` passes, R[0..n], D[0..n])."""
    q = np.ascontiguousarray(q, np.uint32)
    neg = np.ascontiguousarray(neg, np.uint8)
    h, w = q.shape
    R = np.zeros(70, np.int32)
    D = np.zeros(70, np.int64)
    cap = 2 * 24 * 3 * q.size + 64
    out = np.zeros(cap, np.uint8)
    ln = C.c_long(0)
    npass = lib().ebcc_ref_t1_encode(_p(q), _p(neg), w, h, orient, bypass, keep, _p(R), _p(D), _p(out), cap,
                                     C.byref(ln))
    assert npass >= 0
    return out[: ln.value].tobytes(), R[: npass + 1].copy(), D[: npass + 1].copy()


def t1_decode(cw, h, w, orient, P, k, bypass=0):
    buf = np.frombuffer(bytes(cw) + b"\0", np.uint8).copy()
    m = np.zeros((h, w), np.uint32)
    neg = np.zeros((h, w), np.uint8)
    pk = np.zeros((h, w), np.int8)
    rc = lib().ebcc_ref_t1_decode(_p(buf), len(cw), w, h, orient, bypass, P, k, _p(m), _p(neg), _p(pk))
    assert rc == 0
    return m, neg, pk


def t1_rawbits(q, neg, orient):
    """Raw bits after each pass of a block coded with the bypass."""
    q = np.ascontiguousarray(q, np.uint32)
    neg = np.ascontiguousarray(neg, np.uint8)
    h, w = q.shape
    rb = np.zeros(70, np.int64)
    n = lib().ebcc_ref_t1_rawbits(_p(q), _p(neg), w, h, orient, _p(rb))
    return rb[: n + 1].copy()


def pcrd(npass, R, D, budget):
    """npass: [nblk]; R, D: [nblk][stride]. Returns (kb, used bytes)."""
    npass = np.ascontiguousarray(npass, np.int32)
    R = np.ascontiguousarray(R, np.int32)
    D = np.ascontiguousarray(D, np.int64)
    kb = np.zeros(len(npass), np.uint8)
    used = lib().ebcc_ref_pcrd(len(npass), _p(npass), _p(R), _p(D), R.shape[1], int(budget), _p(kb))
    return kb, used


def spiht_encode(q, neg, levels, tile, n_s):
    q = np.ascontiguousarray(q, np.uint32)
    neg = np.ascontiguousarray(neg, np.uint8)
    ny, nx = q.shape
    cap = 16 * q.size + 4096
    out = np.zeros(cap, np.uint8)
    n = lib().ebcc_ref_spiht_encode(_p(q), _p(neg), ny, nx, levels, tile, n_s, _p(out), cap)
    assert n >= 0
    return out[:n].tobytes()


def spiht_decode(sec, ny, nx, levels, tile, n_s):
    buf = np.frombuffer(bytes(sec) + b"\0", np.uint8).copy()
    m = np.zeros((ny, nx), np.uint32)
    neg = np.zeros((ny, nx), np.uint8)
    rc = lib().ebcc_ref_spiht_decode(_p(buf), len(sec), ny, nx, levels, tile, n_s, _p(m), _p(neg))
    return rc, m, neg


def spiht_encode_cut(q, neg, levels, tile, n_s, t):
    """Residual section of q/neg cut at position t of the embedded sequence
    (tiles' codes ordered by plane, then tile), where lo < t <= hi with lo,
    hi the sequence's bits through plane n_s + 1 and through plane n_s.
    Returns (section bytes, or None when t is outside (lo, hi]; (lo, hi))."""
    q = np.ascontiguousarray(q, np.uint32)
    neg = np.ascontiguousarray(neg, np.uint8)
    ny, nx = q.shape
    cap = 16 * q.size + 4096
    out = np.zeros(cap, np.uint8)
    span = np.zeros(2, np.int64)
    n = lib().ebcc_ref_spiht_encode_cut(_p(q), _p(neg), ny, nx, levels, tile, n_s, int(t), _p(out), cap, _p(span))
    return (out[:n].tobytes() if n >= 0 else None), (int(span[0]), int(span[1]))


def spiht_decode_cut(sec, ny, nx, levels, tile, n_s):
    """Decode a byte-cut residual section: (rc, magnitudes, signs, lowest
    known plane per coefficient)."""
    buf = np.frombuffer(bytes(sec) + b"\0", np.uint8).copy()
    m = np.zeros((ny, nx), np.uint32)
    neg = np.zeros((ny, nx), np.uint8)
    pk = np.zeros((ny, nx), np.int8)
    rc = lib().ebcc_ref_spiht_decode_cut(_p(buf), len(sec), ny, nx, levels, tile, n_s, _p(m), _p(neg), _p(pk))
    return rc, m, neg, pk


def checksum(b):
    buf = np.frombuffer(bytes(b) + b"\0", np.uint8).copy()
    return lib().ebcc_ref_checksum(_p(buf), len(b))


def mq_table():
    """The oracle's MQ probability table: list of (Qe, NMPS, NLPS, SWITCH)."""
    rows = []
    for i in range(47):
        v = [C.c_int() for _ in range(4)]
        assert lib().ebcc_ref_mq_table(i, *[C.byref(a) for a in v]) == 0
        rows.append(tuple(a.value for a in v))
    return rows


def quant(y, sh):
    """Base-layer quantised magnitude floor(|y| 2^sh) (capped at 2^23 - 1)."""
    return lib().ebcc_ref_quant(float(y), int(sh))


def mq_counts(reset=False):
    """MQ decisions made by the oracle on the calling thread since the last
    reset: coded (encoder) and decoded (decoder) totals, the code-blocks
    each ran over, and the most decisions in one block (measurement only)."""
    v = np.zeros(6, dtype=np.int64)
    lib().ebcc_ref_mq_counts(v.ctypes.data, 1 if reset else 0)
    return {"enc": int(v[0]), "enc_blocks": int(v[1]), "enc_max_block": int(v[2]),
            "dec": int(v[3]), "dec_blocks": int(v[4]), "dec_max_block": int(v[5])}
