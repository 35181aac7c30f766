"""The C-ABI library loads and exports every entry point include/ebcc.h
declares (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ebcc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ebcc_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_2510_22265_amd import ebcc
    if not os.path.exists(ebcc.LIB_PATH):
        from paper_2510_22265_amd import build
        build.build()
    return ebcc


def test_exports_every_declared_symbol():
    ebcc = _lib()
    lib = ctypes.CDLL(ebcc.LIB_PATH)
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ebcc.SYMBOLS)


def test_host_only_entry_points():
    ebcc = _lib()
    L = ebcc.lib()
    p = ebcc.Params()
    L.ebcc_params_default(ctypes.byref(p))
    assert p.struct_size == ctypes.sizeof(ebcc.Params)
    assert (p.err_bound, p.base_ratio, p.levels, p.cblk_log2w, p.cblk_log2h, p.spiht_tile) == (0.01, 30.0, 5, 5, 5, 1)
    assert (p.q, p.trunc, p.bypass) == (0.0, 0, 0)
    assert L.ebcc_compress_bound(181, 360) == 48 + 4 * 181 * 360
    assert L.ebcc_status_str(-3) == b"corrupt stream"
    hdr = bytearray(48)
    hdr[:4] = b"EBCC"
    hdr[4] = 1
    hdr[5] = 2
    hdr[8:12] = (721).to_bytes(4, "little")
    hdr[12:16] = (1440).to_bytes(4, "little")
    assert ebcc.stream_info(bytes(hdr)) == (721, 1440, 2)
    bad = bytes(b"XBCC" + hdr[4:])
    try:
        ebcc.stream_info(bad)
        assert False
    except ebcc.EbccError as e:
        assert e.code == ebcc.ECORRUPT


def test_params_struct_matches_header():
    """Field order and size of ebcc_params in the binding and the header."""
    src = open(os.path.join(ROOT, "include", "ebcc.h")).read()
    body = src[src.index("typedef struct {"): src.index("} ebcc_params;")]
    fields = re.findall(r"^\s*(?:uint32_t|double)\s+(\w+);", body, flags=re.M)
    from paper_2510_22265_amd import ebcc
    assert fields == [f for f, _ in ebcc.Params._fields_]


def test_tuning_struct_and_round_trip():
    """ebcc_tuning: field order matches the header; set/get round-trips and
    out-of-range values are refused (host-only entry points)."""
    src = open(os.path.join(ROOT, "include", "ebcc.h")).read()
    body = src[src.rindex("typedef struct {"): src.index("} ebcc_tuning;")]
    fields = re.findall(r"^\s*(?:uint32_t|int32_t)\s+(\w+);", body, flags=re.M)
    ebcc = _lib()
    assert fields == [f for f, _ in ebcc.Tuning._fields_]
    old = ebcc.get_tuning()
    assert old == {"t1_encoder": 0, "t1_decoder": 0, "t1_wave_max": 32768, "spiht": 0, "t1_lanes": 0, "t1_split": 10,
                   "t1_persist": 1}
    try:
        ebcc.set_tuning(t1_encoder=2, t1_wave_max=100, spiht=1, t1_lanes=64, t1_split=30, t1_persist=0)
        assert ebcc.get_tuning() == {"t1_encoder": 2, "t1_decoder": 0, "t1_wave_max": 100, "spiht": 1, "t1_lanes": 64,
                                     "t1_split": 30, "t1_persist": 0}
        for bad in (dict(spiht=5), dict(t1_lanes=8), dict(t1_split=101), dict(t1_persist=2)):
            try:
                ebcc.set_tuning(**bad)
                assert False
            except ebcc.EbccError as e:
                assert e.code == ebcc.EINVAL
    finally:
        ebcc.set_tuning(**old)
    assert ebcc.get_tuning() == old


def _hdr(ny, nx, L=5, cbl=(5, 5), T=1, mode=2):
    h = bytearray(48)
    h[:4] = b"EBCC"
    h[4], h[5], h[6], h[7] = 1, mode, L, cbl[0] | (cbl[1] << 4)
    h[8:12] = ny.to_bytes(4, "little")
    h[12:16] = nx.to_bytes(4, "little")
    h[32:34] = T.to_bytes(2, "little")
    return bytes(h)


def test_workspace_size_queries():
    """The workspace-size queries are host-only (plan geometry and the calls'
    own layout code): positive for valid shapes, 0 for invalid arguments,
    growing with the field, a batch needs no more than its fields alone, and
    a decompression no more than the compression of the same shape."""
    ebcc = _lib()
    shapes = [(91, 180), (181, 360), (361, 720), (721, 1440)]
    single = [ebcc.workspace_size(*s) for s in shapes]
    assert all(a > 0 for a in single) and single == sorted(single)
    assert single[-1] > 4 * 721 * 1440
    assert ebcc.workspace_size(0, 5) == 0 and ebcc.workspace_size(1 << 25, 2) == 0
    p = ebcc.params(cblk_log2w=2)           # 4x32 code-blocks: more blocks, more tables
    assert ebcc.workspace_size(721, 1440, p) > single[-1]
    # the tier-1 bypass adds a raw-bit table per block and pass; other values are refused
    assert ebcc.workspace_size(721, 1440, ebcc.params(bypass=1)) > single[-1]
    assert ebcc.workspace_size(721, 1440, ebcc.params(bypass=2)) == 0
    assert ebcc.workspace_size(721, 1440, ebcc.params(trunc=2)) == 0
    mix = [shapes[i % 4] for i in range(37)]
    batch = ebcc.workspace_size_batch(mix)
    assert 0 < batch <= sum(single[i % 4] for i in range(37))
    assert ebcc.workspace_size_batch([shapes[3]]) <= single[3]
    dec = ebcc.workspace_size_batch([shapes[3]], headers=[_hdr(721, 1440)], lengths=[100000])
    assert 0 < dec <= ebcc.workspace_size_batch([shapes[3]])
    # two code-block sizes decode in two calls: the workspace is the larger one
    both = ebcc.workspace_size_batch([shapes[3], shapes[3]], headers=[_hdr(721, 1440), _hdr(721, 1440, cbl=(2, 2))],
                                     lengths=[100000, 100000])
    small = ebcc.workspace_size_batch([shapes[3]], headers=[_hdr(721, 1440, cbl=(2, 2))], lengths=[100000])
    assert both == max(dec, small)
    # constant and raw streams need no field buffers
    const = ebcc.workspace_size_batch([shapes[3]], headers=[_hdr(721, 1440, mode=0)], lengths=[48])
    assert const < dec


def test_async_decode_refuses_bad_arguments():
    """ebcc_decompress_batch_async checks its arguments on the host before it
    enqueues anything: an empty batch is a no-op; negative counts, NULL
    arrays, shapes out of range and invalid parameters are EINVAL (the
    pointers below are never dereferenced)."""
    ebcc = _lib()
    L = ebcc.lib()
    C = ctypes
    fake = C.c_void_p(256)
    p = ebcc.params()

    def call(n, ny, nx, p, status=fake, d_in=fake):
        d_x = (C.c_void_p * max(1, n))(*([fake] * max(1, n)))
        a_ny = (C.c_size_t * max(1, n))(*([ny] * max(1, n)))
        a_nx = (C.c_size_t * max(1, n))(*([nx] * max(1, n)))
        return L.ebcc_decompress_batch_async(n, d_in, fake, fake, d_x, a_ny, a_nx, C.byref(p), status, None)

    assert L.ebcc_decompress_batch_async(0, None, None, None, None, None, None, C.byref(p), None, None) == ebcc.OK
    assert call(-1, 8, 8, p) == ebcc.EINVAL
    assert call(1, 8, 8, p, status=None) == ebcc.EINVAL
    assert call(1, 8, 8, p, d_in=None) == ebcc.EINVAL
    assert call(1, 0, 8, p) == ebcc.EINVAL
    assert call(2, 1 << 25, 8, p) == ebcc.EINVAL
    for bad in (dict(cblk_log2w=7), dict(spiht_tile=0), dict(levels=17), dict(trunc=2), dict(bypass=3)):
        assert call(1, 8, 8, ebcc.params(**bad)) == ebcc.EINVAL, bad


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """No CPU fallback: without libebcc.so every entry point of the binding
    raises, and host tensors are refused rather than compressed another way."""
    import numpy as np
    import pytest
    import torch
    from paper_2510_22265_amd import ebcc
    monkeypatch.setattr(ebcc, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libebcc.so"))
    monkeypatch.setattr(ebcc, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        ebcc.lib()
    with pytest.raises(RuntimeError, match="missing"):
        ebcc.params()
    with pytest.raises((TypeError, RuntimeError)):
        ebcc.compress(torch.from_numpy(np.zeros((8, 8), np.float32)), 0.01)
