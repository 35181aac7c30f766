"""GPU parity of the byte-granular residual truncation (trunc = 1: Algorithm
1's second binary search at byte positions of the tiles' codes read as one
embedded sequence): every stream byte-identical to the oracle's, every
decode bit-identical, the bound met everywhere; single fields of several
shapes, tiles and bounds, the ratio search on top, both SPIHT kernel
families, batches mixing cut and plane-end streams, and full 721x1440
fields."""
import numpy as np
import pytest

from paper_2510_22265_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_22265_amd import ebcc
    ebcc.lib()
    return ebcc


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    return t.cpu().numpy()


def _same(a, b, what):
    if a != b:
        n = min(len(a), len(b))
        d = np.nonzero(np.frombuffer(a[:n], np.uint8) != np.frombuffer(b[:n], np.uint8))[0]
        first = int(d[0]) if d.size else n
        pytest.fail(f"{what}: lengths {len(a)} / {len(b)}, first difference at byte {first}")


def _roundtrip(gpu, ref, x, eps, tile=1, levels=5, q=0.0):
    print(f"byte cut: {x.shape} eps {eps} tile {tile} levels {levels} q {q}", flush=True)
    s_ref, tr = ref.compress(x, eps, tile=tile, levels=levels, q=q, trunc=1, trace=True)
    s_gpu = _host(gpu.compress(_dev(x), eps, spiht_tile=tile, levels=levels, q=q, trunc=1)).tobytes()
    _same(s_gpu, s_ref, "stream")
    y_gpu = _host(gpu.decompress(_dev(np.frombuffer(s_ref, np.uint8).copy()), *x.shape))
    y_ref = ref.decompress(s_ref, *x.shape)
    assert np.array_equal(y_gpu.view(np.uint32), y_ref.view(np.uint32))
    rng_ = float(x.max()) - float(x.min())
    assert np.abs(x.astype(np.float64) - y_gpu.astype(np.float64)).max() <= eps * rng_
    return s_ref, tr


@pytest.mark.parametrize("var,shape,eps,tile", [("u", (181, 360), 0.01, 1), ("v", (181, 360), 0.002, 1),
                                                ("t", (91, 180), 0.005, 1), ("q", (129, 255), 0.003, 2),
                                                ("u", (97, 203), 0.01, 3), ("v", (33, 47), 0.02, 1),
                                                ("u", (8, 8), 0.01, 1), ("t", (64, 96), 0.002, 64),
                                                ("v", (361, 720), 0.01, 1)])
def test_byte_cut_matches_oracle(gpu, ref, var, shape, eps, tile):
    x = synth.field(var, *shape, cfg=7, level=3)
    s, tr = _roundtrip(gpu, ref, x, eps, tile=tile)
    if tr["resid_bytes"]:
        assert s[34] & 1


@pytest.mark.parametrize("q", [1 - 1e-5, 0.5])
def test_byte_cut_with_ratio_search(gpu, ref, q):
    _roundtrip(gpu, ref, synth.field("u", 181, 360, cfg=7, level=5), 0.01, q=q)


@pytest.mark.parametrize("variant", ["global", "lds"])
@pytest.mark.parametrize("shape,levels,tile", [((181, 360), 5, 1), ((97, 203), 3, 3), ((70, 130), 6, 1)])
def test_byte_cut_spiht_kernel_variants(gpu, ref, variant, shape, levels, tile, monkeypatch):
    monkeypatch.setenv("EBCC_SPIHT_KERNEL", variant)
    _roundtrip(gpu, ref, synth.field("v", *shape, cfg=7, level=13), 0.002, tile=tile, levels=levels)


def test_byte_cut_batch_and_mixed_decode(gpu, ref):
    """Batched compression with trunc = 1 gives each field's oracle stream;
    a decode batch mixing cut and plane-end streams decodes each like the
    oracle."""
    xs = [synth.field(v, *sh, cfg=7, level=k) for k, (v, sh) in
          enumerate([("u", (181, 360)), ("t", (91, 180)), ("v", (129, 255)), ("q", (64, 96)), ("u", (33, 47))])]
    eps = [0.01, 0.003, 0.01, 0.002, 0.02]
    print("byte cut batch", flush=True)
    streams = gpu.compress_batch([_dev(x) for x in xs], err_bounds=eps, trunc=1)
    cut = []
    for i, (x, e) in enumerate(zip(xs, eps)):
        s_ref = ref.compress(x, e, trunc=1)
        _same(_host(streams[i]).tobytes(), s_ref, f"field {i}")
        cut.append(s_ref)
    plain = [ref.compress(x, e) for x, e in zip(xs, eps)]
    mix = [cut[i] if i % 2 == 0 else plain[i] for i in range(len(xs))] + [cut[1], plain[0]]
    shapes = [x.shape for x in xs] + [xs[1].shape, xs[0].shape]
    ys = gpu.decompress_batch([_dev(np.frombuffer(s, np.uint8).copy()) for s in mix], shapes)
    for i, (s, sh) in enumerate(zip(mix, shapes)):
        y_ref = ref.decompress(s, *sh)
        assert np.array_equal(_host(ys[i]).view(np.uint32), y_ref.view(np.uint32)), f"stream {i}"


@pytest.mark.parametrize("var", ["u", "v", "q"])
def test_byte_cut_full_size_fields(gpu, ref, var):
    """721x1440 fields (the ERA5-shaped stack's grid) at 1%: the cut stream
    is the oracle's and no longer than the plane-end stream (plus its
    8-byte trailer)."""
    x = synth.field(var, 721, 1440, cfg=1, level=21)
    s, _ = _roundtrip(gpu, ref, x, 0.01)
    assert len(s) <= len(ref.compress(x, 0.01)) + 8


def test_byte_cut_corrupt_trailer_is_reported(gpu, ref):
    """A trailer naming a tile the field does not have is a corrupt stream
    (status), not an out-of-range access."""
    x = synth.field("u", 91, 180, cfg=7, level=2)
    s = bytearray(ref.compress(x, 0.01, trunc=1))
    assert s[34] & 1
    s[-8:-4] = (0x7FFFFFF0).to_bytes(4, "little")
    # the checksum covers the trailer: restore it so that the trailer check is what fails
    import struct
    body = bytes(s[48:])
    ck = 0
    for k in range((len(body) + 3) // 4):
        w = int.from_bytes(body[4 * k: 4 * k + 4].ljust(4, b"\0"), "little")
        ck = (ck + w * (2 * k + 1)) & 0xFFFFFFFF
    s[44:48] = struct.pack("<I", ck)
    assert ref.decompress_rc(bytes(s), *x.shape) != 0
    from paper_2510_22265_amd import ebcc
    with pytest.raises(ebcc.EbccError) as e:
        gpu.decompress(_dev(np.frombuffer(bytes(s), np.uint8).copy()), *x.shape)
    assert e.value.code == ebcc.ECORRUPT
