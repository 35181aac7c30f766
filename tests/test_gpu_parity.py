"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Streams must be byte-identical, stage results (DWT coefficients, planes and
kept passes per code-block, base reconstruction, residual coefficients,
truncation plane) bit-identical, and decoded fields bit-identical (the
contract's tolerance is 1e-6 relative; the arithmetic is the same FP32
sequence on both sides, so the expected difference is exactly 0).  Every
decoded point must satisfy |x - x_hat| <= eps in FP64."""
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


def _bound_ok(x, y, eps):
    return np.abs(x.astype(np.float64) - y.astype(np.float64)).max() <= eps


_GPU_NAMES = {"cbl2w": "cblk_log2w", "cbl2h": "cblk_log2h", "tile": "spiht_tile"}


def _gpu_kw(kw):
    return {_GPU_NAMES.get(k, k): v for k, v in kw.items()}


def _roundtrip(gpu, ref, x, eps_rel, **kw):
    s_ref = ref.compress(x, eps_rel, **kw)
    s_gpu = _host(gpu.compress(_dev(x), eps_rel, **_gpu_kw(kw))).tobytes()
    assert len(s_gpu) == len(s_ref)
    if s_gpu != s_ref:
        d = np.nonzero(np.frombuffer(s_gpu, np.uint8) != np.frombuffer(s_ref, np.uint8))[0]
        pytest.fail(f"streams differ at {d.size} bytes, first at {d[0]} of {len(s_ref)}")
    y_gpu = _host(gpu.decompress(_dev(np.frombuffer(s_ref, np.uint8).copy()), *x.shape))
    y_ref = ref.decompress(s_ref, *x.shape)
    assert np.array_equal(y_gpu.view(np.uint32), y_ref.view(np.uint32))
    rng_ = float(x.max()) - float(x.min())
    eps = eps_rel * rng_ if kw.get("bound_mode", 0) == 0 else eps_rel
    assert _bound_ok(x, y_gpu, eps)
    return s_ref


def test_stage_parity_plain_field(gpu, ref):
    """181x360 temperature-like field, 1% bound, r = 30: every stage."""
    x = synth.plain_field()
    s_ref, tr = ref.compress(x, 0.01, trace=True)
    s_gpu, tg = gpu.compress_trace(_dev(x), 0.01)
    for k in ("mode", "L", "e0", "e_r", "n_max", "n_s", "nblocks", "ntiles", "base_bytes", "resid_bytes"):
        assert tg[k] == tr[k], k
    assert np.array_equal(_host(tg["coef"]).view(np.uint32), tr["coef"].view(np.uint32))
    assert np.array_equal(_host(tg["pb"]), tr["pb"])
    assert np.array_equal(_host(tg["kb"]), tr["kb"])
    assert np.array_equal(_host(tg["abase"]).view(np.uint32), tr["abase"].view(np.uint32))
    assert np.array_equal(_host(tg["cres"]).view(np.uint32), tr["cres"].view(np.uint32))
    assert _host(s_gpu).tobytes() == s_ref


SHAPES = [(1, 1), (1, 7), (9, 1), (2, 2), (3, 3), (5, 64), (33, 17), (64, 64), (100, 3), (91, 180), (129, 255)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("eps", [1e-3, 1e-2, 1e-1])
def test_stream_parity_shapes(gpu, ref, shape, eps):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    x = (rng.standard_normal(shape) * 5 + 280).astype(np.float32)
    if shape[0] >= 8 and shape[1] >= 8:
        x = synth.field("u", *shape, cfg=1, level=shape[0] % 7)
    _roundtrip(gpu, ref, x, eps)


@pytest.mark.parametrize("var", ["t", "u", "v", "q"])
@pytest.mark.parametrize("eps", [1e-3, 1e-2, 1e-1])
def test_stream_parity_era5_like(gpu, ref, var, eps):
    _roundtrip(gpu, ref, synth.field(var, 181, 360, cfg=1, level=5), eps)


@pytest.mark.parametrize("cb", [(2, 2), (4, 6), (6, 6), (5, 3), (6, 2), (3, 5), (6, 4)])
def test_stream_parity_codeblock_sizes(gpu, ref, cb):
    x = synth.field("t", 97, 203, cfg=1, level=2)
    _roundtrip(gpu, ref, x, 0.004, cbl2w=cb[0], cbl2h=cb[1])


@pytest.mark.parametrize("levels", [0, 1, 2, 3, 6, 9])
@pytest.mark.parametrize("tile", [1, 3])
def test_stream_parity_levels_tiles(gpu, ref, levels, tile):
    x = synth.field("v", 70, 130, cfg=1, level=levels)
    _roundtrip(gpu, ref, x, 0.003, levels=levels, tile=tile, base_ratio=12.0)


@pytest.mark.parametrize("ratio", [1.0, 4.0, 100.0, 1000.0])
def test_stream_parity_ratios(gpu, ref, ratio):
    _roundtrip(gpu, ref, synth.field("q", 91, 180, cfg=1, level=1), 0.01, base_ratio=ratio)


def test_absolute_bound(gpu, ref):
    _roundtrip(gpu, ref, synth.field("t", 91, 180, cfg=1), 0.3, bound_mode=1)


def test_special_streams(gpu, ref):
    c = np.full((37, 41), 273.15, np.float32)
    assert _roundtrip(gpu, ref, c, 0.01)[5] == 0          # constant -> header only
    x = synth.field("t", 20, 30)
    assert _roundtrip(gpu, ref, x, 1e-13)[5] == 1         # bound below FP32 -> raw
    z = np.zeros((16, 16), np.float32)
    z[3, 4] = -0.0
    z[5, 5] = 1.0
    _roundtrip(gpu, ref, z, 0.01)


def test_error_paths(gpu):
    import torch
    x = _dev(synth.field("v", 16, 16))
    p = gpu.params(0.01)
    bad = x.clone()
    bad[3, 3] = float("nan")
    out = torch.empty(gpu.compress_bound(16, 16), dtype=torch.uint8, device="cuda")
    rc, _ = gpu.compress_into(bad, out, p)
    assert rc == gpu.EINVAL
    small = torch.empty(10, dtype=torch.uint8, device="cuda")
    rc, need = gpu.compress_into(x, small, p)
    assert rc == gpu.ENOSPC and need > 10
    with pytest.raises(gpu.EbccError) as e:
        gpu.compress(x, 0.01, q=1.5)
    assert e.value.code == gpu.EINVAL
    s = gpu.compress(x, 0.01).clone()
    y = torch.empty((16, 16), dtype=torch.float32, device="cuda")
    assert gpu.decompress_into(s, y) == 0
    assert gpu.decompress_into(s, torch.empty((16, 17), dtype=torch.float32, device="cuda")) == gpu.EINVAL
    c = s.clone()
    c[60] ^= 0x10
    assert gpu.decompress_into(c, y) == gpu.ECORRUPT
    assert gpu.decompress_into(s[:-1].clone(), y) == gpu.ECORRUPT


def test_deterministic(gpu):
    x = _dev(synth.field("q", 181, 360, cfg=1, level=9))
    a = _host(gpu.compress(x, 0.003)).tobytes()
    b = _host(gpu.compress(x, 0.003)).tobytes()
    assert a == b


@pytest.mark.parametrize("var", ["t", "u", "v", "q"])
@pytest.mark.parametrize("eps", [1e-3, 1e-2, 1e-1])
def test_full_size_era5_stack_fields(gpu, ref, var, eps):
    """721x1440 fields (the ERA5-shaped stack's grid), three bounds."""
    _roundtrip(gpu, ref, synth.field(var, 721, 1440, cfg=1, level=17), eps)


@pytest.mark.parametrize("variant", ["lane", "wave", "wave-nopipe"])
@pytest.mark.parametrize("cb", [(5, 5), (6, 6), (2, 3), (6, 4)])
def test_tier1_kernel_variants(gpu, ref, variant, cb, monkeypatch):
    """Both tier-1 kernel families (wave per block for few blocks, lanes per
    block for large batches), and the wave encoder with and without its
    modelling/coding pipeline, produce the oracle's stream and decode."""
    monkeypatch.setenv("EBCC_T1_KERNEL", variant.split("-")[0])
    monkeypatch.setenv("EBCC_T1_PIPE", "0" if variant.endswith("nopipe") else "1")
    x = synth.field("u", 181, 360, cfg=1, level=11)
    _roundtrip(gpu, ref, x, 0.002, cbl2w=cb[0], cbl2h=cb[1])


@pytest.mark.parametrize("variant", ["global", "lds"])
@pytest.mark.parametrize("shape,levels,tile", [((181, 360), 5, 1), ((181, 360), 5, 2), ((97, 203), 3, 3),
                                                ((70, 130), 6, 1), ((33, 17), 2, 2)])
def test_spiht_kernel_variants(gpu, ref, variant, shape, levels, tile, monkeypatch):
    """Both SPIHT kernel families (tile in LDS, lists in global memory)
    produce the oracle's stream and decode."""
    monkeypatch.setenv("EBCC_SPIHT_KERNEL", variant)
    x = synth.field("v", *shape, cfg=1, level=13)
    _roundtrip(gpu, ref, x, 0.002, levels=levels, tile=tile)


@pytest.mark.parametrize("var,shape,eps", [("t", (91, 180), 0.01), ("u", (181, 360), 0.001), ("q", (64, 96), 0.05),
                                           ("v", (129, 255), 0.01), ("u", (33, 47), 0.02), ("t", (5, 64), 0.01)])
@pytest.mark.parametrize("q", [1 - 1e-5, 0.99, 0.5, 1.0])
def test_stream_parity_ratio_search(gpu, ref, var, shape, eps, q):
    """Algorithm 1's base-ratio feedback search (q > 0) and its base-only
    fallback: the oracle's stream, byte for byte."""
    x = synth.field(var, *shape, cfg=1, level=1)
    _roundtrip(gpu, ref, x, eps, q=q)
