"""ebcc_compress_noalloc, the entry point for callers that cannot allocate:
called through the C ABI, its streams must be byte-identical to
ebcc_compress's on the same field (two calls in a row, the second on a
smaller field, so the second call runs over what the first left in the
static scratch), the device's free memory must not move across its calls,
and a field whose workspace does not fit the scratch is refused before any
work is queued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2510_22265_amd import ebcc, synth

pytestmark = pytest.mark.gpu


def _noalloc(x, out, p, stream):
    n = ctypes.c_size_t(0)
    rc = ebcc.lib().ebcc_compress_noalloc(ctypes.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], ctypes.byref(p),
                                          ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(n),
                                          ctypes.c_void_p(stream.cuda_stream))
    return rc, n.value


@pytest.mark.parametrize("q", [0.0, 1 - 1e-5])
def test_noalloc_streams_equal_compress(q):
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    # a 721x1440 wind-like field, then a smaller temperature-like one
    cases = [(synth.field("u", 721, 1440, cfg=1, level=3), 0.01), (synth.plain_field(181, 360, seed=7), 0.001)]
    xs = [torch.from_numpy(h).to(dev) for h, _ in cases]
    ref_out = [torch.empty(ebcc.compress_bound(*h.shape), dtype=torch.uint8, device=dev) for h, _ in cases]
    na_out = [torch.zeros(ebcc.compress_bound(*h.shape), dtype=torch.uint8, device=dev) for h, _ in cases]
    ref_len = []
    for (h, e), x, o in zip(cases, xs, ref_out):
        print(f"ebcc_compress {h.shape} eps {e} q {q}", flush=True)
        rc, n = ebcc.compress_into(x, o, ebcc.params(e, 30.0, q=q), stream)
        assert rc == 0, ebcc.lib().ebcc_last_error()
        ref_len.append(n)
    torch.cuda.synchronize()
    # nothing else touches device memory between the two readings (the
    # comparisons below allocate through torch, so they come after)
    free0, _ = torch.cuda.mem_get_info(dev)
    res = []
    for (h, e), x, o in zip(cases, xs, na_out):
        print(f"ebcc_compress_noalloc {h.shape} eps {e} q {q}", flush=True)
        rc, n = _noalloc(x, o, ebcc.params(e, 30.0, q=q), stream)
        res.append((rc, n, ebcc.lib().ebcc_last_error()))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(dev)
    for k, (rc, n, msg) in enumerate(res):
        assert rc == 0, msg
        assert n == ref_len[k]
        assert torch.equal(na_out[k][:n], ref_out[k][:n]), f"stream of call {k} differs from ebcc_compress's"
    assert free1 == free0, (free0, free1)


def test_noalloc_decodes_within_bound_and_refuses_oversize():
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    h = synth.field("q", 361, 720, cfg=1, level=5)
    x = torch.from_numpy(h).to(dev)
    out = torch.empty(ebcc.compress_bound(*h.shape), dtype=torch.uint8, device=dev)
    rc, n0 = _noalloc(x, out, ebcc.params(0.01, 30.0), stream)
    assert rc == 0, ebcc.lib().ebcc_last_error()
    y = ebcc.decompress(out[:n0], *h.shape).cpu().numpy()
    eps = 0.01 * (float(h.max()) - float(h.min()))
    assert float(np.abs(h.astype(np.float64) - y.astype(np.float64)).max()) <= eps
    # too large for the static scratch: refused with EINVAL, nothing launched
    big = torch.zeros((2048, 4096), dtype=torch.float32, device=dev)
    big_out = torch.empty(64, dtype=torch.uint8, device=dev)
    print("ebcc_compress_noalloc (2048, 4096): expect EINVAL", flush=True)
    rc, n = _noalloc(big, big_out, ebcc.params(0.01, 30.0), stream)
    assert rc == ebcc.EINVAL and n == 0
    assert b"scratch" in ebcc.lib().ebcc_last_error()
    # ENOSPC reports the size needed, as ebcc_compress does
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    rc, need = _noalloc(x, small, ebcc.params(0.01, 30.0), stream)
    assert rc == ebcc.ENOSPC and need == n0
