"""Serving loop on the GPU: continuous batching over two lanes (streams).

Every result, taken from the mix of concurrent compress and decompress
requests, must equal the same request served alone: streams byte for byte,
decoded fields bit for bit (the stated tolerance for decoded fields is 1e-6
relative; the batched path reproduces the single-field arithmetic, so the
difference is exactly zero)."""
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


def test_serving_mix_equals_solo(gpu):
    import torch
    from paper_2510_22265_amd import serve
    specs = synth.batch_specs(n=20, cfg=5)
    xs = [torch.from_numpy(synth.batch_field(s, cfg=5)).cuda() for s in specs]
    eps = [s[3] for s in specs]
    solo_streams = [gpu.compress(x, e).clone() for x, e in zip(xs, eps)]
    solo_fields = [gpu.decompress(s, *x.shape) for s, x in zip(solo_streams, xs)]
    reqs = []
    for i, (x, e) in enumerate(zip(xs, eps)):
        reqs.append(serve.Request(serve.COMPRESS, x, eps=e, tag=("c", i)))
        reqs.append(serve.Request(serve.DECOMPRESS, solo_streams[i], shape=tuple(x.shape), tag=("d", i)))
    order = np.random.default_rng(4).permutation(len(reqs))
    srv = serve.Server(hbm_budget=4 * 10**9, lanes=2).start()
    done, wall = serve.poisson_run(srv, lambda k: reqs[order[k]], rate=400.0, duration=30.0,
                                   max_requests=len(reqs))
    srv.stop()
    assert len(done) == len(reqs)
    for r in done:
        assert r.status == 0, r.tag
        kind, i = r.tag
        if kind == "c":
            assert torch.equal(r.result, solo_streams[i]), f"compress {i} differs in the mix"
        else:
            assert torch.equal(r.result.view(torch.int32), solo_fields[i].view(torch.int32)), f"decompress {i}"
    assert max(srv.batch_sizes) > 1
    assert srv.peak_in_use <= 4 * 10**9
    st = serve.summarize(done, wall)
    assert st["failed"] == 0 and st["p99_ms"] >= st["p50_ms"]


def test_serving_tight_budget(gpu):
    """A budget that holds about one large request at a time still serves a
    mix of sizes correctly (admission waits for memory to free up)."""
    import torch
    from paper_2510_22265_amd import serve
    xs = [torch.from_numpy(synth.field(v, ny, nx, cfg=6, level=k)).cuda()
          for k, (v, ny, nx) in enumerate([("t", 721, 1440), ("u", 91, 180), ("q", 361, 720), ("v", 181, 360),
                                           ("t", 721, 1440), ("u", 361, 720)])]
    solo = [gpu.compress(x, 0.01).clone() for x in xs]
    big = serve.request_cost(serve.Request(serve.COMPRESS, xs[0], eps=0.01))
    srv = serve.Server(hbm_budget=big + 1, lanes=2).start()
    rs = [srv.submit(serve.Request(serve.COMPRESS, x, eps=0.01, tag=i)) for i, x in enumerate(xs)]
    for r in rs:
        r.wait(60)
    srv.stop()
    for r in rs:
        assert r.status == 0 and torch.equal(r.result, solo[r.tag])
    assert srv.peak_in_use <= big + 1
