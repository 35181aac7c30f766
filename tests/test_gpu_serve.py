"""Serving loop on the GPU: continuous batching over two lanes (streams).

Every result taken from the mix of concurrent compress and decompress
requests must equal the CPU oracle's result for that request alone: streams
byte for byte, decoded fields bit for bit (the stated tolerance for decoded
fields is 1e-6 relative; the batched path reproduces the single-field
arithmetic, so the difference is exactly zero).  A request that cannot be
served (a field with a NaN) fails alone; a stream with another code-block
size decodes in the mix.  The memory the server holds is measured on the
device (torch's live allocations plus the library's workspaces and tables)
and must stay within the HBM budget."""
import threading

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


class MemWatch:
    """Peak device memory while a server runs: torch's live allocations
    (max_memory_allocated, relative to the start), the library's workspaces
    and tables (ebcc_device_bytes, sampled), and the device's own free-memory
    reading (hipMemGetInfo, sampled)."""

    def __init__(self, ebcc):
        import torch
        self.torch, self.ebcc = torch, ebcc
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        self.alloc0 = torch.cuda.memory_allocated()
        self.reserved0 = torch.cuda.memory_reserved()
        self.lib0 = ebcc.device_bytes()
        self.free0 = torch.cuda.mem_get_info()[0]
        self.lib_peak, self.free_min = self.lib0, self.free0
        self._stop = threading.Event()
        self._t = threading.Thread(target=self._run, daemon=True)
        self._t.start()

    def _run(self):
        while not self._stop.wait(0.001):
            self.lib_peak = max(self.lib_peak, self.ebcc.device_bytes())
            self.free_min = min(self.free_min, self.torch.cuda.mem_get_info()[0])

    def stop(self):
        self._stop.set()
        self._t.join()
        torch = self.torch
        self.torch_peak = torch.cuda.max_memory_allocated() - self.alloc0
        self.cache_slack = (torch.cuda.max_memory_reserved() - self.reserved0) - self.torch_peak
        self.held = self.torch_peak + (self.lib_peak - self.lib0)
        self.device_peak = self.free0 - self.free_min
        return self


def _host_result(r):
    """on_done: keep a host copy of the result and release the device one."""
    if r.result is not None and hasattr(r.result, "cpu"):
        r.result = r.result.cpu().numpy()


def test_serving_mix_matches_oracle(gpu, ref):
    import torch
    from paper_2510_22265_amd import serve
    specs = synth.batch_specs(n=20, cfg=5)
    xs_h = [synth.batch_field(s, cfg=5) for s in specs]
    eps = [s[3] for s in specs]
    ref_streams = [ref.compress(x, e) for x, e in zip(xs_h, eps)]
    ref_fields = [ref.decompress(s, *x.shape) for s, x in zip(ref_streams, xs_h)]
    # a stream of 64x64 code-blocks and a field with a NaN join the mix
    x64 = synth.field("u", 181, 360, cfg=5, level=30)
    s64 = ref.compress(x64, 0.01, cbl2w=6, cbl2h=6)
    y64 = ref.decompress(s64, *x64.shape)
    xnan = synth.field("t", 91, 180, cfg=5, level=31)
    xnan[40, 50] = np.nan
    xs = [torch.from_numpy(x).cuda() for x in xs_h]
    dstreams = [torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() for s in ref_streams]
    d64 = torch.from_numpy(np.frombuffer(s64, np.uint8).copy()).cuda()
    dnan = torch.from_numpy(xnan).cuda()
    reqs = []
    for i, (x, e) in enumerate(zip(xs, eps)):
        reqs.append(serve.Request(serve.COMPRESS, x, eps=e, tag=("c", i), on_done=_host_result))
        reqs.append(serve.Request(serve.DECOMPRESS, dstreams[i], shape=tuple(x.shape), tag=("d", i),
                                  on_done=_host_result))
    reqs.append(serve.Request(serve.DECOMPRESS, d64, shape=x64.shape, tag=("d64", 0), on_done=_host_result))
    reqs.append(serve.Request(serve.COMPRESS, dnan, eps=0.01, tag=("nan", 0), on_done=_host_result))
    order = np.random.default_rng(4).permutation(len(reqs))
    budget = 4 * 10**9
    watch = MemWatch(gpu)
    srv = serve.Server(hbm_budget=budget, lanes=2).start()
    done, wall = serve.poisson_run(srv, lambda k: reqs[order[k]], rate=800.0, duration=30.0,
                                   max_requests=len(reqs))
    srv.stop()
    watch.stop()
    assert len(done) == len(reqs)
    for r in done:
        kind, i = r.tag
        if kind == "nan":
            assert r.status == gpu.EINVAL and r.result is None
            continue
        assert r.status == 0, r.tag
        if kind == "c":
            assert r.result.tobytes() == ref_streams[i], f"compress {i} differs from the oracle in the mix"
        elif kind == "d":
            assert np.array_equal(r.result.view(np.uint32), ref_fields[i].view(np.uint32)), f"decompress {i}"
        else:
            assert np.array_equal(r.result.view(np.uint32), y64.view(np.uint32))
    assert max(srv.batch_sizes) > 1
    assert srv.peak_in_use <= srv.req_budget
    assert watch.held <= budget, (watch.held, budget)
    st = serve.summarize(done, wall)
    assert st["failed"] == 1 and st["p99_ms"] >= st["p50_ms"]


def test_serving_tight_budget_measured(gpu, ref):
    """A budget that holds the lanes' workspaces and about two large requests
    at a time: every request is submitted at once, admission makes them wait
    for memory, every result is the oracle's, and the device memory the
    server holds (measured) never exceeds the budget."""
    import torch
    from paper_2510_22265_amd import serve
    shapes = [("t", 721, 1440), ("u", 91, 180), ("q", 361, 720), ("v", 181, 360), ("t", 721, 1440),
              ("u", 361, 720), ("v", 721, 1440), ("q", 181, 360)]
    xs_h = [synth.field(v, ny, nx, cfg=6, level=k) for k, (v, ny, nx) in enumerate(shapes)]
    ref_streams = [ref.compress(x, 0.01) for x in xs_h]
    xs = [torch.from_numpy(x).cuda() for x in xs_h]
    p = gpu.params()
    lane_ws = gpu.workspace_size_batch([(721, 1440)], p)
    big = serve.request_cost(serve.Request(serve.COMPRESS, xs[0], eps=0.01))
    budget = 2 * lane_ws + 2 * big + 1
    watch = MemWatch(gpu)
    srv = serve.Server(hbm_budget=budget, lanes=2, lane_workspace=lane_ws).start()
    rs = [srv.submit(serve.Request(serve.COMPRESS, x, eps=0.01, tag=i, on_done=_host_result))
          for i, x in enumerate(xs)]
    for r in rs:
        r.wait(120)
    srv.stop()
    watch.stop()
    for r in rs:
        assert r.status == 0 and r.result.tobytes() == ref_streams[r.tag], r.tag
    assert srv.peak_in_use <= srv.req_budget
    assert watch.held <= budget, (watch.held, budget)
    # the device's own reading also includes what torch's caching allocator
    # keeps beyond the live tensors, and a little HIP runtime memory
    assert watch.device_peak <= budget + max(0, watch.cache_slack) + (64 << 20), \
        (watch.device_peak, budget, watch.cache_slack)
