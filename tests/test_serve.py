"""Serving loop host logic on the CPU (admission by memory budget, FIFO,
continuous batching over lanes), with an executor that stands in for the
GPU.  The GPU executor itself is covered by the GPU serving tests."""
import threading
import time

import numpy as np
import pytest

from paper_2510_22265_amd import serve


class FakeData:
    def __init__(self, shape, value):
        self.shape = shape
        self.value = value

    def numel(self):
        return self.shape[0] * self.shape[1]


class FakeExecutor:
    """Sleeps in proportion to the batch's samples; result = f(value)."""

    def __init__(self, per_sample=2e-8, fail_tag=None):
        self.per_sample = per_sample
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.fail_tag = fail_tag

    def on_submit(self, req):
        pass

    def start_lane(self, lane):
        pass

    def run(self, lane, comp, dec):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        try:
            if any(r.tag == self.fail_tag for r in comp + dec):
                raise RuntimeError("planted executor failure")
            time.sleep(0.001 + self.per_sample * sum(r.samples for r in comp + dec))
            for r in comp:
                r.result, r.status = ("stream", r.data.value * 3 + 1), 0
            for r in dec:
                r.result, r.status = ("field", r.data.value * 5 - 2), 0
        finally:
            with self.lock:
                self.active -= 1

    def close(self):
        pass


SHAPES = [(91, 180), (181, 360), (361, 720), (721, 1440)]


def _make(i, rng):
    sh = SHAPES[rng.integers(0, 4)]
    if rng.random() < 0.5:
        return serve.Request(serve.COMPRESS, FakeData(sh, i), eps=0.01, tag=i)
    return serve.Request(serve.DECOMPRESS, FakeData((1, 4 * sh[0] * sh[1] // 8), i), shape=sh, tag=i)


def _check_results(reqs):
    for r in reqs:
        assert r.status == 0
        if r.kind == serve.COMPRESS:
            assert r.result == ("stream", r.data.value * 3 + 1)
        else:
            assert r.result == ("field", r.data.value * 5 - 2)


def test_all_requests_complete_under_budget():
    rng = np.random.default_rng(1)
    ex = FakeExecutor()
    budget = 3 * serve.request_cost(serve.Request(serve.COMPRESS, FakeData((721, 1440), 0)))
    srv = serve.Server(hbm_budget=budget, lanes=3, executor=ex).start()
    reqs, wall = serve.poisson_run(srv, lambda i: _make(i, rng), rate=2000.0, duration=0.3, seed=3)
    srv.stop()
    assert len(reqs) > 100
    _check_results(reqs)
    assert srv.peak_in_use <= budget
    assert srv.in_use == 0
    assert ex.max_active >= 2                      # batches overlapped on lanes
    assert max(srv.batch_sizes) > 1               # requests were batched
    st = serve.summarize(reqs, wall)
    assert st["requests"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_continuous_batching_admits_during_a_batch():
    """Requests that arrive while a batch runs go into a later batch of a
    free lane, not after the whole queue drains."""
    ex = FakeExecutor(per_sample=1e-7)
    srv = serve.Server(lanes=2, executor=ex).start()
    first = srv.submit(serve.Request(serve.COMPRESS, FakeData((721, 1440), 0), eps=0.01, tag=0))
    time.sleep(0.02)                               # the first batch (about 0.1 s) is running
    later = [srv.submit(serve.Request(serve.COMPRESS, FakeData((91, 180), i), eps=0.01, tag=i)) for i in range(1, 6)]
    for r in later:
        r.wait(5)
    assert not first.done.is_set()                 # served by the other lane meanwhile
    first.wait(5)
    assert all(r.t_done < first.t_done for r in later)
    srv.stop()
    _check_results([first] + later)
    assert len({r.batch_id for r in later}) >= 1 and first.batch_id not in {r.batch_id for r in later}


def test_fifo_admission_with_tight_budget():
    ex = FakeExecutor()
    one = serve.request_cost(serve.Request(serve.COMPRESS, FakeData((361, 720), 0)))
    srv = serve.Server(hbm_budget=one, lanes=2, executor=ex).start()
    reqs = [srv.submit(serve.Request(serve.COMPRESS, FakeData((361, 720), i), eps=0.01, tag=i)) for i in range(8)]
    for r in reqs:
        r.wait(5)
    srv.stop()
    _check_results(reqs)
    assert srv.peak_in_use <= one
    assert ex.max_active == 1                      # only one request fits at a time
    admits = [r.t_admit for r in reqs]
    assert admits == sorted(admits)                # first come, first admitted


def test_oversized_request_is_refused():
    srv = serve.Server(hbm_budget=1000, lanes=1, executor=FakeExecutor()).start()
    with pytest.raises(ValueError):
        srv.submit(serve.Request(serve.COMPRESS, FakeData((91, 180), 0), eps=0.01))
    srv.stop()


def test_executor_failure_is_reported_per_batch():
    ex = FakeExecutor(fail_tag=7)
    srv = serve.Server(lanes=1, max_batch=1, executor=ex).start()
    reqs = [srv.submit(serve.Request(serve.COMPRESS, FakeData((91, 180), i), eps=0.01, tag=i)) for i in range(10)]
    for r in reqs:
        r.wait(5)
    srv.stop()
    assert isinstance(reqs[7].status, RuntimeError)
    _check_results(reqs[:7] + reqs[8:])


class WsExecutor(FakeExecutor):
    """A stand-in with a library workspace: a request needs one byte per
    sample, a batch the sum plus a fixed overhead per call."""

    def __init__(self, overhead=0, **kw):
        super().__init__(**kw)
        self.overhead = overhead
        self.reserved = {}
        self.batch_ws = []

    def workspace(self, req):
        return req.samples + self.overhead

    def batch_workspace(self, comp, dec):
        return max(sum(r.samples for r in comp) + (self.overhead if comp else 0),
                   sum(r.samples for r in dec) + (self.overhead if dec else 0))

    def reserve(self, lane, nbytes):
        self.reserved[lane] = nbytes

    def run(self, lane, comp, dec):
        self.batch_ws.append(self.batch_workspace(comp, dec))
        super().run(lane, comp, dec)


def test_lane_workspaces_bound_batches():
    """Each lane reserves its workspace at start; no batch needs more than
    that; the requests share what the workspaces leave of the budget."""
    ex = WsExecutor(overhead=1000)
    n = 361 * 720
    one = serve.request_cost(serve.Request(serve.COMPRESS, FakeData((361, 720), 0)))
    lane_ws = 3 * (n + 1000)               # three requests by their own sizes
    srv = serve.Server(hbm_budget=2 * lane_ws + 8 * one, lanes=2, lane_workspace=lane_ws, executor=ex).start()
    assert srv.req_budget == 8 * one and srv.reserved == 2 * lane_ws
    reqs = [srv.submit(serve.Request(serve.COMPRESS, FakeData((361, 720), i), eps=0.01, tag=i)) for i in range(24)]
    for r in reqs:
        r.wait(5)
    srv.stop()
    _check_results(reqs)
    assert ex.reserved == {0: lane_ws, 1: lane_ws}
    assert max(ex.batch_ws) <= lane_ws and max(srv.batch_sizes) == 3
    assert srv.peak_in_use <= srv.req_budget
    with pytest.raises(ValueError):     # more workspace than a lane has
        serve.Server(hbm_budget=10**9, lanes=1, lane_workspace=100, executor=WsExecutor()).submit(
            serve.Request(serve.COMPRESS, FakeData((91, 180), 0), eps=0.01))
    with pytest.raises(ValueError):     # the workspaces take the whole budget
        serve.Server(hbm_budget=100, lanes=2, lane_workspace=50, executor=WsExecutor())


def test_batch_workspace_decides_over_the_sum():
    """When the library's sizing of a batch exceeds the lane's workspace
    although the requests' own sizes fit, the last requests go back to the
    front of the queue (FIFO is kept)."""
    ex = WsExecutor(overhead=1000)
    ex.workspace = lambda req: req.samples             # understates each request's need
    n = 181 * 360
    srv = serve.Server(hbm_budget=10**9, lanes=1, lane_workspace=2 * n + 1000, executor=ex).start()
    reqs = [srv.submit(serve.Request(serve.COMPRESS, FakeData((181, 360), i), eps=0.01, tag=i)) for i in range(9)]
    for r in reqs:
        r.wait(5)
    srv.stop()
    _check_results(reqs)
    assert max(ex.batch_ws) <= 2 * n + 1000
    starts = [r.t_start for r in reqs]
    assert starts == sorted(starts)


def test_batch_is_the_longest_prefix_that_fits():
    """A batch shares workspace (the library sizes it below the sum of its
    requests alone): the lane takes the longest FIFO prefix whose batch
    sizing fits its workspace, more requests than their own sizes would
    allow, and never one that does not fit."""
    ex = WsExecutor(per_sample=1e-6)
    n = 181 * 360
    ex.workspace = lambda req: req.samples
    ex.batch_workspace = lambda comp, dec: max(sum(r.samples for r in comp) // 2 + 1000,
                                               sum(r.samples for r in dec) // 2 + 1000)
    lane_ws = 3 * n                         # own sizes: 3 per batch; batch sizing: 5
    srv = serve.Server(hbm_budget=10**9, lanes=1, lane_workspace=lane_ws, executor=ex)
    blocker = srv.submit(serve.Request(serve.COMPRESS, FakeData((181, 360), 99), eps=0.01, tag=99))
    srv.start()
    time.sleep(0.01)                        # the lane is busy with the first request (65 ms)
    reqs = [srv.submit(serve.Request(serve.COMPRESS, FakeData((181, 360), i), eps=0.01, tag=i)) for i in range(12)]
    for r in [blocker] + reqs:
        r.wait(10)
    srv.stop()
    _check_results(reqs)
    assert max(ex.batch_ws) <= lane_ws
    assert max(srv.batch_sizes) == 5
    starts = [r.t_start for r in reqs]
    assert starts == sorted(starts)


def test_on_done_runs_before_completion_is_signalled():
    seen = []
    srv = serve.Server(lanes=1, executor=FakeExecutor()).start()
    reqs = [srv.submit(serve.Request(serve.COMPRESS, FakeData((91, 180), i), eps=0.01, tag=i,
                                     on_done=lambda r: seen.append((r.tag, r.done.is_set(), r.status))))
            for i in range(5)]
    for r in reqs:
        r.wait(5)
    srv.stop()
    assert sorted(seen) == [(i, False, 0) for i in range(5)]
