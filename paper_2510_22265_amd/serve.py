"""Serving loop: continuous batching of compress / decompress requests.

Requests of mixed sizes (device-resident fields to compress, device-resident
streams to decompress) arrive at any time.  An admission controller keeps
the device memory that admitted requests hold (inputs, outputs and the
library's per-sample workspace) under an HBM budget; admitted requests wait
in FIFO order for a lane.  Each lane is one host thread with its own HIP
stream (the library keeps one workspace per stream): when a lane is free it
takes every admitted request that is waiting (up to a batch cap) and runs
them as one `ebcc_compress_batch` and one `ebcc_decompress_batch` call.
Requests that arrive while the lanes are busy are admitted as memory frees
up and go into the next batch of whichever lane frees first, so batches on
different lanes overlap on the device.  Every result is byte-identical to
what the request would produce alone (the batched entry points guarantee
it; the GPU tests check it in the mix).

The executor (what a lane runs for a batch) is a parameter, so the
admission and batching logic can be exercised without a GPU.
"""
import collections
import threading
import time

COMPRESS, DECOMPRESS = "compress", "decompress"

# Device bytes the library's workspace takes per sample of a compressed field
# (eight float planes, four u32 planes, per-code-block pass tables, codeword
# slots and SPIHT slots, rounded up); decompression needs less.
WS_BYTES_PER_SAMPLE = 128


class Request:
    """One request.  kind COMPRESS: `data` is a float32 device tensor
    (ny, nx), `eps` its range-relative bound; result = uint8 stream tensor.
    kind DECOMPRESS: `data` is a uint8 device stream, `shape` = (ny, nx);
    result = float32 field tensor."""

    __slots__ = ("kind", "data", "shape", "eps", "tag", "t_arrive", "t_admit", "t_start", "t_done", "result",
                 "status", "cost", "done", "lane", "batch_id", "ready")

    def __init__(self, kind, data, shape=None, eps=None, tag=None):
        self.kind = kind
        self.data = data
        self.shape = tuple(shape if shape is not None else data.shape)
        self.eps = eps
        self.tag = tag
        self.t_arrive = self.t_admit = self.t_start = self.t_done = None
        self.result = None
        self.status = None
        self.cost = 0
        self.done = threading.Event()
        self.lane = None
        self.batch_id = None
        self.ready = None      # executor's marker that the data is ready

    @property
    def samples(self):
        return self.shape[0] * self.shape[1]

    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive

    def wait(self, timeout=None):
        return self.done.wait(timeout)


def request_cost(req):
    """Device bytes an admitted request holds until it completes."""
    n = req.samples
    if req.kind == COMPRESS:
        return 4 * n + (48 + 4 * n) + WS_BYTES_PER_SAMPLE * n      # field, stream capacity, workspace
    return req.data.numel() + 4 * n + (WS_BYTES_PER_SAMPLE // 2) * n  # stream, field, workspace


class Server:
    """Continuous-batching server.

    hbm_budget   bytes that admitted requests may hold together (a request
                 larger than the whole budget is refused with ValueError)
    lanes        concurrent batches (one stream and host thread each)
    max_batch    requests per batch
    max_samples  samples per batch
    executor     callable(lane, compress_reqs, decompress_reqs) that fills
                 req.result / req.status; default: the GPU executor
    """

    def __init__(self, hbm_budget=64 * 10**9, lanes=2, max_batch=256, max_samples=1 << 27, executor=None,
                 params=None, base_ratio=30.0):
        self.budget = int(hbm_budget)
        self.lanes = int(lanes)
        self.max_batch = int(max_batch)
        self.max_samples = int(max_samples)
        self.params = params or {}
        self.base_ratio = base_ratio
        self.executor = executor or GpuExecutor(self.params, base_ratio)
        self._cv = threading.Condition()
        self._pending = collections.deque()    # arrived, not admitted
        self._ready = collections.deque()      # admitted, waiting for a lane
        self.in_use = 0
        self.peak_in_use = 0
        self._running = False
        self._threads = []
        self._batches = 0
        self.batch_sizes = []
        self.completed = []

    # ---- client side ----
    def submit(self, req):
        req.cost = request_cost(req)
        if req.cost > self.budget:
            raise ValueError(f"request needs {req.cost} B, more than the whole budget {self.budget} B")
        req.t_arrive = time.perf_counter()
        self.executor.on_submit(req)
        with self._cv:
            self._pending.append(req)
            self._admit_locked()
            self._cv.notify_all()
        return req

    # ---- admission: FIFO, as memory frees up ----
    def _admit_locked(self):
        while self._pending and self.in_use + self._pending[0].cost <= self.budget:
            r = self._pending.popleft()
            self.in_use += r.cost
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            r.t_admit = time.perf_counter()
            self._ready.append(r)

    def _take_locked(self):
        batch, samples = [], 0
        while self._ready and len(batch) < self.max_batch:
            r = self._ready[0]
            if batch and samples + r.samples > self.max_samples:
                break
            batch.append(self._ready.popleft())
            samples += r.samples
        return batch

    def _lane(self, lane):
        self.executor.start_lane(lane)
        while True:
            with self._cv:
                while self._running and not self._ready:
                    self._cv.wait()
                if not self._ready and not self._running:
                    return
                batch = self._take_locked()
                bid = self._batches
                self._batches += 1
                self.batch_sizes.append(len(batch))
            t = time.perf_counter()
            for r in batch:
                r.t_start = t
                r.lane = lane
                r.batch_id = bid
            comp = [r for r in batch if r.kind == COMPRESS]
            dec = [r for r in batch if r.kind == DECOMPRESS]
            try:
                self.executor.run(lane, comp, dec)
            except Exception as e:   # every request of the batch learns of it
                for r in batch:
                    if r.status is None:
                        r.status = e
            t = time.perf_counter()
            with self._cv:
                for r in batch:
                    r.t_done = t
                    self.in_use -= r.cost
                    self.completed.append(r)
                self._admit_locked()
                self._cv.notify_all()
            for r in batch:
                r.done.set()

    def start(self):
        self._running = True
        self._threads = [threading.Thread(target=self._lane, args=(i,), daemon=True) for i in range(self.lanes)]
        for t in self._threads:
            t.start()
        return self

    def stop(self):
        """Finish every submitted request, then stop the lanes."""
        with self._cv:
            while self._pending or self._ready:
                self._cv.wait(0.05)
            self._running = False
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        self.executor.close()

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()


_LANE_STREAMS = {}   # (device, lane) -> stream, shared by every server of the process


class GpuExecutor:
    """Runs a lane's batch through the library's batched entry points on the
    lane's own stream (one stream per lane index and device for the whole
    process, so the library's per-stream workspaces are reused by later
    servers)."""

    def __init__(self, params, base_ratio):
        import torch
        from . import ebcc
        self.torch, self.ebcc = torch, ebcc
        self.p = ebcc.params(0.01, base_ratio, **params)
        self.streams = {}
        self.dev = torch.device("cuda", torch.cuda.current_device())

    def on_submit(self, req):
        # the lane's stream waits for the producer of the request's data
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.dev))
        req.ready = ev

    def start_lane(self, lane):
        self.torch.cuda.set_device(self.dev)
        key = (self.dev.index, lane)
        if key not in _LANE_STREAMS:
            _LANE_STREAMS[key] = self.torch.cuda.Stream(self.dev)
        self.streams[lane] = _LANE_STREAMS[key]

    def run(self, lane, comp, dec):
        torch, ebcc = self.torch, self.ebcc
        s = self.streams[lane]
        with torch.cuda.stream(s):
            for r in comp + dec:
                s.wait_event(r.ready)
                r.ready = None
            if comp:
                args = ebcc.BatchArgs([r.data for r in comp], err_bounds=[r.eps for r in comp])
                out = torch.empty(max(1, args.bound()), dtype=torch.uint8, device=self.dev)
                rc = ebcc.compress_batch_into(args, out, self.p, s)
                for i, r in enumerate(comp):
                    r.status = rc
                    if rc == 0:
                        r.result = out[args.offsets[i]: args.offsets[i] + args.lengths[i]]
            if dec:
                outs = [torch.empty(r.shape, dtype=torch.float32, device=self.dev) for r in dec]
                args = ebcc.DecodeArgs([r.data for r in dec], outs)
                ebcc.decompress_batch_into(args, s)
                for i, r in enumerate(dec):
                    r.status = args.status[i]
                    r.result = outs[i] if r.status == 0 else None
            s.synchronize()

    def close(self):
        pass


def poisson_run(server, make_request, rate, duration, seed=0, max_requests=None):
    """Submit requests with exponential inter-arrival times (rate per second)
    for `duration` seconds; wait for all; return them."""
    import random
    rnd = random.Random(seed)
    reqs = []
    t0 = time.perf_counter()
    t_next = t0
    while True:
        t_next += rnd.expovariate(rate)
        if t_next - t0 > duration or (max_requests and len(reqs) >= max_requests):
            break
        now = time.perf_counter()
        if t_next > now:
            time.sleep(t_next - now)
        reqs.append(server.submit(make_request(len(reqs))))
    for r in reqs:
        r.wait()
    return reqs, time.perf_counter() - t0


def summarize(reqs, wall):
    """Latency percentiles (ms), throughput and compression ratio."""
    import numpy as np
    lat = np.array([r.latency() for r in reqs]) * 1e3
    raw = sum(4 * r.samples for r in reqs)
    comp = [r for r in reqs if r.kind == COMPRESS and hasattr(r.result, "numel")]
    cr_in = sum(4 * r.samples for r in comp)
    cr_out = sum(int(r.result.numel()) for r in comp)
    return {"requests": len(reqs), "seconds": wall,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None,
            "GBps": raw / wall / 1e9, "CR": (cr_in / cr_out) if cr_out else None,
            "failed": sum(1 for r in reqs if r.status not in (0, None))}
