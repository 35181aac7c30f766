"""Serving loop: continuous batching of compress / decompress requests.

Requests of mixed sizes (device-resident fields to compress, device-resident
streams to decompress) arrive at any time.  An admission controller bounds
the device memory the server is responsible for by an HBM budget:

  * every lane (one host thread with its own HIP stream) owns one library
    workspace of a fixed size, reserved when the lane starts
    (`ebcc_workspace_reserve`), and never runs a batch whose workspace
    (`ebcc_workspace_size_batch`, the library's own sizing) exceeds it;
  * every admitted request holds its input and output buffers until it
    completes; requests are admitted first come, first served while these
    fit what the lanes' workspaces leave of the budget.

So device memory in use is at most lanes x lane workspace + the admitted
requests' buffers <= budget (plus the library's small per-shape tables).
Admitted requests wait in FIFO order for a lane: when a lane is free it
takes every admitted request that is waiting (up to a batch cap and its
workspace) and runs them as one `ebcc_compress_batch` and one
`ebcc_decompress_batch` call.  Requests that arrive while the lanes are busy
are admitted as memory frees up and go into the next batch of whichever lane
frees first, so batches on different lanes overlap on the device.  Each
request gets its own status: a field that cannot be compressed (non-finite
values) or a stream that cannot be decoded fails alone, and every result is
byte-identical to what the request produces alone (the batched entry points
guarantee it; the GPU tests check it against the CPU oracle in the mix).

The executor (what a lane runs for a batch) is a parameter, so the
admission and batching logic can be exercised without a GPU.
"""
import collections
import threading
import time

COMPRESS, DECOMPRESS = "compress", "decompress"
HDR_BYTES = 48


class Request:
    """One request.  kind COMPRESS: `data` is a float32 device tensor
    (ny, nx), `eps` its range-relative bound; result = uint8 stream tensor.
    kind DECOMPRESS: `data` is a uint8 device stream, `shape` = (ny, nx);
    result = float32 field tensor."""

    __slots__ = ("kind", "data", "shape", "eps", "tag", "t_arrive", "t_admit", "t_start", "t_done", "result",
                 "status", "cost", "ws", "done", "lane", "batch_id", "ready", "header", "on_done")

    def __init__(self, kind, data, shape=None, eps=None, tag=None, header=None, on_done=None):
        self.kind = kind
        self.data = data
        self.shape = tuple(shape if shape is not None else data.shape)
        self.eps = eps
        self.tag = tag
        self.t_arrive = self.t_admit = self.t_start = self.t_done = None
        self.result = None
        self.status = None
        self.cost = 0
        self.ws = 0            # library workspace the request needs alone (bytes)
        self.done = threading.Event()
        self.lane = None
        self.batch_id = None
        self.ready = None      # executor's marker that the data is ready
        self.header = header   # DECOMPRESS: the stream's first 48 bytes (host), read at submit if None
        self.on_done = on_done  # called with the request in the lane thread when it completes

    @property
    def samples(self):
        return self.shape[0] * self.shape[1]

    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive

    def wait(self, timeout=None):
        return self.done.wait(timeout)


def request_cost(req):
    """Device bytes an admitted request holds until it completes: its input
    and its output (the library workspace is the lanes')."""
    n = req.samples
    if req.kind == COMPRESS:
        return 4 * n + (HDR_BYTES + 4 * n)          # field, stream capacity
    return req.data.numel() + 4 * n                 # stream, field


class Server:
    """Continuous-batching server.

    hbm_budget      device bytes the server may hold: the lanes' workspaces
                    plus the admitted requests' buffers
    lanes           concurrent batches (one stream and host thread each)
    lane_workspace  bytes of library workspace reserved per lane (default:
                    a quarter of the budget shared by the lanes; 0 for an
                    executor without workspaces)
    max_batch       requests per batch
    max_samples     samples per batch
    executor        object with on_submit(req), start_lane(lane),
                    run(lane, compress_reqs, decompress_reqs) (fills
                    req.result / req.status) and close(); optionally
                    workspace(req), batch_workspace(comp, dec) and
                    reserve(lane, nbytes).  Default: the GPU executor.
    A request whose buffers exceed what the workspaces leave of the budget,
    or whose workspace exceeds a lane's, is refused with ValueError.
    """

    def __init__(self, hbm_budget=64 * 10**9, lanes=2, max_batch=256, max_samples=1 << 27, executor=None,
                 params=None, base_ratio=30.0, lane_workspace=None):
        self.budget = int(hbm_budget)
        self.lanes = int(lanes)
        self.max_batch = int(max_batch)
        self.max_samples = int(max_samples)
        self.params = params or {}
        self.base_ratio = base_ratio
        self.executor = executor or GpuExecutor(self.params, base_ratio)
        has_ws = hasattr(self.executor, "workspace")
        if lane_workspace is None:
            lane_workspace = self.budget // (4 * self.lanes) if has_ws else 0
        self.lane_ws = int(lane_workspace)
        self.req_budget = self.budget - self.lanes * self.lane_ws
        if self.req_budget <= 0:
            raise ValueError("the lanes' workspaces take the whole budget")
        self._cv = threading.Condition()
        self._pending = collections.deque()    # arrived, not admitted
        self._ready = collections.deque()      # admitted, waiting for a lane
        self.in_use = 0                        # admitted requests' buffers
        self.peak_in_use = 0
        self._running = False
        self._threads = []
        self._batches = 0
        self.batch_sizes = []
        self.completed = []

    @property
    def reserved(self):
        """Device bytes the lanes' workspaces take."""
        return self.lanes * self.lane_ws

    # ---- client side ----
    def submit(self, req):
        req.cost = request_cost(req)
        if req.cost > self.req_budget:
            raise ValueError(f"request needs {req.cost} B, more than the budget leaves for requests "
                             f"({self.req_budget} B)")
        self.executor.on_submit(req)
        if hasattr(self.executor, "workspace"):
            req.ws = int(self.executor.workspace(req))
            if req.ws > self.lane_ws:
                raise ValueError(f"request needs {req.ws} B of workspace, more than a lane's {self.lane_ws} B")
        req.t_arrive = time.perf_counter()
        with self._cv:
            self._pending.append(req)
            self._admit_locked()
            self._cv.notify_all()
        return req

    # ---- admission: FIFO, as memory frees up ----
    def _admit_locked(self):
        while self._pending and self.in_use + self._pending[0].cost <= self.req_budget:
            r = self._pending.popleft()
            self.in_use += r.cost
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            r.t_admit = time.perf_counter()
            self._ready.append(r)

    def _take_locked(self):
        # FIFO candidates up to the batch limits; with the library's sizing
        # of a batch (batch_workspace), the longest prefix that fits the
        # lane's workspace is kept (a batch shares its search candidates'
        # planes, so it needs less than its requests alone), found by
        # bisection, and the rest go back to the front of the queue; without
        # it, the requests' own workspaces must fit together.
        fit = getattr(self.executor, "batch_workspace", None)
        batch, samples, ws = [], 0, 0
        while self._ready and len(batch) < self.max_batch:
            r = self._ready[0]
            if batch and (samples + r.samples > self.max_samples or (fit is None and ws + r.ws > self.lane_ws)):
                break
            batch.append(self._ready.popleft())
            samples += r.samples
            ws += r.ws
        if fit is not None and len(batch) > 1:
            def fits(m):
                part = batch[:m]
                return fit([r for r in part if r.kind == COMPRESS],
                           [r for r in part if r.kind == DECOMPRESS]) <= self.lane_ws
            if not fits(len(batch)):
                lo, hi = 1, len(batch)          # a request alone fits (checked at submit)
                while hi - lo > 1:
                    mid = (lo + hi) // 2
                    if fits(mid):
                        lo = mid
                    else:
                        hi = mid
                for r in reversed(batch[lo:]):
                    self._ready.appendleft(r)
                del batch[lo:]
        return batch

    def _lane(self, lane):
        self.executor.start_lane(lane)
        if self.lane_ws and hasattr(self.executor, "reserve"):
            self.executor.reserve(lane, self.lane_ws)
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
            for r in batch:
                r.t_done = t
                if r.on_done is not None:
                    r.on_done(r)
            with self._cv:
                for r in batch:
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
        if req.kind == DECOMPRESS and req.header is None:
            req.header = bytes(req.data[:HDR_BYTES].cpu().numpy().tobytes())

    def workspace(self, req):
        """Library workspace of the request alone."""
        return self.batch_workspace([req], []) if req.kind == COMPRESS else self.batch_workspace([], [req])

    def batch_workspace(self, comp, dec):
        """Library workspace of one lane batch: its compress call, then its
        decompress call, on the same stream (the larger of the two)."""
        ebcc = self.ebcc
        a = ebcc.workspace_size_batch([r.shape for r in comp], self.p) if comp else 0
        b = ebcc.workspace_size_batch([r.shape for r in dec], headers=[r.header for r in dec],
                                      lengths=[r.data.numel() for r in dec]) if dec else 0
        return max(a, b)

    def start_lane(self, lane):
        self.torch.cuda.set_device(self.dev)
        key = (self.dev.index, lane)
        if key not in _LANE_STREAMS:
            _LANE_STREAMS[key] = self.torch.cuda.Stream(self.dev)
        self.streams[lane] = _LANE_STREAMS[key]

    def reserve(self, lane, nbytes):
        self.ebcc.workspace_reserve(nbytes, self.streams[lane])

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
                per_field = rc in (ebcc.OK, ebcc.EINVAL)
                for i, r in enumerate(comp):
                    r.status = args.status[i] if per_field else rc
                    if r.status == 0:
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
