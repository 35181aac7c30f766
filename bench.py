#!/usr/bin/env python3
"""EBCC compress/decompress throughput on one MI355X.

Headline workload (`value`): the ERA5-shaped stack, plain per-field path:
148 float32 fields of 721x1440 (37 levels x {temperature-, u-, v-,
humidity-like}), range-relative bound 1%, base ratio r = 30, 5 DWT levels,
32x32 code-blocks, one-root SPIHT tiles.  One step = compress every field,
then decompress every stream, one field per call on one stream.  value = fp32
bytes of the stack / step time (GB/s, decimal): round-trip throughput.

Beside it, in the same JSON line:
  c1_bounds     the same stack and loop at 0.1% and 10% of range
  c0            the plain single field (181x360 temperature-like, 1%): per-call
                p50/p99 latency over >= 200 repetitions, GPU and oracle
  batched       the uneven batch (256 fields drawn from 91x180 .. 721x1440,
                per-field bounds log-uniform in [0.1%, 10%] of range) through
                ebcc_compress_batch / ebcc_decompress_batch, the same fields
                through the per-field loop, and the speedup; the headline
                stack through the batched entry points; the autotuned batch
  serving       Poisson arrivals of compress/decompress requests on the
                uneven mix under a 64 GB HBM budget
  ratio_search  Algorithm 1's base-ratio search (q = 1 - 1e-5) on the stack
  q_ablation    relative compression ratio against q = 1 over the uneven mix
  km_scale      1801x3600 fields with embedded vortices, batched and served
  roofline      the dominant kernel of the headline path (its HIP-event time
                per launch, algorithmic bytes per launch N (4 + 4/CR))
  cpu_baseline  the CPU oracle over all host cores on a bounded sample of the
                headline fields (single-thread, uneven-mix and km-scale legs
                beside it)
Inputs are synthetic (seeded generators standing in for ERA5), generated
before the GPU is first touched, and resident in HBM before timing;
verification (bound, compression ratio) is outside the timed regions.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
# Plain-ALU ceiling of MQ decisions: 256 compute units issuing one 64-lane
# vector instruction per cycle at 2.4 GHz (39.3 T lane-operations/s), at
# about 25 lane-operations per decision (context formation, interval update,
# renormalisation).  The coders are chains of dependent decisions per
# code-block, so this is a bound on decisions over all blocks at once.
T1_ALU_CEILING = 256 * 64 * 2.4e9 / 25

# Per-launch figures of the headline path's tier-1 kernels on one 721x1440
# field at eps_rel 1%, measured with rocprofv3 (profiles/
# kernels_era5_721x1440_per_field.md): the average kernel duration
# (--kernel-trace --stats) and the HBM bytes from two --pmc runs (FETCH_SIZE,
# WRITE_SIZE), each scaled by what the counter reads for a plain elementwise
# copy of 1 GiB (FETCH_SIZE x2.0, WRITE_SIZE x1.0).  Valid only while the
# kernel's source is the one measured (checked by hash); otherwise null.
MEASURED = {
    "t1_encode": {"source": "paper_2510_22265_amd/csrc/t1wave.hip",
                  "sha256": "6bccb9e1a87ceff9e73ad4faa539c8c8181f3f2979f9b4cca93cbfaed0f07907",
                  "ny": 721, "nx": 1440, "eps": 0.01, "kernel": "k_t1_encode_pipe<3>", "avg_ms": 1.4465,
                  "bytes": (2.0 * (734.1 + 680.8) / 2 + 1.0 * (868.2 + 1078.6) / 2) * 1024},
    "t1_decode": {"source": "paper_2510_22265_amd/csrc/t1wave.hip",
                  "sha256": "6bccb9e1a87ceff9e73ad4faa539c8c8181f3f2979f9b4cca93cbfaed0f07907",
                  "ny": 721, "nx": 1440, "eps": 0.01, "kernel": "k_t1_decode_wave<u32>", "avg_ms": 1.5401,
                  "bytes": (2.0 * (593.8 + 558.4) / 2 + 1.0 * (4099.5 + 4099.5) / 2) * 1024},
}

SERVE_BUDGET = 64 * 10**9


def measured(kernel, ny, nx, eps):
    m = MEASURED.get(kernel)
    if not m or (m["ny"], m["nx"], m["eps"]) != (ny, nx, eps):
        return None
    with open(os.path.join(ROOT, m["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != m["sha256"]:
            return None
    return m


def _gen(spec):
    from paper_2510_22265_amd import synth
    kind, a = spec
    if kind == "stack":
        var, ny, nx, level = a
        return synth.field(var, ny, nx, cfg=1, level=level)
    if kind == "plain":
        return synth.plain_field(*a)
    if kind == "km":
        var, level = a
        return synth.vortex_field(1801, 3600, var=var, level=level, cfg=4)
    return synth.batch_field(a)


def generate(specs):
    """Host inputs, in worker processes forked before any GPU call."""
    if not specs:
        return []
    from multiprocessing import get_context
    procs = min(16, os.cpu_count() or 1)
    with get_context("fork").Pool(procs) as p:
        return p.map(_gen, specs, chunksize=1)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def verify(xs_h, recs, eps):
    """Count bound violations (FP64) and the largest range-relative error."""
    viol, max_rel = 0, 0.0
    for i, (x, y, e) in enumerate(zip(xs_h, recs, eps)):
        if i and i % 128 == 0:
            log(f"verified {i} of {len(xs_h)} fields")
        rng_ = float(x.max()) - float(x.min())
        yh = y if isinstance(y, np.ndarray) else y.cpu().numpy()
        err = float(np.abs(x.astype(np.float64) - yh.astype(np.float64)).max())
        if err > e * rng_:
            viol += 1
        if rng_ > 0:
            max_rel = max(max_rel, err / rng_)
    return viol, max_rel


def oracle_all_cores(fields, eps, threads, seconds, **kw):
    """The oracle (compress then decompress) over fields in a pool of host
    threads (the oracle's C calls run without the GIL), until `seconds` have
    passed; returns the round-trip rate and what was run."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import ref
    ref.lib()

    def one(i):
        x = fields[i]
        s = ref.compress(x, eps[i], **kw)
        ref.decompress(s, *x.shape)
        return x.nbytes

    t0 = time.perf_counter()
    done = nbytes = 0
    with ThreadPoolExecutor(threads) as ex:
        while done < len(fields) and time.perf_counter() - t0 < seconds:
            k = min(len(fields) - done, threads)
            nbytes += sum(ex.map(one, range(done, done + k)))
            done += k
    el = time.perf_counter() - t0
    return {"GBps": nbytes / el / 1e9, "fields": done, "seconds": el, "threads": threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fields", type=int, default=148)
    ap.add_argument("--ny", type=int, default=721)
    ap.add_argument("--nx", type=int, default=1440)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--ratio", type=float, default=30.0)
    ap.add_argument("--tile", type=int, default=None, help="SPIHT tile side (default: the library's)")
    ap.add_argument("--cblk", default=None, help="code-block log2 sizes w,h (default: the library's)")
    ap.add_argument("--extra-bounds", default="0.001,0.1", help="further bounds of the stack loop (empty: skip)")
    ap.add_argument("--c0-reps", type=int, default=200, help="timed repetitions of the 181x360 field (0: skip)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuned batched run")
    ap.add_argument("--serve-rates", default="200,1000,5000", help="Poisson arrival rates (req/s); empty: skip")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per arrival rate")
    ap.add_argument("--q", type=float, default=1 - 1e-5, help="proportion q of the ratio-search run (0: skip)")
    ap.add_argument("--ablation-fields", type=int, default=256, help="fields of the q ablation (0: skip)")
    ap.add_argument("--byte-cut", type=int, default=1, help="measure the byte-granular residual cut (0: skip)")
    ap.add_argument("--bypass", type=int, default=1,
                    help="measure the tier-1 arithmetic-coding bypass against MQ-only streams (0: skip)")
    ap.add_argument("--km-fields", type=int, default=16, help="km-scale 1801x3600 vortex fields (0: skip)")
    ap.add_argument("--batch-fields", type=int, default=256, help="fields of the uneven batch (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of each oracle baseline leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the batched uneven mix (for kernel profiles); prints its own JSON line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run a plain elementwise copy of MIB MiB three times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the path shards by field with no exchange between GPUs, "
              "and it does not launch multi-GPU runs (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    # ---------------- inputs (host; before the GPU is touched) ----------------
    from paper_2510_22265_amd import synth
    stack_specs = [("stack", (v, args.ny, args.nx, lev)) for lev in range(37) for v in synth.VARS][: args.fields]
    bspecs = synth.batch_specs(n=args.batch_fields) if args.batch_fields else []
    kspecs = [("km", (v, lev)) for lev in range((args.km_fields + 3) // 4) for v in synth.VARS][: args.km_fields]
    c0_specs = [("plain", (181, 360))] if args.c0_reps else []
    if args.calibrate_copy:
        stack_specs, bspecs, kspecs, c0_specs = [], [], [], []
    log(f"generating {len(stack_specs)} fields of {args.ny}x{args.nx}, an uneven batch of {len(bspecs)}, "
        f"{len(kspecs)} km-scale fields")
    fields_h = generate(stack_specs + [("batch", s) for s in bspecs] + kspecs + c0_specs)
    n1, n2, n3 = len(stack_specs), len(stack_specs) + len(bspecs), len(stack_specs) + len(bspecs) + len(kspecs)
    stack_h, batch_h, km_h, c0_h = fields_h[:n1], fields_h[n1:n2], fields_h[n2:n3], fields_h[n3:]

    import torch
    from paper_2510_22265_amd import ebcc
    if not os.path.exists(ebcc.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    ebcc.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)      # reads 4 B and writes 4 B per element
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "elementwise copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "launches": 3}), flush=True)
        return

    xs = [torch.from_numpy(f).to(dev) for f in stack_h]
    fmt = {} if args.tile is None else {"spiht_tile": args.tile}
    if args.cblk:
        fmt["cblk_log2w"], fmt["cblk_log2h"] = (int(v) for v in args.cblk.split(","))
    p = ebcc.params(args.eps, args.ratio, **fmt)
    tile = p.spiht_tile
    cap = ebcc.compress_bound(args.ny, args.nx)
    outs = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in xs]
    recs = [torch.empty((args.ny, args.nx), dtype=torch.float32, device=dev) for _ in xs]
    lens = [0] * len(xs)
    nbytes = sum(f.nbytes for f in stack_h)

    def per_field_step(xs_, outs_, recs_, lens_, p_list, lat_c=None, lat_d=None):
        t0 = time.perf_counter()
        for i, x in enumerate(xs_):
            a = time.perf_counter()
            rc, n = ebcc.compress_into(x, outs_[i], p_list[i], stream)
            if rc != 0:
                raise RuntimeError(f"compress failed on field {i}: {rc} {ebcc.lib().ebcc_last_error()}")
            lens_[i] = n
            if lat_c is not None:
                lat_c.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(len(xs_)):
            a = time.perf_counter()
            rc = ebcc.decompress_into(outs_[i][: lens_[i]], recs_[i], stream)
            if rc != 0:
                raise RuntimeError(f"decompress failed on field {i}: {rc}")
            if lat_d is not None:
                lat_d.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1

    if args.batch_only:
        bx = [torch.from_numpy(f).to(dev) for f in batch_h]
        beps = [s[3] for s in bspecs]
        bbytes = sum(f.nbytes for f in batch_h)
        bargs = ebcc.BatchArgs(bx, err_bounds=beps)
        bout = torch.empty(bargs.bound(), dtype=torch.uint8, device=dev)
        assert ebcc.compress_batch_into(bargs, bout, p, stream) == 0
        bstreams = [bout[bargs.offsets[i]: bargs.offsets[i] + bargs.lengths[i]] for i in range(bargs.n)]
        brecs = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in batch_h]
        dargs = ebcc.DecodeArgs(bstreams, brecs)
        for w in range(args.warmup):
            assert ebcc.compress_batch_into(bargs, bout, p, stream) == 0
            assert ebcc.decompress_batch_into(dargs, stream) == 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            assert ebcc.compress_batch_into(bargs, bout, p, stream) == 0
            assert ebcc.decompress_batch_into(dargs, stream) == 0
            log(f"batched step {s} done")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        viol, _ = verify(batch_h, brecs, beps)
        print(json.dumps({"workload": f"uneven batch of {len(bx)} fields, batched entry points only",
                          "GBps": bbytes * args.steps / dt / 1e9, "steps": args.steps, "violations": viol}),
              flush=True)
        return

    # ---------------- headline: per-field path over the stack ----------------
    plist = [p] * len(xs)
    for w in range(args.warmup):
        per_field_step(xs, outs, recs, lens, plist)
        log(f"warmup step {w} done")
    lat_c, lat_d = [], []
    ebcc.profile_enable(True)
    torch.cuda.synchronize()
    tc = td = 0.0
    t_start = time.perf_counter()
    for s in range(args.steps):
        a, b = per_field_step(xs, outs, recs, lens, plist, lat_c, lat_d)
        tc += a
        td += b
        log(f"step {s}: compress {a * 1e3:.1f} ms, decompress {b * 1e3:.1f} ms")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = ebcc.profile_read()
    ebcc.profile_enable(False)
    viol, max_rel = verify(stack_h, recs, [args.eps] * len(xs))
    stream_bytes = sum(lens)
    headline_lens = list(lens)
    # the headline streams, kept for comparisons after later runs reuse the buffers
    headline_streams = [outs[i][: lens[i]].clone() for i in range(len(xs))]
    steps = args.steps
    value = nbytes * steps / t_total / 1e9
    cr_stack = nbytes / stream_bytes

    # roofline of the dominant kernel: tier-1 coding is one kernel launch per
    # call and stage (HIP events on the library's stream)
    stages = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(stages, key=lambda k: stages[k][0]) if stages else None
    roof = None
    if dom is not None:
        ms, calls = stages[dom]
        avg_s = ms / calls / 1e3
        N = args.ny * args.nx
        algo = N * (4.0 + 4.0 / cr_stack)          # 4 B in + 4/CR B out per sample (4/CR in + 4 out decoding)
        ach = algo / avg_s / 1e9
        m = measured(dom, args.ny, args.nx, args.eps)
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBPS, "traffic": m["bytes"] if m else None,
                "avg_launch_ms": ms / calls, "algo_bytes_per_launch": algo,
                "algo_bytes_per_sample": 4.0 + 4.0 / cr_stack}
        if m:
            roof["rocprof_kernel"] = m["kernel"]
            roof["rocprof_avg_launch_ms"] = m["avg_ms"]
            roof["frac_rocprof"] = algo / (m["avg_ms"] / 1e3) / 1e9 / HBM_PEAK_GBPS
    log(f"headline: {value:.3f} GB/s, CR {cr_stack:.2f}, roofline {roof}")

    # ---------------- the stack at the other bounds ----------------
    c1_bounds = {}
    for e in [float(v) for v in args.extra_bounds.split(",") if v.strip()]:
        pe = [ebcc.params(e, args.ratio, **fmt)] * len(xs)
        elens = [0] * len(xs)
        per_field_step(xs, outs, recs, elens, pe)
        lc, ld = [], []
        ec = ed = 0.0
        for s in range(max(1, steps - 1)):
            a, b = per_field_step(xs, outs, recs, elens, pe, lc, ld)
            ec += a
            ed += b
        k = max(1, steps - 1)
        ev, emax = verify(stack_h, recs, [e] * len(xs))
        c1_bounds[f"eps_{e:g}"] = {
            "GBps": nbytes * k / (ec + ed) / 1e9, "compress_GBps": nbytes * k / ec / 1e9,
            "decompress_GBps": nbytes * k / ed / 1e9, "CR": nbytes / sum(elens), "violations": ev,
            "max_err_rel": emax, "compress_ms_p50": pct(lc, 50) * 1e3, "compress_ms_p99": pct(lc, 99) * 1e3,
            "decompress_ms_p50": pct(ld, 50) * 1e3, "decompress_ms_p99": pct(ld, 99) * 1e3, "steps": k}
        log(f"stack at eps {e:g}: {c1_bounds[f'eps_{e:g}']}")
    c1_bounds[f"eps_{args.eps:g}"] = {"GBps": value, "CR": cr_stack, "violations": viol, "headline": True}

    # ---------------- the plain single field: per-call latency ----------------
    c0 = None
    if c0_h:
        x0h = c0_h[0]
        x0 = torch.from_numpy(x0h).to(dev)
        p0 = ebcc.params(0.01, 30.0)
        o0 = torch.empty(ebcc.compress_bound(*x0h.shape), dtype=torch.uint8, device=dev)
        r0 = torch.empty(x0h.shape, dtype=torch.float32, device=dev)
        for _ in range(3):
            rc, n0 = ebcc.compress_into(x0, o0, p0, stream)
            assert rc == 0 and ebcc.decompress_into(o0[:n0], r0, stream) == 0
        torch.cuda.synchronize()
        gc_, gd_ = [], []
        for _ in range(args.c0_reps):
            a = time.perf_counter()
            rc, n0 = ebcc.compress_into(x0, o0, p0, stream)      # returns after its final length read
            b = time.perf_counter()
            rc2 = ebcc.decompress_into(o0[:n0], r0, stream)       # returns after its status read
            c = time.perf_counter()
            assert rc == 0 and rc2 == 0
            gc_.append(b - a)
            gd_.append(c - b)
        c0v, c0max = verify([x0h], [r0], [0.01])
        s0 = o0[:n0].cpu().numpy().tobytes()
        c0 = {"workload": "plain single field: 181x360 temperature-like, eps_rel 1%, r 30, L 5, 32x32 blocks",
              "reps": args.c0_reps, "warmup": 3, "CR": x0h.nbytes / n0, "violations": c0v, "max_err_rel": c0max,
              "gpu": {"compress_ms_p50": pct(gc_, 50) * 1e3, "compress_ms_p99": pct(gc_, 99) * 1e3,
                      "decompress_ms_p50": pct(gd_, 50) * 1e3, "decompress_ms_p99": pct(gd_, 99) * 1e3,
                      "GBps": x0h.nbytes * args.c0_reps / (sum(gc_) + sum(gd_)) / 1e9}}
        if not args.no_cpu:
            from oracle import ref
            ref.lib()
            for _ in range(3):
                ref.decompress(ref.compress(x0h, 0.01), *x0h.shape)
            oc, od = [], []
            same = True
            for _ in range(args.c0_reps):
                a = time.perf_counter()
                sr = ref.compress(x0h, 0.01)
                b = time.perf_counter()
                ref.decompress(sr, *x0h.shape)
                c = time.perf_counter()
                oc.append(b - a)
                od.append(c - b)
                same &= sr == s0
            c0["oracle"] = {"compress_ms_p50": pct(oc, 50) * 1e3, "compress_ms_p99": pct(oc, 99) * 1e3,
                            "decompress_ms_p50": pct(od, 50) * 1e3, "decompress_ms_p99": pct(od, 99) * 1e3,
                            "GBps": x0h.nbytes * args.c0_reps / (sum(oc) + sum(od)) / 1e9, "threads": 1}
            c0["gpu_stream_equals_oracle"] = bool(same)
        log(f"c0: {c0}")

    # ---------------- batched execution ----------------
    batched = None
    serving = None
    bx = [torch.from_numpy(f).to(dev) for f in batch_h]
    beps = [s[3] for s in bspecs]
    if bspecs:
        bbytes = sum(f.nbytes for f in batch_h)
        bargs = ebcc.BatchArgs(bx, err_bounds=beps)
        bout = torch.empty(bargs.bound(), dtype=torch.uint8, device=dev)

        def batch_compress():
            rc = ebcc.compress_batch_into(bargs, bout, p, stream)
            if rc != 0:
                raise RuntimeError(f"batched compress failed: {rc} {ebcc.lib().ebcc_last_error()}")

        batch_compress()
        bstreams = [bout[bargs.offsets[i]: bargs.offsets[i] + bargs.lengths[i]].clone() for i in range(bargs.n)]
        brecs = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in batch_h]
        dargs = ebcc.DecodeArgs(bstreams, brecs)

        def batch_decompress():
            rc = ebcc.decompress_batch_into(dargs, stream)
            if rc != 0:
                raise RuntimeError(f"batched decompress failed: {rc}")

        batch_decompress()
        torch.cuda.synchronize()
        bc = bd = 0.0
        blat = []
        for s in range(steps):
            a = time.perf_counter()
            batch_compress()
            torch.cuda.synchronize()
            b = time.perf_counter()
            batch_decompress()
            torch.cuda.synchronize()
            c = time.perf_counter()
            bc += b - a
            bd += c - b
            blat.append(c - a)
            log(f"batched step {s}: compress {(b - a) * 1e3:.1f} ms, decompress {(c - b) * 1e3:.1f} ms")
        bviol, bmax = verify(batch_h, brecs, beps)
        bsbytes = sum(bargs.lengths[i] for i in range(bargs.n))
        # decoded fields of the default format, kept for the serving checks
        # (later runs decode other formats into brecs)
        brecs_ref = [r.clone() for r in brecs]
        # the same fields and bounds through the per-field loop (one step)
        bplist = [ebcc.params(e, args.ratio, **fmt) for e in beps]
        bouts = [torch.empty(ebcc.compress_bound(*f.shape), dtype=torch.uint8, device=dev) for f in batch_h]
        blens = [0] * len(bx)
        per_field_step(bx, bouts, brecs, blens, bplist)
        pc, pd = per_field_step(bx, bouts, brecs, blens, bplist)
        same = all(torch.equal(bouts[i][: blens[i]], bstreams[i]) for i in range(len(bx)))
        # stage breakdown of one batched call (profiled separately, not timed)
        ebcc.profile_enable(True)
        batch_compress()
        batch_decompress()
        torch.cuda.synchronize()
        bprof = {k: v[0] for k, v in ebcc.profile_read().items() if v[1] > 0}
        ebcc.profile_enable(False)
        # the headline stack through the batched entry points
        sargs = ebcc.BatchArgs(xs, err_bounds=[args.eps] * len(xs))
        sout = torch.empty(sargs.bound(), dtype=torch.uint8, device=dev)
        assert ebcc.compress_batch_into(sargs, sout, p, stream) == 0
        sstreams = [sout[sargs.offsets[i]: sargs.offsets[i] + sargs.lengths[i]] for i in range(sargs.n)]
        sdargs = ebcc.DecodeArgs(sstreams, recs)
        assert ebcc.decompress_batch_into(sdargs, stream) == 0
        torch.cuda.synchronize()
        s_a = time.perf_counter()
        for s in range(steps):
            assert ebcc.compress_batch_into(sargs, sout, p, stream) == 0
        torch.cuda.synchronize()
        s_b = time.perf_counter()
        for s in range(steps):
            assert ebcc.decompress_batch_into(sdargs, stream) == 0
        torch.cuda.synchronize()
        s_c = time.perf_counter()
        sviol, _ = verify(stack_h, recs, [args.eps] * len(xs))
        stack_same = all(torch.equal(sstreams[i], headline_streams[i]) for i in range(len(xs)))
        log(f"stack batched: compress {(s_b - s_a) / steps * 1e3:.1f} ms, "
            f"decompress {(s_c - s_b) / steps * 1e3:.1f} ms per step")
        # the uneven batch through the asynchronous decoder: streams in one
        # buffer at device offsets, statuses on the device, back-to-back calls
        # with no host wait between them (host enqueue time and device time)
        abuf = torch.cat(bstreams)
        alens = torch.tensor([t.numel() for t in bstreams], dtype=torch.int64)
        aoffs = (torch.cumsum(alens, 0) - alens).to(dev)
        alens = alens.to(dev)
        arecs = [torch.empty_like(r) for r in brecs_ref]
        ashapes = [tuple(f.shape) for f in batch_h]
        for _ in range(2):   # (the second call records the launch sequence)
            _, ast = ebcc.decompress_batch_async(abuf, aoffs, alens, ashapes, stream=stream, outs=arecs, **fmt)
        torch.cuda.synchronize()
        a_enq = 0.0
        a_a = time.perf_counter()
        for s in range(steps):
            q0 = time.perf_counter()
            _, ast = ebcc.decompress_batch_async(abuf, aoffs, alens, ashapes, stream=stream, outs=arecs, **fmt)
            a_enq += time.perf_counter() - q0
        torch.cuda.synchronize()
        a_b = time.perf_counter()
        async_dec = {"GBps": bbytes * steps / (a_b - a_a) / 1e9, "ms_per_batch": (a_b - a_a) / steps * 1e3,
                     "host_enqueue_ms_per_call": a_enq / steps * 1e3,
                     "statuses_ok": bool((ast == 0).all().item()),
                     "identical_to_sync_decode": all(torch.equal(a.view(torch.int32), b.view(torch.int32))
                                                     for a, b in zip(arecs, brecs_ref))}
        log(f"async batched decode: {async_dec}")
        # autotuned batched run: format and kernel choices measured on the batch
        tuned = None
        if not args.no_tune:
            from paper_2510_22265_amd import autotune
            t0 = time.perf_counter()
            res = autotune.tune(bx, beps, base_ratio=args.ratio, stream=stream)
            t_tune = time.perf_counter() - t0
            old = ebcc.set_tuning(**res["tuning"])
            tp = ebcc.params(args.eps, args.ratio, **res["params"])
            targs = ebcc.BatchArgs(bx, err_bounds=beps)
            tout = torch.empty(targs.bound(), dtype=torch.uint8, device=dev)
            assert ebcc.compress_batch_into(targs, tout, tp, stream) == 0
            tstreams = [tout[targs.offsets[i]: targs.offsets[i] + targs.lengths[i]] for i in range(targs.n)]
            tdargs = ebcc.DecodeArgs(tstreams, brecs)
            assert ebcc.decompress_batch_into(tdargs, stream) == 0
            torch.cuda.synchronize()
            t_c = t_d = 0.0
            for s in range(steps):
                u0 = time.perf_counter()
                assert ebcc.compress_batch_into(targs, tout, tp, stream) == 0
                torch.cuda.synchronize()
                u1 = time.perf_counter()
                assert ebcc.decompress_batch_into(tdargs, stream) == 0
                torch.cuda.synchronize()
                u2 = time.perf_counter()
                t_c += u1 - u0
                t_d += u2 - u1
                log(f"tuned batched step {s}: compress {(u1 - u0) * 1e3:.1f} ms, decompress {(u2 - u1) * 1e3:.1f} ms")
            tviol, _ = verify(batch_h, brecs, beps)
            ebcc.set_tuning(**old)
            tsb = sum(targs.lengths[i] for i in range(targs.n))
            tuned = {"params": res["params"], "tuning": res["tuning"], "tune_seconds": t_tune,
                     "candidates": len(res["table"]),
                     "GBps": bbytes * steps / (t_c + t_d) / 1e9, "compress_GBps": bbytes * steps / t_c / 1e9,
                     "decompress_GBps": bbytes * steps / t_d / 1e9, "CR": bbytes / tsb, "violations": tviol,
                     "speedup_vs_per_field": (pc + pd) / ((t_c + t_d) / steps)}
        batched = {
            "workload": f"uneven batch: {len(bx)} fields from {{91x180, 181x360, 361x720, 721x1440}}, "
                        f"eps_rel log-uniform [1e-3, 1e-1], r {args.ratio}",
            "fields": len(bx), "MB": bbytes / 1e6,
            "GBps": bbytes * steps / (bc + bd) / 1e9,
            "compress_GBps": bbytes * steps / bc / 1e9, "decompress_GBps": bbytes * steps / bd / 1e9,
            "per_field_GBps": bbytes / (pc + pd) / 1e9,
            "per_field_compress_GBps": bbytes / pc / 1e9, "per_field_decompress_GBps": bbytes / pd / 1e9,
            "speedup_vs_per_field": (pc + pd) / ((bc + bd) / steps),
            "streams_identical_to_per_field": bool(same),
            "CR": bbytes / bsbytes, "violations": bviol, "max_err_rel": bmax,
            "batch_ms_p50": pct(blat, 50) * 1e3, "batch_ms_p99": pct(blat, 99) * 1e3,
            "stages_ms_per_batch": bprof,
            "stack_GBps": nbytes * steps / (s_c - s_a) / 1e9,
            "stack_compress_GBps": nbytes * steps / (s_b - s_a) / 1e9,
            "stack_decompress_GBps": nbytes * steps / (s_c - s_b) / 1e9,
            "stack_ms_per_step": (s_c - s_a) / steps * 1e3,
            "stack_speedup_vs_per_field": (t_total / steps) / ((s_c - s_a) / steps),
            "stack_streams_identical": bool(stack_same), "stack_violations": sviol,
            "async_decode": async_dec,
            "tuned": tuned,
        }

        # ---------------- serving loop: Poisson arrivals, continuous batching ----------------
        rates = [float(r) for r in args.serve_rates.split(",") if r.strip()]
        if rates:
            from paper_2510_22265_amd import serve
            import random
            hdrs = [bytes(s[:48].cpu().numpy().tobytes()) for s in bstreams]
            serving = {"workload": f"Poisson arrivals of compress/decompress requests (1:1) on the uneven "
                                   f"{len(bx)}-field mix, HBM admission budget 64 GB, 2 lanes",
                       "budget_GB": SERVE_BUDGET / 1e9, "lanes": 2}
            for rate in rates:
                rnd = random.Random(int(rate))
                stat = {"out_bytes": 0, "in_bytes": 0, "mismatch": 0, "checked": 0}

                def on_done(r, stat=stat):
                    # results are checked (a sample against the same request
                    # alone) and released here, so that the run holds only
                    # what is admitted
                    if r.status == 0:
                        if r.kind == serve.COMPRESS:
                            stat["out_bytes"] += int(r.result.numel())
                            stat["in_bytes"] += 4 * r.samples
                            if r.tag % 16 == 0:
                                stat["checked"] += 1
                                stat["mismatch"] += int(not torch.equal(r.result, bstreams[r.tag]))
                        elif r.tag % 16 == 0:
                            stat["checked"] += 1
                            stat["mismatch"] += int(not torch.equal(r.result, brecs_ref[r.tag]))
                    r.result = None

                def make(k):
                    i = rnd.randrange(len(bx))
                    if rnd.random() < 0.5:
                        return serve.Request(serve.COMPRESS, bx[i], eps=beps[i], tag=i, on_done=on_done)
                    return serve.Request(serve.DECOMPRESS, bstreams[i], shape=tuple(bx[i].shape), tag=i,
                                         header=hdrs[i], on_done=on_done)

                srv = serve.Server(hbm_budget=SERVE_BUDGET, lanes=2, params=fmt, base_ratio=args.ratio).start()
                lib0 = ebcc.device_bytes()
                reqs, wall = serve.poisson_run(srv, make, rate=rate, duration=1e9, seed=int(rate),
                                               max_requests=args.serve_requests)
                srv.stop()
                st = serve.summarize(reqs, wall)
                st["CR"] = stat["in_bytes"] / stat["out_bytes"] if stat["out_bytes"] else None
                st["mean_batch"] = float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0
                st["peak_GB_admitted"] = srv.peak_in_use / 1e9
                st["lane_workspace_GB"] = srv.lane_ws / 1e9
                st["library_device_GB"] = max(lib0, ebcc.device_bytes()) / 1e9
                st["mix_vs_solo_checked"] = stat["checked"]
                st["mix_vs_solo_mismatches"] = stat["mismatch"]
                serving[f"{int(rate)}_per_s"] = st
                log(f"serving at {rate:.0f} req/s: {st}")

    # ---------------- Algorithm 1's ratio search on the stack (batched) ----------------
    ratio_search = None
    if args.q > 0:
        qargs = ebcc.BatchArgs(xs, err_bounds=[args.eps] * len(xs))
        qout = torch.empty(qargs.bound(), dtype=torch.uint8, device=dev)
        pq = ebcc.params(args.eps, args.ratio, q=args.q, **fmt)
        assert ebcc.compress_batch_into(qargs, qout, pq, stream) == 0
        torch.cuda.synchronize()
        a = time.perf_counter()
        assert ebcc.compress_batch_into(qargs, qout, pq, stream) == 0
        torch.cuda.synchronize()
        b = time.perf_counter()
        qstreams = [qout[qargs.offsets[i]: qargs.offsets[i] + qargs.lengths[i]] for i in range(qargs.n)]
        qd = ebcc.DecodeArgs(qstreams, recs)
        assert ebcc.decompress_batch_into(qd, stream) == 0
        torch.cuda.synchronize()
        c = time.perf_counter()
        qviol, qmax = verify(stack_h, recs, [args.eps] * len(xs))
        qsb = sum(qargs.lengths[i] for i in range(qargs.n))
        ratio_search = {"workload": f"the stack through the batched entry points with Algorithm 1's base-ratio "
                                    f"search, q = {args.q}, r0 = {args.ratio}",
                        "q": args.q, "compress_GBps": nbytes / (b - a) / 1e9, "decompress_GBps": nbytes / (c - b) / 1e9,
                        "CR": nbytes / qsb, "CR_fixed_ratio": cr_stack, "violations": qviol,
                        "max_err_rel": qmax}
        log(f"ratio search: {ratio_search}")

    # ---------------- byte-granular residual truncation (trunc = 1) ----------------
    byte_cut = None
    if args.byte_cut:
        bcargs = ebcc.BatchArgs(xs, err_bounds=[args.eps] * len(xs))
        bcout = torch.empty(bcargs.bound(), dtype=torch.uint8, device=dev)
        byte_cut = {"workload": f"the stack through the batched entry points, residual cut at byte positions "
                                f"(trunc = 1), eps_rel {args.eps}, r {args.ratio}"}
        for qv in ([0.0, args.q] if args.q > 0 else [0.0]):
            pb = ebcc.params(args.eps, args.ratio, q=qv, trunc=1, **fmt)
            assert ebcc.compress_batch_into(bcargs, bcout, pb, stream) == 0
            torch.cuda.synchronize()
            a = time.perf_counter()
            assert ebcc.compress_batch_into(bcargs, bcout, pb, stream) == 0
            torch.cuda.synchronize()
            b = time.perf_counter()
            bcs = [bcout[bcargs.offsets[i]: bcargs.offsets[i] + bcargs.lengths[i]] for i in range(bcargs.n)]
            assert ebcc.decompress_batch_into(ebcc.DecodeArgs(bcs, recs), stream) == 0
            torch.cuda.synchronize()
            c = time.perf_counter()
            bv, bm = verify(stack_h, recs, [args.eps] * len(xs))
            bsb = sum(bcargs.lengths[i] for i in range(bcargs.n))
            key = "fixed_ratio" if qv == 0 else f"q_{qv:g}"
            byte_cut[key] = {"CR": nbytes / bsb, "CR_plane_ends": cr_stack if qv == 0 else None,
                             "compress_GBps": nbytes / (b - a) / 1e9, "decompress_GBps": nbytes / (c - b) / 1e9,
                             "violations": bv, "max_err_rel": bm}
        # per-call latency of the per-field path with the byte search
        pl1 = ebcc.params(args.eps, args.ratio, trunc=1, **fmt)
        lc = []
        for i in range(min(16, len(xs))):
            torch.cuda.synchronize()
            a = time.perf_counter()
            rc, _ = ebcc.compress_into(xs[i], outs[i], pl1, stream)
            lc.append(time.perf_counter() - a)
            assert rc == 0
        byte_cut["per_field_compress_ms_p50"] = pct(lc, 50) * 1e3
        byte_cut["per_field_fields"] = len(lc)
        log(f"byte cut: {byte_cut}")

    # ---------------- tier-1 arithmetic-coding bypass (bypass = 1) ----------------
    bypass = None
    if args.bypass:
        bypass = {"workload": f"the stack ({len(xs)} fields of {args.ny}x{args.nx}), per-field and batched entry "
                              f"points, r {args.ratio}, with and without the arithmetic-coding bypass "
                              f"(raw SPP/MRP passes after the tenth)"}
        yout = None
        for e in (args.eps, 0.001):
            row = {}
            bargs_y = ebcc.BatchArgs(xs, err_bounds=[e] * len(xs))
            if yout is None:
                yout = torch.empty(bargs_y.bound(), dtype=torch.uint8, device=dev)
            for byp in (0, 1):
                pl = [ebcc.params(e, args.ratio, bypass=byp, **fmt)] * len(xs)
                per_field_step(xs, outs, recs, lens, pl)             # warm-up (graphs, workspace)
                lc, ld = [], []
                ebcc.profile_enable(True)
                torch.cuda.synchronize()
                tcy, tdy = per_field_step(xs, outs, recs, lens, pl, lc, ld)
                prof_y = ebcc.profile_read()
                ebcc.profile_enable(False)
                vy, my = verify(stack_h, recs, [e] * len(xs))
                st = {k: v for k, v in prof_y.items() if k.startswith("t1") and v[1] > 0}
                pb = ebcc.params(e, args.ratio, bypass=byp, **fmt)
                assert ebcc.compress_batch_into(bargs_y, yout, pb, stream) == 0
                torch.cuda.synchronize()
                a = time.perf_counter()
                assert ebcc.compress_batch_into(bargs_y, yout, pb, stream) == 0
                torch.cuda.synchronize()
                b = time.perf_counter()
                ys_ = [yout[bargs_y.offsets[i]: bargs_y.offsets[i] + bargs_y.lengths[i]] for i in range(bargs_y.n)]
                assert ebcc.decompress_batch_into(ebcc.DecodeArgs(ys_, recs), stream) == 0
                torch.cuda.synchronize()
                c = time.perf_counter()
                vb, _ = verify(stack_h, recs, [e] * len(xs))
                row["bypass" if byp else "mq_only"] = {
                    "CR": nbytes / sum(lens), "per_field_compress_ms_p50": pct(lc, 50) * 1e3,
                    "per_field_decompress_ms_p50": pct(ld, 50) * 1e3, "per_field_GBps": nbytes / (tcy + tdy) / 1e9,
                    "tier1_stage_ms_per_call": {k: v[0] / v[1] for k, v in st.items()},
                    "batched_compress_GBps": nbytes / (b - a) / 1e9, "batched_decompress_GBps": nbytes / (c - b) / 1e9,
                    "violations": vy + vb, "max_err_rel": my}
            row["CR_cost_pct"] = 100.0 * (1.0 - row["bypass"]["CR"] / row["mq_only"]["CR"])
            bypass[f"eps_{e:g}"] = row
        log(f"bypass: {bypass}")

    # ---------------- ablation of q (relative CR against q = 1) ----------------
    q_ablation = None
    if args.ablation_fields and bx:
        ab = bx[: args.ablation_fields]
        qs = [1 - 1e-3, 1 - 1e-4, 1 - 1e-5, 1 - 1e-6, 1.0]
        q_ablation = {"workload": f"uneven mix, first {len(ab)} fields, each bound in {{0.1%, 1%, 10%}}, "
                                  f"q in {{1-1e-3 .. 1-1e-6, 1}}, r0 {args.ratio}; CR relative to q = 1 per field",
                      "q": qs}
        aargs = ebcc.BatchArgs(ab)
        aout = torch.empty(aargs.bound(), dtype=torch.uint8, device=dev)
        for e in (0.001, 0.01, 0.1):
            lens_q = {}
            for qv in qs:
                pa = ebcc.params(e, args.ratio, q=qv, **fmt)
                assert ebcc.compress_batch_into(aargs, aout, pa, stream) == 0
                lens_q[qv] = np.array([aargs.lengths[i] for i in range(aargs.n)], dtype=np.float64)
            per_q = {}
            for qv in qs[:-1]:
                rel = lens_q[1.0] / lens_q[qv]          # CR(q) / CR(q = 1)
                per_q[f"{qv:.6f}"] = {"min": float(rel.min()), "p10": pct(rel, 10), "median": pct(rel, 50),
                                      "p90": pct(rel, 90), "max": float(rel.max()), "mean": float(rel.mean()),
                                      "frac_ge_1": float(np.mean(rel >= 1.0))}
            q_ablation[f"eps_{e:g}"] = per_q
        log(f"q ablation: {q_ablation}")

    # ---------------- km-scale stress fields (batched and served) ----------------
    km = None
    if km_h:
        kx = [torch.from_numpy(f).to(dev) for f in km_h]
        kbytes = sum(f.nbytes for f in km_h)
        kargs = ebcc.BatchArgs(kx, err_bounds=[0.001] * len(kx))
        kout = torch.empty(kargs.bound(), dtype=torch.uint8, device=dev)
        pk = ebcc.params(0.001, args.ratio, levels=6, **fmt)
        assert ebcc.compress_batch_into(kargs, kout, pk, stream) == 0
        torch.cuda.synchronize()
        a = time.perf_counter()
        assert ebcc.compress_batch_into(kargs, kout, pk, stream) == 0
        torch.cuda.synchronize()
        b = time.perf_counter()
        kst = [kout[kargs.offsets[i]: kargs.offsets[i] + kargs.lengths[i]] for i in range(kargs.n)]
        krec = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in km_h]
        kd = ebcc.DecodeArgs(kst, krec)
        assert ebcc.decompress_batch_into(kd, stream) == 0
        torch.cuda.synchronize()
        c = time.perf_counter()
        kviol, kmax = verify(km_h, krec, [0.001] * len(kx))
        ext_err = 0.0
        for i, (f, y) in enumerate(zip(km_h, krec)):   # error at the vortex cores (top 0.01% of |x|)
            if i and i % 128 == 0:
                log(f"vortex-core errors of {i} of {len(km_h)} fields")
            a64 = np.abs(f.astype(np.float64))
            m = a64 >= np.quantile(a64, 0.9999)
            e = np.abs(f.astype(np.float64) - y.cpu().numpy().astype(np.float64))[m].max()
            ext_err = max(ext_err, e / (float(f.max()) - float(f.min())))
        km = {"workload": f"{len(kx)} km-scale 1801x3600 fields (8 Rankine vortices each), bound 0.1% of range, "
                          f"6 levels", "MB": kbytes / 1e6,
              "compress_GBps": kbytes / (b - a) / 1e9, "decompress_GBps": kbytes / (c - b) / 1e9,
              "CR": kbytes / sum(kargs.lengths[i] for i in range(kargs.n)), "violations": kviol,
              "max_err_rel": kmax, "max_err_rel_at_extremes": float(ext_err)}
        # served: every field compressed and its stream decompressed through the loop
        from paper_2510_22265_amd import serve
        kres = {}

        def kdone(r):
            if r.status == 0:
                kres[(r.kind, r.tag)] = r.result if r.kind == serve.COMPRESS else r.result.cpu().numpy()
            r.result = None

        srv = serve.Server(hbm_budget=SERVE_BUDGET, lanes=2, params=dict(fmt, levels=6),
                           base_ratio=args.ratio).start()
        t0 = time.perf_counter()
        rs = [srv.submit(serve.Request(serve.COMPRESS, x, eps=0.001, tag=i, on_done=kdone)) for i, x in enumerate(kx)]
        rs += [srv.submit(serve.Request(serve.DECOMPRESS, s, shape=tuple(kx[i].shape), tag=i, on_done=kdone))
               for i, s in enumerate(kst)]
        for r in rs:
            r.wait()
        wall = time.perf_counter() - t0
        srv.stop()
        st = serve.summarize(rs, wall)
        same = all(torch.equal(kres.get((serve.COMPRESS, i), torch.empty(0, dtype=torch.uint8, device=dev)), kst[i])
                   for i in range(len(kx)))
        sv, _ = verify(km_h, [kres[(serve.DECOMPRESS, i)] for i in range(len(kx))], [0.001] * len(kx))
        km["served"] = {"requests": len(rs), "seconds": wall, "GBps": 2 * kbytes / wall / 1e9,
                        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "failed": st["failed"],
                        "streams_identical_to_batched": bool(same), "violations": sv}
        log(f"km-scale: {km}")

    # ---------------- CPU oracle baselines ----------------
    cpu = cpu_single = cpu_legs = tier1 = None
    if not args.no_cpu:
        from oracle import ref
        ref.lib()
        threads = min(16, os.cpu_count() or 1)
        model = cpu_model()
        # all cores on the headline workload: the reported baseline
        r = oracle_all_cores(stack_h, [args.eps] * len(stack_h), threads, args.cpu_seconds, base_ratio=args.ratio)
        cpu = {"value": r["GBps"], "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"{r['fields']} of {len(stack_h)} fields ({args.ny}x{args.nx}, eps_rel {args.eps}), "
                         f"compress + decompress, {threads} threads over fields, {r['seconds']:.1f} s",
               "cpu_model": model}
        log(f"oracle all cores: {cpu}")
        # one thread (the paper's protocol)
        # (the oracle's work counters give the MQ decisions of these fields:
        # what the tier-1 kernels execute, for a decisions/s figure)
        t0 = time.perf_counter()
        done = sb = 0
        enc_c, dec_c = [], []
        while done < len(stack_h) and time.perf_counter() - t0 < args.cpu_seconds:
            ref.mq_counts(reset=True)
            s = ref.compress(stack_h[done], args.eps, base_ratio=args.ratio)
            enc_c.append(ref.mq_counts(reset=True))
            ref.decompress(s, args.ny, args.nx)
            dec_c.append(ref.mq_counts(reset=True))
            sb += stack_h[done].nbytes
            done += 1
        el = time.perf_counter() - t0
        cpu_single = {"value": sb / el / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
                      "sample": f"{done} of {len(stack_h)} fields, single thread, {el:.1f} s", "cpu_model": model}
        if done and "t1_encode" in stages and "t1_decode" in stages:
            enc = float(np.mean([c["enc"] for c in enc_c]))
            dec = float(np.mean([c["dec"] for c in dec_c]))
            emax = float(np.mean([c["enc_max_block"] for c in enc_c]))
            dmax = float(np.mean([c["dec_max_block"] for c in dec_c]))
            t_enc = stages["t1_encode"][0] / stages["t1_encode"][1] / 1e3    # s per launch (one field)
            t_dec = stages["t1_decode"][0] / stages["t1_decode"][1] / 1e3
            tier1 = {"fields": done, "samples_per_field": args.ny * args.nx,
                     "enc_decisions_per_field": enc, "enc_decisions_per_sample": enc / (args.ny * args.nx),
                     "enc_max_block_decisions": emax,
                     "dec_decisions_per_field": dec, "dec_decisions_per_sample": dec / (args.ny * args.nx),
                     "dec_max_block_decisions": dmax,
                     "t1_encode_ms": t_enc * 1e3, "t1_decode_ms": t_dec * 1e3,
                     "enc_decisions_per_s": enc / t_enc, "dec_decisions_per_s": dec / t_dec,
                     "enc_ns_per_decision_heaviest_block": t_enc / emax * 1e9,
                     "dec_ns_per_decision_heaviest_block": t_dec / dmax * 1e9,
                     "alu_ceiling_decisions_per_s": T1_ALU_CEILING,
                     "enc_frac_of_alu_ceiling": enc / t_enc / T1_ALU_CEILING,
                     "dec_frac_of_alu_ceiling": dec / t_dec / T1_ALU_CEILING}
            log(f"tier-1 decisions: {tier1}")
        cpu_legs = {}
        if batch_h:
            rb = oracle_all_cores(batch_h, beps, threads, args.cpu_seconds, base_ratio=args.ratio)
            cpu_legs["uneven_batch"] = dict(rb, sample=f"{rb['fields']} of {len(batch_h)} uneven-mix fields")
        if km_h:
            kk = km_h[:4]
            rk = oracle_all_cores(kk, [0.001] * len(kk), threads, 10 * args.cpu_seconds, base_ratio=args.ratio,
                                  levels=6)
            cpu_legs["km_scale"] = dict(rk, sample=f"{rk['fields']} of {len(km_h)} km-scale fields (one per "
                                                   f"variable); the stack's time extrapolates by field count")
        log(f"oracle legs: {cpu_legs}")

    out = {
        "metric": "compress/decompress GB/s (fp32 in) at max-err<=1% range; CR; p50/p99 latency",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": t_total / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ERA5-shaped stack, plain per-field path: {len(xs)} fields {args.ny}x{args.nx} "
                               f"(37 levels x t,u,v,q), eps_rel {args.eps}, r {args.ratio}, L 5, "
                               f"{1 << p.cblk_log2w}x{1 << p.cblk_log2h} blocks, "
                               f"{tile}x{tile}-root SPIHT tiles",
                   "fields": len(xs), "ny": args.ny, "nx": args.nx, "eps_rel": args.eps, "base_ratio": args.ratio},
        "compress_GBps": nbytes * steps / tc / 1e9, "decompress_GBps": nbytes * steps / td / 1e9,
        "CR": cr_stack, "violations": viol, "max_err_rel": max_rel,
        "compress_ms_p50": pct(lat_c, 50) * 1e3, "compress_ms_p99": pct(lat_c, 99) * 1e3,
        "decompress_ms_p50": pct(lat_d, 50) * 1e3, "decompress_ms_p99": pct(lat_d, 99) * 1e3,
        "stages_ms_per_step": {k: v[0] / steps for k, v in stages.items()},
        "c1_bounds": c1_bounds,
        "c0": c0,
        "batched": batched,
        "serving": serving,
        "ratio_search": ratio_search,
        "byte_cut": byte_cut,
        "bypass": bypass,
        "q_ablation": q_ablation,
        "km_scale": km,
        "tier1_decisions": tier1,
        "roofline": roof, "cpu_baseline": cpu, "cpu_single_thread": cpu_single, "cpu_legs": cpu_legs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
