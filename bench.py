#!/usr/bin/env python3
"""EBCC compress/decompress throughput on one MI355X.

Headline workload (`value`): the ERA5-shaped stack, plain per-field path:
148 float32 fields of 721x1440 (37 levels x {temperature-, u-, v-,
humidity-like}), range-relative bound 1%, base ratio r = 30, 5 DWT levels,
32x32 code-blocks, one-root SPIHT tiles.  One step = compress every field,
then decompress every stream, one field per call on one stream.  value = fp32
bytes of the stack / step time (GB/s, decimal): round-trip throughput.

Beside it, in the same JSON line:
  batched   the uneven batch (256 fields drawn from 91x180 .. 721x1440,
            per-field bounds log-uniform in [0.1%, 10%] of range) through
            ebcc_compress_batch / ebcc_decompress_batch, the same fields
            through the per-field loop, and the speedup; also the headline
            stack through the batched entry points;
  roofline  the dominant kernel of the headline path (its HIP-event time
            per launch, algorithmic bytes per launch);
  cpu_baseline  the CPU oracle on a bounded sample of the headline fields.
Inputs are synthetic (seeded generators standing in for ERA5) and resident
in HBM before timing; verification (bound, compression ratio) is outside the
timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E

# HBM bytes per launch of the headline path's tier-1 kernels on one
# 721x1440 field at eps_rel 1%, from two rocprofv3 --pmc runs (FETCH_SIZE,
# WRITE_SIZE; profiles/kernels_era5_721x1440_per_field.md), each scaled by
# what the counter reads for a plain elementwise copy of 1 GiB (FETCH_SIZE
# x2.0, WRITE_SIZE x1.0).  Valid only while the kernel's source is the one
# measured (checked by hash); otherwise traffic is reported as null.
MEASURED_TRAFFIC = {
    "t1_encode": {"source": "paper_2510_22265_amd/csrc/t1wave.hip",
                  "sha256": "ae2148ef88020237e02003971584fdb66d708c9add6b03aa4a1e1025b48d1a0e",
                  "ny": 721, "nx": 1440, "eps": 0.01,
                  "bytes": (2.0 * (3869.4 + 3747.1) / 2 + 1.0 * (986.7 + 1230.2) / 2) * 1024},
    "t1_decode": {"source": "paper_2510_22265_amd/csrc/t1wave.hip",
                  "sha256": "ae2148ef88020237e02003971584fdb66d708c9add6b03aa4a1e1025b48d1a0e",
                  "ny": 721, "nx": 1440, "eps": 0.01,
                  "bytes": (2.0 * (593.8 + 558.4) / 2 + 1.0 * (4099.5 + 4099.5) / 2) * 1024},
}


def measured_traffic(kernel, ny, nx, eps):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if not m or (m["ny"], m["nx"], m["eps"]) != (ny, nx, eps):
        return None
    with open(os.path.join(ROOT, m["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != m["sha256"]:
            return None
    return m["bytes"]


def _gen(spec):
    from paper_2510_22265_amd import synth
    kind, a = spec
    if kind == "stack":
        var, ny, nx, level = a
        return synth.field(var, ny, nx, cfg=1, level=level)
    return synth.batch_field(a)


def _gen_km(a):
    from paper_2510_22265_amd import synth
    var, level = a
    return synth.vortex_field(1801, 3600, var=var, level=level, cfg=4)


def generate(specs):
    from multiprocessing import Pool
    procs = min(16, os.cpu_count() or 1)
    with Pool(procs) as p:
        return p.map(_gen, specs, chunksize=4)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def verify(xs_h, recs, eps):
    """Count bound violations (FP64) and the largest range-relative error."""
    viol, max_rel = 0, 0.0
    for x, y, e in zip(xs_h, recs, eps):
        rng_ = float(x.max()) - float(x.min())
        err = float(np.abs(x.astype(np.float64) - y.cpu().numpy().astype(np.float64)).max())
        if err > e * rng_:
            viol += 1
        if rng_ > 0:
            max_rel = max(max_rel, err / rng_)
    return viol, max_rel


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
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuned batched run")
    ap.add_argument("--serve-rates", default="200,1000,5000", help="Poisson arrival rates (req/s); empty: skip")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window per rate")
    ap.add_argument("--q", type=float, default=1 - 1e-5, help="proportion q of the ratio-search run (0: skip)")
    ap.add_argument("--km-fields", type=int, default=8, help="km-scale 1801x3600 vortex fields (0: skip)")
    ap.add_argument("--batch-fields", type=int, default=256, help="fields of the uneven batch (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle baseline sample")
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

    import torch
    from paper_2510_22265_amd import ebcc, synth
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

    # ---------------- inputs ----------------
    stack_specs = [("stack", (v, args.ny, args.nx, lev)) for lev in range(37) for v in synth.VARS][: args.fields]
    bspecs = synth.batch_specs(n=args.batch_fields) if args.batch_fields else []
    log(f"generating {len(stack_specs)} fields of {args.ny}x{args.nx} and an uneven batch of {len(bspecs)}")
    fields_h = generate(stack_specs + [("batch", s) for s in bspecs])
    stack_h, batch_h = fields_h[: len(stack_specs)], fields_h[len(stack_specs):]
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
    steps = args.steps
    value = nbytes * steps / t_total / 1e9

    # roofline of the dominant kernel (each timed stage is one kernel launch
    # per call for tier-1; HIP events on the library's stream)
    stages = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(stages, key=lambda k: stages[k][0]) if stages else None
    roof = None
    if dom is not None:
        ms, calls = stages[dom]
        avg_s = ms / calls / 1e3
        N = args.ny * args.nx
        if dom in ("t1_encode", "t1_decode"):
            # algorithmic bytes of one launch: the field's coefficients (4 B
            # per sample) and the base-layer codewords of one stream
            algo = 4.0 * N + stream_bytes / len(xs) / 2
        else:
            algo = 8.0 * N
        ach = algo / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBPS, "traffic": measured_traffic(dom, args.ny, args.nx, args.eps),
                "avg_launch_ms": ms / calls, "algo_bytes_per_launch": algo}

    # ---------------- batched execution ----------------
    batched = None
    if bspecs:
        bx = [torch.from_numpy(f).to(dev) for f in batch_h]
        beps = [s[3] for s in bspecs]
        bbytes = sum(f.nbytes for f in batch_h)
        bargs = ebcc.BatchArgs(bx, err_bounds=beps)
        bout = torch.empty(bargs.bound(), dtype=torch.uint8, device=dev)

        def batch_compress():
            rc = ebcc.compress_batch_into(bargs, bout, p, stream)
            if rc != 0:
                raise RuntimeError(f"batched compress failed: {rc} {ebcc.lib().ebcc_last_error()}")

        batch_compress()
        bstreams = [bout[bargs.offsets[i]: bargs.offsets[i] + bargs.lengths[i]] for i in range(bargs.n)]
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
        a = time.perf_counter()
        for s in range(steps):
            assert ebcc.compress_batch_into(sargs, sout, p, stream) == 0
        torch.cuda.synchronize()
        b = time.perf_counter()
        for s in range(steps):
            assert ebcc.decompress_batch_into(sdargs, stream) == 0
        torch.cuda.synchronize()
        c = time.perf_counter()
        sviol, _ = verify(stack_h, recs, [args.eps] * len(xs))
        stack_same = all(torch.equal(sstreams[i], outs[i][: lens[i]]) for i in range(len(xs)))
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
            tc_ = td_ = 0.0
            for s in range(steps):
                a = time.perf_counter()
                assert ebcc.compress_batch_into(targs, tout, tp, stream) == 0
                torch.cuda.synchronize()
                b = time.perf_counter()
                assert ebcc.decompress_batch_into(tdargs, stream) == 0
                torch.cuda.synchronize()
                c = time.perf_counter()
                tc_ += b - a
                td_ += c - b
                log(f"tuned batched step {s}: compress {(b - a) * 1e3:.1f} ms, decompress {(c - b) * 1e3:.1f} ms")
            tviol, _ = verify(batch_h, brecs, beps)
            ebcc.set_tuning(**old)
            tsb = sum(targs.lengths[i] for i in range(targs.n))
            tuned = {"params": res["params"], "tuning": res["tuning"], "tune_seconds": t_tune,
                     "candidates": len(res["table"]),
                     "GBps": bbytes * steps / (tc_ + td_) / 1e9, "compress_GBps": bbytes * steps / tc_ / 1e9,
                     "decompress_GBps": bbytes * steps / td_ / 1e9, "CR": bbytes / tsb, "violations": tviol,
                     "speedup_vs_per_field": (pc + pd) / ((tc_ + td_) / steps)}
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
            "stack_GBps": nbytes * steps / (c - a) / 1e9,
            "stack_compress_GBps": nbytes * steps / (b - a) / 1e9,
            "stack_decompress_GBps": nbytes * steps / (c - b) / 1e9,
            "stack_speedup_vs_per_field": (t_total / steps) / ((c - a) / steps),
            "stack_streams_identical": bool(stack_same), "stack_violations": sviol,
            "tuned": tuned,
        }

    # ---------------- serving loop: Poisson arrivals, continuous batching ----------------
    serving = None
    rates = [float(r) for r in args.serve_rates.split(",") if r.strip()] if bspecs else []
    if rates:
        from paper_2510_22265_amd import serve
        import random
        # half the requests compress a field of the uneven mix, half decompress one of its streams
        sstreams_c = [s.clone() for s in bstreams]
        serving = {"workload": f"Poisson arrivals of compress/decompress requests (1:1) on the uneven "
                               f"{len(bx)}-field mix, HBM admission budget 64 GB, 2 lanes",
                   "budget_GB": 64, "lanes": 2}
        for rate in rates:
            rnd = random.Random(int(rate))

            def make(k):
                i = rnd.randrange(len(bx))
                if rnd.random() < 0.5:
                    return serve.Request(serve.COMPRESS, bx[i], eps=beps[i], tag=i)
                return serve.Request(serve.DECOMPRESS, sstreams_c[i], shape=tuple(bx[i].shape), tag=i)

            srv = serve.Server(hbm_budget=64 * 10**9, lanes=2, params=fmt, base_ratio=args.ratio).start()
            reqs, wall = serve.poisson_run(srv, make, rate=rate, duration=args.serve_seconds, seed=int(rate),
                                           max_requests=int(rate * args.serve_seconds * 2) + 10)
            srv.stop()
            st = serve.summarize(reqs, wall)
            st["mean_batch"] = float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0
            st["peak_GB_admitted"] = srv.peak_in_use / 1e9
            bad = 0
            for r in reqs:   # results in the mix against the same request alone (a sample)
                if r.kind == serve.COMPRESS and r.tag % 16 == 0 and r.status == 0:
                    bad += int(not torch.equal(r.result, bstreams[r.tag]))
            st["mix_vs_solo_mismatches"] = bad
            serving[f"{int(rate)}_per_s"] = st
            log(f"serving at {rate:.0f} req/s: {st}")
        batched["serving"] = serving

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
                        "CR": nbytes / qsb, "CR_fixed_ratio": nbytes / stream_bytes, "violations": qviol,
                        "max_err_rel": qmax}
        log(f"ratio search: {ratio_search}")

    # ---------------- km-scale stress fields (batched) ----------------
    km = None
    if args.km_fields:
        kspecs = [("km", (v, lev)) for lev in range((args.km_fields + 1) // 2) for v in ("u", "v")][: args.km_fields]
        from multiprocessing import Pool
        with Pool(min(16, os.cpu_count() or 1)) as pool:
            kh = pool.map(_gen_km, [k[1] for k in kspecs])
        kx = [torch.from_numpy(f).to(dev) for f in kh]
        kbytes = sum(f.nbytes for f in kh)
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
        krec = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in kh]
        kd = ebcc.DecodeArgs(kst, krec)
        assert ebcc.decompress_batch_into(kd, stream) == 0
        torch.cuda.synchronize()
        c = time.perf_counter()
        kviol, kmax = verify(kh, krec, [0.001] * len(kx))
        ext_err = 0.0
        for f, y in zip(kh, krec):   # error at the vortex cores (top 0.01% of |x|)
            a64 = np.abs(f.astype(np.float64))
            m = a64 >= np.quantile(a64, 0.9999)
            e = np.abs(f.astype(np.float64) - y.cpu().numpy().astype(np.float64))[m].max()
            ext_err = max(ext_err, e / (float(f.max()) - float(f.min())))
        km = {"workload": f"{len(kx)} km-scale 1801x3600 fields (8 Rankine vortices each), bound 0.1% of range, "
                          f"6 levels, batched", "MB": kbytes / 1e6,
              "compress_GBps": kbytes / (b - a) / 1e9, "decompress_GBps": kbytes / (c - b) / 1e9,
              "CR": kbytes / sum(kargs.lengths[i] for i in range(kargs.n)), "violations": kviol,
              "max_err_rel": kmax, "max_err_rel_at_extremes": ext_err}
        log(f"km-scale: {km}")

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu:
        from oracle import ref
        ref.lib()
        t0 = time.perf_counter()
        done = 0
        sb = 0
        while done < len(stack_h) and time.perf_counter() - t0 < args.cpu_seconds:
            s = ref.compress(stack_h[done], args.eps, base_ratio=args.ratio)
            ref.decompress(s, args.ny, args.nx)
            sb += stack_h[done].nbytes
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": sb / el / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} of {len(stack_h)} fields ({args.ny}x{args.nx}), compress + decompress, "
                         f"single thread, {el:.1f} s"}

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
        "CR": nbytes / stream_bytes, "violations": viol, "max_err_rel": max_rel,
        "compress_ms_p50": pct(lat_c, 50) * 1e3, "compress_ms_p99": pct(lat_c, 99) * 1e3,
        "decompress_ms_p50": pct(lat_d, 50) * 1e3, "decompress_ms_p99": pct(lat_d, 99) * 1e3,
        "stages_ms_per_step": {k: v[0] / steps for k, v in stages.items()},
        "batched": batched,
        "ratio_search": ratio_search,
        "km_scale": km,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
