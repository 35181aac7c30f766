#!/usr/bin/env python3
"""EBCC compress/decompress throughput on one MI355X.

Workload (default): the ERA5-shaped stack, plain per-field path: 148 float32
fields of 721x1440 (37 levels x {temperature-, u-, v-, humidity-like}),
range-relative bound 1% (the headline bound), base ratio r = 30, 5 DWT
levels, 32x32 code-blocks, 2x2-root SPIHT tiles.  Inputs are synthetic
(seeded generators standing in for ERA5) and resident in HBM before timing.

One step = compress every field, then decompress every stream, one field at
a time on one stream.  value = fp32 bytes of the stack / step time (GB/s,
decimal), i.e. round-trip throughput; compress and decompress rates,
compression ratio, per-call p50/p99 latency, the stage breakdown, the
roofline of the dominant kernel and the CPU oracle baseline are printed in
the same JSON line.
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
# Integer/ALU peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def _gen(args):
    from paper_2510_22265_amd import synth
    var, ny, nx, level = args
    return synth.field(var, ny, nx, cfg=1, level=level)


def make_fields(nfields, ny, nx):
    from multiprocessing import Pool
    specs = []
    for lev in range(37):
        for v in ("t", "u", "v", "q"):
            specs.append((v, ny, nx, lev))
    specs = specs[:nfields]
    procs = min(16, os.cpu_count() or 1)
    with Pool(procs) as p:
        fields = p.map(_gen, specs)
    return specs, fields


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


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
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the path shards by field with no exchange between GPUs, "
              "and multi-GPU runs are not part of this build (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_22265_amd import ebcc
    if not os.path.exists(ebcc.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    ebcc.lib()
    dev = torch.device("cuda:0")
    print(f"bench: generating {args.fields} fields of {args.ny}x{args.nx}", file=sys.stderr, flush=True)
    specs, fields_h = make_fields(args.fields, args.ny, args.nx)
    xs = [torch.from_numpy(f).to(dev) for f in fields_h]
    p = ebcc.params(args.eps, args.ratio)
    cap = ebcc.compress_bound(args.ny, args.nx)
    outs = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in xs]
    recs = [torch.empty((args.ny, args.nx), dtype=torch.float32, device=dev) for _ in xs]
    lens = [0] * len(xs)
    stream = torch.cuda.current_stream()
    nbytes = sum(f.nbytes for f in fields_h)

    def step(lat_c=None, lat_d=None):
        t0 = time.perf_counter()
        for i, x in enumerate(xs):
            a = time.perf_counter()
            rc, n = ebcc.compress_into(x, outs[i], p, stream)
            if rc != 0:
                raise RuntimeError(f"compress failed on field {specs[i]}: {rc} {ebcc.lib().ebcc_last_error()}")
            lens[i] = n
            if lat_c is not None:
                lat_c.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(len(xs)):
            a = time.perf_counter()
            rc = ebcc.decompress_into(outs[i][: lens[i]], recs[i], stream)
            if rc != 0:
                raise RuntimeError(f"decompress failed on field {specs[i]}: {rc}")
            if lat_d is not None:
                lat_d.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    for w in range(args.warmup):
        step()
        print(f"bench: warmup step {w} done", file=sys.stderr, flush=True)
    lat_c, lat_d = [], []
    ebcc.profile_enable(True)
    torch.cuda.synchronize()
    tc = td = 0.0
    t_start = time.perf_counter()
    for s in range(args.steps):
        a, b = step(lat_c, lat_d)
        tc += a
        td += b
        print(f"bench: step {s}: compress {a * 1e3:.1f} ms, decompress {b * 1e3:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = ebcc.profile_read()
    ebcc.profile_enable(False)

    # verification outside the timed region: bound and compression ratio
    viol = 0
    max_rel = 0.0
    for i, x in enumerate(xs):
        xd = x.double()
        rng_ = float(fields_h[i].max()) - float(fields_h[i].min())
        err = float((xd - recs[i].double()).abs().max())
        if err > args.eps * rng_:
            viol += 1
        if rng_ > 0:
            max_rel = max(max_rel, err / rng_)
    stream_bytes = sum(lens)
    cr = nbytes / stream_bytes

    steps = args.steps
    value = nbytes * steps / t_total / 1e9
    comp_gbps = nbytes * steps / tc / 1e9
    dec_gbps = nbytes * steps / td / 1e9

    # roofline of the dominant stage (a single kernel: tier-1 encode)
    stages = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(stages, key=lambda k: stages[k][0]) if stages else None
    roof = None
    if dom is not None:
        ms, calls = stages[dom]
        avg_s = ms / calls / 1e3
        N = args.ny * args.nx
        # algorithmic bytes of one launch of the dominant kernel
        if dom == "t1_encode":
            # reads the field's quantised bit-plane masks and coefficients and
            # writes the codewords: ~4 B/sample in + codeword bytes out
            algo = 4.0 * N + stream_bytes / len(xs)
        else:
            algo = 8.0 * N
        ach = algo / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBPS, "traffic": None, "avg_launch_ms": ms / calls}

    cpu = None
    if not args.no_cpu:
        from oracle import ref
        ref.lib()
        t0 = time.perf_counter()
        done = 0
        sb = 0
        while done < len(fields_h) and time.perf_counter() - t0 < args.cpu_seconds:
            s = ref.compress(fields_h[done], args.eps, base_ratio=args.ratio)
            ref.decompress(s, args.ny, args.nx)
            sb += fields_h[done].nbytes
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": sb / el / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} of {len(fields_h)} fields ({args.ny}x{args.nx}), compress + decompress, "
                         f"single thread, {el:.1f} s"}

    out = {
        "metric": "compress/decompress GB/s (fp32 in) at max-err<=1% range; CR; p50/p99 latency",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": t_total / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ERA5-shaped stack, plain per-field path: {len(xs)} fields {args.ny}x{args.nx} "
                               f"(37 levels x t,u,v,q), eps_rel {args.eps}, r {args.ratio}, L 5, 32x32 blocks",
                   "fields": len(xs), "ny": args.ny, "nx": args.nx, "eps_rel": args.eps, "base_ratio": args.ratio},
        "compress_GBps": comp_gbps, "decompress_GBps": dec_gbps, "CR": cr, "violations": viol,
        "max_err_rel": max_rel,
        "compress_ms_p50": pct(lat_c, 50) * 1e3, "compress_ms_p99": pct(lat_c, 99) * 1e3,
        "decompress_ms_p50": pct(lat_d, 50) * 1e3, "decompress_ms_p99": pct(lat_d, 99) * 1e3,
        "stages_ms_per_step": {k: v[0] / steps for k, v in stages.items()},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
