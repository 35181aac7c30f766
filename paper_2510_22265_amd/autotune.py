"""Autotuner of batched execution.

Picks, by measurement on the caller's own fields, the code-block size and
SPIHT tile (which change the stream, so a compression-ratio constraint
applies) and the kernel choices of `ebcc_tuning` (which never change the
stream: only speed).  Every candidate is a full batched round trip
(`ebcc_compress_batch` then `ebcc_decompress_batch`) on the fields, or on a
size-stratified sample of them; the fastest candidate whose compression
ratio is within `cr_tol` of the default format's wins.  Results are cached
per (device, field-shape histogram, bounds, base ratio) in memory and,
optionally, in a JSON file.
"""
import json
import os
import time

import torch

from . import ebcc

# (cblk_log2w, cblk_log2h, spiht_tile); the first entry is the default format
FORMATS = ((5, 5, 1), (5, 5, 2), (5, 4, 1), (6, 5, 1), (6, 6, 1), (6, 6, 2), (4, 4, 1))
# kernel choices (ebcc_tuning fields); the first entry is the library default
KERNELS = (
    dict(t1_encoder=0, t1_decoder=0, spiht=0),
    dict(t1_encoder=2, t1_decoder=1, spiht=0),
    dict(t1_encoder=1, t1_decoder=1, spiht=0),
    dict(t1_encoder=2, t1_decoder=2, spiht=0),
    dict(t1_encoder=0, t1_decoder=0, spiht=1),
)

_CACHE = {}


def _signature(xs, eps, base_ratio, bound_mode, levels):
    shapes = {}
    for x in xs:
        shapes[tuple(x.shape)] = shapes.get(tuple(x.shape), 0) + 1
    dev = torch.cuda.get_device_name(xs[0].device) if xs else ""
    e = sorted(round(float(v), 6) for v in eps)
    return json.dumps([dev, sorted((list(k), v) for k, v in shapes.items()), e[:: max(1, len(e) // 16)],
                       base_ratio, bound_mode, levels])


def sample_fields(xs, eps, k):
    """Up to k fields, taken round-robin over the distinct shapes so that the
    sample keeps the batch's mix of sizes."""
    if k is None or k >= len(xs):
        return list(xs), list(eps)
    groups = {}
    for x, e in zip(xs, eps):
        groups.setdefault(tuple(x.shape), []).append((x, e))
    out = []
    while len(out) < k:
        for g in groups.values():
            if g and len(out) < k:
                out.append(g.pop(0))
    return [x for x, _ in out], [e for _, e in out]


def measure(xs, eps, p, stream=None, reps=1):
    """(seconds per batched round trip, compression ratio) for params p."""
    args = ebcc.BatchArgs(xs, err_bounds=eps)
    out = torch.empty(args.bound(), dtype=torch.uint8, device=xs[0].device)
    if ebcc.compress_batch_into(args, out, p, stream) != 0:
        raise ebcc.EbccError(-1, ebcc.lib().ebcc_last_error().decode())
    streams = [out[args.offsets[i]: args.offsets[i] + args.lengths[i]] for i in range(args.n)]
    recs = [torch.empty(tuple(x.shape), dtype=torch.float32, device=x.device) for x in xs]
    dargs = ebcc.DecodeArgs(streams, recs)
    if ebcc.decompress_batch_into(dargs, stream) != 0:
        raise ebcc.EbccError(-1, ebcc.lib().ebcc_last_error().decode())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ebcc.compress_batch_into(args, out, p, stream)
        ebcc.decompress_batch_into(dargs, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    nbytes = sum(x.numel() * 4 for x in xs)
    sbytes = sum(args.lengths[i] for i in range(args.n))
    return dt, nbytes / sbytes


def tune(xs, err_bounds, base_ratio=30.0, bound_mode=ebcc.BOUND_REL, levels=5, sample=None, cr_tol=0.01,
         formats=FORMATS, kernels=KERNELS, stream=None, cache_file=None, log=None):
    """Measure the candidates on the fields `xs` (device tensors) with
    per-field bounds `err_bounds`; return a dict with `params` (keyword
    arguments of ebcc.params), `tuning` (of ebcc.set_tuning) and the measured
    `table`.  Leaves the library's tuning as it found it."""
    key = _signature(xs, err_bounds, base_ratio, bound_mode, levels)
    if key in _CACHE:
        return _CACHE[key]
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as f:
            disk = json.load(f)
        if key in disk:
            _CACHE[key] = disk[key]
            return disk[key]
    sx, se = sample_fields(xs, err_bounds, sample)
    nbytes = sum(x.numel() * 4 for x in sx)
    saved = ebcc.get_tuning()
    table = []

    def run(fmt, kern):
        ebcc.set_tuning(**{**saved, **kern})
        p = ebcc.params(1.0, base_ratio, bound_mode=bound_mode, levels=levels, cblk_log2w=fmt[0],
                        cblk_log2h=fmt[1], spiht_tile=fmt[2])
        dt, cr = measure(sx, se, p, stream)
        row = {"cblk_log2w": fmt[0], "cblk_log2h": fmt[1], "spiht_tile": fmt[2], **kern,
               "ms": dt * 1e3, "GBps": nbytes / dt / 1e9, "CR": cr}
        table.append(row)
        if log:
            log(f"autotune: {row}")
        return row

    try:
        # kernel choices at the default format, then the formats with the best kernels
        rows = [run(formats[0], k) for k in kernels]
        best_k = {k: rows[min(range(len(rows)), key=lambda i: rows[i]["ms"])][k] for k in kernels[0]}
        cr_ref = rows[0]["CR"]
        frows = [rows[min(range(len(rows)), key=lambda i: rows[i]["ms"])]]
        frows += [run(f, best_k) for f in formats[1:]]
        ok = [r for r in frows if r["CR"] >= (1.0 - cr_tol) * cr_ref]
        best = min(ok, key=lambda r: r["ms"])
        # the kernel choice again at the chosen format
        if (best["cblk_log2w"], best["cblk_log2h"], best["spiht_tile"]) != tuple(formats[0]):
            fmt = (best["cblk_log2w"], best["cblk_log2h"], best["spiht_tile"])
            krows = [run(fmt, k) for k in kernels if any(k[q] != best_k[q] for q in k)]
            best = min([best] + krows, key=lambda r: r["ms"])
    finally:
        ebcc.set_tuning(**saved)
    res = {"params": {"cblk_log2w": best["cblk_log2w"], "cblk_log2h": best["cblk_log2h"],
                      "spiht_tile": best["spiht_tile"]},
           "tuning": {k: best[k] for k in kernels[0]},
           "GBps": best["GBps"], "CR": best["CR"], "CR_default": cr_ref, "table": table,
           "fields_measured": len(sx)}
    _CACHE[key] = res
    if cache_file:
        disk = {}
        if os.path.exists(cache_file):
            with open(cache_file) as f:
                disk = json.load(f)
        disk[key] = res
        with open(cache_file, "w") as f:
            json.dump(disk, f)
    return res
