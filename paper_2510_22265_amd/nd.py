"""N-D arrays: chunking and flattening to 2-D fields (Method section).

The paper splits a four-dimensional array (time, level, latitude,
longitude) into chunks of one shape, flattens each chunk (T, P, H, W) into
(T*P*H, W) and compresses every chunk on its own (its own minimum, maximum
and range-relative bound).  Here the chunks of an array are one batched
call: every chunk is a field of ebcc_compress_batch.

Container (host bytes, little-endian): "EBCN", u32 ndim, u64 shape[ndim],
u64 chunk[ndim], u32 n_chunks, then per chunk u64 offset and u64 length of
its stream in the payload, then the payload (the streams back to back).
Edge chunks are smaller when a dimension is not a multiple of the chunk.
"""
import itertools
import struct

import torch

from . import ebcc

MAGIC = b"EBCN"


def chunk_grid(shape, chunk):
    """Chunk origins and extents covering `shape` in row-major chunk order."""
    if len(chunk) != len(shape) or any(c < 1 for c in chunk):
        raise ValueError("chunk must have one positive extent per dimension")
    ranges = [range(0, n, c) for n, c in zip(shape, chunk)]
    out = []
    for origin in itertools.product(*ranges):
        ext = tuple(min(c, n - o) for o, c, n in zip(origin, chunk, shape))
        out.append((origin, ext))
    return out


def flat_shape(ext):
    """(T, P, H, W) -> (T * P * H, W); a 1-D chunk is one row."""
    if len(ext) == 1:
        return (1, ext[0])
    rows = 1
    for e in ext[:-1]:
        rows *= e
    return (rows, ext[-1])


def chunks_2d(x, chunk):
    """Contiguous 2-D float32 copies of the chunks of `x` (device tensor)."""
    out = []
    for origin, ext in chunk_grid(tuple(x.shape), chunk):
        v = x[tuple(slice(o, o + e) for o, e in zip(origin, ext))]
        out.append(v.contiguous().reshape(flat_shape(ext)))
    return out


def compress_nd(x, chunk, err_bound=0.01, base_ratio=30.0, stream=None, **kw):
    """Compress an N-D float32 device tensor chunk by chunk; returns the
    container as bytes (the chunks' streams are copied to the host)."""
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() >= 1):
        raise TypeError("expected a float32 tensor on the GPU")
    parts = chunks_2d(x, tuple(chunk))
    streams = ebcc.compress_batch(parts, err_bound=err_bound, base_ratio=base_ratio, stream=stream, **kw)
    head = MAGIC + struct.pack("<I", x.dim()) + struct.pack(f"<{x.dim()}Q", *x.shape)
    head += struct.pack(f"<{x.dim()}Q", *chunk) + struct.pack("<I", len(streams))
    payload = [s.cpu().numpy().tobytes() for s in streams]
    off = 0
    for p in payload:
        head += struct.pack("<QQ", off, len(p))
        off += len(p)
    return head + b"".join(payload)


def parse_nd(blob):
    """(shape, chunk, [(offset, length)], payload start) of a container."""
    if blob[:4] != MAGIC:
        raise ValueError("not an EBCN container")
    (nd,) = struct.unpack_from("<I", blob, 4)
    shape = struct.unpack_from(f"<{nd}Q", blob, 8)
    chunk = struct.unpack_from(f"<{nd}Q", blob, 8 + 8 * nd)
    (n,) = struct.unpack_from("<I", blob, 8 + 16 * nd)
    pos = 12 + 16 * nd
    table = [struct.unpack_from("<QQ", blob, pos + 16 * i) for i in range(n)]
    return tuple(shape), tuple(chunk), table, pos + 16 * n


def decompress_nd(blob, device="cuda", stream=None):
    """Decompress a container into an N-D float32 device tensor."""
    shape, chunk, table, start = parse_nd(blob)
    grid = chunk_grid(shape, chunk)
    if len(grid) != len(table):
        raise ValueError("chunk table does not match the shape")
    streams = [torch.frombuffer(bytearray(blob[start + o: start + o + n]), dtype=torch.uint8).to(device)
               for o, n in table]
    fields = ebcc.decompress_batch(streams, [flat_shape(ext) for _, ext in grid], stream=stream)
    out = torch.empty(shape, dtype=torch.float32, device=device)
    for (origin, ext), f in zip(grid, fields):
        out[tuple(slice(o, o + e) for o, e in zip(origin, ext))] = f.reshape(ext)
    return out
