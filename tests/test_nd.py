"""N-D chunking and flattening (Method section): chunk grids cover the array
exactly once, (T, P, H, W) chunks flatten to (T*P*H, W), and the container
header round-trips.  The GPU round trip is in test_gpu_batch.py."""
import itertools

import numpy as np
import pytest
import torch

from paper_2510_22265_amd import nd


@pytest.mark.parametrize("shape,chunk", [((4, 3, 10, 17), (2, 3, 5, 17)), ((5, 7), (2, 3)), ((9,), (4,)),
                                         ((3, 2, 6, 8), (3, 2, 6, 8)), ((2, 5, 4, 7), (1, 2, 3, 4))])
def test_chunk_grid_covers_once(shape, chunk):
    hits = np.zeros(shape, np.int32)
    for origin, ext in nd.chunk_grid(shape, chunk):
        assert all(1 <= e <= c for e, c in zip(ext, chunk))
        hits[tuple(slice(o, o + e) for o, e in zip(origin, ext))] += 1
    assert (hits == 1).all()


def test_flatten_is_the_papers():
    assert nd.flat_shape((2, 3, 5, 7)) == (30, 7)
    assert nd.flat_shape((5, 7)) == (5, 7)
    assert nd.flat_shape((9,)) == (1, 9)
    x = torch.arange(2 * 3 * 5 * 7, dtype=torch.float32).reshape(2, 3, 5, 7)
    parts = [v.reshape(nd.flat_shape(tuple(v.shape))) for v in [x]]
    assert torch.equal(parts[0][7], x[0, 1, 2])        # row t*P*H + p*H + h


def test_chunks_reassemble():
    x = torch.randn(3, 4, 9, 11)
    chunk = (2, 3, 4, 5)
    grid = nd.chunk_grid(tuple(x.shape), chunk)
    parts = []
    for origin, ext in grid:
        parts.append(x[tuple(slice(o, o + e) for o, e in zip(origin, ext))].contiguous().reshape(nd.flat_shape(ext)))
    y = torch.empty_like(x)
    for (origin, ext), p in zip(grid, parts):
        y[tuple(slice(o, o + e) for o, e in zip(origin, ext))] = p.reshape(ext)
    assert torch.equal(x, y)


def test_container_header():
    import struct
    shape, chunk = (4, 3, 10, 17), (2, 3, 5, 17)
    head = nd.MAGIC + struct.pack("<I", 4) + struct.pack("<4Q", *shape) + struct.pack("<4Q", *chunk)
    head += struct.pack("<I", 2) + struct.pack("<QQ", 0, 5) + struct.pack("<QQ", 5, 3)
    s, c, table, start = nd.parse_nd(head + b"abcdefgh")
    assert (s, c, table, start) == (shape, chunk, [(0, 5), (5, 3)], len(head))
    with pytest.raises(ValueError):
        nd.parse_nd(b"XXXX" + head[4:])
