"""CPU model of the persistent lanes-per-block tier-1 launch, with bounds
assertions, checked before the kernel runs on a GPU.

It restates the index arithmetic of `order_by_key` (`k_t1_order`,
`k_t1_order_dec`: block order by a key of 24 values, bit-planes coded or
decoded, largest first: per-thread counts over contiguous shares, a scan
over (key, thread), a scatter) and of the work loop of `k_t1_encode` and
`k_t1_decode` (each workgroup
takes group g = counter++ and its lanes the entries g * LANES + lane of the
order, until g reaches the number of groups), and checks for every case:
every index stays inside its array, the order is a permutation sorted by
P_b (largest first, stable), every block is coded exactly once whatever the
interleaving of the workgroups, and every workgroup leaves the loop."""
import numpy as np
import pytest

KQBITS = 23
THREADS = 1024


def model_order(pb):
    nblk = len(pb)
    per = (nblk + THREADS - 1) // THREADS
    cnt = np.zeros((KQBITS + 1, THREADS), np.int64)
    key = lambda b: KQBITS - min(int(pb[b]), KQBITS)
    for t in range(THREADS):
        b0 = min(t * per, nblk)
        b1 = min(b0 + per, nblk)
        assert 0 <= b0 <= b1 <= nblk
        for b in range(b0, b1):
            k = key(b)
            assert 0 <= k <= KQBITS
            cnt[k][t] += 1
    base = np.zeros(KQBITS + 1, np.int64)
    for t in range(KQBITS + 1):          # threads 0..23 scan one row each
        s = 0
        for u in range(THREADS):
            v = cnt[t][u]
            cnt[t][u] = s
            s += v
        base[t] = s
    s = 0
    for k in range(KQBITS + 1):          # thread 0
        v = base[k]
        base[k] = s
        s += v
    assert s == nblk
    order = np.full(nblk, -1, np.int64)
    for t in range(THREADS):
        b0 = min(t * per, nblk)
        b1 = min(b0 + per, nblk)
        for b in range(b0, b1):
            k = key(b)
            i = base[k] + cnt[k][t]
            assert 0 <= i < nblk and order[i] == -1
            order[i] = b
            cnt[k][t] += 1
    return order


def model_queue(order, lanes, grid, rng):
    nblk = len(order)
    ngroups = (nblk + lanes - 1) // lanes
    counter = 0
    done = np.zeros(nblk, np.int64)
    live = list(range(grid))
    steps = 0
    while live:
        w = live[int(rng.integers(len(live)))]      # any workgroup may take the next group
        g = counter
        counter += 1
        if g >= ngroups:
            live.remove(w)
            continue
        for lane in range(lanes):
            i = g * lanes + lane
            if i < nblk:
                assert 0 <= i < len(order)
                b = order[i]
                assert 0 <= b < nblk
                done[b] += 1
        steps += 1
        assert steps <= ngroups + grid
    assert counter == ngroups + grid
    return done


@pytest.mark.parametrize("nblk", [1, 15, 16, 17, 255, 256, 257, 1000, 4097, 20011])
@pytest.mark.parametrize("lanes", [1, 4, 16, 64])
def test_persistent_dispatch_model(nblk, lanes):
    if lanes == 1 and nblk > 5000:
        pytest.skip("covered by the smaller cases (one block per group)")
    rng = np.random.default_rng(nblk * 131 + lanes)
    pb = rng.integers(0, KQBITS + 1, nblk).astype(np.uint8)
    if nblk > 100:
        pb[: nblk // 3] = 0                      # empty blocks, as in smooth bands
    order = model_order(pb)
    assert sorted(order.tolist()) == list(range(nblk))
    keys = [int(pb[b]) for b in order]
    assert keys == sorted(keys, reverse=True)
    for p in set(keys):                          # stable within a P_b
        idx = [b for b in order if pb[b] == p]
        assert idx == sorted(idx)
    ngroups = (nblk + lanes - 1) // lanes
    for grid in sorted({1, 2, min(ngroups, 7), ngroups, ngroups + 5}):
        done = model_queue(order, lanes, grid, rng)
        assert (done == 1).all()


def test_lds_of_persistent_launch_is_the_plain_launch():
    """The persistent kernel is the plain lanes-per-block kernel with a loop
    around the per-lane body: it declares the same shared block (no
    per-wavefront slices), sized per lane, and its launches use the same
    workgroup size LANES <= 64 (one wavefront, so the group index is shared
    with a shuffle, no barrier inside the loop)."""
    import os
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2510_22265_amd", "csrc", "t1.hip")).read()
    for name, fn in (("k_t1_encode", "t1_enc_block"), ("k_t1_decode", "t1_dec_block")):
        kern = src[src.index(f"__global__ __launch_bounds__(LANES) void {name}("):]
        kern = kern[: kern.index("\n}\n")]
        assert kern.count("__shared__") == 1 and re.search(r"T1Shared<M, ROWS, LANES, (true|false)> S;", kern)
        loop = kern[kern.index("for (;;)"):]
        assert "__syncthreads" not in loop
        assert re.search(r"g = __shfl\(g, 0\)", loop)
        body = src[src.index(f"__device__ __forceinline__ void {fn}("):]
        body = body[: body.index("\n}\n")]
        assert "__syncthreads" not in body
