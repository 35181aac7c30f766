"""Launch sequences from cached HIP graphs: calls of one shape replay the
graph recorded by an earlier one (the second), with the program's own eager work and
synchronisations between the replays.  Every replay's stream must be the
oracle's, byte for byte, and every decode the oracle's, bit for bit; the
same calls with graphs switched off (EBCC_GRAPHS=0) give the same bytes."""
import numpy as np
import pytest

from paper_2510_22265_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_22265_amd import ebcc
    ebcc.lib()
    return ebcc


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _eager_work():
    import torch
    a = torch.randn(1 << 20, device="cuda")
    b = (a * 2.0 + 1.0).sum()
    torch.cuda.synchronize()
    return float(b)


@pytest.mark.parametrize("kw", [dict(), dict(trunc=1), dict(q=1 - 1e-5)])
def test_single_field_replays(gpu, ref, kw, monkeypatch):
    import torch
    stream = torch.cuda.Stream()          # a stream of its own (its workspace records the graphs)
    for graphs in ("1", "0"):
        monkeypatch.setenv("EBCC_GRAPHS", graphs)
        for rep in range(4):
            x = synth.field(["u", "v", "t", "q"][rep], 181, 360, cfg=8, level=rep)
            print(f"graphs {graphs} rep {rep} {kw}", flush=True)
            with torch.cuda.stream(stream):
                s = gpu.compress(_dev(x), 0.01, **kw)
                y = gpu.decompress(s, *x.shape)
            stream.synchronize()
            s_ref = ref.compress(x, 0.01, **kw)
            assert s.cpu().numpy().tobytes() == s_ref, f"replay {rep}: stream differs from the oracle's"
            assert np.array_equal(y.cpu().numpy().view(np.uint32), ref.decompress(s_ref, *x.shape).view(np.uint32))
            _eager_work()


def test_batch_replays(gpu, ref, monkeypatch):
    import torch
    shapes = [(91, 180), (181, 360), (64, 96), (181, 360)]
    for graphs in ("1", "0"):
        monkeypatch.setenv("EBCC_GRAPHS", graphs)
        for rep in range(3):
            xs = [synth.field(["t", "u", "v", "q"][k], *sh, cfg=9, level=rep) for k, sh in enumerate(shapes)]
            eps = [0.01, 0.003, 0.02, 0.01]
            print(f"batch graphs {graphs} rep {rep}", flush=True)
            streams = gpu.compress_batch([_dev(x) for x in xs], err_bounds=eps)
            ys = gpu.decompress_batch(streams, shapes)
            torch.cuda.synchronize()
            for i, (x, e) in enumerate(zip(xs, eps)):
                s_ref = ref.compress(x, e)
                assert streams[i].cpu().numpy().tobytes() == s_ref, f"rep {rep} field {i}"
                assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                                      ref.decompress(s_ref, *x.shape).view(np.uint32))
            _eager_work()
