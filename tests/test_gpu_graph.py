"""HIP-graph capture of whole calls: every replay (with eager work and
synchronisations in between) must reproduce the eager result bit for bit --
the kernels are deterministic and clear their own counters with kernels, not
memset nodes."""
import numpy as np
import pytest

from paper_1401_7962_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gj():
    import torch  # noqa: F401
    import paper_1401_7962_amd as m
    m.load_library()
    return m


def _capture(fn):
    import torch
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn(s)
    torch.cuda.synchronize()
    return g


GRAPH_BATCHES = {
    "mixed": [5, 17, 40, 64, 70, 128, 140, 260],
    # streaming members in several chunk groups: the groups split over two streams
    "groups": [9, 40, 130, 200, 257, 333, 420, 512],
}


@pytest.mark.parametrize("batch", sorted(GRAPH_BATCHES))
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_graph_replays(gj, precision, batch):
    import torch
    sizes = np.array(GRAPH_BATCHES[batch], dtype=np.int32)
    rng = inputs.rng_for(0, 7500)
    mats = [inputs.conditioned(int(n), 1e3, rng) for n in sizes]
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    A = torch.from_numpy(np.concatenate([m.ravel() for m in mats])).cuda()
    opts = gj.make_opts(precision=precision)
    X, ip, jp, res, poff = gj.gj_invert_batched(sizes, offs, A, opts=opts)   # eager; uploads the plan
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, len(sizes), sizes, opts),
                     dtype=torch.uint8, device="cuda")
    gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, opts, ws)
    torch.cuda.synchronize()
    want = (X.cpu().numpy().copy(), ip.cpu().numpy().copy(), res.cpu().numpy().copy())
    reuse = gj.make_opts(precision=precision, flags=gj.GJ_FLAG_REUSE_PLAN)
    g = _capture(lambda s: gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, reuse, ws, s))
    for rep in range(4):
        X.zero_()
        res.zero_()
        _ = torch.ones(1000, device="cuda").sum()     # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert X.cpu().numpy().tobytes() == want[0].tobytes(), rep
        assert np.array_equal(ip.cpu().numpy(), want[1]), rep
        assert res.cpu().numpy().tobytes() == want[2].tobytes(), rep


@pytest.mark.parametrize("n,precision", [(64, 0), (300, 0), (300, 1)])
def test_single_graph_replays(gj, n, precision):
    import torch
    A = torch.from_numpy(inputs.conditioned(n, 1e3, inputs.rng_for(0, 7600 + n))).cuda()
    opts = gj.make_opts(precision=precision)
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, opts), dtype=torch.uint8,
                     device="cuda")
    X, ip, jp, res = gj.gj_invert(A, opts=opts, ws=ws)
    torch.cuda.synchronize()
    want = X.cpu().numpy().copy()
    g = _capture(lambda s: gj.gj_invert(A, X, ip, jp, res, opts, ws, s))
    for rep in range(3):
        X.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert X.cpu().numpy().tobytes() == want.tobytes(), rep
