"""Caller buffers that are too short, on the wrong device or of the wrong
type are refused before anything is launched (GJError), and a batched plan
reused with other buffers than the upload it reuses is refused by the
library; reused with the same buffers it gives the eager call's results bit
for bit."""
import sys

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


def test_single_matrix_buffers_refused(gj):
    import torch
    n = 300
    A = torch.from_numpy(inputs.single_normal(n, offset=40)).to("cuda")
    dev = A.device
    cases = {
        "X short": dict(X=torch.empty((n - 1, n), dtype=torch.float64, device=dev)),
        "X float32": dict(X=torch.empty((n, n), dtype=torch.float32, device=dev)),
        "X on host": dict(X=torch.empty((n, n), dtype=torch.float64)),
        "ipiv short": dict(ipiv=torch.empty(n - 1, dtype=torch.int32, device=dev)),
        "jpiv int64": dict(jpiv=torch.empty(n, dtype=torch.int64, device=dev)),
        "res short": dict(res=torch.empty(gj.RESULT_BYTES - 1, dtype=torch.uint8, device=dev)),
        "ws short": dict(ws=torch.empty(1024, dtype=torch.uint8, device=dev)),
    }
    for name, kw in cases.items():
        with pytest.raises(gj.GJError):
            gj.gj_invert(A, **kw)
        print(f"refused: {name}", file=sys.stderr, flush=True)
    with pytest.raises(gj.GJError):
        gj.gj_det(A, ipiv=torch.empty(2, dtype=torch.int32, device=dev))
    B = torch.ones((n, 3), dtype=torch.float64, device=dev)
    with pytest.raises(gj.GJError):
        gj.gj_solve(A, B, X=torch.empty((n, 2), dtype=torch.float64, device=dev))


def _batch(gj, sizes, seed):
    import torch
    sizes = np.asarray(sizes, dtype=np.int32)
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    packed = np.concatenate([inputs.rng_for(0, seed + b).standard_normal(int(n) * int(n))
                             for b, n in enumerate(sizes)])
    return sizes, offs, torch.from_numpy(packed).to("cuda")


def test_batched_buffers_refused(gj):
    import torch
    sizes, offs, A = _batch(gj, [30, 200, 70], 4100)
    dev = A.device
    span = int(offs[-1] + sizes[-1] ** 2)
    cases = {
        "A short": dict(A=A[: span - 1]),
        "X short": dict(X=torch.empty(span - 1, dtype=torch.float64, device=dev)),
        "ipiv short": dict(ipiv=torch.empty(int(sizes.sum()) - 1, dtype=torch.int32, device=dev)),
        "res short": dict(res=torch.empty(3 * gj.RESULT_BYTES - 8, dtype=torch.uint8, device=dev)),
        "ws short": dict(ws=torch.empty(4096, dtype=torch.uint8, device=dev)),
    }
    for name, kw in cases.items():
        args = dict(A=A)
        args.update(kw)
        with pytest.raises(gj.GJError):
            gj.gj_invert_batched(sizes, offs, args.pop("A"), **args)
        print(f"refused: batched {name}", file=sys.stderr, flush=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_reuse_plan_requires_same_buffers(gj, precision):
    import torch
    sizes, offs, A = _batch(gj, [40, 150, 128, 9, 300], 4200)
    opts = gj.make_opts(precision=precision)
    reuse = gj.make_opts(precision=precision, flags=gj.GJ_FLAG_REUSE_PLAN)
    print(f"reuse plan, precision {precision}", file=sys.stderr, flush=True)
    X, ip, jp, res, poff = gj.gj_invert_batched(sizes, offs, A, opts=opts)
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, len(sizes), sizes, opts),
                     dtype=torch.uint8, device="cuda")
    X1 = torch.empty_like(A)
    gj.gj_invert_batched(sizes, offs, A, X1, poff, ip, jp, res, opts, ws)     # uploads
    torch.cuda.synchronize()
    X2 = torch.full_like(A, 7.0)
    with pytest.raises(gj.GJError):                                            # other X
        gj.gj_invert_batched(sizes, offs, A, X2, poff, ip, jp, res, reuse, ws)
    torch.cuda.synchronize()
    assert bool((X2 == 7.0).all())                                             # nothing ran
    X1.fill_(0.0)
    gj.gj_invert_batched(sizes, offs, A, X1, poff, ip, jp, res, reuse, ws)    # same buffers
    torch.cuda.synchronize()
    assert X1.cpu().numpy().tobytes() == X.cpu().numpy().tobytes()
