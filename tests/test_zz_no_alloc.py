"""gj_invert_noalloc (the entry point that allocates nothing: its kernels
use the library's built-in scratch array) against gj_invert with a caller
workspace: bit for bit on X, the pivots and the determinant record, on two
calls in a row, the second with a smaller input (the array keeps the first
call's contents), plus an on-chip order, the refined precision and the
size limit."""
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


def _both(gj, A_h, opts=None):
    import torch
    A = torch.from_numpy(A_h).to("cuda")
    print(f"noalloc vs workspace: n={A_h.shape[0]}", file=sys.stderr, flush=True)
    ref = gj.gj_invert(A, opts=opts)
    got = gj.gj_invert_noalloc(A, opts=opts)
    torch.cuda.synchronize()
    return ref, got


def _assert_same(gj, ref, got):
    Xr, ir, jr, rr = ref
    Xg, ig, jg, rg = got
    assert Xg.cpu().numpy().tobytes() == Xr.cpu().numpy().tobytes()
    assert np.array_equal(ig.cpu().numpy(), ir.cpu().numpy())
    assert np.array_equal(jg.cpu().numpy(), jr.cpu().numpy())
    dr, dg = gj.results_to_dicts(rr)[0], gj.results_to_dicts(rg)[0]
    for key in ("code", "rank", "det_sign", "det_mant", "det_exp", "refine_iters"):
        assert dg[key] == dr[key], key


def test_noalloc_two_calls_second_smaller(gj):
    first = _both(gj, inputs.single_dominant(1500, offset=31))
    second = _both(gj, inputs.single_normal(700, offset=32))
    _assert_same(gj, *first)
    _assert_same(gj, *second)
    assert gj.results_to_dicts(second[1][3])[0]["code"] == 0


def test_noalloc_onchip_refined_and_singular(gj):
    _assert_same(gj, *_both(gj, inputs.single_normal(100, offset=33)))
    A = inputs.conditioned(900, 1e6, inputs.rng_for(0, 34))
    _assert_same(gj, *_both(gj, A, gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)))
    H = inputs.sylvester_hadamard(256)
    H[:, 255] = H[:, 0] + H[:, 1]
    ref, got = _both(gj, H)
    _assert_same(gj, ref, got)
    assert gj.results_to_dicts(got[3])[0]["code"] == gj.GJ_RES_SINGULAR


def test_noalloc_size_limit(gj):
    import torch
    A = torch.empty((4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(gj.GJError):
        gj.gj_invert_noalloc(A)
