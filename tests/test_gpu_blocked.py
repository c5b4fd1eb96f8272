"""GPU parity for the blocked elimination (GJ_FLAG_BLOCKED, delayed updates).

Each step eliminates on the trailing block only, and the block's values are
the unblocked elimination's, operation for operation; so the pivot sequence,
rank, result code and determinant (sign, mantissa, exponent) must equal the
FP64 oracle's bit for bit.  The other rows and columns receive the panel's
eqs. 14-15 as matrix-core products, which sum in another order: the inverse
is compared by its forward error against the long-double oracle, which may be
at most 4x the FP64 oracle's own plus 1e-15 (relative Frobenius; the same bar
as the refined path's, R-16), up to order 520 (the long-double oracle's time);
at every order its residual ||A X - I||_F / (||A||_F ||X||_F) may be at most
4x the FP64 oracle's own plus 1e-16, and X within 1e-12 of the oracle's (the
inputs have cond <= 1e4).  With
a single panel nothing is delayed and X must be the oracle's bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1401_7962_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gj():
    import torch  # noqa: F401
    import paper_1401_7962_amd as m
    m.load_library()
    return m


def _blocked(gj, A, flags=None):
    import torch
    opts = gj.make_opts(flags=gj.GJ_FLAG_BLOCKED if flags is None else flags)
    Ad = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to("cuda")
    X, ipiv, jpiv, res = gj.gj_invert(Ad, opts=opts)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy(), gj.results_to_dicts(res)[0]


def _rel(Y, Z):
    return float(np.linalg.norm(Y - Z) / np.linalg.norm(Z))


def _resid(A, X):
    R = A @ X
    R[np.diag_indices_from(R)] -= 1.0
    return float(np.linalg.norm(R) / (np.linalg.norm(A) * np.linalg.norm(X)))


def _accurate(A, X, Xo, where):
    """X from the blocked elimination against the FP64 oracle's Xo: the inputs
    here have cond <= 1e4, for which the bar is 1e-12 relative Frobenius."""
    assert np.linalg.cond(A) <= 1e4, where
    assert _resid(A, X) <= 4 * _resid(A, Xo) + 1e-16, where
    assert _rel(X, Xo) <= 1e-12, where
    if A.shape[0] <= 520:
        Xt, _, _, _ = oracle.gj_invert_f80(A)
        err, err_o = _rel(X, Xt), _rel(Xo, Xt)
        assert err <= 4 * err_o + 1e-15, (where, err, err_o)


def _same_pivots(got, want, where):
    _, ipiv, jpiv, r = got
    _, io, jo, ro = want
    assert r["code"] == ro["code"] and r["rank"] == ro["rank"], (where, r, ro)
    assert np.array_equal(ipiv, io) and np.array_equal(jpiv, jo), where
    if ro["code"] == 0:
        assert r["det_sign"] == ro["det_sign"], where
        assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"], where


@pytest.mark.parametrize("n,nb", [(150, 32), (300, 64), (300, 128), (517, 128), (777, 96),
                                  (1000, 128), (640, 2)])
def test_blocked_matches_oracle(gj, n, nb, monkeypatch):
    """Several panels, a ragged last panel, panel widths from 2 to 128."""
    monkeypatch.setenv("GJ_BLK_NB", str(nb))
    A = inputs.rng_for(0, 7000 + n + nb).standard_normal((n, n))
    got = _blocked(gj, A)
    want = oracle.gj_invert_f64(A)
    _same_pivots(got, want, f"n={n} nb={nb}")
    _accurate(A, got[0], want[0], f"n={n} nb={nb}")


@pytest.mark.parametrize("n,nb", [(200, 256), (300, 300), (129, 128)])
def test_blocked_one_panel_is_bitwise(gj, n, nb, monkeypatch):
    """With one panel nothing is delayed: the copy into pivot order, the
    deferred division and the gather must reproduce the oracle's X bit for
    bit.  129 with 128-step panels leaves a second panel of one step (checked
    for pivots and accuracy)."""
    monkeypatch.setenv("GJ_BLK_NB", str(nb))
    A = inputs.rng_for(0, 7100 + n).standard_normal((n, n))
    got = _blocked(gj, A)
    want = oracle.gj_invert_f64(A)
    _same_pivots(got, want, f"n={n} nb={nb}")
    if nb >= n:
        assert got[0].tobytes() == want[0].tobytes()
    else:
        _accurate(A, got[0], want[0], f"n={n} nb={nb}")


def test_blocked_small_order_on_chip(gj):
    """Orders up to 128 ignore the flag (the on-chip kernel): bit for bit."""
    A = inputs.rng_for(0, 7200).standard_normal((100, 100))
    got = _blocked(gj, A)
    want = oracle.gj_invert_f64(A)
    _same_pivots(got, want, "n=100")
    assert got[0].tobytes() == want[0].tobytes()


@pytest.mark.parametrize("n,rank,nb", [(300, 200, 64), (300, 40, 64), (260, 128, 128)])
def test_blocked_singular(gj, n, rank, nb, monkeypatch):
    """Rank-deficient input: the elimination stops in the panel where the
    oracle stops (a later panel, the first one, or exactly at a panel
    boundary), with the same rank, code and pivots; X is NaN."""
    monkeypatch.setenv("GJ_BLK_NB", str(nb))
    rng = inputs.rng_for(0, 7300 + n + rank)
    A = rng.standard_normal((n, rank)) @ rng.standard_normal((rank, n))
    got = _blocked(gj, A)
    want = oracle.gj_invert_f64(A)
    _same_pivots(got, want, f"n={n} rank={rank}")
    assert want[3]["code"] != 0
    assert np.isnan(got[0]).all()


def test_blocked_nonfinite(gj):
    A = inputs.rng_for(0, 7400).standard_normal((200, 200))
    A[5, 7] = np.inf
    got = _blocked(gj, A)
    want = oracle.gj_invert_f64(A)
    _same_pivots(got, want, "inf")
    assert np.isnan(got[0]).all()


@pytest.mark.parametrize("n,nb", [(256, 64), (512, 128)])
def test_blocked_hadamard_ties(gj, n, nb, monkeypatch):
    """Every candidate ties at every step: the tie-break on logical positions
    must survive the copies into pivot order.  H^-1 = H^T / n exactly."""
    monkeypatch.setenv("GJ_BLK_NB", str(nb))
    H = inputs.sylvester_hadamard(n)
    got = _blocked(gj, H)
    want = oracle.gj_invert_f64(H)
    _same_pivots(got, want, f"H{n}")
    assert _rel(got[0], H.T / n) <= 1e-15


def test_blocked_headline_size(gj):
    """4096^2 headline input, default panel width: the same pivots and
    determinant as the unblocked elimination (itself the oracle's bit for bit
    at smaller orders), X within 1e-13 of it, and sampled rows of X A - I."""
    n = 4096
    A = inputs.single_dominant(n)
    Xb, ib, jb, rb = _blocked(gj, A)
    Xu, iu, ju, ru = _blocked(gj, A, flags=0)
    assert rb["code"] == ru["code"] == 0
    assert np.array_equal(ib, iu) and np.array_equal(jb, ju)
    assert (rb["det_sign"], rb["det_mant"], rb["det_exp"]) == (ru["det_sign"], ru["det_mant"], ru["det_exp"])
    assert _rel(Xb, Xu) <= 1e-13
    rows = inputs.rng_for(0, 7500).choice(n, size=16, replace=False)
    R = Xb[rows] @ A
    R[np.arange(16), rows] -= 1.0
    assert np.abs(R).max() <= 1e-12


def test_blocked_with_residual(gj):
    """want_resid with delayed updates: the residual's workspace follows the
    blocked layout, and the reported ||A X - I||_F / (||A||_F ||X||_F) is the
    returned X's."""
    import torch
    n = 300
    A = inputs.conditioned(n, 1e3, inputs.rng_for(0, 7600))
    opts = gj.make_opts(flags=gj.GJ_FLAG_BLOCKED, want_resid=True)
    X, _, _, res = gj.gj_invert(torch.from_numpy(A).to("cuda"), opts=opts)
    torch.cuda.synchronize()
    r = gj.results_to_dicts(res)[0]
    assert r["code"] == 0
    want = oracle.residual(A, X.cpu().numpy())
    assert abs(r["resid"] - want) <= 1e-2 * want + 1e-18
