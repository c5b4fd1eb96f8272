"""GPU parity for gj_solve (A X = B through the elimination of [A | B]): the
HIP path against the FP64 oracle's augmented elimination with D^0 = B, bit
for bit (the same division and fma per element), plus, at the benchmark's
order, the property that right-hand sides taken from the identity reproduce
the corresponding columns of gj_invert's inverse bit for bit."""
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


def _dev(M):
    import torch
    return torch.from_numpy(np.ascontiguousarray(M, dtype=np.float64)).to("cuda")


def _solve(gj, A, B, **kw):
    import torch
    opts = gj.make_opts(**kw) if kw else None
    X, ipiv, jpiv, res = gj.gj_solve(_dev(A), _dev(B), opts=opts)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy(), gj.results_to_dicts(res)[0]


def _assert_same(got, want, where):
    X, ipiv, jpiv, r = got
    Xo, io, jo, ro = want
    assert r["code"] == ro["code"] and r["rank"] == ro["rank"], where
    assert np.array_equal(ipiv, io) and np.array_equal(jpiv, jo), where
    if ro["code"] == 0:
        assert X.tobytes() == Xo.tobytes(), (where, np.nanmax(np.abs(X - Xo)))
        assert r["det_sign"] == ro["det_sign"], where
        assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"], where
    else:
        assert np.isnan(X).all(), where
        assert r["det_sign"] == 0, where


# (1000, 3), (1000, 24), (2000, 128): A fills all register chunks, B is the
# extra partial chunk (odd m, and m at the chunk's width); (1000, 200): B too
# wide for it, [A | B] shaped as one array; the rest: B right after A.
@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (3, 2), (17, 1), (64, 5), (129, 3), (300, 7),
                                 (777, 1), (1000, 3), (1000, 24), (1000, 200), (1500, 40),
                                 (2000, 128)])
def test_solve_matches_oracle(gj, n, m):
    rng = inputs.rng_for(0, 8000 + n)
    A = rng.standard_normal((n, n))
    B = rng.standard_normal((n, m))
    _assert_same(_solve(gj, A, B), oracle.gj_solve_f64(A, B), f"n={n} m={m}")


def test_solve_pascal_and_ties(gj):
    """The program's default matrix with an integer right-hand side, and a
    Hadamard matrix, where every candidate ties at every step."""
    P = inputs.pascal(3)
    B = np.array([[1.0, 2.0], [3.0, -1.0], [0.5, 4.0]])
    _assert_same(_solve(gj, P, B), oracle.gj_solve_f64(P, B), "pascal3")
    H = inputs.sylvester_hadamard(64)
    Bh = inputs.rng_for(0, 8100).standard_normal((64, 9))
    _assert_same(_solve(gj, H, Bh), oracle.gj_solve_f64(H, Bh), "hadamard64")


@pytest.mark.parametrize("n", [5, 200])
def test_solve_singular(gj, n):
    rng = inputs.rng_for(0, 8200 + n)
    A = rng.standard_normal((n, n))
    A[:, n - 1] = A[:, 0] + A[:, 1]
    B = rng.standard_normal((n, 4))
    got = _solve(gj, A, B)
    assert got[3]["code"] == 1 and got[3]["rank"] == n - 1
    _assert_same(got, oracle.gj_solve_f64(A, B), f"singular n={n}")


@pytest.mark.parametrize("stat", [1, 2])
def test_solve_counted_units(gj, stat, monkeypatch):
    """[A | B] = 896 + 128 columns: A alone uses 7 register chunks, the
    array as a whole all 8, so some work units come from the step kernel's
    counter."""
    monkeypatch.setenv("GJ_BIG_STATIC", str(stat))
    monkeypatch.setenv("GJ_BIG_ROWS", "32")
    rng = inputs.rng_for(0, 8300 + stat)
    A = rng.standard_normal((896, 896))
    B = rng.standard_normal((896, 128))
    _assert_same(_solve(gj, A, B), oracle.gj_solve_f64(A, B), f"counted static={stat}")


def test_solve_identity_columns_at_4096(gj):
    """At the benchmark's order and input: right-hand sides taken from the
    identity give the inverse's columns bit for bit (each column of B is
    carried independently, and B = I is the inversion), with the same pivots
    and determinant as gj_invert."""
    import torch
    n = 4096
    A = _dev(inputs.single_dominant(n))
    cols = np.array([0, 1, 977, 2048, 3001, 4095])
    B = torch.zeros((n, len(cols)), dtype=torch.float64, device="cuda")
    B[torch.from_numpy(cols).cuda(), torch.arange(len(cols), device="cuda")] = 1.0
    Xs, ips, jps, rs = gj.gj_solve(A, B)
    Xi, ipi, jpi, ri = gj.gj_invert(A)
    torch.cuda.synchronize()
    assert torch.equal(ips, ipi) and torch.equal(jps, jpi)
    assert torch.equal(Xs, Xi[:, torch.from_numpy(cols).cuda()])
    r1, r2 = gj.results_to_dicts(rs)[0], gj.results_to_dicts(ri)[0]
    assert r1["det_mant"] == r2["det_mant"] and r1["det_exp"] == r2["det_exp"]
    assert r1["det_sign"] == r2["det_sign"]
