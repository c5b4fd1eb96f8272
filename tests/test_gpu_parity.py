"""GPU parity for the plain FP64 path: the HIP kernels against the FP64
oracle, element by element.  The FP64 path performs exactly the oracle's
operations (same division, one fma per element, same total-order pivot
search), so the bar is bit-for-bit equality of X, the pivot sequence and the
determinant's (sign, mantissa, exponent); log|det| within 4 ulp (device log).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1401_7962_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def gj():
    import torch  # noqa: F401
    import paper_1401_7962_amd as m
    m.load_library()
    return m


def _dev(A):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to("cuda")


def _run_invert(gj, A, **kw):
    import torch
    opts = gj.make_opts(**kw) if kw else None
    X, ipiv, jpiv, res = gj.gj_invert(_dev(A), opts=opts)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy(), gj.results_to_dicts(res)[0]


def _assert_same(A, got, want, where=""):
    X, ipiv, jpiv, r = got
    Xo, io, jo, ro = want
    assert r["code"] == ro["code"], where
    assert r["rank"] == ro["rank"], where
    assert np.array_equal(ipiv, io), where
    assert np.array_equal(jpiv, jo), where
    if ro["code"] == 0:
        assert X.tobytes() == Xo.tobytes(), (where, np.max(np.abs(X - Xo)))
        assert r["det_sign"] == ro["det_sign"], where
        assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"], where
        if np.isfinite(ro["det"]):
            assert r["det"] == ro["det"], where
        assert abs(r["logabsdet"] - ro["logabsdet"]) <= 4 * np.spacing(max(1.0, abs(ro["logabsdet"])))
    else:
        assert np.isnan(X).all(), where
        assert r["det_sign"] == 0


def test_pascal3_default_matrix(gj):
    g = json.load(open(os.path.join(GOLDEN, "pascal3.json")))
    A = np.array(g["A"], dtype=np.float64)
    got = _run_invert(gj, A)
    _assert_same(A, got, oracle.gj_invert_f64(A))
    assert got[1].tolist() == g["ipiv"] and got[3]["det"] == 1.0


def test_golden_small_cases(gj):
    for case in json.load(open(os.path.join(GOLDEN, "small_cases.json")))["cases"]:
        A = np.array(case["A"], dtype=np.float64)
        got = _run_invert(gj, A)
        _assert_same(A, got, oracle.gj_invert_f64(A), case["name"])
        assert got[3]["code"] == case["code"] and got[1].tolist() == case["ipiv"]


def test_single_normal_64(gj):
    A = inputs.single_normal(64)
    _assert_same(A, _run_invert(gj, A), oracle.gj_invert_f64(A))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128])
def test_onchip_sizes(gj, n):
    A = inputs.rng_for(0, 2000 + n).standard_normal((n, n))
    _assert_same(A, _run_invert(gj, A), oracle.gj_invert_f64(A), f"n={n}")


@pytest.mark.parametrize("n", [129, 200, 257, 333, 440, 512, 777, 1000, 1400])
def test_streaming_sizes(gj, n):
    """Orders whose rows fill 4 (200, 512, 777, 1000), 5 (129, 257), 6 (333,
    1400) and 7 (440) register chunks per thread: each runs the step kernel
    of its own chunk count."""
    A = inputs.rng_for(0, 3000 + n).standard_normal((n, n))
    _assert_same(A, _run_invert(gj, A), oracle.gj_invert_f64(A), f"n={n}")


@pytest.mark.parametrize("n", [2600, 3500])
def test_streaming_sizes_large(gj, n):
    """256 threads per row filling 6 (2600) and 7 (3500) chunks, against the
    oracle's OpenMP form (bitwise the serial oracle)."""
    A = inputs.rng_for(0, 3000 + n).standard_normal((n, n))
    _assert_same(A, _run_invert(gj, A), oracle.gj_invert_f64_par(A), f"n={n}")


@pytest.mark.parametrize("n,nt,rows", [(300, 1, 0), (777, 1, 0), (1000, 1, 3), (1000, 0, 64),
                                         (1025, 1, 0), (2049, 0, 0)])
def test_streaming_variants(gj, n, nt, rows, monkeypatch):
    """The step kernel's instantiations: nontemporal row loads (chosen by the
    library only past the Infinity Cache, forced here), full or partial
    register chunks, and rows per workgroup away from the tuned value."""
    monkeypatch.setenv("GJ_BIG_NT", str(nt))
    if rows:
        monkeypatch.setenv("GJ_BIG_ROWS", str(rows))
    A = inputs.rng_for(0, 3100 + n).standard_normal((n, n))
    _assert_same(A, _run_invert(gj, A), oracle.gj_invert_f64(A), f"n={n} nt={nt} rows={rows}")


@pytest.mark.parametrize("n,rows,stat", [(250, 64, 1), (500, 64, 2), (1000, 32, 1), (1000, 32, 2),
                                           (2000, 16, 3), (1000, 32, 100), (777, 16, 2)])
def test_streaming_work_units(gj, n, rows, stat, monkeypatch):
    """Work units of the step kernel taken by index and from the per-step
    counter: one, two or three units per workgroup by index and the rest from
    the counter (with one, the first counter read happens during the only own
    unit; 250 and 500 end in a partial unit), every unit by index (100 is
    clamped to the workgroup's share), and a size whose threads do not use all
    their register chunks (no counter: every unit by index).  The inverse and
    the determinant-only sweep (which skips the rows already eliminated) must
    match the oracle bit for bit."""
    import torch
    monkeypatch.setenv("GJ_BIG_STATIC", str(stat))
    if rows:
        monkeypatch.setenv("GJ_BIG_ROWS", str(rows))
    A = inputs.rng_for(0, 3200 + n).standard_normal((n, n))
    want = oracle.gj_invert_f64(A)
    _assert_same(A, _run_invert(gj, A), want, f"n={n} rows={rows} static={stat}")
    ipiv, jpiv, res = gj.gj_det(_dev(A))
    torch.cuda.synchronize()
    r = gj.results_to_dicts(res)[0]
    assert np.array_equal(ipiv.cpu().numpy(), want[1]) and np.array_equal(jpiv.cpu().numpy(), want[2])
    assert r["det_mant"] == want[3]["det_mant"] and r["det_exp"] == want[3]["det_exp"]
    assert r["det_sign"] == want[3]["det_sign"]


@pytest.mark.parametrize("n,chunks", [(1100, 4), (1100, 2), (2100, 4), (1500, 1), (2000, 4)])
def test_streaming_chunks_per_thread(gj, n, chunks, monkeypatch):
    """Wider rows than the default shape (fewer register chunks per thread,
    more threads per row; 1 chunk clamps the row to the workgroup; at 2000
    with 4 chunks every thread fills all 4, the 4-chunk step kernel): the
    inverse and the pivots must still match the oracle bit for bit."""
    monkeypatch.setenv("GJ_BIG_CHUNKS", str(chunks))
    A = inputs.rng_for(0, 3300 + n + chunks).standard_normal((n, n))
    _assert_same(A, _run_invert(gj, A), oracle.gj_invert_f64(A), f"n={n} chunks={chunks}")


@pytest.mark.parametrize("n", [4, 16, 64, 128, 256, 512])
def test_hadamard_ties(gj, n):
    """Every candidate ties at every step: the tie-break on the swapped
    positions decides each pivot (virtual swaps on the streaming path)."""
    H = inputs.sylvester_hadamard(n)
    got = _run_invert(gj, H)
    _assert_same(H, got, oracle.gj_invert_f64(H), f"H{n}")
    assert np.array_equal(got[0], H.T / n)


@pytest.mark.parametrize("n", [16, 128, 256])
def test_exactly_singular(gj, n):
    H = inputs.sylvester_hadamard(n)
    A = H.copy()
    A[:, n - 1] = H[:, 0] + H[:, 1]
    got = _run_invert(gj, A)
    _assert_same(A, got, oracle.gj_invert_f64(A), f"singular H{n}")
    assert got[3]["code"] == 1 and got[3]["rank"] == n - 1


@pytest.mark.parametrize("n", [20, 300])
def test_nonfinite(gj, n):
    A = inputs.rng_for(0, 4000 + n).standard_normal((n, n))
    A[n // 2, n // 3] = np.nan
    got = _run_invert(gj, A)
    _assert_same(A, got, oracle.gj_invert_f64(A), "nan")
    assert got[3]["code"] == 2
    B = inputs.rng_for(0, 4100 + n).standard_normal((n, n))
    B[1, 2] = np.inf
    got = _run_invert(gj, B)
    assert got[3]["code"] == 2


@pytest.mark.parametrize("n", [40, 260])
def test_zero_threshold(gj, n):
    A = inputs.rng_for(0, 4200 + n).standard_normal((n, n))
    A[:, 5] = A[:, 1] * 0.5 + A[:, 2] * 0.25 + 1e-15 * A[:, 3]   # nearly rank-deficient
    for tol in (-1.0, 0.0, 1e-3):
        got = _run_invert(gj, A, zero_tol=tol)
        _assert_same(A, got, oracle.gj_invert_f64(A, zero_tol=tol), f"tol={tol}")


@pytest.mark.parametrize("n", [50, 128, 300])
def test_det_matches_invert(gj, n):
    import torch
    A = inputs.rng_for(0, 4300 + n).standard_normal((n, n))
    ipiv, jpiv, res = gj.gj_det(_dev(A))
    torch.cuda.synchronize()
    r = gj.results_to_dicts(res)[0]
    _, io, jo, ro = oracle.gj_invert_f64(A)
    assert np.array_equal(ipiv.cpu().numpy(), io) and np.array_equal(jpiv.cpu().numpy(), jo)
    assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"]
    assert r["det_sign"] == ro["det_sign"]


def test_batched_counted_units(gj, monkeypatch):
    """A batch whose streaming members all use their full register chunks
    (n = 900, 1000, 1000) runs one step launch with the work-unit counter:
    each member has its own counters; small members go on chip.  Every member
    must match the oracle bit for bit."""
    import torch
    monkeypatch.setenv("GJ_BIG_STATIC", "1")
    monkeypatch.setenv("GJ_BIG_ROWS", "32")
    sizes = np.array([1000, 64, 900, 1000, 5], dtype=np.int32)
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    rng = inputs.rng_for(0, 3300)
    mats = [rng.standard_normal((int(n), int(n))) for n in sizes]
    packed = np.concatenate([m.ravel() for m in mats])
    A = torch.from_numpy(packed).to("cuda")
    X, ipiv, jpiv, res, poff = gj.gj_invert_batched(sizes, offs, A)
    torch.cuda.synchronize()
    Xh, ih, jh = X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy()
    rs = gj.results_to_dicts(res)
    for b, M in enumerate(mats):
        n = int(sizes[b])
        got = (Xh[offs[b]:offs[b] + n * n].reshape(n, n), ih[poff[b]:poff[b] + n],
               jh[poff[b]:poff[b] + n], rs[b])
        _assert_same(M, got, oracle.gj_invert_f64(M), f"member {b} n={n}")


def test_batched_mixed(gj):
    """A packed batch spanning the wavefront, workgroup and streaming paths,
    with planted rank-(n-1) members."""
    import torch
    sizes, offs, packed, singular = inputs.batch_uneven(batch=240, nmin=1, nmax=300,
                                                        singular_frac=0.05, offset=77)
    A = torch.from_numpy(packed).to("cuda")
    X, ipiv, jpiv, res, poff = gj.gj_invert_batched(sizes, offs, A)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    ih, jh = ipiv.cpu().numpy(), jpiv.cpu().numpy()
    rs = gj.results_to_dicts(res)
    n_sing = 0
    for b in range(len(sizes)):
        n = int(sizes[b])
        Ab = packed[offs[b]:offs[b] + n * n].reshape(n, n)
        got = (Xh[offs[b]:offs[b] + n * n].reshape(n, n), ih[poff[b]:poff[b] + n],
               jh[poff[b]:poff[b] + n], rs[b])
        _assert_same(Ab, got, oracle.gj_invert_f64(Ab), f"member {b} n={n}")
        n_sing += rs[b]["code"] == 1
    assert n_sing >= len(singular) - 2   # tiny members (n < 3) cannot host the planted sum


@pytest.mark.parametrize("chunks", ["2", "4"])
def test_batched_chunk_groups(gj, chunks, monkeypatch):
    """Streaming members of several orders with fewer register chunks per
    thread than the default: the members fall into groups by the chunk count
    their rows fill (1-4 here), one launch sequence each, and every member of
    every group must be inverted (bit for bit against the oracle)."""
    monkeypatch.setenv("GJ_BIG_CHUNKS", chunks)
    rng = inputs.rng_for(0, 8600 + int(chunks))
    mats = [rng.standard_normal((n, n)) for n in (130, 200, 257, 300, 384, 500, 64)]
    _batched_vs_oracle(gj, mats, f"chunks={chunks}")


def _batched_vs_oracle(gj, mats, where):
    import torch
    sizes = np.array([M.shape[0] for M in mats], dtype=np.int32)
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    packed = np.concatenate([M.ravel() for M in mats])
    A = torch.from_numpy(packed).to("cuda")
    X, ipiv, jpiv, res, poff = gj.gj_invert_batched(sizes, offs, A)
    torch.cuda.synchronize()
    Xh, ih, jh = X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy()
    rs = gj.results_to_dicts(res)
    for b, M in enumerate(mats):
        n = M.shape[0]
        got = (Xh[offs[b]:offs[b] + n * n].reshape(n, n), ih[poff[b]:poff[b] + n],
               jh[poff[b]:poff[b] + n], rs[b])
        _assert_same(M, got, oracle.gj_invert_f64(M), f"{where} member {b} n={n}")
    return rs


BOUNDARY_ORDERS = [1, 2, 7, 8, 9, 15, 16, 17, 24, 25, 32, 33, 40, 41, 48, 49, 56, 57, 63, 64,
                   65, 79, 80, 81, 96, 97, 111, 112, 113, 127, 128]


def test_batched_every_onchip_class(gj):
    """Every on-chip task class (one matrix per wavefront for n <= 64, per
    workgroup above, register blocks of 1..8 per thread and dimension) at
    both ends of its range, three members each, interleaved."""
    rng = inputs.rng_for(0, 8800)
    mats = [rng.standard_normal((n, n)) for n in BOUNDARY_ORDERS for _ in range(3)]
    rng.shuffle(mats)
    _batched_vs_oracle(gj, mats, "classes")


def test_batched_onchip_ties_and_singular(gj):
    """Hadamard members (a tie at every step, exact arithmetic), exactly
    singular ones, a zero matrix, and scaled copies with ties across
    wavefronts, in one batch."""
    mats = []
    for n in (4, 8, 16, 32, 64, 128):
        H = inputs.sylvester_hadamard(n)
        mats.append(H)
        S = H.copy()
        S[:, n - 1] = S[:, 0] + S[:, 1]
        if n >= 4:
            mats.append(S)
        mats.append(np.kron(np.eye(2), inputs.sylvester_hadamard(n // 2)) if n >= 2 else H)
    mats.append(np.zeros((20, 20)))
    mats.append(np.ones((70, 70)))
    rs = _batched_vs_oracle(gj, mats, "ties")
    assert sum(r["code"] == 1 for r in rs) >= 8


@pytest.mark.parametrize("n", [1, 5, 16, 17, 33, 64, 65, 100, 128])
def test_det_only_onchip(gj, n):
    """gj_det on the on-chip path: the pivots and determinant of gj_invert."""
    import torch
    A = inputs.single_normal(n, offset=900 + n)
    ipiv, jpiv, res = gj.gj_det(_dev(A))
    torch.cuda.synchronize()
    _, io, jo, ro = oracle.gj_invert_f64(A)
    r = gj.results_to_dicts(res)[0]
    assert np.array_equal(ipiv.cpu().numpy(), io) and np.array_equal(jpiv.cpu().numpy(), jo)
    assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"]
    assert r["det_sign"] == ro["det_sign"]
