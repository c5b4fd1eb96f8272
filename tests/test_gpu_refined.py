"""GPU parity for the FP32-elimination + FP64-refinement path.

Bars (each tolerance follows from the arithmetic of its stage):
* the FP32 elimination is the oracle's FP32 model operation for operation, so
  the returned pivot sequence equals the FP32 oracle's bit for bit;
* for cond <= 1e4 the refined inverse is within 1e-12 (relative Frobenius) of
  the FP64 oracle's inverse;
* for every condition number its forward error against the long-double
  oracle is at most 4x the FP64 oracle's own error plus 1e-14;
* the Newton-Schulz update count is within one of the oracle's loop run from
  the same FP32 starting inverse;
* the FP64 determinant agrees with the static-pivot LU oracle (same pivot
  order) to 1e-11 relative in log|det| (both are backward stable in that
  order; measured at most 3e-13 up to cond 1e8), and with the closed form
  n ln(cond) / 2 of the test matrices.
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


def _refined(gj, A, det_only=False, **kw):
    import torch
    opts = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED, **kw)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to("cuda")
    if det_only:
        ipiv, jpiv, res = gj.gj_det(Ad, opts=opts)
        torch.cuda.synchronize()
        return None, ipiv.cpu().numpy(), jpiv.cpu().numpy(), gj.results_to_dicts(res)[0]
    X, ipiv, jpiv, res = gj.gj_invert(Ad, opts=opts)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy(), gj.results_to_dicts(res)[0]


def _rel(Y, Z):
    return float(np.linalg.norm(Y - Z) / np.linalg.norm(Z))


CASES = [(n, c) for n in (48, 128, 200, 333) for c in (1e2, 1e4, 1e6, 1e8)]


@pytest.mark.parametrize("n,cond", CASES)
def test_refined_inverse(gj, n, cond):
    A = inputs.conditioned(n, cond, inputs.rng_for(0, 6000 + n))
    X, ipiv, jpiv, r = _refined(gj, A)
    assert r["code"] == 0, r
    # FP32 stage: pivot sequence identical to the FP32 oracle
    X32, i32, j32, _ = oracle.gj_invert_f32(A.astype(np.float32))
    assert np.array_equal(ipiv, i32) and np.array_equal(jpiv, j32)
    Xo, _, _, ro = oracle.gj_invert_f64(A)
    Xt, _, _, _ = oracle.gj_invert_f80(A)
    if cond <= 1e4:
        assert _rel(X, Xo) <= 1e-12
    assert _rel(X, Xt) <= 4 * _rel(Xo, Xt) + 1e-14
    # Newton-Schulz: same number of kept updates (within one) as the oracle loop
    _, upd, norms, acc = oracle.newton_schulz(A, X32.astype(np.float64))
    assert abs(r["refine_iters"] - upd) <= 1, (r["refine_iters"], upd, norms)
    # FP64 determinant
    lu = oracle.lu_static_det_f64(A, i32, j32)
    assert r["det_sign"] == lu["det_sign"] == 1
    assert abs(r["logabsdet"] - lu["logabsdet"]) <= 1e-11 * abs(lu["logabsdet"])
    if cond <= 1e6:
        cf = inputs.closed_form_logdet(n, cond)
        assert abs(r["logabsdet"] - cf) <= 1e-9 * abs(cf)


@pytest.mark.parametrize("stat", [1, 3])
def test_refined_counted_units(gj, stat, monkeypatch):
    """FP32 elimination with work units from the step kernel's counter (all
    register chunks in use at n = 1000): the pivot sequence must be the FP32
    oracle's, and the refined inverse as accurate as with the default split."""
    monkeypatch.setenv("GJ_BIG_STATIC", str(stat))
    monkeypatch.setenv("GJ_BIG_ROWS", "32")
    n = 1000
    A = inputs.conditioned(n, 1e4, inputs.rng_for(0, 6050 + stat))
    X, ipiv, jpiv, r = _refined(gj, A)
    assert r["code"] == 0, r
    _, i32, j32, _ = oracle.gj_invert_f32(A.astype(np.float32))
    assert np.array_equal(ipiv, i32) and np.array_equal(jpiv, j32)
    Xo, _, _, _ = oracle.gj_invert_f64(A)
    assert _rel(X, Xo) <= 1e-12


@pytest.mark.parametrize("n", [1100, 2100, 2000, 4000])
def test_refined_chunks_per_thread(gj, n, monkeypatch):
    """The FP32 elimination's default row shape (1-2 register chunks per
    thread up to 2048, the table's 4 above; each on the step kernel of the chunk
    count its rows fill) against the 8-chunk shape: the same FP32 pivot
    sequence as the oracle, and the same refined inverse bit for bit (each
    element's update does not depend on which thread holds it)."""
    A = inputs.conditioned(n, 1e4, inputs.rng_for(0, 6070 + n))
    X4, ip4, jp4, r4 = _refined(gj, A)
    monkeypatch.setenv("GJ_BIG_CHUNKS", "8")
    X8, ip8, jp8, r8 = _refined(gj, A)
    assert r4["code"] == 0 and r8["code"] == 0, (r4, r8)
    _, i32, j32, _ = oracle.gj_invert_f32_par(A.astype(np.float32))
    assert np.array_equal(ip4, i32) and np.array_equal(jp4, j32)
    assert np.array_equal(ip8, i32) and np.array_equal(jp8, j32)
    assert np.array_equal(X4, X8)
    assert r4["det_mant"] == r8["det_mant"] and r4["det_exp"] == r8["det_exp"]


def _exact_pair(n, span, seed):
    """A = H D H^T with H Sylvester-Hadamard (entries +-1) and D a diagonal of
    powers of two spanning 2^span (cond(A) = 2^span): every entry of A and of
    A^-1 = H D^-1 H^T / n^2 is an exact sum of powers of two, so both are
    exact in FP64 and the forward error of a computed inverse is known."""
    H = inputs.sylvester_hadamard(n)
    rng = inputs.rng_for(0, seed)
    e = rng.integers(0, span + 1, size=n)
    e[0], e[1] = 0, span
    A = (H * np.ldexp(1.0, e)) @ H.T
    Ainv = (H * np.ldexp(1.0, -e)) @ H.T / float(n * n)
    return A, Ainv


@pytest.mark.parametrize("n,span", [(64, 20), (256, 20), (256, 24), (512, 16)])
def test_accurate_residual_phase(gj, n, span):
    """GJ_FLAG_ACCURATE: the FP64-residual loop leaves a forward error of
    about n u cond(A); the updates with error-free split residuals bring it to
    a few u, against an exactly known inverse."""
    A, Ainv = _exact_pair(n, span, 6200 + n + span)
    Xr, _, _, rr = _refined(gj, A)
    Xa, _, _, ra = _refined(gj, A, flags=gj.GJ_FLAG_ACCURATE)
    assert rr["code"] == 0 and ra["code"] == 0, (rr, ra)
    err_r = _rel(Xr, Ainv)
    err_a = _rel(Xa, Ainv)
    assert err_a <= 8 * 2.0 ** -53, (err_a, err_r)
    assert ra["refine_iters"] > rr["refine_iters"]
    if span >= 20:
        assert err_r >= 100 * err_a, (err_a, err_r)


def test_accurate_phase_skipped_on_fallback(gj):
    """When the FP32 elimination fails the plain FP64 result stands, with or
    without the accurate phase."""
    A = inputs.rng_for(0, 6300).standard_normal((40, 40)) * 1e-50
    Xr, _, _, rr = _refined(gj, A)
    Xa, _, _, ra = _refined(gj, A, flags=gj.GJ_FLAG_ACCURATE)
    assert rr["code"] == ra["code"]
    assert Xr.tobytes() == Xa.tobytes()


@pytest.mark.parametrize("n", [64, 300])
def test_refined_det_only(gj, n):
    A = inputs.conditioned(n, 1e3, inputs.rng_for(0, 6100 + n))
    _, ipiv, jpiv, r = _refined(gj, A, det_only=True)
    _, i32, j32, _ = oracle.gj_invert_f32(A.astype(np.float32))
    assert np.array_equal(ipiv, i32) and np.array_equal(jpiv, j32)
    lu = oracle.lu_static_det_f64(A, i32, j32)
    assert r["det_sign"] == lu["det_sign"]
    assert abs(r["logabsdet"] - lu["logabsdet"]) <= 1e-12 * abs(lu["logabsdet"])


@pytest.mark.parametrize("n", [40, 260])
def test_fallback_when_fp32_underflows(gj, n):
    """Entries below the FP32 range: the FP32 elimination sees a zero matrix
    (singular), so the FP64 elimination produces the result, bit for bit."""
    A = inputs.rng_for(0, 6200 + n).standard_normal((n, n)) * 1e-50
    X, ipiv, jpiv, r = _refined(gj, A)
    Xo, io, jo, ro = oracle.gj_invert_f64(A)
    assert r["code"] == 3
    assert X.tobytes() == Xo.tobytes()
    assert np.array_equal(ipiv, io) and np.array_equal(jpiv, jo)
    assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"]


@pytest.mark.parametrize("n", [40, 260])
def test_fallback_on_caller_stream(gj, n):
    """Outside graph capture the FP64 fallback runs on the library's second
    stream; synchronising only the caller's stream must cover it (the call
    makes that stream wait for the second one before its last work)."""
    import torch
    A = inputs.rng_for(0, 6250 + n).standard_normal((n, n)) * 1e-50
    opts = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)
    Ad = torch.from_numpy(A).to("cuda")
    X = torch.full((n, n), 7.0, dtype=torch.float64, device="cuda")
    ip = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    jp = ip.clone()
    res = torch.zeros(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, opts), dtype=torch.uint8,
                     device="cuda")
    torch.cuda.synchronize()
    s2 = torch.cuda.Stream()
    gj.gj_invert(Ad, X, ip, jp, res, opts, ws, s2)
    s2.synchronize()
    r = gj.results_to_dicts(res)[0]
    Xo, io, jo, ro = oracle.gj_invert_f64(A)
    assert r["code"] == 3
    assert X.cpu().numpy().tobytes() == Xo.tobytes()
    assert np.array_equal(ip.cpu().numpy(), io) and np.array_equal(jp.cpu().numpy(), jo)
    assert r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"]


@pytest.mark.parametrize("n", [64, 256])
def test_singular_through_refined_path(gj, n):
    H = inputs.sylvester_hadamard(n)
    A = H.copy()
    A[:, n - 1] = H[:, 0] + H[:, 1]
    X, ipiv, jpiv, r = _refined(gj, A)
    assert r["code"] == 1 and r["rank"] == n - 1
    assert np.isnan(X).all()


@pytest.mark.parametrize("n,prec", [(70, 0), (300, 0), (70, 1), (300, 1)])
def test_want_resid(gj, n, prec):
    import torch
    A = inputs.conditioned(n, 1e3, inputs.rng_for(0, 6300 + n))
    opts = gj.make_opts(precision=prec, want_resid=True)
    X, _, _, res = gj.gj_invert(torch.from_numpy(A).to("cuda"), opts=opts)
    torch.cuda.synchronize()
    r = gj.results_to_dicts(res)[0]
    want = oracle.residual(A, X.cpu().numpy())
    assert abs(r["resid"] - want) <= 1e-2 * want + 1e-18


def test_refined_batched_mixed(gj):
    """A packed batch through the refined path: every on-chip class, the
    streaming FP32 path, an exactly singular member and one whose entries
    underflow FP32 (fallback), each against the same bars as a single call."""
    import torch
    rng = inputs.rng_for(0, 6400)
    sizes = [1, 3, 7, 8, 12, 16, 20, 33, 40, 64, 65, 90, 128, 129, 150, 200, 256, 300]
    conds = [10.0 ** rng.uniform(1, 8) for _ in sizes]
    mats = [inputs.conditioned(n, c, rng) if n > 1 else np.array([[2.5]]) for n, c in zip(sizes, conds)]
    H = inputs.sylvester_hadamard(64)
    Hs = H.copy()
    Hs[:, 63] = H[:, 0] + H[:, 1]
    mats.append(Hs)
    sizes.append(64)
    conds.append(np.inf)
    mats.append(rng.standard_normal((70, 70)) * 1e-50)
    sizes.append(70)
    conds.append(np.nan)
    sizes = np.array(sizes, dtype=np.int32)
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    packed = np.concatenate([m.ravel() for m in mats])
    opts = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)
    X, ipiv, jpiv, res, poff = gj.gj_invert_batched(sizes, offs, torch.from_numpy(packed).to("cuda"),
                                                     opts=opts)
    torch.cuda.synchronize()
    Xh, ih, jh = X.cpu().numpy(), ipiv.cpu().numpy(), jpiv.cpu().numpy()
    rs = gj.results_to_dicts(res)
    for b, (n, A) in enumerate(zip(sizes, mats)):
        n = int(n)
        Xb = Xh[offs[b]:offs[b] + n * n].reshape(n, n)
        ib, jb = ih[poff[b]:poff[b] + n], jh[poff[b]:poff[b] + n]
        r = rs[b]
        where = f"member {b} n={n} cond={conds[b]:.2g}"
        if np.isinf(conds[b]):
            assert r["code"] == 1 and r["rank"] == n - 1, where
            continue
        if np.isnan(conds[b]):
            Xo, io, jo, ro = oracle.gj_invert_f64(A)
            assert r["code"] == 3 and Xb.tobytes() == Xo.tobytes(), where
            assert np.array_equal(ib, io) and np.array_equal(jb, jo), where
            continue
        assert r["code"] == 0, (where, r)
        X32, i32, j32, _ = oracle.gj_invert_f32(A.astype(np.float32))
        assert np.array_equal(ib, i32) and np.array_equal(jb, j32), where
        Xo, _, _, _ = oracle.gj_invert_f64(A)
        Xt, _, _, _ = oracle.gj_invert_f80(A)
        if conds[b] <= 1e4:
            assert _rel(Xb, Xo) <= 1e-12, where
        assert _rel(Xb, Xt) <= 4 * _rel(Xo, Xt) + 1e-14, where
        _, upd, _, _ = oracle.newton_schulz(A, X32.astype(np.float64))
        assert abs(r["refine_iters"] - upd) <= 1, where
        lu = oracle.lu_static_det_f64(A, i32, j32)
        assert r["det_sign"] == lu["det_sign"], where
        assert abs(r["logabsdet"] - lu["logabsdet"]) <= 1e-11 * max(1.0, abs(lu["logabsdet"])), where


@pytest.mark.parametrize("n,cond,nb", [(300, 1e4, 64), (333, 1e8, 128), (777, 1e6, 96),
                                       (1000, 1e2, 256)])
def test_refined_blocked(gj, n, cond, nb, monkeypatch):
    """GJ_FLAG_BLOCKED on the refined path: the FP32 stage eliminates with
    delayed updates (FP32 matrix-core products between panels), which leaves
    the trailing block's values, so the pivot sequence is the FP32 oracle's
    bit for bit; the refined inverse and determinant are held to the same bars
    as the unblocked refined path."""
    monkeypatch.setenv("GJ_BLK_NB", str(nb))
    A = inputs.conditioned(n, cond, inputs.rng_for(0, 6500 + n))
    X, ipiv, jpiv, r = _refined(gj, A, flags=gj.GJ_FLAG_BLOCKED)
    assert r["code"] == 0, r
    X32, i32, j32, _ = oracle.gj_invert_f32(A.astype(np.float32))
    assert np.array_equal(ipiv, i32) and np.array_equal(jpiv, j32)
    Xo, _, _, _ = oracle.gj_invert_f64(A)
    if cond <= 1e4:
        assert _rel(X, Xo) <= 1e-12
    if n <= 520:
        Xt, _, _, _ = oracle.gj_invert_f80(A)
        assert _rel(X, Xt) <= 4 * _rel(Xo, Xt) + 1e-14
    else:
        Xt = oracle.inverse_truth(A, Xo)
        assert _rel(X, Xt) <= 4 * _rel(Xo, Xt) + 1e-14
    lu = oracle.lu_static_det_f64(A, i32, j32)
    assert r["det_sign"] == lu["det_sign"] == 1
    assert abs(r["logabsdet"] - lu["logabsdet"]) <= 1e-11 * abs(lu["logabsdet"])
    # the same call without the flag: same pivots, refined X within rounding
    X2, i2, j2, r2 = _refined(gj, A)
    assert np.array_equal(i2, ipiv) and np.array_equal(j2, jpiv)
    assert _rel(X, X2) <= 1e-12 if cond <= 1e4 else _rel(X, Xt) <= 4 * _rel(X2, Xt) + 1e-14


def test_refined_blocked_singular(gj, monkeypatch):
    """A rank-deficient input stops the FP32 stage inside a panel; the FP64
    fallback then reports the oracle's rank and code."""
    monkeypatch.setenv("GJ_BLK_NB", "64")
    rng = inputs.rng_for(0, 6600)
    n, rank = 300, 200
    A = rng.standard_normal((n, rank)) @ rng.standard_normal((rank, n))
    X, ipiv, jpiv, r = _refined(gj, A, flags=gj.GJ_FLAG_BLOCKED)
    _, io, jo, ro = oracle.gj_invert_f64(A)
    assert r["code"] == ro["code"] != 0 and r["rank"] == ro["rank"]
    assert np.array_equal(ipiv, io) and np.array_equal(jpiv, jo)


def test_refined_blocked_large_order(gj):
    """An order whose first panels take the tuned whole-inversion row shape
    (FP32 blocks above 6144): the blocked FP32 stage keeps the unblocked FP32
    stage's pivot sequence bit for bit, and both refined inverses agree to
    1e-12 (the input is diagonally dominant, cond ~ 2)."""
    import torch
    n = 6400
    A = torch.from_numpy(inputs.single_dominant(n, offset=77)).to("cuda")
    out = {}
    for name, flags in (("blocked", gj.GJ_FLAG_BLOCKED), ("unblocked", 0)):
        X, ip, jp, res = gj.gj_invert(A, opts=gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED, flags=flags))
        torch.cuda.synchronize()
        out[name] = (X, ip.cpu().numpy(), jp.cpu().numpy(), gj.results_to_dicts(res)[0])
    Xb, ib, jb, rb = out["blocked"]
    Xu, iu, ju, ru = out["unblocked"]
    assert rb["code"] == ru["code"] == 0
    assert np.array_equal(ib, iu) and np.array_equal(jb, ju)
    assert float(torch.linalg.norm(Xb - Xu) / torch.linalg.norm(Xu)) <= 1e-12
    assert abs(rb["logabsdet"] - ru["logabsdet"]) <= 1e-11 * abs(ru["logabsdet"])
