"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code (worked examples, closed forms,
exact arithmetic, invariants, brute force, a LAPACK routine, higher
precision).  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1401_7962_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- worked cases

def test_pascal3_default_matrix():
    g = _golden("pascal3.json")
    A = np.array(g["A"], dtype=np.float64)
    X, ipiv, jpiv, res = oracle.gj_invert_f64(A)
    assert res["code"] == 0 and res["rank"] == 3
    assert ipiv.tolist() == g["ipiv"] and jpiv.tolist() == g["jpiv"]
    assert res["det_sign"] == g["det_sign"]
    # exact integers in rational arithmetic; allow rounding in FP64
    assert np.array_equal(np.rint(X), np.array(g["inverse"], dtype=np.float64))
    assert np.max(np.abs(X - np.array(g["inverse"]))) <= 1e-14
    assert abs(res["det"] - g["det"]) <= 1e-14
    # the product of the printed pivots is the determinant (eq. 13)
    assert abs(np.prod(g["pivots"]) - res["det"]) <= 1e-15


@pytest.mark.parametrize("case", _golden("small_cases.json")["cases"], ids=lambda c: c["name"])
def test_exact_small_cases(case):
    A = np.array(case["A"], dtype=np.float64)
    X, ipiv, jpiv, res = oracle.gj_invert_f64(A)
    assert res["code"] == case["code"]
    assert res["rank"] == case["rank"]
    assert ipiv.tolist() == case["ipiv"] and jpiv.tolist() == case["jpiv"]
    if case["code"] == 0:
        assert np.array_equal(X, np.array(case["inverse"], dtype=np.float64))
        assert res["det"] == case["det"]
    else:
        assert np.isnan(X).all()
        assert res["det_sign"] == 0 and res["det"] == 0.0
        assert res["logabsdet"] == -math.inf


def _pascal_inverse_exact(n):
    """P = L L^T with L_ij = C(i,j); (L^-1)_ij = (-1)^(i-j) C(i,j)."""
    Li = [[(-1) ** (i - j) * math.comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)]
    return [[sum(Li[k][i] * Li[k][j] for k in range(n)) for j in range(n)] for i in range(n)]


@pytest.mark.parametrize("n", range(1, 10))
def test_pascal_closed_form(n):
    A = inputs.pascal(n)
    X, _, _, res = oracle.gj_invert_f64(A)
    exact = np.array(_pascal_inverse_exact(n), dtype=np.float64)
    assert np.array_equal(np.rint(X), exact)
    cond = np.linalg.cond(A)
    assert np.max(np.abs(X - exact)) <= 8 * n * cond * U64 * np.max(np.abs(exact))
    assert abs(res["det"] - 1.0) <= 8 * n * cond * U64


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64])
def test_hadamard_exact_and_ties(n):
    """Every |a| ties at every step: the tie-break picks (k,k), no swaps, and
    all arithmetic is exact, so X == H^T / n bit for bit and det = +-n^(n/2)."""
    H = inputs.sylvester_hadamard(n)
    X, ipiv, jpiv, res = oracle.gj_invert_f64(H)
    assert np.array_equal(X, H.T / n)
    assert ipiv.tolist() == list(range(n)) and jpiv.tolist() == list(range(n))
    m = int(round(math.log2(n)))
    # n^(n/2) = 2^(m n / 2) = 0.5 * 2^(m n/2 + 1)
    assert res["det_mant"] == 0.5 and res["det_exp"] == m * n // 2 + 1
    assert res["det_sign"] == (-1 if n == 2 else 1)


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_hadamard_exactly_singular(n):
    H = inputs.sylvester_hadamard(n)
    A = H.copy()
    A[:, n - 1] = H[:, 0] + H[:, 1]
    _, ipiv, _, res = oracle.gj_invert_f64(A)
    assert res["code"] == 1 and res["rank"] == n - 1 and ipiv[n - 1] == -1
    B = H.copy()
    B[n - 1] = H[0]
    _, _, _, res = oracle.gj_invert_f64(B)
    assert res["code"] == 1 and res["rank"] == n - 1


def test_closed_form_n1_n2():
    for a in (3.0, -0.125, 7.5e-300, 1e300):
        X, _, _, res = oracle.gj_invert_f64(np.array([[a]]))
        assert X[0, 0] == 1.0 / a and res["det"] == a
    rng = inputs.rng_for(0, 101)
    for _ in range(200):
        A = rng.standard_normal((2, 2))
        a, b, c, d = A.ravel()
        det = a * d - b * c
        exact = np.array([[d, -b], [-c, a]]) / det
        X, _, _, res = oracle.gj_invert_f64(A)
        cond = np.linalg.cond(A)
        assert np.max(np.abs(X - exact)) <= 8 * cond * U64 * np.max(np.abs(exact))
        assert abs(res["det"] - det) <= 8 * cond * U64 * abs(det)


# ----------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(6))
def test_power_of_two_scaling_is_bitwise(seed):
    rng = inputs.rng_for(0, 200 + seed)
    n = int(rng.integers(2, 20))
    A = rng.standard_normal((n, n))
    s = int(rng.integers(-20, 20))
    X, ipiv, jpiv, res = oracle.gj_invert_f64(A)
    Xs, ipiv_s, jpiv_s, res_s = oracle.gj_invert_f64(np.ldexp(A, s))
    assert np.array_equal(Xs, np.ldexp(X, -s))
    assert np.array_equal(ipiv, ipiv_s) and np.array_equal(jpiv, jpiv_s)
    assert res_s["det_mant"] == res["det_mant"] and res_s["det_exp"] == res["det_exp"] + s * n


@pytest.mark.parametrize("seed", range(6))
def test_permutation_equivariance_is_bitwise(seed):
    """Full pivoting picks the same elements whatever the row/column order
    (tie-free input), so inv(A[p][:,q]) == inv(A)[q][:,p] exactly."""
    rng = inputs.rng_for(0, 300 + seed)
    n = int(rng.integers(2, 24))
    A = rng.standard_normal((n, n))
    p, q = rng.permutation(n), rng.permutation(n)
    X, _, _, res = oracle.gj_invert_f64(A)
    Xp, _, _, res_p = oracle.gj_invert_f64(A[p][:, q])
    assert np.array_equal(Xp, X[q][:, p])
    assert res_p["det_mant"] == res["det_mant"] and res_p["det_exp"] == res["det_exp"]


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_cofactor_determinant(n):
    rng = inputs.rng_for(0, 400 + n)
    for _ in range(3):
        A = rng.standard_normal((n, n))
        exact = oracle.cofactor_det(A)
        _, _, _, res = oracle.gj_invert_f64(A)
        cond = np.linalg.cond(A)
        rel = abs(Fraction(res["det"]) - exact) / abs(exact)
        assert float(rel) <= 16 * n * cond * U64
        assert res["det_sign"] == (1 if exact > 0 else -1)


@pytest.mark.parametrize("n", [5, 17, 64, 130])
def test_residual_bound(n):
    A = inputs.rng_for(0, 500 + n).standard_normal((n, n))
    X, _, _, res = oracle.gj_invert_f64(A)
    assert oracle.residual(A, X) <= 10 * n * U64


def test_lapack_complete_pivoting_sequence():
    """LAPACK dgetc2 (complete-pivot LU) chooses the same pivots as GJ with full
    pivoting on tie-free inputs: both search the same trailing block, whose
    entries agree to rounding."""
    from scipy.linalg import lapack
    rng = inputs.rng_for(0, 600)
    for _ in range(40):
        n = int(rng.integers(1, 24))
        A = rng.standard_normal((n, n))
        _, ipiv_l, jpiv_l, info = lapack.dgetc2(A)
        _, ipiv, jpiv, res = oracle.gj_invert_f64(A)
        assert info == 0
        assert np.array_equal(ipiv, ipiv_l) and np.array_equal(jpiv, jpiv_l)
        sign, logdet = np.linalg.slogdet(A)
        assert res["det_sign"] == sign
        assert abs(res["logabsdet"] - logdet) <= 1e-12 * max(1.0, abs(logdet))


def test_augmented_form_is_bitwise_equal():
    """The in-place array and the literal [A|D] form of eqs. 14-15 agree bit
    for bit (the structural zeros and ones of D do not change any value)."""
    rng = inputs.rng_for(0, 700)
    for _ in range(30):
        n = int(rng.integers(1, 20))
        A = rng.standard_normal((n, n))
        X, ipiv, jpiv, res = oracle.gj_invert_f64(A)
        X2, ipiv2, jpiv2, res2 = oracle.gj_augmented_f64(A)
        assert X.tobytes() == X2.tobytes()
        assert np.array_equal(ipiv, ipiv2) and np.array_equal(jpiv, jpiv2)
        assert res["det_mant"] == res2["det_mant"] and res["det_exp"] == res2["det_exp"]


def _exact_solve(A, B):
    """A^-1 B in rationals: Gauss-Jordan with exact arithmetic (textbook; any
    nonzero pivot will do when nothing is rounded)."""
    n, m = len(A), len(B[0])
    M = [[Fraction(x) for x in list(A[i]) + list(B[i])] for i in range(n)]
    for k in range(n):
        r = next(i for i in range(k, n) if M[i][k] != 0)
        M[k], M[r] = M[r], M[k]
        p = M[k][k]
        M[k] = [x / p for x in M[k]]
        for i in range(n):
            if i != k and M[i][k] != 0:
                q = M[i][k]
                M[i] = [a - q * b for a, b in zip(M[i], M[k])]
    return [[M[i][n + j] for j in range(m)] for i in range(n)]


def test_solve_with_identity_is_the_inverse():
    """D^0 = B in eq. 2: with B = I the augmented elimination is the inversion,
    bit for bit, including ties (Hadamard), a permutation and singular input."""
    rng = inputs.rng_for(0, 710)
    mats = [rng.standard_normal((n, n)) for n in (1, 2, 5, 17, 40)]
    mats += [inputs.sylvester_hadamard(8), inputs.pascal(3), np.zeros((3, 3)),
             np.ones((4, 4))]
    for A in mats:
        n = A.shape[0]
        X, ipiv, jpiv, res = oracle.gj_invert_f64(A)
        Xs, ips, jps, rs = oracle.gj_solve_f64(A, np.eye(n))
        assert np.array_equal(ipiv, ips) and np.array_equal(jpiv, jps)
        assert res["code"] == rs["code"] and res["rank"] == rs["rank"]
        if res["code"] == 0:
            assert X.tobytes() == Xs.tobytes()
            assert res["det_mant"] == rs["det_mant"] and res["det_exp"] == rs["det_exp"]
            assert res["det_sign"] == rs["det_sign"]
        else:
            assert np.isnan(Xs).all()


def test_solve_exact_cases():
    """Inputs where every operation is exact: a permutation matrix (X = P^T B,
    with column swaps undone as row swaps) and a power-of-two diagonal."""
    rng = inputs.rng_for(0, 711)
    B = rng.integers(-50, 50, size=(4, 3)).astype(np.float64)
    s = [2, 0, 3, 1]
    Pm = np.zeros((4, 4))
    Pm[np.arange(4), s] = 1
    X, ipiv, jpiv, res = oracle.gj_solve_f64(Pm, B)
    assert res["code"] == 0 and res["det"] == -1
    assert np.array_equal(X, Pm.T @ B)
    D = np.diag([2.0, -0.25, 8.0, 0.5])
    X, _, _, res = oracle.gj_solve_f64(D, B)
    assert np.array_equal(X, B / np.diag(D)[:, None])
    assert res["det"] == -2.0


@pytest.mark.parametrize("seed", range(6))
def test_solve_against_exact_rationals(seed):
    """Small integer systems solved exactly in rationals; the FP64 result must
    be within the normwise bound c * n * u * cond(A) of the exact one."""
    rng = inputs.rng_for(0, 720 + seed)
    n, m = int(rng.integers(2, 7)), int(rng.integers(1, 4))
    A = rng.integers(-9, 10, size=(n, n)).astype(np.float64)
    while abs(np.linalg.det(A)) < 0.5:
        A = rng.integers(-9, 10, size=(n, n)).astype(np.float64)
    B = rng.integers(-9, 10, size=(n, m)).astype(np.float64)
    Xe = np.array([[float(x) for x in row] for row in _exact_solve(A.tolist(), B.tolist())])
    X, _, _, res = oracle.gj_solve_f64(A, B)
    assert res["code"] == 0
    cond = np.linalg.cond(A)
    err = np.abs(X - Xe).max() / np.abs(Xe).max()
    assert err <= 8 * n * 2.0 ** -53 * cond, (err, cond)


def test_solve_columns_are_independent():
    """Each column of B is carried by the same row operations: solving for
    [B1 B2] gives, bit for bit, the solutions for B1 and B2 separately."""
    rng = inputs.rng_for(0, 730)
    A = rng.standard_normal((30, 30))
    B = rng.standard_normal((30, 5))
    X, *_ = oracle.gj_solve_f64(A, B)
    X1, *_ = oracle.gj_solve_f64(A, B[:, :2])
    X2, *_ = oracle.gj_solve_f64(A, B[:, 2:])
    assert X.tobytes() == np.hstack([X1, X2]).tobytes()


RULES = {"full": 0, "partial": 1, "program": 2}


@pytest.mark.parametrize("case", _golden("pivot_rules.json")["cases"], ids=lambda c: c["name"])
def test_pivot_rules_golden(case):
    A = np.array(case["A"], dtype=np.float64)
    for name, rule in RULES.items():
        want = case[name]
        X, ipiv, jpiv, res = oracle.gj_invert_rule_f64(A, rule)
        assert res["code"] == want["code"], name
        assert ipiv.tolist() == want["ipiv"] and jpiv.tolist() == want["jpiv"], name
        if want["code"] == 0:
            assert res["det"] == want["det"], name
            if "inverse" in want:
                assert np.array_equal(X, np.array(want["inverse"])), name
        else:
            assert res["rank"] == want["rank"] and np.isnan(X).all(), name


def test_partial_rule_matches_lapack_getrf():
    """Partial pivoting on |a| picks, step by step, the rows LAPACK's getrf
    (partial-pivoting LU) picks; no column is swapped.  The full rule with the
    same inputs is the default entry point, bit for bit."""
    from scipy.linalg import lu_factor
    rng = inputs.rng_for(0, 740)
    for _ in range(10):
        n = int(rng.integers(2, 40))
        A = rng.standard_normal((n, n))
        X, ipiv, jpiv, res = oracle.gj_invert_rule_f64(A, 1)
        _, piv = lu_factor(A)
        assert np.array_equal(ipiv, piv) and np.array_equal(jpiv, np.arange(n))
        assert oracle.residual(A, X) <= 10 * n * 2.0 ** -53
        X0, i0, j0, r0 = oracle.gj_invert_rule_f64(A, 0)
        X1, i1, j1, r1 = oracle.gj_invert_f64(A)
        assert X0.tobytes() == X1.tobytes() and np.array_equal(i0, i1) and np.array_equal(j0, j1)


def test_program_rule_loses_accuracy_where_max_abs_does_not():
    """The conclusion's claim: bringing the largest |a| to the pivot position
    reduces rounding error.  The program's rule takes the only positive entry
    of a column however small it is: with tiny positive diagonal entries and
    negative off-diagonal ones its pivots are tiny, the elements grow, and its
    forward error (against the long-double run) is orders of magnitude above
    that of either |a|-maximising rule."""
    rng = inputs.rng_for(0, 741)
    n = 12
    A = -np.abs(rng.standard_normal((n, n)))
    np.fill_diagonal(A, 1e-6)
    Xt, _, _, rt = oracle.gj_invert_f80(A)
    assert rt["code"] == 0
    err = {}
    for name, rule in RULES.items():
        X, ipiv, _, res = oracle.gj_invert_rule_f64(A, rule)
        assert res["code"] == 0, name
        err[name] = np.abs(X - Xt).max() / np.abs(Xt).max()
    assert err["full"] <= 1e-13 and err["partial"] <= 1e-13, err
    assert err["program"] >= 1e4 * max(err["full"], err["partial"]), err


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_forward_error_against_long_double(cond):
    n = 48
    A = inputs.conditioned(n, cond, inputs.rng_for(0, 800))
    X, ipiv, jpiv, _ = oracle.gj_invert_f64(A)
    Xt, ipiv_t, jpiv_t, _ = oracle.gj_invert_f80(A)
    err = np.linalg.norm(X - Xt) / np.linalg.norm(Xt)
    assert err <= 4 * n * cond * U64
    # the long double run itself is far more accurate: compare with scipy's inverse
    assert np.linalg.norm(Xt - np.linalg.inv(A)) / np.linalg.norm(Xt) <= 8 * n * cond * U64


def test_float_model_matches_its_precision():
    A = inputs.conditioned(40, 1e3, inputs.rng_for(0, 900))
    X32, _, _, res = oracle.gj_invert_f32(A.astype(np.float32))
    assert X32.dtype == np.float32 and res["code"] == 0
    r = oracle.residual(A.astype(np.float32).astype(np.float64), X32)
    assert r <= 10 * 40 * 2.0 ** -24


def test_nonfinite_and_threshold():
    A = np.eye(4)
    A[2, 1] = np.nan
    X, ipiv, _, res = oracle.gj_invert_f64(A)
    assert res["code"] == 2 and res["rank"] == 0 and np.isnan(X).all() and ipiv[0] == -1
    A = np.eye(4)
    A[3, 0] = np.inf
    assert oracle.gj_invert_f64(A)[3]["code"] == 2
    # tiny but non-zero pivot: singular under the default threshold, not under tau = 0
    B = np.diag([1.0, 1.0, 1.0, 1e-17])
    assert oracle.gj_invert_f64(B)[3]["code"] == 1
    X, _, _, res = oracle.gj_invert_f64(B, zero_tol=0.0)
    assert res["code"] == 0 and X[3, 3] == 1e17


def test_lu_static_det_agrees():
    rng = inputs.rng_for(0, 1000)
    for _ in range(10):
        n = int(rng.integers(2, 40))
        A = rng.standard_normal((n, n))
        _, ipiv, jpiv, res = oracle.gj_invert_f64(A)
        lu = oracle.lu_static_det_f64(A, ipiv, jpiv)
        assert lu["det_sign"] == res["det_sign"]
        assert abs(lu["logabsdet"] - res["logabsdet"]) <= 1e-12 * max(1.0, abs(res["logabsdet"]))
    # exact on a diagonal matrix with swaps
    D = np.diag([2.0, -5.0, 0.5, 5.0])
    lu = oracle.lu_static_det_f64(D, [1, 3, 3, 3], [1, 3, 3, 3])
    assert lu["det"] == -25.0


def test_conditioned_generator_closed_form_logdet():
    n, cond = 64, 1e6
    A = inputs.conditioned(n, cond, inputs.rng_for(0, 1100))
    _, _, _, res = oracle.gj_invert_f64(A)
    assert res["det_sign"] == 1
    assert abs(res["logabsdet"] - inputs.closed_form_logdet(n, cond)) <= 1e-9 * n * math.log(cond)


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_newton_schulz_squares_the_residual(cond):
    """One update maps R to R^2 (X' = X + X R gives I - A X' = R^2), and the
    iteration from an FP32 inverse reaches the FP64 oracle's accuracy."""
    n = 64
    A = inputs.conditioned(n, cond, inputs.rng_for(0, 1200))
    X32, _, _, _ = oracle.gj_invert_f32(A.astype(np.float32))
    X0 = X32.astype(np.float64)
    R0 = np.eye(n) - A @ X0
    X1 = X0 + X0 @ R0
    R1 = np.eye(n) - A @ X1
    assert np.linalg.norm(R1 - R0 @ R0) <= 64 * n * U64 * np.linalg.norm(A) * np.linalg.norm(X1)
    X, updates, norms, accepted = oracle.newton_schulz(A, X0)
    assert accepted and 1 <= updates <= 6
    Xt, _, _, _ = oracle.gj_invert_f80(A)
    Xo, _, _, _ = oracle.gj_invert_f64(A)
    err_ns = np.linalg.norm(X - Xt) / np.linalg.norm(Xt)
    err_or = np.linalg.norm(Xo - Xt) / np.linalg.norm(Xt)
    assert err_ns <= 2 * max(err_or, 1e-14)


def _ns_diag_case(e, d, max_iters=10):
    """A = diag(d), X0 = diag((1 - e_i) / d_i): R_0 = I - A X0 = diag(e_i),
    and each update squares it, R_k = diag(e_i^(2^k)).  With d_i powers of
    two and e_i dyadic, every operation is exact until 1 - e_i^(2^k) needs
    more than 53 bits; R becomes exactly 0 once e_i^(2^k) < 2^-54 (1 - e
    then rounds to 1)."""
    A = np.diag(np.asarray(d, dtype=np.float64))
    X0 = np.diag((1.0 - np.asarray(e, dtype=np.float64)) / np.asarray(d, dtype=np.float64))
    return oracle.newton_schulz(A, X0, max_iters=max_iters)


def test_newton_schulz_stop_rule_slow_start_below_one():
    """||R_0||_F = 7/8: the exact norms are (7/8)^(2^k) = 0.875, 0.766, 0.586,
    0.344, 0.118, 0.0139, 1.9e-4, 3.8e-8, 1.4e-15 (k = 0..8), every kept
    update within the quadratic bound, and R_9 = 0 exactly ((7/8)^512 <
    2^-54).  So exactly 9 updates, ending at 0, accepted.  An update from
    0.875 to 0.766 does not halve the norm: a rule that stops at the first
    such update below 1 would keep 1 update and fall back."""
    X, updates, norms, accepted = _ns_diag_case([0.875], [2.0])
    assert updates == 9 and accepted and norms[-1] == 0.0
    for k in range(5):                       # exact while (7/8)^(2^k) fits 53 bits
        assert norms[k] == 0.875 ** (2 ** k)
    assert X[0, 0] == 0.5                    # the exact inverse


def test_newton_schulz_stop_rule_slow_fall_above_one():
    """Sixteen diagonal entries with e = 7/8: ||R_k||_F = 4 (7/8)^(2^k) =
    3.5, 3.06, 2.34, 1.37, 0.47, 0.056, 7.8e-4, 1.5e-7, 5.7e-15, then 0:
    9 updates, accepted, although the first three fall by less than half."""
    X, updates, norms, accepted = _ns_diag_case([0.875] * 16, [4.0] * 16)
    assert updates == 9 and accepted and norms[-1] == 0.0
    assert norms[0] == 3.5 and 3.0 < norms[1] < 3.1
    assert np.array_equal(X, np.eye(16) / 4.0)


def test_newton_schulz_accept_threshold():
    """e = 1/2: ||R_k|| = 2^-(2^k).  Capped at 3 updates the loop ends at
    2^-8 <= 1e-2 (accepted); capped at 2 it ends at 2^-4 > 1e-2 (not
    accepted: the caller falls back to the FP64 elimination)."""
    _, updates, norms, accepted = _ns_diag_case([0.5], [1.0], max_iters=3)
    assert updates == 3 and norms == [0.5, 0.25, 0.0625, 2.0 ** -8] and accepted
    _, updates, norms, accepted = _ns_diag_case([0.5], [1.0], max_iters=2)
    assert updates == 2 and norms[-1] == 0.0625 and not accepted


def test_newton_schulz_no_progress_keeps_previous_iterate():
    """X0 = 2 A^-1 (A = diag(4)): R_0 = -1, and X1 = X0 + X0 R0 = 0 gives
    R_1 = I, no decrease: no update is kept and X0 is returned."""
    A = np.diag([4.0])
    X0 = np.diag([0.5])
    X, updates, norms, accepted = oracle.newton_schulz(A, X0)
    assert updates == 0 and norms == [1.0, 1.0] and not accepted
    assert X[0, 0] == 0.5


@pytest.mark.parametrize("cond", [1e2, 1e6, 1e8])
def test_exact_residual_against_rationals(cond):
    """I - A X from bit-slice products equals the exact rational residual of
    the two FP64 matrices, rounded (n = 10; every double is a rational)."""
    n = 10
    A = inputs.conditioned(n, cond, inputs.rng_for(0, 1400))
    X, _, _, _ = oracle.gj_invert_f64(A)
    R = oracle.exact_residual(A, X)
    Fa = [[Fraction(float(v)) for v in row] for row in A]
    Fx = [[Fraction(float(v)) for v in row] for row in X]
    for i in range(n):
        for j in range(n):
            exact = Fraction(int(i == j)) - sum(Fa[i][k] * Fx[k][j] for k in range(n))
            assert abs(Fraction(float(R[i, j])) - exact) <= abs(exact) * Fraction(2, 2 ** 52), (i, j)


def test_inverse_truth_exact_and_against_long_double():
    """On A = H D H^T (H Sylvester-Hadamard, D powers of two spanning 2^20)
    A^-1 = H D^-1 H^T / n^2 is exact in FP64, and the Newton steps with the
    exact residual reach it from the FP64 oracle's inverse (error 1e-11).  On
    a U diag(s) V^T matrix they agree with the long-double elimination far
    below the FP64 oracle's own error."""
    n = 256
    H = inputs.sylvester_hadamard(n)
    e = inputs.rng_for(0, 1410).integers(0, 21, n)
    e[0], e[1] = 0, 20
    A = (H * np.ldexp(1.0, e)) @ H.T
    Ainv = (H * np.ldexp(1.0, -e)) @ H.T / float(n * n)
    Xo, _, _, _ = oracle.gj_invert_f64(A)
    assert np.linalg.norm(Xo - Ainv) > 1e-13 * np.linalg.norm(Ainv)
    T = oracle.inverse_truth(A, Xo)
    assert np.linalg.norm(T - Ainv) <= 2 * U64 * np.linalg.norm(Ainv)
    A = inputs.conditioned(150, 1e6, inputs.rng_for(0, 1420))
    Xo, _, _, _ = oracle.gj_invert_f64(A)
    Xt, _, _, _ = oracle.gj_invert_f80(A)
    T = oracle.inverse_truth(A, Xo)
    err_o = np.linalg.norm(Xo - Xt) / np.linalg.norm(Xt)
    assert np.linalg.norm(T - Xt) / np.linalg.norm(Xt) <= max(1e-3 * err_o, 1e-14)


def test_pivots_to_permutations():
    A = inputs.rng_for(0, 1300).standard_normal((12, 12))
    X, ipiv, jpiv, _ = oracle.gj_invert_f64(A)
    rows, cols = oracle.perms_from_pivots(ipiv, jpiv)
    B = A[rows][:, cols]
    # after the permutation, no search is needed: the diagonal is the pivot order
    Xb, ipiv_b, jpiv_b, _ = oracle.gj_invert_f64(B)
    assert ipiv_b.tolist() == list(range(12)) and jpiv_b.tolist() == list(range(12))
    assert np.array_equal(Xb, X[cols][:, rows])
