"""Planted mistakes: each mutant is a copy of the oracle's C source with one
plausible error (a flipped sign, a dropped term, a wrong index, a transposed
operand, a different tie-break or pivot rule), compiled on the CPU.  The pin
battery below -- the same kinds of check as test_oracle_pins.py -- must
reject every one of them, which shows the pins can tell a wrong oracle from
the right one.  The product library is not involved."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1401_7962_amd import inputs

SRC = os.path.join(os.path.dirname(oracle.__file__), "gj_oracle.c")

MUTANTS = {
    "tie_break_last_max": ("if (v > best) { best = v; r = i; c = j; }",
                           "if (v >= best) { best = v; r = i; c = j; }"),
    "eq15_sign": ("W[(int64_t)i * n + j] = FMA(-q,", "W[(int64_t)i * n + j] = FMA(q,"),
    "eq15_transposed": ("FMA(-q, W[(int64_t)k * n + j],", "FMA(-q, W[(int64_t)j * n + k],"),
    "pivot_column_not_cleared": ("W[(int64_t)i * n + k] = (T)0;", "(void)0;"),
    "pivot_slot_not_one": ("W[(int64_t)k * n + k] = (T)1;", "(void)0;"),
    "unscramble_roles_swapped": ("int r = ipiv[k], c = jpiv[k];", "int r = jpiv[k], c = ipiv[k];"),
    "det_sign_flipped": ("res->det_sign = (m_acc < 0) ? -sign : sign;",
                         "res->det_sign = (m_acc < 0) ? sign : -sign;"),
    "partial_pivoting": ("for (int j = k; j < n; ++j) {", "for (int j = k; j <= k; ++j) {"),
    "search_includes_done_rows": ("for (int i = k; i < n; ++i)                                                \\",
                                  "for (int i = 0; i < n; ++i)                                                \\"),
    "no_zero_test": ("if (best == (T)0 || best < tau) {", "if (best < tau) {"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(so), str(c), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    fn = lib.ora_gj_invert_f64
    P = ctypes.c_void_p
    fn.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, P, P, P,
                   ctypes.POINTER(oracle.OraResult)]
    return fn


def _invert(fn, A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    X = np.empty_like(A)
    ipiv = np.full(n, -1, np.int32)
    jpiv = np.full(n, -1, np.int32)
    res = oracle.OraResult()
    fn(n, A.ctypes.data_as(ctypes.c_void_p), n, -1.0, X.ctypes.data_as(ctypes.c_void_p),
       ipiv.ctypes.data_as(ctypes.c_void_p), jpiv.ctypes.data_as(ctypes.c_void_p),
       ctypes.byref(res))
    return X, ipiv, jpiv, res.as_dict()


def _pin_battery(fn):
    """Returns the list of pins that fail."""
    failed = []
    with np.errstate(all="ignore"):
        P = inputs.pascal(3)
        X, ipiv, jpiv, res = _invert(fn, P)
        if not (np.array_equal(np.rint(X), [[3, -3, 1], [-3, 5, -2], [1, -2, 1]])
                and ipiv.tolist() == [2, 2, 2] and jpiv.tolist() == [2, 2, 2]
                and res["det_sign"] == 1):
            failed.append("pascal3")
        H = inputs.sylvester_hadamard(8)
        X, ipiv, jpiv, res = _invert(fn, H)
        if not (np.array_equal(X, H.T / 8) and ipiv.tolist() == list(range(8))):
            failed.append("hadamard8")
        s = [2, 0, 3, 1]
        Pm = np.zeros((4, 4))
        Pm[np.arange(4), s] = 1
        X, ipiv, jpiv, res = _invert(fn, Pm)
        if not (np.array_equal(X, Pm.T) and res["det"] == -1 and jpiv.tolist() == [2, 2, 3, 3]):
            failed.append("permutation")
        X, ipiv, jpiv, res = _invert(fn, np.zeros((3, 3)))
        if not (res["code"] == 1 and res["rank"] == 0):
            failed.append("zero_matrix")
        from scipy.linalg import lapack
        rng = inputs.rng_for(0, 77)
        for t in range(5):
            n = int(rng.integers(3, 16))
            A = rng.standard_normal((n, n))
            X, ipiv, jpiv, res = _invert(fn, A)
            _, il, jl, _ = lapack.dgetc2(A)
            if not (np.isfinite(X).all() and oracle.residual(A, X) <= 10 * n * 2.0 ** -53):
                failed.append(f"residual{t}")
                break
            if not (np.array_equal(ipiv, il) and np.array_equal(jpiv, jl)):
                failed.append(f"dgetc2_{t}")
                break
            if res["det_sign"] != np.linalg.slogdet(A)[0]:
                failed.append(f"det_sign{t}")
                break
    return failed


def test_unmutated_source_passes_battery(tmp_path):
    fn = _build(tmp_path, "identity", "#include <math.h>", "#include <math.h>")
    assert _pin_battery(fn) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    fn = _build(tmp_path, name, old, new)
    failed = _pin_battery(fn)
    assert failed, f"mutant {name} passed every pin"


# Planted mistakes in the right-hand-side half of the augmented elimination
# (the solve); checked by a battery of the solve pins' kinds.
SOLVE_MUTANTS = {
    "rhs_not_divided": ("for (int j = 0; j < m; ++j) d[(int64_t)k * m + j] = d[(int64_t)k * m + j] / p;",
                        "(void)0;"),
    "rhs_not_row_swapped": ("                double t = d[(int64_t)k * m + j];\n                d[(int64_t)k * m + j] = d[(int64_t)r * m + j];",
                            "                double t = d[(int64_t)k * m + j];\n                d[(int64_t)k * m + j] = d[(int64_t)k * m + j];"),
    "no_final_row_permutation": ("for (int k = n - 1; k >= 0; --k) {                                              /* A^-1 B = Q D */",
                                 "for (int k = n - 1; k >= 0 && 0; --k) {"),
    "rhs_update_sign": ("d[(int64_t)i * m + j] = fma(-q, d[(int64_t)k * m + j], d[(int64_t)i * m + j]);",
                        "d[(int64_t)i * m + j] = fma(q, d[(int64_t)k * m + j], d[(int64_t)i * m + j]);"),
}


def _build_solve(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(so), str(c), "-lm"], check=True)
    fn = ctypes.CDLL(str(so)).ora_gj_solve_f64
    P = ctypes.c_void_p
    fn.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int64,
                   ctypes.c_double, P, ctypes.c_int64, P, P, ctypes.POINTER(oracle.OraResult)]
    return fn


def _solve(fn, A, B):
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    n, m = A.shape[0], B.shape[1]
    X = np.empty((n, m))
    ipiv = np.full(n, -1, np.int32)
    jpiv = np.full(n, -1, np.int32)
    res = oracle.OraResult()
    P = ctypes.c_void_p
    fn(n, m, A.ctypes.data_as(P), n, B.ctypes.data_as(P), m, -1.0, X.ctypes.data_as(P), m,
       ipiv.ctypes.data_as(P), jpiv.ctypes.data_as(P), ctypes.byref(res))
    return X, res.as_dict()


def _solve_battery(fn):
    failed = []
    with np.errstate(all="ignore"):
        rng = inputs.rng_for(0, 711)
        B = rng.integers(-50, 50, size=(4, 3)).astype(np.float64)
        Pm = np.zeros((4, 4))
        Pm[np.arange(4), [2, 0, 3, 1]] = 1
        X, res = _solve(fn, Pm, B)
        if not np.array_equal(X, Pm.T @ B):
            failed.append("permutation")
        D = np.diag([2.0, -0.25, 8.0, 0.5])
        X, res = _solve(fn, D, B)
        if not np.array_equal(X, B / np.diag(D)[:, None]):
            failed.append("diagonal")
        A = rng.standard_normal((12, 12))
        Bn = rng.standard_normal((12, 3))
        X, res = _solve(fn, A, Bn)
        if not (res["code"] == 0 and np.abs(A @ X - Bn).max() <= 1e-12 * np.abs(Bn).max() * np.linalg.cond(A)):
            failed.append("residual")
    return failed


def test_unmutated_solve_passes_battery(tmp_path):
    fn = _build_solve(tmp_path, "solve_identity", "#include <math.h>", "#include <math.h>")
    assert _solve_battery(fn) == []


@pytest.mark.parametrize("name", sorted(SOLVE_MUTANTS))
def test_solve_mutant_is_caught(tmp_path, name):
    old, new = SOLVE_MUTANTS[name]
    fn = _build_solve(tmp_path, name, old, new)
    assert _solve_battery(fn), f"mutant {name} passed every pin"


# Planted mistakes in the other pivot rules, checked by the golden cases
# worked by hand for each rule.
RULE_MUTANTS = {
    "program_rule_on_abs": ("} else if (v > q) {", "} else if (FABS(v) > q) {"),
    "partial_rule_last_max": ("if (FABS(v) > best) { best = FABS(v); r = i; }",
                              "if (FABS(v) >= best) { best = FABS(v); r = i; }"),
    "partial_rule_full_threshold": ("tau = (rule == 0) ? (T)n * (T)(EPS_DEFAULT) * best : (T)0;",
                                    "tau = (T)n * (T)(EPS_DEFAULT) * best;"),
}


def _build_rule(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(so), str(c), "-lm"], check=True)
    fn = ctypes.CDLL(str(so)).ora_gj_invert_f64_rule
    P = ctypes.c_void_p
    fn.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int, P, P, P,
                   ctypes.POINTER(oracle.OraResult)]
    return fn


def _rule_battery(fn):
    import json
    cases = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pivot_rules.json")))["cases"]
    failed = []
    P = ctypes.c_void_p
    with np.errstate(all="ignore"):
        for case in cases:
            A = np.ascontiguousarray(case["A"], dtype=np.float64)
            n = A.shape[0]
            for name, rule in (("partial", 1), ("program", 2)):
                want = case[name]
                X = np.empty_like(A)
                ipiv = np.full(n, -1, np.int32)
                jpiv = np.full(n, -1, np.int32)
                res = oracle.OraResult()
                fn(n, A.ctypes.data_as(P), n, -1.0, rule, X.ctypes.data_as(P),
                   ipiv.ctypes.data_as(P), jpiv.ctypes.data_as(P), ctypes.byref(res))
                if res.code != want["code"] or ipiv.tolist() != want["ipiv"]:
                    failed.append(f"{case['name']}/{name}")
        # a later pivot far below n * 2^-52 * (first pivot), but nonzero: not
        # singular without a preset threshold
        A = np.array([[1.0, 0.0], [0.0, 1e-300]])
        X = np.empty_like(A)
        ipiv = np.full(2, -1, np.int32)
        jpiv = np.full(2, -1, np.int32)
        res = oracle.OraResult()
        fn(2, A.ctypes.data_as(P), 2, -1.0, 1, X.ctypes.data_as(P), ipiv.ctypes.data_as(P),
           jpiv.ctypes.data_as(P), ctypes.byref(res))
        if res.code != 0:
            failed.append("tiny_pivot")
    return failed


def test_unmutated_rules_pass_battery(tmp_path):
    fn = _build_rule(tmp_path, "rule_identity", "#include <math.h>", "#include <math.h>")
    assert _rule_battery(fn) == []


@pytest.mark.parametrize("name", sorted(RULE_MUTANTS))
def test_rule_mutant_is_caught(tmp_path, name):
    old, new = RULE_MUTANTS[name]
    fn = _build_rule(tmp_path, name, old, new)
    assert _rule_battery(fn), f"mutant {name} passed every pin"


# Planted mistakes in the Newton-Schulz stopping rule (Python source of
# oracle.newton_schulz, rewritten and re-executed).  The exact diagonal pins
# of test_oracle_pins.py must reject each one.
NS_MUTANTS = {
    # the floor test applied whenever ||R|| < 1 (halving only)
    "halving_below_one": ("rn > max(stall * prev, 2.0 * prev * prev)",
                          "(prev < 1.0 and rn > stall * prev)"),
    # the floor test applied at any norm, above 1 too
    "halving_above_one": ("rn > max(stall * prev, 2.0 * prev * prev)", "rn > stall * prev"),
    # a much stricter acceptance threshold
    "accept_1e-6": ("accepted = bool(np.isfinite(r) and r <= accept)",
                    "accepted = bool(np.isfinite(r) and r <= 1e-6)"),
    # a rejected update replaces the iterate anyway
    "keep_failed_update": ("if not rn < r:\n                break",
                           "if not rn < r:\n                X, R, r = Xn, Rn, rn\n                break"),
}


def _ns_mutant(name):
    import inspect
    import textwrap
    old, new = NS_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(oracle.newton_schulz))
    assert old in src, f"mutation anchor for {name} not found"
    ns = {"np": np}
    exec(compile(src.replace(old, new), f"<ns mutant {name}>", "exec"), ns)
    return ns["newton_schulz"]


def _ns_battery(fn):
    """The exact diagonal cases of the stopping-rule pins; returns the failing ones."""
    failed = []

    def case(e, d, max_iters=10):
        A = np.diag(np.asarray(d, dtype=np.float64))
        X0 = np.diag((1.0 - np.asarray(e)) / np.asarray(d, dtype=np.float64))
        return fn(A, X0, max_iters=max_iters)

    _, u, norms, acc = case([0.875], [2.0])
    if not (u == 9 and acc and norms[-1] == 0.0):
        failed.append("slow_start_below_one")
    _, u, norms, acc = case([0.875] * 16, [4.0] * 16)
    if not (u == 9 and acc and norms[-1] == 0.0):
        failed.append("slow_fall_above_one")
    _, u, norms, acc = case([0.5], [1.0], max_iters=3)
    if not (u == 3 and acc):
        failed.append("accept_threshold")
    X, u, norms, acc = fn(np.diag([4.0]), np.diag([0.5]))
    if not (u == 0 and X[0, 0] == 0.5):
        failed.append("no_progress")
    return failed


def test_unmutated_newton_schulz_passes_battery():
    assert _ns_battery(oracle.newton_schulz) == []


@pytest.mark.parametrize("name", sorted(NS_MUTANTS))
def test_newton_schulz_mutant_is_caught(name):
    assert _ns_battery(_ns_mutant(name)), f"mutant {name} passed every stopping-rule pin"


# Planted mistakes in the exact residual (Python source of
# oracle.exact_residual): a dropped slice product, the last slice of A lost,
# the diagonal's I dropped.
RESID_MUTANTS = {
    "dropped_product": ("if i + j > 0)", "if 0 < i + j < 4)"),
    "remainder_dropped": ("As = _slices(A, 1, bits, 3)", "As = _slices(A, 1, bits, 2) + [0.0 * A]"),
    "no_identity": ("R = np.eye(n) - As[0] @ Xs[0]", "R = -(As[0] @ Xs[0])"),
}


@pytest.mark.parametrize("name", sorted(RESID_MUTANTS))
def test_exact_residual_mutant_is_caught(name):
    import inspect
    import textwrap
    from fractions import Fraction
    old, new = RESID_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(oracle.exact_residual))
    assert old in src, f"mutation anchor for {name} not found"
    ns = {"np": np, "_slices": oracle._slices}
    exec(compile(src.replace(old, new), f"<resid mutant {name}>", "exec"), ns)
    fn = ns["exact_residual"]
    n = 10
    A = inputs.conditioned(n, 1e6, inputs.rng_for(0, 1400))
    X, _, _, _ = oracle.gj_invert_f64(A)
    R = fn(A, X)
    worst = Fraction(0)
    for i in range(n):
        for j in range(n):
            exact = Fraction(int(i == j)) - sum(Fraction(float(A[i, k])) * Fraction(float(X[k, j]))
                                                for k in range(n))
            if exact != 0:
                worst = max(worst, abs(Fraction(float(R[i, j])) - exact) / abs(exact))
    assert worst > Fraction(2, 2 ** 52), f"mutant {name} passed the exact-residual pin"
