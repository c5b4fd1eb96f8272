"""CPU oracle for full-pivot Gauss-Jordan inversion -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it,
and it shares no code with the HIP path: the only thing the two have in
common is the seeded inputs they are handed.

The arithmetic lives in ``gj_oracle.c`` (plain C, one element at a time,
correctly rounded division and one ``fma`` per eq. 15 element, following the
paper's section 2: eqs. 1-2 initialisation, Obs. 2-3 pivot search and swaps,
eq. 14 pivot-row scaling, eq. 15 elimination, eq. 13 determinant, Obs. 3
depivoting).  This module loads it through ctypes and adds the few pieces
that are plain definitions written out in NumPy / Python:

* ``newton_schulz`` -- the refinement X <- X + X (I - A X), matmul as the
  only library step (parity: pinned by the contraction property
  R_{k+1} = R_k^2 checked in the tests);
* ``residual`` -- ||A X - I||_F / (||A||_F ||X||_F);
* ``exact_residual`` / ``inverse_truth`` -- I - A X with the large products
  formed exactly from bit slices, and Newton steps with it: a reference
  inverse for forward errors at orders where the long-double elimination is
  too slow (pinned against that elimination and against exact inverses);
* ``cofactor_det`` -- exact rational Laplace expansion (n <= 7), the
  brute-force determinant pin;
* ``gj_solve_f64`` -- the augmented elimination with a general right-hand
  side B in place of I (eq. 2), giving A^-1 B;
* ``perms_from_pivots`` -- original-index permutations from ipiv / jpiv.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gj_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RES_OK, RES_SINGULAR, RES_NONFINITE, RES_REFINE_FALLBACK = 0, 1, 2, 3


class OraResult(ctypes.Structure):
    _fields_ = [
        ("code", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("det_sign", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("det_mant", ctypes.c_double),
        ("det_exp", ctypes.c_int64),
        ("det", ctypes.c_double),
        ("logabsdet", ctypes.c_double),
        ("resid", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        for name in ("ora_gj_invert_f64", "ora_gj_invert_f32", "ora_gj_invert_f80",
                     "ora_gj_augmented_f64"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, P, P, P,
                           ctypes.POINTER(OraResult)]
            fn.restype = ctypes.c_int
        lib.ora_gj_invert_f64_rule.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double,
                                               ctypes.c_int, P, P, P, ctypes.POINTER(OraResult)]
        lib.ora_gj_invert_f64_rule.restype = ctypes.c_int
        for name in ("ora_gj_invert_f64_first_steps", "ora_gj_invert_f32_first_steps"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, P, P, P,
                           ctypes.POINTER(OraResult), ctypes.c_int, P]
            fn.restype = ctypes.c_int
        lib.ora_gj_solve_f64.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int64, P,
                                         ctypes.c_int64, ctypes.c_double, P, ctypes.c_int64,
                                         P, P, ctypes.POINTER(OraResult)]
        lib.ora_gj_solve_f64.restype = ctypes.c_int
        lib.ora_lu_static_det_f64.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P,
                                              ctypes.POINTER(OraResult)]
        lib.ora_lu_static_det_f64.restype = ctypes.c_int
        lib.ora_gj_invert_f64_par.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, P,
                                              P, P, ctypes.POINTER(OraResult), ctypes.c_int,
                                              ctypes.c_int]
        lib.ora_gj_invert_f64_par.restype = ctypes.c_int
        lib.ora_gj_invert_f32_par.argtypes = lib.ora_gj_invert_f64_par.argtypes
        lib.ora_gj_invert_f32_par.restype = ctypes.c_int
        lib.ora_gj_invert_f80_par.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, P,
                                              P, P, ctypes.POINTER(OraResult), ctypes.c_int]
        lib.ora_gj_invert_f80_par.restype = ctypes.c_int
        lib.ora_gj_invert_batched.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, P,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_int]
        lib.ora_gj_invert_batched.restype = ctypes.c_int
        lib.ora_result_size.restype = ctypes.c_int
        assert lib.ora_result_size() == ctypes.sizeof(OraResult)
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _run(fname: str, A: np.ndarray, zero_tol: float, in_dtype, out_dtype):
    A = np.ascontiguousarray(A, dtype=in_dtype)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    X = np.empty((n, n), dtype=out_dtype)
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    res = OraResult()
    getattr(_load(), fname)(n, _ptr(A), n, float(zero_tol), _ptr(X), _ptr(ipiv), _ptr(jpiv),
                            ctypes.byref(res))
    return X, ipiv, jpiv, res.as_dict()


def gj_invert_f64(A, zero_tol: float = -1.0):
    """FP64 in-place full-pivot GJ.  Returns (X, ipiv, jpiv, result dict)."""
    return _run("ora_gj_invert_f64", A, zero_tol, np.float64, np.float64)


PIVOT_FULL, PIVOT_PARTIAL, PIVOT_PROGRAM = 0, 1, 2


def gj_invert_rule_f64(A, rule: int, zero_tol: float = -1.0):
    """FP64 in-place GJ with another pivot rule: PIVOT_PARTIAL (largest |a|
    in column k, row swaps only) or PIVOT_PROGRAM (the section-3 program's
    largest positive value in column k, else row k).  No preset threshold for
    these two: with zero_tol < 0 only a zero pivot is singular."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    X = np.empty((n, n))
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    res = OraResult()
    _load().ora_gj_invert_f64_rule(n, _ptr(A), n, float(zero_tol), int(rule), _ptr(X), _ptr(ipiv),
                                   _ptr(jpiv), ctypes.byref(res))
    return X, ipiv, jpiv, res.as_dict()


def host_threads() -> int:
    """Host cores this process may run on, capped by OMP_NUM_THREADS when set."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def gj_invert_f64_par(A, nthreads: int | None = None, zero_tol: float = -1.0,
                      max_steps: int | None = None):
    """The FP64 oracle with each step's row work shared among ``nthreads``
    OpenMP threads (bitwise the serial result).  ``max_steps`` < n stops
    after that many steps with no depivoting (a timing sample).  Returns
    (X, ipiv, jpiv, result dict)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    X = np.empty((n, n))
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    res = OraResult()
    code = _load().ora_gj_invert_f64_par(n, _ptr(A), n, float(zero_tol), _ptr(X), _ptr(ipiv),
                                         _ptr(jpiv), ctypes.byref(res),
                                         int(nthreads or host_threads()),
                                         n if max_steps is None else int(max_steps))
    if code < 0:
        raise MemoryError("oracle: allocation failed")
    return X, ipiv, jpiv, res.as_dict()


def gj_invert_f32_par(A, nthreads: int | None = None, zero_tol: float = 0.0):
    """The FP32 model on ``nthreads`` threads (bitwise the serial FP32 model)."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    n = A.shape[0]
    X = np.empty((n, n), dtype=np.float32)
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    res = OraResult()
    code = _load().ora_gj_invert_f32_par(n, _ptr(A), n, float(zero_tol), _ptr(X), _ptr(ipiv),
                                         _ptr(jpiv), ctypes.byref(res),
                                         int(nthreads or host_threads()), n)
    if code < 0:
        raise MemoryError("oracle: allocation failed")
    return X, ipiv, jpiv, res.as_dict()


def gj_invert_f80_par(A, nthreads: int | None = None, zero_tol: float = -1.0):
    """The long-double oracle on ``nthreads`` threads (bitwise the serial
    long-double result)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    X = np.empty((n, n))
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    res = OraResult()
    code = _load().ora_gj_invert_f80_par(n, _ptr(A), n, float(zero_tol), _ptr(X), _ptr(ipiv),
                                         _ptr(jpiv), ctypes.byref(res),
                                         int(nthreads or host_threads()))
    if code < 0:
        raise MemoryError("oracle: allocation failed")
    return X, ipiv, jpiv, res.as_dict()


def gj_invert_batched(sizes, offs, packed, nthreads: int | None = None, zero_tol: float = -1.0,
                      fp32: bool = False):
    """One serial oracle run per member of a packed batch (member b: order
    sizes[b] at packed[offs[b]:], ld sizes[b]), members shared among
    ``nthreads`` OpenMP threads.  ``fp32``: the FP32 model instead of FP64.
    Returns (X packed like the input, ipiv, jpiv (concatenated in member
    order), list of result dicts)."""
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    packed = np.ascontiguousarray(packed, dtype=np.float64)
    batch = len(sizes)
    if batch and int(offs[-1]) + int(sizes[-1]) ** 2 > packed.size:
        raise ValueError("packed buffer too short for the last member")
    poff = np.zeros(batch, dtype=np.int64)
    poff[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    X = np.full(packed.size, np.nan)
    ipiv = np.full(int(sizes.sum()), -1, dtype=np.int32)
    jpiv = np.full(int(sizes.sum()), -1, dtype=np.int32)
    res = (OraResult * max(batch, 1))()
    code = _load().ora_gj_invert_batched(batch, _ptr(sizes), _ptr(offs), _ptr(packed), _ptr(X),
                                         _ptr(poff), _ptr(ipiv), _ptr(jpiv), res,
                                         float(zero_tol), 1 if fp32 else 0,
                                         int(nthreads or host_threads()))
    if code < 0:
        raise MemoryError("oracle: allocation failed")
    return X, ipiv, jpiv, [res[b].as_dict() for b in range(batch)]


def gj_invert_f32(A, zero_tol: float = 0.0):
    """FP32 model of the same algorithm (default zero threshold: exact 0)."""
    return _run("ora_gj_invert_f32", A, zero_tol, np.float32, np.float32)


def gj_invert_f80(A, zero_tol: float = -1.0):
    """Same algorithm in x87 long double (u = 2^-64); X rounded to double."""
    return _run("ora_gj_invert_f80", A, zero_tol, np.float64, np.float64)


def gj_augmented_f64(A, zero_tol: float = -1.0):
    """Literal eqs. 1-2, 14-15 on separate A and D arrays."""
    return _run("ora_gj_augmented_f64", A, zero_tol, np.float64, np.float64)


def gj_solve_f64(A, B, zero_tol: float = -1.0):
    """X = A^-1 B by the augmented elimination with D^0 = B (eqs. 1-2, 14-15;
    column swaps undone as row swaps of D).  B is n x m.  Returns
    (X, ipiv, jpiv, result dict); X is all NaN when the run stops early."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    if A.ndim != 2 or A.shape[0] != A.shape[1] or B.ndim != 2 or B.shape[0] != A.shape[0]:
        raise ValueError("A must be n x n and B n x m")
    n, m = A.shape[0], B.shape[1]
    X = np.empty((n, m), dtype=np.float64)
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    res = OraResult()
    code = _load().ora_gj_solve_f64(n, m, _ptr(A), n, _ptr(B), m, float(zero_tol), _ptr(X), m,
                                    _ptr(ipiv), _ptr(jpiv), ctypes.byref(res))
    if code < 0:
        raise MemoryError("oracle solve: allocation failed")
    return X, ipiv, jpiv, res.as_dict()


def gj_first_steps(A, steps: int, zero_tol: float = -1.0, fp32: bool = False):
    """Run only the first ``steps`` steps (same arithmetic as the full run).
    Returns (ipiv, jpiv, pivot values, result dict); entries past the steps
    taken are -1 / NaN.  Cost: steps * n^2 fma."""
    dt = np.float32 if fp32 else np.float64
    A = np.ascontiguousarray(A, dtype=dt)
    n = A.shape[0]
    X = np.empty((n, n), dtype=dt)
    ipiv = np.full(n, -1, dtype=np.int32)
    jpiv = np.full(n, -1, dtype=np.int32)
    piv = np.full(n, np.nan)
    res = OraResult()
    name = "ora_gj_invert_f32_first_steps" if fp32 else "ora_gj_invert_f64_first_steps"
    getattr(_load(), name)(n, _ptr(A), n, float(zero_tol), _ptr(X), _ptr(ipiv), _ptr(jpiv),
                           ctypes.byref(res), int(steps), _ptr(piv))
    k = min(int(steps), n)
    return ipiv[:k], jpiv[:k], piv[:k], res.as_dict()


def lu_static_det_f64(A, ipiv, jpiv) -> dict:
    """FP64 determinant by LU with a fixed (previously chosen) pivot order."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    jpiv = np.ascontiguousarray(jpiv, dtype=np.int32)
    res = OraResult()
    _load().ora_lu_static_det_f64(n, _ptr(A), n, _ptr(ipiv), _ptr(jpiv), ctypes.byref(res))
    return res.as_dict()


def gj_det_f64(A, zero_tol: float = -1.0) -> dict:
    """Determinant (and pivots) of the FP64 full-pivot run."""
    _, ipiv, jpiv, res = gj_invert_f64(A, zero_tol)
    res = dict(res)
    res["ipiv"], res["jpiv"] = ipiv, jpiv
    return res


def residual(A, X) -> float:
    """Normwise residual ||A X - I||_F / (||A||_F ||X||_F) in FP64."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    R = A @ X - np.eye(A.shape[0])
    return float(np.linalg.norm(R) / (np.linalg.norm(A) * np.linalg.norm(X)))


def newton_schulz(A, X0, max_iters: int = 10, stall: float = 0.5, accept: float = 1e-2):
    """Newton-Schulz refinement X <- X + X (I - A X) in FP64.

    The loop: R = I - A X.  An update is kept only if ||R||_F decreases.
    In exact arithmetic an update squares the residual (I - A (X + X R) =
    R^2), so ||R_{k+1}||_F <= ||R_k||_F^2.  The FP64 rounding floor is
    recognised as a kept update that contracted neither by the factor
    ``stall`` nor to within twice that quadratic bound, rn > max(stall r,
    2 r^2); the loop ends there.  For r >= 1/2 the bound 2 r^2 is at least r,
    so the loop goes on for as long as the norm falls, however slowly (a
    residual above 1 can still converge when the spectral radius of R is
    below 1).  At most ``max_iters`` updates.  The result is accepted when
    its final ||R||_F is at most ``accept``; otherwise the caller falls back
    to the plain FP64 run.
    Returns (X, updates kept, [||R_k||_F for every R computed], accepted).
    """
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X0, dtype=np.float64).copy()
    n = A.shape[0]
    eye = np.eye(n)
    R = eye - A @ X
    r = float(np.linalg.norm(R))
    norms = [r]
    updates = 0
    if np.isfinite(r) and r > 0.0:
        for it in range(1, max_iters + 1):
            Xn = X + X @ R
            Rn = eye - A @ Xn
            rn = float(np.linalg.norm(Rn))
            norms.append(rn)
            if not rn < r:
                break                      # no progress: keep the previous iterate
            prev = r
            X, R, r = Xn, Rn, rn
            updates = it
            if rn == 0.0 or rn > max(stall * prev, 2.0 * prev * prev):
                break                      # the rounding floor is reached
    accepted = bool(np.isfinite(r) and r <= accept)
    return X, updates, norms, accepted


def _slices(M, axis: int, bits: int, parts: int):
    """M = sum of ``parts`` slices.  Along ``axis`` (1: per row, 0: per
    column) let 2^e bound the largest |entry|; slice p holds the bits of M
    from 2^(e - bits p) down to the grid 2^(e - bits (p+1)) (rounded to that
    grid), so every slice but the last is an integer multiple of its grid with
    at most ``bits`` + 1 bits; the last slice is what remains.  Every
    subtraction is exact (a value minus its rounding to a coarser grid)."""
    amax = np.max(np.abs(M), axis=axis, keepdims=True)
    _, e = np.frexp(amax)
    rest = np.array(M, dtype=np.float64, copy=True)
    out = []
    for p in range(parts - 1):
        unit = np.ldexp(1.0, e - bits * (p + 1))
        S = np.rint(rest / unit) * unit
        out.append(S)
        rest = rest - S
    out.append(rest)
    return out


def exact_residual(A, X, bits: int = 20):
    """R = I - A X with the large products formed without rounding.

    A is split per row and X per column into three slices (``_slices``).  A
    product of two leading slices is a sum of n terms that are integer
    multiples of the two grids' product and at most 2^(2 bits) of them each,
    so for n <= 2^(53 - 2 bits) (8192 with 20 bits) every partial sum is
    exact, in any summation order.  I - A0 X0 is exact too (Sterbenz on the
    diagonal).  The remaining slice products, at most 2^-bits of the leading
    one, are added from the largest down, each rounding at about u times a
    partial sum of size 2^-bits: R is accurate to about 2^-bits u |A||X|
    absolutely, far below the FP64 residual's n u |A||X|.  The products are
    library matmuls (the only library step)."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = A.shape[0]
    if n > 2 ** (53 - 2 * bits):
        raise ValueError("order too large for exact slice products at this slice width")
    As = _slices(A, 1, bits, 3)
    Xs = _slices(X, 0, bits, 3)
    R = np.eye(n) - As[0] @ Xs[0]
    # remaining products, largest first: (0,1) (1,0), then (1,1) (0,2) (2,0), ...
    for i, j in sorted(((i, j) for i in range(3) for j in range(3) if i + j > 0),
                       key=lambda ij: (ij[0] + ij[1], ij)):
        R = R - As[i] @ Xs[j]
    return R


def inverse_truth(A, X0, max_steps: int = 3):
    """A reference inverse far more accurate than X0 (an FP64 inverse of A):
    Newton steps X <- X + X R with R = exact_residual(A, X).  A step from an
    inverse with relative error e leaves about cond(A) e^2 + u, so from the
    FP64 oracle's inverse (e ~ cond u) one or two steps reach about u for
    cond up to 1e8.  Stops when the correction stops shrinking."""
    X = np.array(X0, dtype=np.float64, copy=True)
    last = np.inf
    for _ in range(max_steps):
        C = X @ exact_residual(A, X)
        c = float(np.linalg.norm(C))
        if not c < last:
            break
        X = X + C
        last = c
        if c <= 1e-17 * float(np.linalg.norm(X)):
            break
    return X


def cofactor_det(A) -> Fraction:
    """Exact determinant of the (binary floating point) input by Laplace
    expansion over rationals.  Brute force; n <= 7."""
    M = [[Fraction(float(v)) for v in row] for row in np.asarray(A, dtype=np.float64)]
    n = len(M)
    if n > 7:
        raise ValueError("cofactor expansion is for n <= 7")

    def det(rows, cols):
        if len(rows) == 1:
            return M[rows[0]][cols[0]]
        total = Fraction(0)
        r0 = rows[0]
        for idx, c in enumerate(cols):
            if M[r0][c] == 0:
                continue
            minor = det(rows[1:], cols[:idx] + cols[idx + 1:])
            total += (-1) ** idx * M[r0][c] * minor
        return total

    return det(list(range(n)), list(range(n)))


def perms_from_pivots(ipiv, jpiv):
    """Original-index row and column orders after applying the swaps:
    the pivoted matrix is A[rows][:, cols]."""
    n = len(ipiv)
    rows = np.arange(n)
    cols = np.arange(n)
    for k in range(n):
        r, c = int(ipiv[k]), int(jpiv[k])
        if r < 0:
            break
        rows[[k, r]] = rows[[r, k]]
        cols[[k, c]] = cols[[c, k]]
    return rows, cols
