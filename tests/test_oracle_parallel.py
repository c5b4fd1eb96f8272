"""The oracle's OpenMP forms (used to time it on every host core, and to
write the large-order digests under tests/golden/) against the serial oracle:
bit for bit on X, the pivots and the determinant record, across thread
counts that split the rows unevenly, ties, singular and non-finite input.
The batched form against one serial run per member."""
import numpy as np
import pytest

import oracle
from paper_1401_7962_amd import inputs


def _same(a, b):
    Xa, ia, ja, ra = a
    Xb, ib, jb, rb = b
    assert Xa.tobytes() == Xb.tobytes()
    assert np.array_equal(ia, ib) and np.array_equal(ja, jb)
    for key in ("code", "rank", "det_sign", "det_mant", "det_exp", "det", "logabsdet"):
        va, vb = ra[key], rb[key]
        assert va == vb or (np.isnan(va) and np.isnan(vb)), key


@pytest.mark.parametrize("n,threads", [(1, 3), (2, 8), (7, 3), (64, 5), (250, 8), (333, 7)])
def test_parallel_oracle_bitwise_normal(n, threads):
    A = inputs.single_normal(n, offset=500 + n)
    _same(oracle.gj_invert_f64_par(A, threads), oracle.gj_invert_f64(A))


def test_parallel_oracle_bitwise_dominant_and_ties():
    A = inputs.single_dominant(400, offset=9)
    _same(oracle.gj_invert_f64_par(A, 6), oracle.gj_invert_f64(A))
    H = inputs.sylvester_hadamard(64)          # a tie at every step
    got = oracle.gj_invert_f64_par(H, 5)
    _same(got, oracle.gj_invert_f64(H))
    assert np.array_equal(got[0], H.T / 64)


def test_parallel_oracle_singular_and_nonfinite():
    H = inputs.sylvester_hadamard(32)
    H[:, 31] = H[:, 0] + H[:, 1]               # exactly singular
    got = oracle.gj_invert_f64_par(H, 4)
    _same(got, oracle.gj_invert_f64(H))
    assert got[3]["code"] == oracle.RES_SINGULAR and got[3]["rank"] == 31
    A = inputs.single_normal(50, offset=3)
    A[17, 3] = np.inf
    got = oracle.gj_invert_f64_par(A, 4)
    _same(got, oracle.gj_invert_f64(A))
    assert got[3]["code"] == oracle.RES_NONFINITE


def test_parallel_oracle_sample_steps():
    """max_steps stops early with the same pivots as the full run."""
    A = inputs.single_dominant(300, offset=5)
    _, i_full, j_full, _ = oracle.gj_invert_f64(A)
    _, i_part, j_part, r = oracle.gj_invert_f64_par(A, 4, max_steps=40)
    assert np.array_equal(i_part[:40], i_full[:40]) and np.array_equal(j_part[:40], j_full[:40])
    assert (i_part[40:] == -1).all()


def test_parallel_fp32_bitwise():
    A = inputs.conditioned(150, 1e4, inputs.rng_for(0, 2300)).astype(np.float32)
    _same(oracle.gj_invert_f32_par(A, 6), oracle.gj_invert_f32(A))


def test_parallel_long_double_bitwise():
    A = inputs.conditioned(120, 1e6, inputs.rng_for(0, 2200))
    _same(oracle.gj_invert_f80_par(A, 5), oracle.gj_invert_f80(A))


@pytest.mark.parametrize("fp32", [False, True])
def test_batched_oracle_matches_member_runs(fp32):
    sizes, offs, packed, singular = inputs.batch_uneven(300, nmin=1, nmax=40, singular_frac=0.05,
                                                        offset=11)
    X, ipiv, jpiv, res = oracle.gj_invert_batched(sizes, offs, packed, nthreads=5, fp32=fp32)
    p = 0
    for b in range(len(sizes)):
        n = int(sizes[b])
        A = packed[offs[b]: offs[b] + n * n].reshape(n, n)
        if fp32:
            Xo, io, jo, ro = oracle.gj_invert_f32(A.astype(np.float32))
            Xo = Xo.astype(np.float64)
        else:
            Xo, io, jo, ro = oracle.gj_invert_f64(A)
        assert X[offs[b]: offs[b] + n * n].tobytes() == Xo.ravel().tobytes(), b
        assert np.array_equal(ipiv[p: p + n], io) and np.array_equal(jpiv[p: p + n], jo), b
        assert res[b]["code"] == ro["code"] and res[b]["det_exp"] == ro["det_exp"], b
        p += n
    if not fp32:
        flagged = {b for b in range(len(sizes)) if res[b]["code"] == oracle.RES_SINGULAR}
        assert flagged == {int(b) for b in singular if sizes[b] >= 3}
