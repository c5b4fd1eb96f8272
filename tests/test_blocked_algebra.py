"""CPU check of the algebra behind the blocked elimination (delayed updates).

A plain NumPy model, independent of the HIP code: full-pivot Gauss-Jordan
steps (eqs. 14-15) on the trailing block only, the array then reordered so
that the panel's pivots follow the earlier ones, and the panel's steps
applied to the other rows and columns at once by three products,
    W_b1 = T W_b1,  W_31 += W_3b W_b1(old),  W_1* -= W_1b(old) W_b*,
with W_1b zeroed first (T = the panel's inverted pivot block, held in W_bb
after the trailing steps).  The section-1 theorem (the inverse is the product
of the elimination's left factors) is what allows the grouping.  The result
must be the oracle's inverse up to rounding, for any panel width.
"""
import numpy as np
import pytest

import oracle
from paper_1401_7962_amd import inputs


def _trailing_steps(S, nsteps):
    """In-place full-pivot steps on S; returns the pivots' (row, col) positions."""
    m = S.shape[0]
    used_r, used_c, piv = [], [], []
    for _ in range(nsteps):
        mask = np.abs(S)
        mask[used_r, :] = -1.0
        mask[:, used_c] = -1.0
        p, q = np.unravel_index(np.argmax(mask), mask.shape)
        pv = S[p, q]
        row = S[p, :] / pv
        row[q] = 1.0 / pv
        col = S[:, q].copy()
        for i in range(m):
            if i != p:
                S[i, :] -= col[i] * row
                S[i, q] = -col[i] / pv
        S[p, :] = row
        used_r.append(p)
        used_c.append(q)
        piv.append((p, q))
    return piv


def _blocked_inverse(A, nb, skip_w31=False):
    n = A.shape[0]
    W = A.copy()
    prow, pcol = np.arange(n), np.arange(n)
    for k0 in range(0, n, nb):
        m, nbp = n - k0, min(nb, n - k0)
        S = W[k0:, k0:].copy()
        piv = _trailing_steps(S, nbp)
        W[k0:, k0:] = S
        pr = [p for p, _ in piv]
        pc = [q for _, q in piv]
        rsrc = np.r_[np.arange(k0), k0 + np.array(pr + [i for i in range(m) if i not in pr], dtype=int)]
        csrc = np.r_[np.arange(k0), k0 + np.array(pc + [j for j in range(m) if j not in pc], dtype=int)]
        W = W[rsrc][:, csrc]
        prow, pcol = prow[rsrc], pcol[csrc]
        if k0 == 0:
            continue
        b, one, three = slice(k0, k0 + nbp), slice(0, k0), slice(k0 + nbp, n)
        tB, tA = W[b, one].copy(), W[one, b].copy()
        W[one, b] = 0.0
        W[b, one] = W[b, b] @ tB
        if not skip_w31:
            W[three, one] += W[three, b] @ tB
        W[one, :] -= tA @ W[b, :]
    rowinv, colinv = np.empty(n, dtype=int), np.empty(n, dtype=int)
    rowinv[prow] = np.arange(n)
    colinv[pcol] = np.arange(n)
    return W[colinv][:, rowinv]


@pytest.mark.parametrize("n,nb", [(10, 4), (33, 8), (64, 16), (70, 32), (50, 50), (17, 2), (40, 64)])
def test_grouped_panel_updates_give_the_inverse(n, nb):
    A = inputs.rng_for(0, 9100 + n + nb).standard_normal((n, n))
    X = _blocked_inverse(A, nb)
    Xo, _, _, ro = oracle.gj_invert_f64(A)
    assert ro["code"] == 0
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


def test_dropping_a_delayed_product_is_caught():
    """Without the W_31 product the result is not the inverse: the check above
    tells a wrong grouping from rounding."""
    n, nb = 40, 8
    A = inputs.rng_for(0, 9200).standard_normal((n, n))
    Xo, _, _, _ = oracle.gj_invert_f64(A)
    X_bad = _blocked_inverse(A, nb, skip_w31=True)
    assert np.linalg.norm(X_bad - Xo) / np.linalg.norm(Xo) > 1e-3
