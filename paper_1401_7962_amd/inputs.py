"""Seeded synthetic inputs for full-pivot Gauss-Jordan inversion.

This module holds random-number plumbing and matrix construction only -- none
of the inversion's arithmetic -- so that the CPU oracle and the HIP library can
be handed the same bytes without sharing any code.

Workloads (every one seeded from ``SEED_BASE + index``):

1. ``single_normal``     one 64 x 64 matrix, entries iid N(0,1); plus the 3 x 3
                         symmetric Pascal matrix, the default matrix of the
                         paper's program (section 3).
2. ``single_dominant``   one 4096 x 4096 matrix, entries iid U[-1,1] plus 4 on
                         the diagonal.
3. ``batch_uneven``      100,000 matrices, n uniform in [8,128], entries iid
                         N(0,1); 1% of them made rank n-1 by replacing one
                         column with the sum of two others.
4. ``single_conditioned`` one n x n matrix U diag(s) V^T, U and V Haar
                         orthogonal with determinant +1, s log-spaced from 1 to
                         1e6 (n = 8192; a 2048 instance with seed offset 40 for
                         the CPU cross-check).
5. ``batch_conditioned`` 20,000 matrices, n log-uniform in [32,512], built as
                         U diag(s) V^T with cond log-uniform in [1e2,1e8].
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 14017962


def rng_for(index: int, offset: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + index + offset)


def pascal(n: int) -> np.ndarray:
    """Symmetric Pascal matrix P_ij = C(i+j, i) (the program's default is n=3)."""
    from math import comb
    return np.array([[comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)


def sylvester_hadamard(n: int) -> np.ndarray:
    """Sylvester-Hadamard matrix of order n = 2^m (entries +-1)."""
    if n < 1 or n & (n - 1):
        raise ValueError("n must be a power of two")
    H = np.ones((1, 1))
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def single_normal(n: int = 64, offset: int = 0) -> np.ndarray:
    return rng_for(1, offset).standard_normal((n, n))


def single_dominant(n: int = 4096, offset: int = 0) -> np.ndarray:
    A = rng_for(2, offset).uniform(-1.0, 1.0, (n, n))
    A[np.arange(n), np.arange(n)] += 4.0
    return A


def batch_uneven(batch: int = 100_000, nmin: int = 8, nmax: int = 128,
                 singular_frac: float = 0.01, offset: int = 0):
    """Packed batch.  Returns (sizes int32, offsets int64 (elements), packed
    float64 buffer, sorted singular member ids).  Member b is
    packed[off[b]: off[b] + n_b^2].reshape(n_b, n_b)."""
    rng = rng_for(3, offset)
    sizes = rng.integers(nmin, nmax + 1, batch).astype(np.int32)
    n_sing = int(round(batch * singular_frac))
    singular = np.sort(rng.choice(batch, n_sing, replace=False)) if n_sing else np.zeros(0, np.int64)
    sq = sizes.astype(np.int64) ** 2
    offs = np.zeros(batch, dtype=np.int64)
    offs[1:] = np.cumsum(sq)[:-1]
    packed = rng.standard_normal(int(sq.sum()))
    for b in singular:
        n = int(sizes[b])
        if n < 3:
            continue          # too small to hold a column that is the sum of two others
        a, bb, c = rng.choice(n, 3, replace=False)
        M = packed[offs[b]: offs[b] + n * n].reshape(n, n)
        M[:, c] = M[:, a] + M[:, bb]
    return sizes, offs, packed, singular


def haar_orthogonal(n: int, rng: np.random.Generator, device=None):
    """Haar-distributed orthogonal matrix with determinant +1: QR of a
    Gaussian matrix with the signs of diag(R) moved into Q, then column 0
    negated if the determinant is -1.  With ``device`` (a torch device) the
    same Gaussian draws are factored there (for large n) and a torch tensor
    is returned."""
    Z = rng.standard_normal((n, n))
    if device is not None:
        import torch
        Zt = torch.from_numpy(Z).to(device)
        del Z
        Q, R = torch.linalg.qr(Zt)
        del Zt
        Q *= torch.sign(torch.diagonal(R))[None, :]
        del R
        if torch.linalg.slogdet(Q)[0].item() < 0:
            Q[:, 0] = -Q[:, 0]
        return Q
    Q, R = np.linalg.qr(Z)
    Q *= np.sign(np.diag(R))[None, :]
    if np.linalg.slogdet(Q)[0] < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def conditioned(n: int, cond: float, rng: np.random.Generator, device=None):
    """U diag(s) V^T with s_i = cond^(i/(n-1)); det = prod s_i > 0, so
    log|det| = n ln(cond) / 2 in closed form.  ``device``: build it there
    with torch (returns a torch tensor)."""
    U = haar_orthogonal(n, rng, device)
    V = haar_orthogonal(n, rng, device)
    s = cond ** (np.arange(n) / max(n - 1, 1))
    if device is not None:
        import torch
        st = torch.from_numpy(s).to(device)
        return (U * st[None, :]) @ V.T.contiguous()
    return (U * s[None, :]) @ V.T


def single_conditioned(n: int = 8192, cond: float = 1e6, offset: int = 0, device=None):
    return conditioned(n, cond, rng_for(4, offset), device)


def batch_conditioned(batch: int = 20_000, nmin: int = 32, nmax: int = 512,
                      log10_cond: tuple = (2.0, 8.0), offset: int = 0, device=None):
    """Packed batch of U diag(s) V^T members.  Returns (sizes, offsets,
    packed buffer, conds).  Without ``device`` every member is built with
    NumPy in index order (float64 array, det U = det V = +1).  With
    ``device`` (a torch device) the members of each order are built together
    there: Gaussian draws from torch's device generator seeded with the same
    seed, orthonormalised by Cholesky QR applied twice (the Q of the QR with
    positive diag(R), i.e. Haar), orders ascending; the determinant signs are
    left as drawn (|det A| = prod s still holds), and the packed buffer is a
    device tensor."""
    rng = rng_for(5, offset)
    u = rng.random(batch)
    sizes = np.rint(nmin * (nmax / nmin) ** u).astype(np.int32)
    conds = 10.0 ** rng.uniform(log10_cond[0], log10_cond[1], batch)
    sq = sizes.astype(np.int64) ** 2
    offs = np.zeros(batch, dtype=np.int64)
    offs[1:] = np.cumsum(sq)[:-1]
    if device is None:
        packed = np.empty(int(sq.sum()))
        for b in range(batch):
            n = int(sizes[b])
            packed[offs[b]: offs[b] + n * n] = conditioned(n, float(conds[b]), rng).ravel()
        return sizes, offs, packed, conds
    import torch
    packed = torch.empty(int(sq.sum()), dtype=torch.float64, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + 5 + offset)

    def haar(count, n):
        # Q of Z = QR with diag(R) > 0 (Haar), by Cholesky QR applied twice:
        # R^T R = Z^T Z, Q = Z R^-1.  The determinant sign is left as drawn.
        Q = torch.randn((count, n, n), generator=gen, dtype=torch.float64, device=device)
        for _ in range(2):
            G = torch.bmm(Q.transpose(1, 2).contiguous(), Q)
            L = torch.linalg.cholesky(G)
            Q = torch.linalg.solve_triangular(L, Q.transpose(1, 2).contiguous(),
                                              upper=False).transpose(1, 2).contiguous()
        return Q

    for n in np.unique(sizes):
        n = int(n)
        idx = np.nonzero(sizes == n)[0]
        U = haar(len(idx), n)
        V = haar(len(idx), n)
        s = torch.from_numpy(conds[idx][:, None] ** (np.arange(n) / max(n - 1, 1))[None, :]).to(device)
        A = torch.bmm((U * s[:, None, :]).contiguous(), V.transpose(1, 2).contiguous())
        flat = (torch.from_numpy(offs[idx]).to(device)[:, None]
                + torch.arange(n * n, device=device)[None, :]).reshape(-1)
        packed[flat] = A.reshape(-1)
        del U, V, A, flat
    return sizes, offs, packed, conds


def closed_form_logdet(n: int, cond: float) -> float:
    """log|det| of ``conditioned(n, cond, .)``: sum_i ln s_i = n ln(cond)/2."""
    return n * np.log(cond) / 2.0
