"""The regrouping behind the blocked tangent solve, checked on the CPU.

The HIP path builds the exact tangent's blocks W_i = J_ii^{-1} B_i (eqs. 6,
7) from the band LU with partial pivoting that LAPACK's gbtrf computes (the
interchange of step k, then the multipliers below the pivot), regrouped 16
steps at a time: the steps of one block act on a window of 16 + kl rows and
compose to L_b^{-1} P_b, so the forward elimination of a block is the
gather X' = P_b X followed by X <- [0; X'_2] + G_b X'_1 with
G_b = [L11^{-1}; -L21 L11^{-1}], where L_b holds each step's multipliers at
the rows' positions after the whole block; the backward substitution goes
up in blocks of 16 rows, X_1 <- U11^{-1} (Y_1 - U12 X_2).  This test carries
that regrouping out in numpy, on factors from scipy's gbtrf, and compares it
with a dense solve: a mistake in the position maps, the block boundaries or
the strip (a wrong sign, an index off by one, a missed last partial block)
fails it.  It checks the method the kernels implement; the kernels
themselves are compared with the per-lane sweeps and with the oracle by the
GPU tests.
"""
import numpy as np
import pytest
from scipy.linalg import lapack

NB = 16


def _band_problem(rng, n, kl, ku, ng):
    A = np.zeros((n, n))
    for i in range(n):
        lo, hi = max(0, i - kl), min(n, i + ku + 1)
        A[i, lo:hi] = rng.normal(size=hi - lo)
    A += np.diag(0.3 * rng.normal(size=n))  # a weak diagonal: interchanges happen
    B = np.zeros((n, ng))
    for c in range(ng):
        rows = rng.choice(n, size=int(rng.integers(1, 6)), replace=False)
        B[rows, c] = rng.normal(size=len(rows))
    return A, B


def _gbtrf(A, kl, ku):
    """Multipliers Lf[k, j] (row k + 1 + j at step k), pivots and U by
    columns Uf[k, t] = U[k - t, k], from LAPACK's band LU."""
    n = A.shape[0]
    ab = np.zeros((2 * kl + ku + 1, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[kl + ku + i - j, j] = A[i, j]
    lub, piv, info = lapack.dgbtrf(ab, kl, ku)
    assert info == 0
    kw = kl + ku
    Lf = np.zeros((n, max(kl, 1)))
    for k in range(n):
        for j in range(kl):
            if k + 1 + j < n:
                Lf[k, j] = lub[kw + 1 + j, k]
    Uf = np.zeros((n, kw + 1))
    for k in range(n):
        for t in range(min(kw, k) + 1):
            Uf[k, t] = lub[kw - t, k]
    return Lf, np.asarray(piv), Uf


def _block_pieces(Lf, piv, Uf, n, kl, kw, k0):
    """sigma_b, G_b ((16 + kl) x 16) and U11^{-1} of the block at row k0."""
    ns, R = min(NB, n - k0), NB + kl
    sigma = list(range(R))
    for s in range(ns):
        d = piv[k0 + s] - k0
        assert s <= d < R
        sigma[s], sigma[d] = sigma[d], sigma[s]
    Lb = np.zeros((R, NB))
    m = list(range(R))  # position after step s -> position after the block
    for s in range(ns - 1, -1, -1):
        k = k0 + s
        for q in range(s + 1, min(s + kl, R - 1) + 1):
            j = q - s - 1
            if k + 1 + j < n:
                Lb[m[q], s] = Lf[k, j]
        d = piv[k] - k0
        m[s], m[d] = m[d], m[s]
    L11 = np.eye(NB) + np.tril(Lb[:NB], -1)
    L11i = np.linalg.solve(L11, np.eye(NB))
    G = np.vstack([L11i, -Lb[NB:] @ L11i])
    U11 = np.eye(NB)
    for r in range(NB):
        for c in range(r, NB):
            if c < ns and c - r <= kw:
                U11[r, c] = Uf[k0 + c, c - r]
    return np.array(sigma), G, np.linalg.inv(U11)


def _blocked_solve(Lf, piv, Uf, B, n, kl, ku):
    kw = kl + ku
    nb = (n + NB - 1) // NB
    R = NB + kl
    pieces = [_block_pieces(Lf, piv, Uf, n, kl, kw, NB * b) for b in range(nb)]
    X = np.zeros((nb * NB + R, B.shape[1]))
    X[:n] = B
    for b, (sigma, G, _) in enumerate(pieces):
        k0 = NB * b
        Xp = X[k0 + sigma]
        X[k0:k0 + R] = G @ Xp[:NB]
        X[k0 + NB:k0 + R] += Xp[NB:]
    W = np.zeros((nb * NB + NB + kw, B.shape[1]))
    for b in range(nb - 1, -1, -1):
        k0 = NB * b
        strip = np.zeros((NB, kw))
        for r in range(NB):
            for j in range(kw):
                cu, t = k0 + NB + j, NB + j - r
                if cu < n and t <= kw:
                    strip[r, j] = Uf[cu, t]
        W[k0:k0 + NB] = pieces[b][2] @ (X[k0:k0 + NB] - strip @ W[k0 + NB:k0 + NB + kw])
    return W[:n]


@pytest.mark.parametrize("n,kl,ku,ng,seed", [
    (100, 5, 7, 20, 0),      # ragged last block
    (203, 36, 36, 40, 1),    # the benchmark's band width
    (64, 48, 48, 17, 2),     # the widest band of the blocked path, whole blocks
    (37, 16, 16, 33, 3),
    (7, 2, 3, 5, 4),         # a single partial block
    (16, 3, 3, 3, 5),        # exactly one block
    (129, 20, 76, 31, 6),    # wide upper band (strip of 96 columns)
])
def test_blocked_regrouping_matches_dense_solve(n, kl, ku, ng, seed):
    rng = np.random.default_rng(seed)
    A, B = _band_problem(rng, n, kl, ku, ng)
    Lf, piv, Uf = _gbtrf(A, kl, ku)
    W = _blocked_solve(Lf, piv, Uf, B, n, kl, ku)
    ref = np.linalg.solve(A, B)
    err = np.abs(W - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, f"{err:.3e}"


def test_a_dropped_interchange_is_caught():
    """The same regrouping with the block permutation left out must fail:
    the pivots of these matrices are not all on the diagonal."""
    rng = np.random.default_rng(1)
    n, kl, ku = 203, 36, 36
    A, B = _band_problem(rng, n, kl, ku, 8)
    Lf, piv, Uf = _gbtrf(A, kl, ku)
    assert np.any(piv != np.arange(n))
    W = _blocked_solve(Lf, np.arange(n), Uf, B, n, kl, ku)
    ref = np.linalg.solve(A, B)
    assert np.abs(W - ref).max() / np.abs(ref).max() > 1e-6
