"""CPU model of the batched bordered LU's launch order (one matrix).

The library factors [[1 - Pi, B], [B^T, 0]] without back substitution; the
trailing diagonal then holds -b_r^T (1 - Pi)^-1 b_r.  Its launches reorder the
right-looking elimination in two ways, modelled here step by step in NumPy
(each function does what one launch does) and checked against a direct solve:

* groups of up to three 64-column panels share one wide trailing update; a
  later panel of a group first receives the group's earlier panels on its own
  columns, and its U rows subtract their contribution (`kpre`);
* inside a panel, column blocks go in pairs: an even block updates only the
  next block's columns, the odd block subtracts the even block's deferred
  contribution from its U rows and then updates the rest of the panel with
  both blocks at once.
"""
import numpy as np
import pytest

NBO = 64


def _factor_block(P, k0, kb, n_piv):
    # partial pivoting among rows < n_piv, rank-1 updates inside the block;
    # a pivot swap moves whole rows (the net row moves reach every column)
    for c in range(k0, k0 + kb):
        p = c + int(np.argmax(np.abs(P[c:n_piv, c].real) + np.abs(P[c:n_piv, c].imag)))
        P[[c, p], :] = P[[p, c], :]
        P[c + 1:, c] /= P[c, c]
        P[c + 1:, c + 1:k0 + kb] -= np.outer(P[c + 1:, c], P[c, c + 1:k0 + kb])


def _panel(A, N, K0, W, pairs):
    """Factor columns K0..K0+64 (rows >= K0) in blocks of W columns."""
    kend = min(K0 + NBO, N)
    P = A[:, :]                                   # rows move across the whole matrix
    for k0 in range(K0, kend, W):
        kb = min(W, kend - k0)
        ke = k0 + kb
        _factor_block(P, k0, kb, N)
        if ke >= kend:
            continue
        odd = pairs and ((k0 - K0) // W) % 2 == 1
        L = np.tril(P[k0:ke, k0:ke], -1) + np.eye(kb)
        X = P[k0:ke, ke:kend].copy()
        if odd:
            X -= P[k0:ke, k0 - W:k0] @ P[k0 - W:k0, ke:kend]
        P[k0:ke, ke:kend] = np.linalg.solve(L, X)
        if not pairs:
            P[ke:, ke:kend] -= P[ke:, k0:ke] @ P[k0:ke, ke:kend]
        elif odd:
            P[ke:, ke:kend] -= P[ke:, k0 - W:ke] @ P[k0 - W:ke, ke:kend]
        else:
            ce = min(ke + W, kend)
            P[ke:, ke:ce] -= P[ke:, k0:ke] @ P[k0:ke, ke:ce]


def _u12(A, N, K0, c0, kpre):
    """U rows of the panel at K0 on columns c0.. (after the group's earlier
    panels' contribution when kpre >= 0)."""
    kbo = min(NBO, N - K0)
    X = A[K0:K0 + kbo, c0:].copy()
    if kpre >= 0:
        X -= A[K0:K0 + kbo, kpre:K0] @ A[kpre:K0, c0:]
    L = np.tril(A[K0:K0 + kbo, K0:K0 + kbo], -1) + np.eye(kbo)
    A[K0:K0 + kbo, c0:] = np.linalg.solve(L, X)


def _trailing(A, r0, c0, c1, ks, kl):
    A[r0:, c0:c1] -= A[r0:, ks:ks + kl] @ A[ks:ks + kl, c0:c1]


def bordered_lu(A, N, group, W, pairs):
    n = A.shape[0]
    K0 = 0
    while K0 < N:
        g = min(group, (N - K0) // NBO)
        if g >= 2:
            a, e = K0, K0 + g * NBO
            for p in range(g):
                b = a + p * NBO
                if p > 0:
                    _trailing(A, b, b, b + NBO, a, p * NBO)
                _panel(A, N, b, W, pairs)
                _u12(A, N, b, b + NBO, a if p > 0 else -1)
            _trailing(A, e, e, n, a, g * NBO)
            K0 = e
        else:
            kend = min(K0 + NBO, N)
            _panel(A, N, K0, W, pairs)
            _u12(A, N, K0, kend, -1)
            _trailing(A, kend, kend, n, K0, kend - K0)
            K0 = kend
    return np.diag(A[N:, N:]).copy()


@pytest.mark.parametrize("group", [1, 2, 3, 4])
@pytest.mark.parametrize("W,pairs", [(8, False), (8, True), (4, True), (1, True)])
@pytest.mark.parametrize("N,R", [(300, 3), (129, 1), (200, 40), (64, 2), (191, 5)])
def test_schedule_gives_the_schur_complement(group, W, pairs, N, R):
    rng = np.random.default_rng(N * 7 + R)
    M = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    B = rng.normal(size=(N, R))
    A = np.zeros((N + R, N + R), complex)
    A[:N, :N], A[:N, N:], A[N:, :N] = M, B, B.T
    S = bordered_lu(A, N, group, W, pairs)
    ref = -np.einsum("ir,ir->r", B, np.linalg.solve(M, B))
    assert np.max(np.abs(S - ref) / np.abs(ref)) < 1e-10


def test_pairs_reproduce_the_right_looking_panel():
    """Same pivots and the same factored panel, to rounding, with and without
    the pair order (ragged last blocks included)."""
    rng = np.random.default_rng(5)
    for n, N, K0 in ((300, 299, 0), (130, 129, 64), (90, 88, 48), (65, 64, 0)):
        A0 = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        A1, A2 = A0.copy(), A0.copy()
        _panel(A1, N, K0, 8, pairs=False)
        _panel(A2, N, K0, 8, pairs=True)
        kend = min(K0 + NBO, N)
        assert np.max(np.abs(A1[:, K0:kend] - A2[:, K0:kend])) <= 1e-12 * np.max(np.abs(A1[:, K0:kend]))
