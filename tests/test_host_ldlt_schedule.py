"""CPU model of the batched bordered LDL^T's launch order (one matrix).

1 - Pi(z) is complex symmetric; on the real axis (z = x + i eta, x > 0) its
imaginary part L |Im chi| L^T is positive semidefinite, on the imaginary axis
the matrix is real symmetric positive definite.  Either way every leading
principal minor is nonsingular, so the bordered matrix [[1 - Pi, B], [B^T, 0]]
has an LDL^T factorisation without pivoting whose first N steps leave the
Schur complement -B^T (1 - Pi)^-1 B in the border block.  The launches, each
modelled here by one NumPy function:

* D: the 64 x 64 diagonal block is factored L11 D1 L11^T, L11^-1 formed and
  D1^-1 kept per pivot;
* T: every row block below it: W = A21 L11^-T, stored transposed in the row
  part (the upper triangle): W^T = D1 L21^T;
* G: the lower-triangle tiles of the trailing matrix take A -= L21 (W^T) with
  both operands read from the row part, L21[r][k] = W^T[k][r] D^-1[k]
  (off-diagonal border-border tiles skipped: only the diagonal of the Schur
  complement is read).

Groups of up to four panels share one trailing update; a later panel of a
group first receives the group's earlier panels on its own columns.
"""
import numpy as np
import pytest

NBO = 64


def _diag(A, N, K0, dinv):
    """L11 D1 L11^T of the diagonal block (lower triangle read); D1^-1 goes to
    dinv[K0..]; returns (L11^-1, zero pivot seen)."""
    kb = min(NBO, N - K0)
    X = np.tril(A[K0:K0 + kb, K0:K0 + kb]).astype(complex)
    zero = False
    for t in range(kb):
        d = X[t, t]
        if d == 0:
            zero = True
            continue
        col = X[t + 1:, t].copy()
        X[t + 1:, t + 1:] -= np.tril(np.outer(col, col) / d)
        X[t + 1:, t] = col / d
    L = np.tril(X, -1) + np.eye(kb)
    D = np.diag(X).copy()
    with np.errstate(divide="ignore", invalid="ignore"):
        dinv[K0:K0 + kb] = np.where(D != 0, 1.0 / D, 0.0)
    return np.linalg.inv(L), zero


def _trsm(A, N, K0, Linv):
    """Row part of the panel: W^T with W = A21 L11^-T (rows below the panel)."""
    kb = min(NBO, N - K0)
    r0 = K0 + kb
    A[K0:K0 + kb, r0:] = (A[r0:, K0:K0 + kb] @ Linv.T).T


def _lower_operand(A, dinv, rows, ks, kl):
    """L21 rows `rows` over the K range, from the row part: W^T[k][r] D^-1[k]."""
    return (A[ks:ks + kl, rows] * dinv[ks:ks + kl, None]).T


def _tiles_lower(A, N, r0, ks, kl, dinv):
    n = A.shape[0]
    mt = (n - r0 + 63) // 64
    for ti in range(mt):
        for tj in range(ti + 1):
            ra, ca = r0 + 64 * ti, r0 + 64 * tj
            if ra >= N and ca >= N and ca + 64 <= ra:
                continue
            rows = slice(ra, min(ra + 64, n))
            A[rows, ca:ca + 64] -= _lower_operand(A, dinv, rows, ks, kl) @ A[ks:ks + kl, ca:ca + 64]


def _columns(A, r0, c0, c1, ks, kl, dinv):
    rows = slice(r0, A.shape[0])
    A[rows, c0:c1] -= _lower_operand(A, dinv, rows, ks, kl) @ A[ks:ks + kl, c0:c1]


def bordered_ldlt(A, N, group):
    n = A.shape[0]
    dinv = np.zeros(N, complex)
    K0 = 0
    zero = False
    while K0 < N:
        g = min(group, (N - K0) // NBO)
        if g >= 2:
            a, e = K0, K0 + g * NBO
            for p in range(g):
                b = a + p * NBO
                if p > 0:
                    _columns(A, b, b, b + NBO, a, p * NBO, dinv)
                Linv, z = _diag(A, N, b, dinv)
                zero |= z
                _trsm(A, N, b, Linv)
            _tiles_lower(A, N, e, a, g * NBO, dinv)
            K0 = e
        else:
            kend = min(K0 + NBO, N)
            Linv, z = _diag(A, N, K0, dinv)
            zero |= z
            _trsm(A, N, K0, Linv)
            _tiles_lower(A, N, kend, K0, kend - K0, dinv)
            K0 = kend
    return np.diag(A[N:, N:]).copy(), zero


def _bordered(M, B):
    N, R = B.shape
    A = np.zeros((N + R, N + R), complex)
    A[:N, :N], A[:N, N:], A[N:, :N] = M, B, B.T
    return A


def _stale_upper(A, rng):
    """The factorisation must read only the lower triangle: scramble the rest."""
    iu = np.triu_indices(A.shape[0], 1)
    A[iu] = rng.normal(size=len(iu[0])) * 1e3
    return A


@pytest.mark.parametrize("group", [1, 2, 3, 4])
@pytest.mark.parametrize("N,R", [(300, 3), (129, 1), (200, 40), (64, 2), (191, 5), (1200, 1)])
def test_schedule_gives_the_schur_complement(group, N, R):
    """Complex symmetric with positive definite imaginary part (a residue
    matrix), and real symmetric positive definite (an imaginary-axis matrix)."""
    rng = np.random.default_rng(N * 7 + R)
    X = rng.normal(size=(N, N)) / np.sqrt(N)
    G = rng.normal(size=(N, 2 * N)) / np.sqrt(2 * N)
    B = rng.normal(size=(N, R))
    for M in (np.eye(N) + 3.0 * (X + X.T) + 1j * 0.05 * (G @ G.T),
              np.eye(N) + 0.3 * (G @ G.T) + 0j):
        A = _stale_upper(_bordered(M, B), rng)
        S, zero = bordered_ldlt(A, N, group)
        assert not zero
        ref = -np.einsum("ir,ir->r", B, np.linalg.solve(M, B))
        assert np.max(np.abs(S - ref) / np.abs(ref)) < 1e-10


def test_groups_do_not_change_the_result():
    rng = np.random.default_rng(3)
    N, R = 400, 7
    X = rng.normal(size=(N, N)) / np.sqrt(N)
    G = rng.normal(size=(N, N)) / np.sqrt(N)
    M = np.eye(N) + 2.0 * (X + X.T) + 1j * 0.1 * (G @ G.T)
    B = rng.normal(size=(N, R))
    out = [bordered_ldlt(_bordered(M, B), N, g)[0] for g in (1, 2, 3, 4)]
    for s in out[1:]:
        assert np.max(np.abs(s - out[0])) <= 1e-12 * np.max(np.abs(out[0]))


def test_zero_pivot_is_reported():
    """An exactly zero leading entry (possible only when Im(1 - Pi) vanishes)
    is flagged, not divided by."""
    N, R = 70, 1
    M = np.eye(N, dtype=complex)
    M[0, 0] = 0.0
    M[0, 1] = M[1, 0] = 1.0
    B = np.ones((N, R))
    _, zero = bordered_ldlt(_bordered(M, B), N, 1)
    assert zero
