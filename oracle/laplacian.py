"""Quantised spherical Laplacian Delta_N (oracle; test infrastructure only).

Two independent constructions:

* ``delta_tridiag(N, m)`` writes out the tridiagonal block Delta^m of eq. (delta_tria)
  (Sec. 3.2): the restriction of the Laplacian to the m-th diagonal of an N x N matrix,
  with s = (N-1)/2 and 0-based index i <-> matrix entry (i+m, i).  As printed the block is
  positive semidefinite with spectrum {l(l+1) : l = m..N-1}; the Laplacian itself has the
  eigenvalues -l(l+1) of eq. (lap_prop), so Delta_N restricted to diagonal m is -Delta^m.

* ``brute_laplacian(N)`` builds the dense N^2 x N^2 operator X -> -sum_a [J_a, [J_a, X]]
  from the textbook spin-s matrices J_1, J_2, J_3 (J_3 = diag(s, s-1, ..., -s)).  It is the
  quadratic Casimir of the adjoint action, whose eigenvalues on u(N) are l(l+1), l = 0..N-1,
  with multiplicity 2l+1 -- the spectrum eq. (lap_prop) states.  It shares nothing with
  ``delta_tridiag`` and is used only to pin it on tiny N.
"""

import numpy as np


def delta_tridiag(N: int, m: int):
    """Diagonal d (length N-m) and off-diagonal e (length N-m-1) of Delta^m, eq. (delta_tria).

    d_i = 2 (s (2i+1+m) - i (i+m)),
    e_i = -sqrt((i+m+1)(N-1-i-m)) sqrt((i+1)(N-1-i)),   i = 0..N-m-2,
    the block being symmetric (the sub-diagonal term of eq. (delta_tria) is e_{i-1}).
    """
    if not (0 <= m < N):
        raise ValueError("need 0 <= m < N")
    s = (N - 1) / 2.0
    n = N - m
    i = np.arange(n, dtype=np.float64)
    d = 2.0 * (s * (2.0 * i + 1.0 + m) - i * (i + m))
    k = np.arange(n - 1, dtype=np.float64)
    e = -np.sqrt((k + m + 1.0) * (N - 1.0 - k - m)) * np.sqrt((k + 1.0) * (N - 1.0 - k))
    return d, e


def spin_matrices(N: int):
    """Spin-s representation (s = (N-1)/2) of su(2): J_1, J_2, J_3 with [J_1, J_2] = i J_3.

    Basis index i carries J_3 eigenvalue s - i; J_+ raises it by one (index i -> i-1) with
    the standard coefficient sqrt(s(s+1) - mu(mu+1)).
    """
    s = (N - 1) / 2.0
    mu = s - np.arange(N)
    Jp = np.zeros((N, N))
    for i in range(1, N):
        Jp[i - 1, i] = np.sqrt(s * (s + 1.0) - mu[i] * (mu[i] + 1.0))
    Jm = Jp.T.copy()
    J1 = (Jp + Jm) / 2.0
    J2 = (Jp - Jm) / 2.0j
    J3 = np.diag(mu).astype(np.complex128)
    return J1.astype(np.complex128), J2, J3


def brute_laplacian(N: int) -> np.ndarray:
    """Dense N^2 x N^2 matrix of X -> -sum_a [J_a, [J_a, X]] acting on row-major vec(X).

    For row-major vec, vec(A X B) = (A kron B^T) vec(X).
    """
    I = np.eye(N)
    L = np.zeros((N * N, N * N), dtype=np.complex128)
    for J in spin_matrices(N):
        ad = np.kron(J, I) - np.kron(I, J.T)
        L += ad @ ad
    return -L


def apply_laplacian(X: np.ndarray) -> np.ndarray:
    """Delta_N X = -sum_a [J_a, [J_a, X]] by explicit commutators (O(N^3); any N)."""
    N = X.shape[0]
    out = np.zeros_like(X, dtype=np.complex128)
    for J in spin_matrices(N):
        c = J @ X - X @ J
        out -= J @ c - c @ J
    return out
