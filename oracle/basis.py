"""Quantised basis T_lm and the projection omega_lm <-> W (oracle).

Sec. 3.2: since Delta_N T_lm = -l(l+1) T_lm (eq. (lap_prop)) and the Laplacian splits into
the tridiagonal blocks Delta^m of eq. (delta_tria), the basis elements with m >= 0 are the
eigenvectors of Delta^m placed on the m-th sub-diagonal; those with m < 0 follow by
skew-symmetry.  W is then assembled as W = sum_lm i omega_lm T_lm, eq. (W0).  Here the
eigenvectors come from LAPACK (``scipy.linalg.eigh_tridiagonal``), standing in for the
paper's ``pdstedc``.

Readings taken here:

* l runs over m..N-1 on diagonal m (l = 0 is the identity direction on m = 0); the
  eigenvalues of Delta^m, in ascending order, are l(l+1) for l = m, m+1, ..., N-1;
* each eigenvector has unit 2-norm (so T_lm has unit Frobenius norm).  The paper leaves its
  sign open; here, among the entries with index 0..floor((n-1)/2) whose magnitude is within a
  relative 1e-8 of the largest there, the one with the lowest index is made positive.  (The
  first entry alone is no good: it underflows for large N.  The largest entry alone is no
  good either: these blocks have eigenvectors with exactly equal magnitudes at different
  indices, e.g. N = 8, l = 3, m = 0 at indices 0 and 2, with opposite signs.)
* T_{l,-m} = (-1)^m T_lm^H, so W[i+m, i] = i sum_l omega_lm v^{lm}_i and
  W[i, i+m] = i (-1)^m sum_l omega_{l,-m} v^{lm}_i; real vorticity,
  omega_{l,-m} = (-1)^m conj(omega_lm), makes W skew-Hermitian;
* coefficients are stored flat at index l*l + l + m (length N*N).
"""

import numpy as np
from scipy.linalg import eigh_tridiagonal

from .laplacian import delta_tridiag

SIGN_TIE_REL = 1e-8  # magnitudes within this relative distance of the largest count as ties


def eigvecs(N: int, m: int, count: int | None = None):
    """Eigenvalues (ascending) and sign-fixed unit eigenvectors (columns) of Delta^m.

    ``count`` limits the result to the lowest ``count`` eigenpairs (l = m..m+count-1).
    """
    d, e = delta_tridiag(N, m)
    n = N - m
    if n == 1:
        return d.copy(), np.ones((1, 1))
    if count is None or count >= n:
        w, V = eigh_tridiagonal(d, e)
    else:
        w, V = eigh_tridiagonal(d, e, select="i", select_range=(0, count - 1))
    half = (n - 1) // 2 + 1
    a = np.abs(V[:half, :])
    k = np.argmax(a >= (1.0 - SIGN_TIE_REL) * a.max(axis=0), axis=0)  # lowest such index
    sgn = np.sign(V[k, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return w, V * sgn


def _diagonal(args):
    """Entries of diagonal m of W: the lower one (i+m, i) and, for m > 0, the upper (i, i+m)."""
    N, m, top, om_pos, om_neg = args
    _, V = eigvecs(N, m, top - m + 1)
    low = 1j * (V @ om_pos)
    up = 1j * (-1) ** m * (V @ om_neg) if m > 0 else None
    return low, up


def assemble(N: int, omega: np.ndarray, lmax: int | None = None, workers: int = 1) -> np.ndarray:
    """W = sum_{l,m} i omega_lm T_lm (eq. (W0)) from flat coefficients omega[l*l+l+m].

    With ``lmax`` the coefficients of degree l > lmax must be zero, and only the basis
    elements up to degree lmax are computed (the large-scale initial conditions).
    ``workers`` > 1 forms the diagonals in that many processes (each diagonal is independent
    of the others; the result is the same bit for bit).
    """
    omega = np.asarray(omega, dtype=np.complex128)
    W = np.zeros((N, N), dtype=np.complex128)
    top = N - 1 if lmax is None else min(int(lmax), N - 1)
    if np.any(omega[(top + 1) ** 2:] != 0):
        raise ValueError("coefficients beyond lmax must be zero")

    def jobs():
        for m in range(top + 1):
            l = np.arange(m, top + 1)
            yield N, m, top, omega[l * l + l + m], omega[l * l + l - m]

    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor

        with ProcessPoolExecutor(max_workers=workers) as ex:
            diags = list(ex.map(_diagonal, jobs(), chunksize=4))
    else:
        diags = map(_diagonal, jobs())
    for m, (low, up) in enumerate(diags):
        i = np.arange(N - m)
        W[i + m, i] = low
        if m > 0:
            W[i, i + m] = up
    return W


def extract(W: np.ndarray) -> np.ndarray:
    """omega_lm = -i <T_lm, W>_F, the inverse of ``assemble`` on u(N) (Sec. 3.2, post-processing)."""
    W = np.asarray(W, dtype=np.complex128)
    N = W.shape[0]
    omega = np.zeros(N * N, dtype=np.complex128)
    for m in range(N):
        _, V = eigvecs(N, m)
        n = N - m
        i = np.arange(n)
        l = np.arange(m, N)
        c = -1j * (V.T @ W[i + m, i])
        omega[l * l + l + m] = c
        if m > 0:
            omega[l * l + l - m] = (-1) ** m * np.conj(c)
    return omega


def energy_spectrum(omega: np.ndarray, N: int) -> np.ndarray:
    """Kinetic energy per degree l (the spectrum of Sec. 4): E_l = sum_m |omega_lm|^2 / (l(l+1)).

    The stream matrix P = Delta_N^{-1} W has coefficients -omega_lm / (l(l+1)) (eq. (lap_prop)),
    so sum_l E_l = tr(P W) and sum_l l(l+1) E_l = ||W||_F^2 (the T_lm are orthonormal).
    E_0 = 0 (l = 0 carries no kinetic energy).
    """
    omega = np.asarray(omega, dtype=np.complex128)
    E = np.zeros(N)
    for l in range(1, N):
        E[l] = np.sum(np.abs(omega[l * l:(l + 1) * (l + 1)]) ** 2) / (l * (l + 1))
    return E
