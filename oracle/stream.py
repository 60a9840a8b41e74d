"""Stream solve P = Delta_N^+ W, one tridiagonal system per diagonal (oracle).

Follows Sec. 3.3, eq. (sub_tria_W): the Laplacian maps the m-th diagonal of P to the m-th
diagonal of W, through the tridiagonal block of eq. (delta_tria); the lower triangle of P
comes from the N systems m = 0..N-1, the upper triangle from skew-Hermitian symmetry, and
each system is solved with LAPACK's positive-definite tridiagonal routines (the paper uses
``zpttrs``; here ``dpttrf``/``dpttrs`` on the real and imaginary parts, which is the same
real factorisation applied to a complex right-hand side).

Readings of the paper taken here (the paper is silent or inconsistent on each):

* Sign.  Delta_N has eigenvalues -l(l+1) (eq. (lap_prop)) while the block of
  eq. (delta_tria) is positive semidefinite with eigenvalues +l(l+1); so on diagonal m the
  Laplacian is -Delta^m, and P_m = -(Delta^m)^{-1} W_m.
* Singular block m = 0.  Delta^0 annihilates the identity (l = 0).  The solve is the
  pseudo-inverse: the trace part tr(W)/N is removed from the m = 0 right-hand side, the
  leading (N-1) x (N-1) block (positive definite) is solved with the last unknown set to 0,
  and the mean is subtracted, which gives the minimum-norm solution, so P is traceless
  (P in su(N), Sec. 2) even when W is not.
* Upper triangle.  P[i, i+m] = -conj(P[i+m, i]) (P skew-Hermitian, Sec. 3.3).
"""

import numpy as np
from scipy.linalg import lapack

from .laplacian import delta_tridiag


def _pt_solve(d: np.ndarray, e: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve T x = b for symmetric positive-definite tridiagonal T = tridiag(e, d, e)."""
    if d.size == 0:
        return np.zeros(0, dtype=np.complex128)
    if d.size == 1:
        return b / d[0]
    df, ef, info = lapack.dpttrf(d, e)
    if info != 0:
        raise np.linalg.LinAlgError(f"dpttrf info={info}")
    B = np.stack([b.real, b.imag], axis=1)
    x, info = lapack.dpttrs(df, ef, B)
    if info != 0:
        raise np.linalg.LinAlgError(f"dpttrs info={info}")
    return x[:, 0] + 1j * x[:, 1]


def stream_solve(W: np.ndarray) -> np.ndarray:
    """P = Delta_N^+ W for a skew-Hermitian N x N matrix W (complex128).

    Only the lower triangle (with the diagonal) of W is read: the m-th diagonal, entries
    W[i+m, i], is the right-hand side of system m.
    """
    W = np.asarray(W, dtype=np.complex128)
    N = W.shape[0]
    P = np.zeros((N, N), dtype=np.complex128)
    tr = np.trace(W) / N
    for m in range(N):
        n = N - m
        i = np.arange(n)
        b = W[i + m, i].copy()
        d, e = delta_tridiag(N, m)
        if m == 0:
            b = b - tr
            x = np.zeros(n, dtype=np.complex128)
            x[: n - 1] = _pt_solve(d[: n - 1], e[: n - 2], b[: n - 1])
            x -= x.mean()
        else:
            x = _pt_solve(d, e, b)
        P[i + m, i] = -x
        if m > 0:
            P[i, i + m] = np.conj(x)
    return P
