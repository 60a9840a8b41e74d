"""Isospectral midpoint (IsoMP) step by fixed-point iteration (oracle).

The scheme is eq. (isomp) (Sec. 2): with the stream matrix P~ = Delta_N^{-1} W~ of an
implicitly defined W~,

    W_n     = (I - h/2 P~) W~ (I + h/2 P~),
    W_{n+1} = (I + h/2 P~) W~ (I - h/2 P~).

Expanding the first line gives the fixed-point map of eq. (isomp_iter),

    W~ <- W_n + h/2 (P W~ - W~ P) + h^2/4 P W~ P,      P = Delta_N^{-1} W~,

iterated until the infinity norm of the change of W~ drops below the tolerance (Sec. 2).
Because P and W~ are skew-Hermitian, W~ P = (P W~)^H, so the commutator is A - A^H with
the single product A = P W~, and P W~ P = A P (Sec. 3.1).

Readings taken here (the paper does not state them):

* the iteration starts from W~ = W_n; optionally (``isomp_run(..., extrapolate=True)``),
  every step after the first starts from the linear extrapolation 2 W_n - F_prev of the
  previous step's converged midpoint (F_prev, the map's output at its last evaluation), since
  W~ approximates W half a step ahead; the converged result is the same fixed point;
* the norm is the matrix infinity norm, max_i sum_j |F_ij - W~_ij|, of the change
  F - W~ between the map's output F and its input W~;
* W_{n+1} is the second line of eq. (isomp) evaluated at the same W~ whose change is
  below the tolerance, reusing that evaluation's products:
  W_{n+1} = W~ + h/2 C - h^2/4 Q, with C = A - A^H and Q = A P;
* Q is skew-Hermitian in exact arithmetic and is projected, Q <- (Q - Q^H)/2;
* with ``maxit`` reached first, W_{n+1} comes from the last W~ and the caller is told the
  residual (a fixed iteration count, as in the paper's timing runs, is ``tol = 0``);
* P = Delta_N^+ W~ is the pseudo-inverse stream solve of ``stream.py``.
"""

import numpy as np

from .stream import stream_solve


def isomp_step(Wn: np.ndarray, h: float, tol: float = 1e-12, maxit: int = 50,
               guess: np.ndarray | None = None, return_midpoint: bool = False):
    """One IsoMP step.  Returns (W_{n+1}, iterations, final residual).

    ``guess`` replaces the starting iterate W~ = W_n; with ``return_midpoint`` the map's last
    output F (the converged midpoint) is returned as a fourth value.
    """
    Wn = np.asarray(Wn, dtype=np.complex128)
    Wt = Wn.copy() if guess is None else np.asarray(guess, dtype=np.complex128).copy()
    for k in range(1, maxit + 1):
        P = stream_solve(Wt)
        A = P @ Wt
        C = A - A.conj().T
        Q = A @ P
        Q = 0.5 * (Q - Q.conj().T)
        F = Wn + (0.5 * h) * C + (0.25 * h * h) * Q
        r = float(np.abs(F - Wt).sum(axis=1).max())
        if r < tol or k == maxit:
            W1 = Wt + (0.5 * h) * C - (0.25 * h * h) * Q
            return (W1, k, r, F) if return_midpoint else (W1, k, r)
        Wt = F
    raise ValueError("maxit must be >= 1")


def isomp_run(W0: np.ndarray, h: float, nsteps: int, tol: float = 1e-12, maxit: int = 50,
              extrapolate: bool = False):
    """nsteps IsoMP steps from W0.  Returns (W, [iterations], [residuals])."""
    W = np.asarray(W0, dtype=np.complex128).copy()
    iters, res = [], []
    mid = None
    for _ in range(nsteps):
        guess = 2.0 * W - mid if (extrapolate and mid is not None) else None
        W, k, r, mid = isomp_step(W, h, tol, maxit, guess=guess, return_midpoint=True)
        iters.append(k)
        res.append(r)
    return W, iters, res
