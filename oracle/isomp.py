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
* with ``degree`` d >= 2 as well, a step with k >= 2 earlier steps in the run starts from the
  polynomial of degree min(k - 1, d) through the last min(k, d + 1) midpoints, evaluated one
  step ahead (``extrapolate_midpoints``): the midpoints are equally spaced samples of a
  smooth curve, so the start is within O(h^(d+1)) of the fixed point; k = 1 keeps the
  linear start above.  With the difference form of W_{n+1} the trajectory carries residual
  noise only at O(h ||P|| r) and a step then takes one evaluation; with the second-line form
  the O(r) kinks that accepted one-evaluation steps leave, amplified by the extrapolation
  weights, push every few steps back to two;
* with ``solution_differences`` as well (degree 3), the third and fourth steps of a run
  (k = 2, 3 earlier steps) use the run's states too (``start_from_history``): adding the two
  lines of eq. (isomp) gives W_k + W_{k+1} = 2 W~_k + h^2/2 P~_k W~_k P~_k, so each midpoint
  is F_k = (W_k + W_{k+1})/2 + delta_k with delta_k = -h^2/4 P~_k F_k P~_k of order h^2; the
  start is (W_k + W*_{k+1})/2 + delta*_k with W*_{k+1} from the polynomial of degree k
  through the states W_0 .. W_k and delta*_k from the one of degree k - 1 through
  delta_0 .. delta_{k-1}, both one step ahead: an error of O(h^(k+1)) against O(h^k) for the
  midpoints alone (measured: 1e-9 -> 1e-13 and 1e-11 -> 1e-15 for the sigma_l = (l+1)^-1.5
  and (l+1)^-1 fields at h = 0.005), so those steps take one evaluation where they took two.
  Later steps keep the midpoint polynomial, already at the rounding level there.  With the
  difference form of W_{n+1}, the second step (k = 1) uses the slope D_0 = P_0 W_0 - W_0 P_0
  of the states at W_0 (P_0 = Delta_N^+ W_0, the right-hand side of the continuous equation;
  the states of the symmetric second-order map lie on a smooth curve whose slope there
  differs from D_0 by O(h^2)): the quadratic through W_0 with that slope and through W_1
  predicts W_2 to O(h^3), delta_1 = delta_0 + O(h^3), and (W_1 + W*_2)/2 + delta_0 works out to
  F_0 + 2 (W_1 - W_0) - h D_0 (``start_second_step``; measured 1e-9 -> 1e-14 at h = 0.005);
  the GPU takes h D_0 from the first evaluation of the first step, whose W_{n+1} is
  W_0 + h D_0 in that form;
* the norm is the matrix infinity norm, max_i sum_j |F_ij - W~_ij|, of the change
  F - W~ between the map's output F and its input W~;
* W_{n+1} is the second line of eq. (isomp) evaluated at the same W~ whose change is below
  the tolerance, reusing that evaluation's products (``update="second_line"``, the default):
  W_{n+1} = W~ + h/2 C - h^2/4 Q, with C = A - A^H and Q = A P.  Optionally
  (``update="difference"``) W_{n+1} = W_n + h C: the two lines of eq. (isomp) differ by
  exactly h (P~ W~ - W~ P~), so at the fixed point both forms agree; at a stopped iterate the
  second line is a unitary conjugate of W_n - (F - W~) (spectrum off by O(r), r the
  residual), while W_n + h C differs from that by F - W~ itself, which cancels the residual
  to first order (spectrum off by O(h ||P|| r));
* Q is skew-Hermitian in exact arithmetic and is projected, Q <- (Q - Q^H)/2;
* with ``maxit`` reached first, W_{n+1} comes from the last W~ and the caller is told the
  residual (a fixed iteration count, as in the paper's timing runs, is ``tol = 0``);
* P = Delta_N^+ W~ is the pseudo-inverse stream solve of ``stream.py``.

Higher order (``composition_weights``, ``isomp_composed_run``).  Sec. 2 places the midpoint
map in the family of isospectral integrators obtained from symplectic Runge--Kutta methods
and names higher-order members without giving them.  The higher-order members built here are
symmetric compositions of the midpoint map itself: every substep is isospectral and
Lie--Poisson, so their composition is too, and because the midpoint map is symmetric (its
adjoint is itself) the triple jump Phi_{g1 h} o Phi_{g2 h} o Phi_{g1 h}, with 2 g1 + g2 = 1
and 2 g1^(p+1) + g2^(p+1) = 0, raises an even order p to p + 2 (the composition method of
Yoshida, Phys. Lett. A 150, 1990).  Readings taken here: the order-6 method is the triple jump
applied twice (9 substeps); with ``extrapolate`` every substep after the first of a run starts
from W + rho (W - F_prev), rho being the ratio of its step to the previous substep's (rho = 1,
the plain 2 W - F_prev, between the equal substeps of the midpoint rule).
"""

import numpy as np

from .stream import stream_solve


UPDATE_FORMS = ("second_line", "difference")


def isomp_step(Wn: np.ndarray, h: float, tol: float = 1e-12, maxit: int = 50,
               guess: np.ndarray | None = None, return_midpoint: bool = False,
               update: str = "second_line"):
    """One IsoMP step.  Returns (W_{n+1}, iterations, final residual).

    ``guess`` replaces the starting iterate W~ = W_n; with ``return_midpoint`` the map's last
    output F (the converged midpoint) is returned as a fourth value; ``update`` selects the
    form of W_{n+1} (see the module notes).
    """
    if update not in UPDATE_FORMS:
        raise ValueError("update must be 'second_line' or 'difference'")
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
            if update == "difference":
                W1 = Wn + h * C
            else:
                W1 = Wt + (0.5 * h) * C - (0.25 * h * h) * Q
            return (W1, k, r, F) if return_midpoint else (W1, k, r)
        Wt = F
    raise ValueError("maxit must be >= 1")


def extrapolate_midpoints(mids: list, degree: int) -> np.ndarray:
    """Value one step ahead of the polynomial of degree ``degree`` through the equally spaced
    samples mids[-1], mids[-2], ..., mids[-(degree+1)] (newest last): by Newton's forward
    differences, sum_{j=1}^{d+1} (-1)^(j+1) binom(d+1, j) mids[-j]."""
    from math import comb

    d = int(degree)
    if d < 0 or len(mids) < d + 1:
        raise ValueError("need degree + 1 samples")
    out = np.zeros_like(np.asarray(mids[-1], dtype=np.complex128))
    for j in range(1, d + 2):
        out = out + ((-1) ** (j + 1) * comb(d + 1, j)) * np.asarray(mids[-j], dtype=np.complex128)
    return out


def start_from_history(mids: list, states: list) -> np.ndarray:
    """Starting iterate of step k = len(mids) of a run from its k midpoints F_0 .. F_{k-1} and
    its k + 1 states W_0 .. W_k (both lists oldest first): with delta_j = F_j - (W_j +
    W_{j+1})/2, the value (W_k + W*_{k+1})/2 + delta*_k, where W*_{k+1} extrapolates the states
    by the polynomial of degree k and delta*_k the deltas by the one of degree k - 1 (see the
    module notes)."""
    k = len(mids)
    if k < 1 or len(states) != k + 1:
        raise ValueError("need k >= 1 midpoints and k + 1 states")
    states = [np.asarray(w, dtype=np.complex128) for w in states]
    deltas = [np.asarray(mids[j], dtype=np.complex128) - 0.5 * (states[j] + states[j + 1])
              for j in range(k)]
    w_next = extrapolate_midpoints(states, k)
    d_next = extrapolate_midpoints(deltas, k - 1)
    return 0.5 * (states[k] + w_next) + d_next


def start_second_step(F0: np.ndarray, W0: np.ndarray, W1: np.ndarray, h: float,
                      D0: np.ndarray | None = None) -> np.ndarray:
    """Starting iterate of the second step of a run from the first step's midpoint F0, the
    states W0, W1 and the slope D0 = P_0 W0 - W0 P_0 (P_0 = Delta_N^+ W0; formed here when not
    given): with W*_2 = W0 + 2 h D0 + 4 a h^2 the quadratic through W0 with slope D0 and
    through W1 (a h^2 = W1 - W0 - h D0), the value (W1 + W*_2)/2 + (F0 - (W0 + W1)/2)."""
    W0 = np.asarray(W0, dtype=np.complex128)
    W1 = np.asarray(W1, dtype=np.complex128)
    if D0 is None:
        A = stream_solve(W0) @ W0
        D0 = A - A.conj().T
    ah2 = W1 - W0 - h * D0
    W2 = W0 + 2.0 * h * D0 + 4.0 * ah2
    delta0 = np.asarray(F0, dtype=np.complex128) - 0.5 * (W0 + W1)
    return 0.5 * (W1 + W2) + delta0


def composition_weights(order: int) -> list:
    """Substep fractions c_j (summing to 1) of the symmetric composition of order ``order``
    (2, 4 or 6): order 2 is the midpoint map alone; each triple jump from order p uses
    g1 = 1 / (2 - 2^(1/(p+1))) on both outer substeps and g2 = 1 - 2 g1 in the middle."""
    if order not in (2, 4, 6):
        raise ValueError("order must be 2, 4 or 6")
    w = [1.0]
    for p in range(2, order, 2):
        r = 2.0 ** (1.0 / (p + 1))
        g1 = 1.0 / (2.0 - r)
        g2 = 1.0 - 2.0 * g1
        w = [g1 * c for c in w] + [g2 * c for c in w] + [g1 * c for c in w]
    return w


def isomp_composed_run(W0: np.ndarray, h: float, nsteps: int, order: int, tol: float = 1e-12,
                       maxit: int = 50, extrapolate: bool = False, update: str = "second_line",
                       degree: int = 1):
    """nsteps steps of the composition of ``order`` from W0: each step is one midpoint substep
    of size c_j h for every c_j of ``composition_weights(order)``, in that order.  Returns
    (W, [evaluations per step], [largest substep residual per step]).

    With ``extrapolate`` a substep starts from W + rho (W - F_prev) (the previous substep's
    midpoint F_prev, rho the ratio of the two substeps); with ``degree`` d >= 2 as well, substep
    j of a step with k >= 2 earlier steps in the run starts from the polynomial of degree
    min(k - 1, d) through the last min(k, d + 1) midpoints of substep j (equally spaced, one
    step apart).  For order 2 this is ``isomp_run``'s start."""
    if degree not in (1, 2, 3):
        raise ValueError("degree must be 1, 2 or 3")
    w = composition_weights(order)
    W = np.asarray(W0, dtype=np.complex128).copy()
    iters, res = [], []
    mid, prev = None, None
    hist = [[] for _ in w]
    for _ in range(nsteps):
        its, rmax = 0, 0.0
        for j, c in enumerate(w):
            guess = None
            if extrapolate and degree >= 2 and len(hist[j]) >= 2:
                guess = extrapolate_midpoints(hist[j], min(len(hist[j]) - 1, degree))
            elif extrapolate and mid is not None:
                rho = c / prev
                guess = 2.0 * W - mid if rho == 1.0 else W + rho * (W - mid)
            W, k, r, mid = isomp_step(W, c * h, tol, maxit, guess=guess, return_midpoint=True,
                                      update=update)
            hist[j] = (hist[j] + [mid])[-(degree + 1):]
            prev = c
            its += k
            rmax = max(rmax, r)
        iters.append(its)
        res.append(rmax)
    return W, iters, res


def isomp_run(W0: np.ndarray, h: float, nsteps: int, tol: float = 1e-12, maxit: int = 50,
              extrapolate: bool = False, degree: int = 1, update: str = "second_line",
              on_step=None, solution_differences: bool = False):
    """nsteps IsoMP steps from W0.  Returns (W, [iterations], [residuals]).

    ``extrapolate``: starting iterates from the previous midpoints of this run (see the
    module notes); ``degree`` (1..3): the highest polynomial degree of that extrapolation;
    ``solution_differences`` (with degree 3): the third and fourth steps start from the
    midpoints and the states (``start_from_history``), and with the difference form the
    second from the first midpoint, the states and the slope at W_0 (``start_second_step``).
    ``on_step(n, W)`` is called after step n (1-based) with the current state."""
    if degree not in (1, 2, 3):
        raise ValueError("degree must be 1, 2 or 3")
    if solution_differences and not (extrapolate and degree == 3):
        raise ValueError("solution_differences needs extrapolate=True and degree=3")
    W = np.asarray(W0, dtype=np.complex128).copy()
    iters, res = [], []
    mids, states = [], [W.copy()]
    for n in range(nsteps):
        guess = None
        if solution_differences and n in (2, 3):
            guess = start_from_history(mids[-n:], states[-(n + 1):])
        elif solution_differences and n == 1 and update == "difference":
            guess = start_second_step(mids[-1], states[0], states[1], h)
        elif extrapolate and len(mids) == 1 or (extrapolate and degree == 1 and mids):
            guess = 2.0 * W - mids[-1]
        elif extrapolate and len(mids) >= 2:
            d = min(len(mids) - 1, degree)
            guess = extrapolate_midpoints(mids, d)
        W, k, r, mid = isomp_step(W, h, tol, maxit, guess=guess, return_midpoint=True,
                                  update=update)
        mids = (mids + [mid])[-(degree + 1):]
        if solution_differences:
            states = (states + [W.copy()])[-4:]
        iters.append(k)
        res.append(r)
        if on_step is not None:
            on_step(len(iters), W)
    return W, iters, res
