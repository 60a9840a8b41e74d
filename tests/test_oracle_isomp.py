"""Pins of the oracle's IsoMP step (eqs. (isomp), (isomp_iter)).

No numeric worked example is printed in the paper, so the step is pinned by what the
scheme and the mathematics fix:

* convergence to the continuous flow dW/dt = [P, W], Delta_N P = W (eq. (Euler_vort_mat))
  at second order, against an independent high-order ODE integration whose right-hand
  side uses the dense pseudo-inverse Laplacian (this pins the sign of time and every term);
* isospectrality and Casimir conservation to the fixed-point tolerance (Sec. 2);
* skew-Hermitian, traceless output; reversibility under h -> -h (midpoint rule symmetry);
* steady states: zonal (and by rotation, degree-1) vorticity is exactly stationary; for a
  single degree l >= 2 the commutator vanishes and the step drifts only at O(h^3);
* SU(2) rotation equivariance;
* iteration counts of a few (2..5) at tolerance 1e-12 (Sec. 2 reports 2 to 3).

The order-4 and order-6 compositions of the step are pinned the same way: fourth and sixth
order against the independent ODE integration, isospectrality and reversibility of the
composed step, the order-2 composition being the midpoint run itself, and the extrapolated
substep starts reaching the same fixed points in fewer evaluations.
"""

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import oracle as O
from workloads import omega_coeffs


def w0(N, seed=0, law="inv1", lmax=None):
    return O.assemble(N, omega_coeffs(N, seed, law, lmax))


def spec(W):
    return np.linalg.eigvalsh(1j * W)


def test_structure_and_isospectral_n64():
    W = w0(64)
    W1, k, r = O.isomp_step(W, 0.01, 1e-12, 50)
    assert 2 <= k <= 5 and r < 1e-12
    assert np.abs(W1 + W1.conj().T).max() < 1e-15
    assert abs(np.trace(W1)) < 1e-13
    assert np.abs(spec(W1) - spec(W)).max() < 1e-12
    c0, c1 = O.casimirs(W, 4), O.casimirs(W1, 4)
    assert np.abs(c1 - c0)[1:].max() < 1e-12 * np.abs(c0[1])
    assert np.abs(W1 - W).max() > 1e-6  # it moved


def test_fixed_iteration_count_with_zero_tol():
    W = w0(16)
    _, k, r = O.isomp_step(W, 0.05, 0.0, 3)
    assert k == 3 and r > 0


def test_reversible():
    W = w0(24, 1)
    W1, _, _ = O.isomp_step(W, 0.05, 1e-14, 50)
    Wb, _, _ = O.isomp_step(W1, -0.05, 1e-14, 50)
    assert np.abs(Wb - W).max() < 1e-13


def _ode_reference(W0, T):
    """dW/dt = [P, W], P = pinv(Delta_N) W, integrated with DOP853 at tight tolerance."""
    N = W0.shape[0]
    Lp = np.linalg.pinv(O.brute_laplacian(N), rcond=1e-10)

    def rhs(_, y):
        W = (y[: N * N] + 1j * y[N * N:]).reshape(N, N)
        P = (Lp @ W.reshape(-1)).reshape(N, N)
        D = (P @ W - W @ P).reshape(-1)
        return np.concatenate([D.real, D.imag])

    y0 = np.concatenate([W0.real.reshape(-1), W0.imag.reshape(-1)])
    sol = solve_ivp(rhs, (0.0, T), y0, method="DOP853", rtol=1e-13, atol=1e-15)
    y = sol.y[:, -1]
    return (y[: N * N] + 1j * y[N * N:]).reshape(N, N)


def test_second_order_against_independent_ode():
    N = 8
    W = 3.0 * w0(N, 2)
    T = 0.8
    ref = _ode_reference(W, T)
    errs = []
    for nsteps in (4, 8, 16):
        Wh, _, _ = O.isomp_run(W, T / nsteps, nsteps, 1e-14, 100)
        errs.append(np.abs(Wh - ref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs
    assert errs[-1] < 1e-3 * np.abs(W).max()


def test_zonal_and_degree_one_are_steady():
    N = 16
    om = np.zeros(N * N, complex)
    for l in range(1, N):
        om[l * l + l] = 1.0 / (l + 1)  # m = 0 only: zonal
    Wz = O.assemble(N, om)
    W1, _, _ = O.isomp_step(Wz, 0.1, 1e-14, 50)
    assert np.abs(W1 - Wz).max() < 1e-14
    om = np.zeros(N * N, complex)
    om[1 * 1 + 1 + 1] = 0.3 - 0.2j
    om[1 * 1 + 1 - 1] = -np.conj(om[3])
    om[1 * 1 + 1] = 0.5
    Wr = O.assemble(N, om)
    W1, _, _ = O.isomp_step(Wr, 0.1, 1e-14, 50)
    assert np.abs(W1 - Wr).max() < 1e-13


def test_single_degree_commutator_vanishes_and_drift_is_cubic():
    N, l = 32, 3
    rng = np.random.default_rng(4)
    om = np.zeros(N * N, complex)
    om[l * l + l] = rng.standard_normal()
    for m in range(1, l + 1):
        c = rng.standard_normal() + 1j * rng.standard_normal()
        om[l * l + l + m] = c
        om[l * l + l - m] = (-1) ** m * np.conj(c)
    W = O.assemble(N, om)
    W /= np.linalg.norm(W, 2)
    P = O.stream_solve(W)
    assert np.abs(P @ W - W @ P).max() < 1e-15
    d = []
    for h in (0.1, 0.05, 0.025):
        W1, _, _ = O.isomp_step(W, h, 1e-15, 50)
        d.append(np.abs(W1 - W).max())
    assert 7.0 < d[0] / d[1] < 9.0 and 7.0 < d[1] / d[2] < 9.0, d


@pytest.mark.parametrize("axis", [0, 2])
def test_su2_equivariance(axis):
    N = 12
    W = w0(N, 3)
    U = expm(0.9j * O.spin_matrices(N)[axis])
    W1, _, _ = O.isomp_step(W, 0.05, 1e-14, 50)
    W1r, _, _ = O.isomp_step(U @ W @ U.conj().T, 0.05, 1e-14, 50)
    assert np.abs(W1r - U @ W1 @ U.conj().T).max() < 1e-13


def test_ten_steps_casimir_drift_n64():
    W = w0(64, 0)
    W10, iters, res = O.isomp_run(W, 0.01, 10, 1e-12, 50)
    assert all(2 <= k <= 5 for k in iters) and max(res) < 1e-12
    c0, c1 = O.casimirs(W, 4), O.casimirs(W10, 4)
    rel = np.abs(c1 - c0) / np.abs(c0)
    assert rel[1] < 1e-11 and rel[3] < 1e-11
    assert abs(c1[2] - c0[2]) / np.linalg.norm(W) ** 3 < 1e-11


def test_isospectral_in_strong_regime():
    """Large h ||P||: the step must still be an exact similarity (to the tolerance);
    a wrong h^2 term (e.g. P P W~ for P W~ P) shows up here at O(h^3)."""
    N = 10
    W = 4.0 * w0(N, 5)
    W1, k, r = O.isomp_step(W, 0.25, 1e-14, 200)
    assert r < 1e-14
    assert np.abs(spec(W1) - spec(W)).max() < 1e-12 * np.abs(spec(W)).max()
    assert np.abs(W1 - W).max() > 1e-2


def test_extrapolated_guess_same_fixed_point_fewer_evaluations():
    """Starting each step from 2 W_n - F_prev reaches the same fixed point (to the tolerance)
    in one evaluation fewer than starting from W_n (h = 0.005, N = 128)."""
    W = w0(128, 0)
    Wa, ia, ra = O.isomp_run(W, 0.005, 4, 1e-12, 50)
    Wb, ib, rb = O.isomp_run(W, 0.005, 4, 1e-12, 50, extrapolate=True)
    assert ia[0] == ib[0] and all(b == a - 1 for a, b in zip(ia[1:], ib[1:])), (ia, ib)
    assert max(rb) < 1e-12
    assert np.abs(Wa - Wb).max() < 1e-14
    # a deliberately wrong guess still converges to the same point (it is only a start)
    W1, _, _ = O.isomp_step(W, 0.005, 1e-13, 50)
    W1g, _, _ = O.isomp_step(W, 0.005, 1e-13, 50, guess=W + 0.01 * w0(128, 9))
    assert np.abs(W1 - W1g).max() < 1e-13


@pytest.mark.parametrize("order,lo,hi", [(4, 14.5, 17.0), (6, 54.0, 70.0)])
def test_composition_order_against_independent_ode(order, lo, hi):
    """Halving h divides the error at T by 2^order (the ODE reference is ~1e-13 accurate)."""
    N = 8
    W = 3.0 * w0(N, 2)
    T = 0.8
    ref = _ode_reference(W, T)
    errs = []
    for nsteps in (4, 8, 16):
        Wh, _, _ = O.isomp_composed_run(W, T / nsteps, nsteps, order, 1e-14, 100)
        errs.append(np.abs(Wh - ref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert lo < r1 < hi and lo < r2 < hi, (errs, r1, r2)
    # at equal h the higher order is the more accurate one
    W2, _, _ = O.isomp_run(W, T / 8, 8, 1e-14, 100)
    assert errs[1] < 0.1 * np.abs(W2 - ref).max()


def test_composition_weights_closed_form_properties():
    """Consistency (sum 1), symmetry, the order-4 condition sum c^3 = 0 of a symmetric
    composition, sum c^5 = 0 as well at order 6, and the known negative middle step."""
    assert O.composition_weights(2) == [1.0]
    for order, n in ((4, 3), (6, 9)):
        w = np.array(O.composition_weights(order))
        assert len(w) == n and abs(w.sum() - 1.0) < 1e-15
        assert np.array_equal(w, w[::-1])
        assert abs((w ** 3).sum()) < 1e-15 * (np.abs(w) ** 3).sum()
    w6 = np.array(O.composition_weights(6))
    assert abs((w6 ** 5).sum()) < 1e-15 * (np.abs(w6) ** 5).sum()
    g1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
    assert abs(O.composition_weights(4)[1] + 2.0 ** (1.0 / 3.0) * g1) < 1e-15  # g2 < 0
    with pytest.raises(ValueError):
        O.composition_weights(3)


@pytest.mark.parametrize("order", [4, 6])
def test_composition_isospectral_and_reversible(order):
    N = 16
    W = 2.0 * w0(N, 6)
    W1, its, res = O.isomp_composed_run(W, 0.1, 2, order, 1e-14, 100)
    assert max(res) < 1e-14 and len(its) == 2
    assert np.abs(spec(W1) - spec(W)).max() < 1e-12 * np.abs(spec(W)).max()
    assert np.abs(W1 + W1.conj().T).max() < 1e-15
    Wb, _, _ = O.isomp_composed_run(W1, -0.1, 2, order, 1e-14, 100)
    assert np.abs(Wb - W).max() < 1e-12 * np.abs(W).max()


def test_composition_order2_is_the_midpoint_run_and_extrapolation():
    W = w0(24, 7)
    for ex in (False, True):
        Wa, ia, ra = O.isomp_run(W, 0.02, 3, 1e-12, 50, extrapolate=ex)
        Wb, ib, rb = O.isomp_composed_run(W, 0.02, 3, 2, 1e-12, 50, extrapolate=ex)
        assert np.array_equal(Wa, Wb) and ia == ib and ra == rb
    Wa, ia, _ = O.isomp_composed_run(W, 0.02, 3, 4, 1e-13, 50)
    Wb, ib, rb = O.isomp_composed_run(W, 0.02, 3, 4, 1e-13, 50, extrapolate=True)
    assert max(rb) < 1e-13 and sum(ib) < sum(ia), (ia, ib)
    assert np.abs(Wa - Wb).max() < 1e-13


def test_stopped_iterate_stays_isospectral_to_order_h_p_r():
    """The difference form W_{n+1} = W_n + h C at an iterate stopped early (maxit 1..3,
    residual r up to 1e-2): W_{n+1} = U (W_n - E) U^H + E with U the Cayley transform of h P~
    and E = F - W~ (||E||_2 <= r for skew-Hermitian E), so by Weyl its eigenvalues move by at
    most ||U E U^H - E|| <= 2 h ||P~|| r / (1 - h ||P~|| / 2).  The second line of eq. (isomp)
    evaluated at the stopped iterate (the default form) moves them by O(r): after two
    evaluations it exceeds that bound."""
    W = w0(16, 3)
    ev = spec(W)
    hp = np.linalg.norm(O.stream_solve(W), 2)
    for h in (0.05, 0.1):
        for m in (1, 2, 3):
            W1, k, r = O.isomp_step(W, h, 0.0, m, update="difference")
            drift = np.abs(spec(W1) - ev).max()
            assert drift <= 2.5 * h * hp * r, (h, m, drift, r)
            assert drift < 0.02 * r
            assert np.abs(W1 + W1.conj().T).max() < 1e-15
            if m == 2:
                W2, _, r2 = O.isomp_step(W, h, 0.0, m)
                assert r2 == r and np.abs(spec(W2) - ev).max() > 2.5 * h * hp * r


def test_extrapolate_midpoints_exact_on_polynomials():
    """Newton extrapolation of degree d reproduces every matrix polynomial of degree <= d one
    step ahead, and misses a degree d + 1 term by exactly its (d+1)-th difference."""
    rng = np.random.default_rng(3)
    M = [rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5)) for _ in range(4)]

    def p(t, deg):
        return sum(M[i] * float(t) ** i for i in range(deg + 1))

    for d in (1, 2, 3):
        samples = [p(t, d) for t in range(d + 1)]
        got = O.extrapolate_midpoints(samples, d)
        assert np.abs(got - p(d + 1, d)).max() < 1e-12 * np.abs(p(d + 1, d)).max()
    # degree 2 on a cubic: p(4) - extrapolation = 3! M3 (the third difference of t^3)
    samples = [p(t, 3) for t in range(1, 4)]
    got = O.extrapolate_midpoints(samples, 2)
    assert np.abs((p(4, 3) - got) - 6.0 * M[3]).max() < 1e-11
    with pytest.raises(ValueError):
        O.extrapolate_midpoints(samples, 3)


def test_polynomial_start_one_evaluation_same_fixed_point():
    """Starting each step from the cubic extrapolation of the previous midpoints, with the
    difference form of W_{n+1}: after the start-up (W_n, linear, then degrees 1 and 2) a step
    needs one evaluation at tol = 1e-12, the residuals stay below it, and the trajectory agrees
    with the W_n-started one to the tolerance.  With the second-line form the same start
    reaches the same trajectory but needs a second evaluation every few steps."""
    W = O.assemble(256, omega_coeffs(256, 0, "inv1.5"))
    Wa, ia, ra = O.isomp_run(W, 0.005, 24, 1e-12, 50, update="difference")
    Wb, ib, rb = O.isomp_run(W, 0.005, 24, 1e-12, 50, extrapolate=True, degree=3,
                             update="difference")
    assert ib[0] == ia[0] and all(k == 1 for k in ib[4:]), ib
    assert max(rb) < 1e-12
    assert np.linalg.norm(Wa - Wb) < 1e-12 * np.linalg.norm(Wa)
    Wc, ic, rc = O.isomp_run(W, 0.005, 24, 1e-12, 50, extrapolate=True, degree=3)
    assert max(rc) < 1e-12 and 1.0 < sum(ic[4:]) / len(ic[4:]) < 2.0, ic
    assert np.linalg.norm(Wa - Wc) < 1e-12 * np.linalg.norm(Wa)
    with pytest.raises(ValueError):
        O.isomp_run(W, 0.005, 1, degree=4)


def test_start_from_history_exact_on_polynomial_states_and_offsets():
    """With states W_j = p(j) of degree k and midpoint offsets delta_j = q(j) of degree k - 1
    (F_j = (W_j + W_{j+1})/2 + delta_j), the start of step k is exactly F_k; a degree k + 1
    term c t^(k+1) in the states is missed by exactly half its (k+1)-th difference, (k+1)! c / 2
    (the state extrapolation enters the start with weight 1/2); and the start equals the
    midpoint polynomial of degree k - 1 plus the k-th backward difference of the states."""
    from math import comb, factorial

    rng = np.random.default_rng(11)
    M = [rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)) for _ in range(5)]
    D = [rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)) for _ in range(4)]

    def p(t, deg):
        return sum(M[i] * float(t) ** i for i in range(deg + 1))

    def q(t, deg):
        return sum(D[i] * float(t) ** i for i in range(deg + 1))

    for k in (1, 2, 3):
        states = [p(j, k) for j in range(k + 1)]
        mids = [0.5 * (p(j, k) + p(j + 1, k)) + q(j, k - 1) for j in range(k)]
        want = 0.5 * (p(k, k) + p(k + 1, k)) + q(k, k - 1)
        got = O.start_from_history(mids, states)
        assert np.abs(got - want).max() < 1e-11 * np.abs(want).max(), k
        # the simplified form: midpoint polynomial of degree k - 1 + k-th difference of states
        diff = sum((-1) ** j * comb(k, j) * states[k - j] for j in range(k + 1))
        alt = O.extrapolate_midpoints(mids, k - 1) + diff
        assert np.abs(got - alt).max() < 1e-11 * np.abs(want).max(), k
        # one degree too many in the states
        states1 = [p(j, k + 1) for j in range(k + 1)]
        mids1 = [0.5 * (p(j, k + 1) + p(j + 1, k + 1)) + q(j, k - 1) for j in range(k)]
        want1 = 0.5 * (p(k, k + 1) + p(k + 1, k + 1)) + q(k, k - 1)
        miss = want1 - O.start_from_history(mids1, states1)
        assert np.abs(miss - 0.5 * factorial(k + 1) * M[k + 1]).max() < 1e-10, k
    with pytest.raises(ValueError):
        O.start_from_history([M[0]], [M[0]])


def test_start_second_step_exact_on_quadratic_states():
    """States on a quadratic W(t) = a + b t + c t^2 sampled at t = 0, h, 2h (slope b at t = 0)
    with a constant midpoint offset: the second step's start is exactly F_1; with a cubic term
    d t^3 as well it misses F_1 by exactly 2 d h^3 (half of what the quadratic misses W(2h)
    by); and the slope formed from Delta_N^+ when not given is P W_0 - W_0 P."""
    rng = np.random.default_rng(5)
    a, b, c, d, e = [rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5)) for _ in range(5)]
    h = 0.3

    def W(t, cubic=0.0):
        return a + b * t + c * t * t + cubic * d * t ** 3

    F0 = 0.5 * (W(0) + W(h)) + e
    F1 = 0.5 * (W(h) + W(2 * h)) + e
    got = O.start_second_step(F0, W(0), W(h), h, D0=b)
    assert np.abs(got - F1).max() < 1e-12 * np.abs(F1).max()
    # with d t^3: the quadratic (W0, slope b, W1) extrapolates W(2h) = ... + 8 d h^3 as
    # 4 W(h) - 3 W(0) - 2 h b = ... + 4 d h^3, so the start misses F_1 by (8 - 4) d h^3 / 2
    F0c = 0.5 * (W(0, 1) + W(h, 1)) + e
    F1c = 0.5 * (W(h, 1) + W(2 * h, 1)) + e
    miss = F1c - O.start_second_step(F0c, W(0, 1), W(h, 1), h, D0=b)
    assert np.abs(miss - 2.0 * d * h ** 3).max() < 1e-12
    # the slope from the definition: D0 = P W0 - W0 P with P = Delta_N^+ W0
    W0 = O.assemble(12, omega_coeffs(12, 3, "inv1"))
    P = O.stream_solve(W0)
    D0 = P @ W0 - W0 @ P
    F = W0 + 0.1 * D0
    diff = O.start_second_step(F, W0, F, 0.01) - O.start_second_step(F, W0, F, 0.01, D0=D0)
    assert np.abs(diff).max() < 1e-15


def test_start_from_history_orders_on_a_trajectory():
    """On an IsoMP trajectory (N = 24, sigma_l = (l+1)^-1), halving h shrinks the distance of
    the start of step 2 to that step's converged midpoint about 8x (O(h^3)) and of step 3
    about 16x (O(h^4)); the midpoint polynomials alone give 4x and 8x."""
    W0 = O.assemble(24, omega_coeffs(24, 0, "inv1"))

    def errs(h):
        Ws, Fs = [W0], []
        for _ in range(4):
            W1, _, _, F = O.isomp_step(Ws[-1], h, 1e-15, 80, return_midpoint=True,
                                       update="difference")
            Ws.append(W1)
            Fs.append(F)
        e = lambda a, b: float(np.abs(a - b).sum(axis=1).max())  # noqa: E731
        return (e(O.start_from_history(Fs[:2], Ws[:3]), Fs[2]),
                e(O.start_from_history(Fs[:3], Ws[:4]), Fs[3]),
                e(O.extrapolate_midpoints(Fs[:2], 1), Fs[2]),
                e(O.extrapolate_midpoints(Fs[:3], 2), Fs[3]),
                e(O.start_second_step(Fs[0], Ws[0], Ws[1], h), Fs[1]),
                e(2.0 * Ws[1] - Fs[0], Fs[1]))

    a, b = errs(0.04), errs(0.02)
    r = [x / y for x, y in zip(a, b)]
    assert 6.5 < r[0] < 10 and 13 < r[1] < 20, r
    assert 3.3 < r[2] < 4.8 and 6.5 < r[3] < 10, r
    assert 6.5 < r[4] < 10 and 3.3 < r[5] < 4.8, r  # second step: O(h^3) against O(h^2)
    assert b[0] < 0.01 * b[2] and b[1] < 0.01 * b[3] and b[4] < 0.01 * b[5], b


def test_solution_difference_start_saves_an_evaluation():
    """The n4096 field law at N = 256, h = 0.005, difference form: with the slope at W_0 in
    the second step's start and the states in the third's and fourth's the run takes
    3, 1, 1, ... evaluations (the midpoints alone: 3, 2, 2, 1, ...), its residuals stay below
    tol and it reaches the W_n-started trajectory to 1e-12; with the second-line form the second
    step keeps the linear start."""
    W = O.assemble(256, omega_coeffs(256, 0, "inv1.5"))
    Wa, ia, _ = O.isomp_run(W, 0.005, 12, 1e-12, 50, update="difference")
    Wb, ib, _ = O.isomp_run(W, 0.005, 12, 1e-12, 50, extrapolate=True, degree=3,
                            update="difference")
    Wc, ic, rc = O.isomp_run(W, 0.005, 12, 1e-12, 50, extrapolate=True, degree=3,
                             update="difference", solution_differences=True)
    assert ib[:4] == [3, 2, 2, 1], ib
    assert ic[0] == 3 and all(k == 1 for k in ic[1:]), ic
    assert max(rc) < 1e-12
    assert np.linalg.norm(Wa - Wc) < 1e-12 * np.linalg.norm(Wa)
    _, idd, _ = O.isomp_run(W, 0.005, 5, 1e-12, 50, extrapolate=True, degree=3,
                            solution_differences=True)
    _, ie, _ = O.isomp_run(W, 0.005, 5, 1e-12, 50, extrapolate=True, degree=3)
    assert idd[:2] == ie[:2], (idd, ie)
    with pytest.raises(ValueError):
        O.isomp_run(W, 0.005, 1, extrapolate=True, degree=2, solution_differences=True)


def test_composition_polynomial_substep_starts():
    """Per-substep polynomial starts: for order 2 the composed run is the midpoint run with the
    same start, bit for bit; for orders 4 and 6 (difference form) every substep takes one
    evaluation after the start-up and the trajectory matches the W_n-started one to 1e-12."""
    W = w0(64, 0)
    for d in (2, 3):
        for u in ("second_line", "difference"):
            a = O.isomp_run(W, 0.01, 7, 1e-12, 50, extrapolate=True, degree=d, update=u)
            b = O.isomp_composed_run(W, 0.01, 7, 2, 1e-12, 50, extrapolate=True, update=u, degree=d)
            assert a[1] == b[1] and np.array_equal(a[0], b[0])
    W = O.assemble(128, omega_coeffs(128, 0, "inv1.5"))
    for order, ns in ((4, 3), (6, 9)):
        Wa, ia, _ = O.isomp_composed_run(W, 0.02, 8, order, 1e-12, 50, update="difference")
        Wb, ib, rb = O.isomp_composed_run(W, 0.02, 8, order, 1e-12, 50, extrapolate=True,
                                          update="difference", degree=3)
        assert all(k == ns for k in ib[4:]) and max(rb) < 1e-12, ib
        assert np.linalg.norm(Wa - Wb) < 1e-12 * np.linalg.norm(Wa)
    with pytest.raises(ValueError):
        O.isomp_composed_run(W, 0.02, 1, 4, degree=0)
