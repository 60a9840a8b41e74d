"""Runs split into calls with ze_set_continuation (eqs. (isomp), (isomp_iter); the starting
iterates of the polynomial modes): a trajectory taken as several ze_isomp_run calls equals,
bit for bit, the same trajectory taken as one call, and the oracle's run of the whole length,
for each starting-iterate mode, the order-4 composition, the on-device stopping rule and a
steady cap.  A call that differs (h, mode, a single ze_isomp_step in between, a mode-3
trajectory shorter than four steps) starts over at step 0, as without continuation."""

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05466_amd import load_library

    load_library()
    return torch.device("cuda", 0)


def field(N, seed):
    from workloads import omega_coeffs

    return O.assemble(N, omega_coeffs(N, seed, "inv1"))


def run_calls(z, W0, h, chunks, tol=1e-12, maxit=50):
    W = torch.from_numpy(W0).cuda()
    its = []
    for k in chunks:
        i, _ = z.isomp_run(W, h, k, tol, maxit)
        its += i
    torch.cuda.synchronize()
    return W.cpu().numpy(), its


@pytest.mark.parametrize("mode,order,stop", [(3, 2, 0), (2, 2, 0), (1, 2, 0), (0, 2, 0),
                                             (3, 2, 1), (3, 4, 0)])
def test_split_run_equals_one_run(dev, mode, order, stop):
    from paper_2206_05466_amd import Zeuler

    N, h = 64, 0.01
    W0 = field(N, 11)
    with Zeuler(N) as z:
        z.set_initial_guess(mode)
        z.set_update_form(1)
        z.set_order(order)
        z.set_stopping(stop)
        Wa, ia = run_calls(z, W0, h, [12])
        z.set_continuation(True)
        Wb, ib = run_calls(z, W0, h, [5, 1, 6])
    assert ia == ib, (ia, ib)
    assert np.array_equal(Wa, Wb)
    if order == 2 and stop == 0:
        Wr, ir, _ = O.isomp_run(W0, h, 12, 1e-12, 50, extrapolate=mode > 0,
                                degree=1 if mode == 1 else 3, update="difference",
                                solution_differences=mode == 3)
        assert ib == ir, (ib, ir)
        assert np.linalg.norm(Wb - Wr) <= 1e-12 * np.linalg.norm(Wr)


def test_continuation_across_stopping_modes(dev):
    """The stopping rule's place (host or device) may change between continued calls: both take
    the same evaluations, so the trajectory is that of one call."""
    from paper_2206_05466_amd import Zeuler

    N, h = 64, 0.01
    W0 = field(N, 14)
    with Zeuler(N) as z:
        z.set_initial_guess(3)
        z.set_update_form(1)
        Wa, ia = run_calls(z, W0, h, [11])
        z.set_continuation(True)
        W = torch.from_numpy(W0).cuda()
        ib = []
        for k, stop in ((5, 0), (3, 1), (3, 0)):
            z.set_stopping(stop)
            i, _ = z.isomp_run(W, h, k, 1e-12, 50)
            ib += i
        torch.cuda.synchronize()
    assert ia == ib, (ia, ib)
    assert np.array_equal(Wa, W.cpu().numpy())


def test_continuation_with_steady_cap(dev):
    """The steady cap goes by the trajectory's step index: a continued call's steps are capped
    from the trajectory's step 4 on, as in one call."""
    from paper_2206_05466_amd import Zeuler

    N, h = 96, 0.01
    W0 = field(N, 12)
    with Zeuler(N) as z:
        z.set_initial_guess(3)
        z.set_update_form(1)
        z.set_steady_cap(2, 4)
        Wa, ia = run_calls(z, W0, h, [10])
        z.set_continuation(True)
        Wb, ib = run_calls(z, W0, h, [4, 3, 3])
    assert ia == ib and np.array_equal(Wa, Wb)


def test_what_starts_over(dev):
    """Each of these makes the next call start at step 0: it then equals a fresh run on the
    same input (a second context without continuation)."""
    from paper_2206_05466_amd import Zeuler

    N, h = 64, 0.01
    W0 = field(N, 13)
    with Zeuler(N) as z, Zeuler(N) as fresh:
        for zz in (z, fresh):
            zz.set_initial_guess(3)
            zz.set_update_form(1)
        z.set_continuation(True)

        def check(W, h2, k):
            Wf = W.clone()
            i1, _ = z.isomp_run(W, h2, k, 1e-12, 50)
            i2, _ = fresh.isomp_run(Wf, h2, k, 1e-12, 50)
            torch.cuda.synchronize()
            assert i1 == i2 and torch.equal(W, Wf), (i1, i2)

        W = torch.from_numpy(W0).cuda()
        z.isomp_run(W, h, 6, 1e-12, 50)
        check(W, 0.5 * h, 3)            # another h
        z.isomp_run(W, h, 5, 1e-12, 50)
        z.isomp_step(W, h, 1e-12, 50)   # a single step in between
        check(W, h, 3)
        z.isomp_run(W, h, 3, 1e-12, 50)  # three steps: mode 3 cannot continue them
        check(W, h, 4)
        z.isomp_run(W, h, 5, 1e-12, 50)
        W2 = W.clone()                   # another buffer
        check(W2, h, 3)
        z.isomp_run(W, h, 5, 1e-12, 50)
        z.set_initial_guess(3)           # a step-option setter in between, even to the same
        check(W, h, 3)
        z.set_continuation(False)        # off
        check(W, h, 3)


@pytest.mark.parametrize("prec_name,mode", [("fp64", 3), ("fp64", 2), ("fp64", 1), ("split", 3)])
def test_ensemble_split_run_equals_one_run(dev, prec_name, mode):
    """The ensemble's trajectories taken as calls of 5, 1 and 6 steps with continuation equal,
    bit for bit, one call of 12 (matrices and the last step's counts and residuals); with a
    steady cap from step 4 as well."""
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Ensemble

    sizes = [40, 64, 96, 17]
    h, tol, K = 0.01, 1e-12, 8
    prec = PREC_SPLIT if prec_name == "split" else PREC_FP64
    W0s = [field(n, 20 + j) for j, n in enumerate(sizes)]
    out = []
    with Ensemble(sizes) as ens:  # one ensemble: the autotuner's choice is the same for both
        ens.set_initial_guess(mode)
        ens.set_update_form(1)
        ens.set_steady_cap(3, 4)
        if prec == PREC_SPLIT:
            ens.set_split_slices(5)
        ens.set_continuation(True)
        for chunks in ([12], [5, 1, 6]):  # the second set of matrices starts at step 0
            Wd = [torch.from_numpy(W).cuda() for W in W0s]
            for k in chunks:
                ens.run(Wd, h, k, tol, K, prec=prec)
            its, res = ens.stats()
            torch.cuda.synchronize()
            out.append(([W.cpu().numpy() for W in Wd], list(its), list(res)))
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
    if prec == PREC_FP64 and mode == 3:
        for j in range(len(sizes)):
            Wr, ir, _ = O.isomp_run(W0s[j], h, 12, tol, K, extrapolate=True, degree=3,
                                    update="difference", solution_differences=True)
            assert np.linalg.norm(out[1][0][j] - Wr) <= 1e-12 * np.linalg.norm(Wr)
