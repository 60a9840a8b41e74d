"""On-device stopping rule (ze_set_stopping 1): the tolerance test of eq. (isomp_iter) taken on
the GPU, every evaluation up to maxit enqueued and skipped once the step has converged.

The kernels and their order are those of the host-tested loop, so the results are compared
with it bit for bit (W, evaluation counts, residuals), and with the oracle at the FP64 bar.
A run captured into a HIP graph is replayed several times, with eager work and
synchronisations between the replays, each replay checked against an eager run on a second
context.
"""

import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, omega_coeffs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05466_amd import load_library

    load_library()
    return torch.device("cuda", 0)


def field(N, seed=0, law="inv1"):
    return O.assemble(N, omega_coeffs(N, seed, law))


def run(z, W0, h, steps, tol, maxit, mode, guess, form, order=2, prec=0):
    z.set_stopping(mode)
    z.set_initial_guess(guess)
    z.set_update_form(form)
    z.set_order(order)
    W = torch.from_numpy(W0).cuda()
    if mode == 1:  # every step runs; the counts come back whatever the status
        z.isomp_run_async(W, h, steps, tol, maxit, prec)
        its, res, _ = z.run_stats(steps)
    else:
        its, res = z.isomp_run(W, h, steps, tol, maxit, prec)
    torch.cuda.synchronize()
    return W.cpu().numpy(), its, res


@pytest.mark.parametrize("N,guess,form", [(64, 0, 0), (64, 2, 1), (129, 1, 0), (512, 2, 1)])
def test_device_stopping_bit_identical_to_host_loop(dev, N, guess, form):
    from paper_2206_05466_amd import Zeuler

    h, tol, maxit, steps = 0.01, 1e-12, 6, 8
    W0 = field(N)
    with Zeuler(N) as z:
        Wh, ith, rh = run(z, W0, h, steps, tol, maxit, 0, guess, form)
        Wd, itd, rd = run(z, W0, h, steps, tol, maxit, 1, guess, form)
    assert itd == ith and rd == rh
    assert np.array_equal(Wd, Wh)
    if N == 64:
        Wr, itr, _ = O.isomp_run(W0, h, steps, tol, maxit, extrapolate=guess > 0,
                                 degree=3 if guess == 2 else 1,
                                 update="difference" if form == 1 else "second_line")
        assert itd == itr
        assert np.linalg.norm(Wd - Wr) / np.linalg.norm(Wr) < 1e-12


@pytest.mark.parametrize("prec_name,N", [("split", 160), ("mixed", 160), ("crt", 160),
                                         ("crt", 512), ("split", 512)])
def test_device_stopping_other_precisions_bit_identical(dev, prec_name, N):
    """The split (4 slices), mixed and modular products with the rule on the device: the same
    W, evaluation counts and residuals as their host loop, bit for bit (polynomial start,
    difference form), and the oracle's trajectory within each form's bar."""
    from paper_2206_05466_amd import PREC_CRT, PREC_MIXED, PREC_SPLIT, Zeuler

    prec = {"split": PREC_SPLIT, "mixed": PREC_MIXED, "crt": PREC_CRT}[prec_name]
    h, tol, maxit, steps = 0.01, 1e-12, 6, 8
    W0 = field(N, 5)
    with Zeuler(N) as z:
        z.set_split_slices(4)
        Wh, ith, rh = run(z, W0, h, steps, tol, maxit, 0, 2, 1, prec=prec)
        Wd, itd, rd = run(z, W0, h, steps, tol, maxit, 1, 2, 1, prec=prec)
        _, _, st = z.run_stats(steps)
    assert itd == ith and rd == rh and st == 0, (itd, ith)
    assert np.array_equal(Wd, Wh)
    if N == 160:
        Wr, itr, _ = O.isomp_run(W0, h, steps, tol, maxit, extrapolate=True, degree=3,
                                 update="difference")
        e = np.linalg.norm(Wd - Wr) / np.linalg.norm(Wr)
        assert e < (1e-12 if prec_name != "split" else 1e-9), e


def test_device_stopping_fixed_count_and_order4(dev):
    """tol = 0 runs exactly maxit evaluations and reports non-convergence; the order-4
    composition (three substeps per step) matches the host loop bit for bit."""
    from paper_2206_05466_amd import Zeuler
    from paper_2206_05466_amd.zeuler import ZE_ENOTCONV

    N, h = 96, 0.02
    W0 = field(N, 3)
    with Zeuler(N) as z:
        # the host loop stops a run at its first unconverged step: step it one call at a time
        z.set_stopping(0)
        Wt = torch.from_numpy(W0).cuda()
        infos = [z.isomp_step(Wt, h, 0.0, 3) for _ in range(3)]
        torch.cuda.synchronize()
        Wh = Wt.cpu().numpy()
        assert all(i.iters == 3 and not i.converged for i in infos)
        Wd, itd, rd = run(z, W0, h, 3, 0.0, 3, 1, 0, 0)
        assert itd == [3, 3, 3] and rd == [i.resid for i in infos] and np.array_equal(Wd, Wh)
        _, _, st = z.run_stats(3)
        assert st == ZE_ENOTCONV
        Wh, ith, rh = run(z, W0, h, 4, 1e-12, 6, 0, 2, 1, order=4)
        Wd, itd, rd = run(z, W0, h, 4, 1e-12, 6, 1, 2, 1, order=4)
    assert itd == ith and rd == rh and np.array_equal(Wd, Wh)


def test_steady_cap_same_steps(dev):
    """A steady cap of 2 from the fourth step (guess mode 3, difference form; no step needs more
    there) gives the uncapped run's W, counts and residuals bit for bit, on the host and on the
    device; a cap of 1 from the first step reports the start-up steps as not converged."""
    from paper_2206_05466_amd import Zeuler
    from paper_2206_05466_amd.zeuler import ZE_ENOTCONV

    N, h, tol, maxit, steps = 200, 0.005, 1e-12, 6, 9
    W0 = field(N, 6, "inv1.5")
    with Zeuler(N) as z:
        base = run(z, W0, h, steps, tol, maxit, 0, 3, 1)
        z.set_steady_cap(2, 3)
        for mode in (0, 1):
            got = run(z, W0, h, steps, tol, maxit, mode, 3, 1)
            assert got[1] == base[1] and got[2] == base[2] and np.array_equal(got[0], base[0]), mode
        z.set_steady_cap(1, 0)
        run(z, W0, h, steps, tol, maxit, 1, 3, 1)
        its, _, st = z.run_stats(steps)
        assert its[0] == 1 and st == ZE_ENOTCONV, its
        z.set_steady_cap(0, 0)
        from paper_2206_05466_amd import ZeulerError

        for cap, frm in ((-1, 0), (2, -1)):
            with pytest.raises(ZeulerError):
                z.set_steady_cap(cap, frm)


def test_device_stopping_graph_capture_replays(dev):
    """A 6-step run (polynomial start, difference form) captured into a graph on the context's
    stream and replayed three times; after each replay W and the run's counts equal those of
    an eager 6-step run from the same state on a second context."""
    from paper_2206_05466_amd import Zeuler

    cfg = WORKLOADS["n512"]
    N, h, tol, maxit, steps = 256, cfg["h"], 1e-12, 5, 6
    W0 = field(N, 1)
    s = torch.cuda.Stream()
    zg = Zeuler(N, stream=s)
    ze = Zeuler(N)
    for z in (zg, ze):
        z.set_stopping(1)
        z.set_initial_guess(2)
        z.set_update_form(1)
    Wg = torch.from_numpy(W0).cuda()
    We = Wg.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        zg.isomp_run_async(Wg, h, steps, tol, maxit)
    torch.cuda.synchronize()
    assert torch.equal(Wg, We)  # capture records, it does not run
    for rep in range(3):
        g.replay()  # on the current stream
        torch.cuda.synchronize()
        its_g, res_g, st_g = zg.run_stats(steps)
        its_e, res_e = ze.isomp_run(We, h, steps, tol, maxit)
        torch.cuda.synchronize()
        assert its_g == its_e and res_g == res_e and st_g == 0, (rep, its_g, its_e)
        assert torch.equal(Wg, We), rep
        # eager work between the replays
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        del junk
    Wr = W0
    for _ in range(3):
        Wr, _, _ = O.isomp_run(Wr, h, steps, tol, maxit, extrapolate=True, degree=3, update="difference")
    got = Wg.cpu().numpy()
    assert np.linalg.norm(got - Wr) / np.linalg.norm(Wr) < 1e-12
    zg.close()
    ze.close()
