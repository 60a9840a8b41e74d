"""Guess mode 3: the third and fourth steps of a run start from the midpoint polynomial plus the
backward difference of the run's states, and with the difference form the second from the first
midpoint, the states and the slope at W_0 (the oracle's ``solution_differences``).

Checked against the oracle: evaluation counts equal and states within 1e-12 (relative
Frobenius) for both update forms and runs of every length up to 6 steps (the states rotate
through four buffers in the first steps, so each length ends in a different one and exercises
the copy back); at order 4 the mode is mode 2, bit for bit; with the stopping rule on the device
the results equal the host loop's bit for bit, also replayed from a captured graph.
"""

import numpy as np
import pytest

import oracle as O
from workloads import omega_coeffs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05466_amd import load_library

    load_library()
    return torch.device("cuda", 0)


def run_gpu(z, W0, h, steps, tol=1e-12, maxit=50):
    W = torch.from_numpy(W0).cuda()
    its, res = z.isomp_run(W, h, steps, tol, maxit)
    torch.cuda.synchronize()
    return W.cpu().numpy(), its, res


@pytest.mark.parametrize("N,law,form", [(64, "inv1", 1), (129, "inv1.5", 1), (256, "inv1.5", 1),
                                        (96, "inv1", 0)])
def test_history_start_matches_oracle(dev, N, law, form):
    from paper_2206_05466_amd import Zeuler

    h, steps = 0.005, 8
    W0 = O.assemble(N, omega_coeffs(N, 2, law))
    upd = "difference" if form == 1 else "second_line"
    Wr, itr, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3, update=upd,
                             solution_differences=True)
    _, it2, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3, update=upd)
    with Zeuler(N) as z:
        z.set_initial_guess(3)
        z.set_update_form(form)
        Wd, itd, rd = run_gpu(z, W0, h, steps)
    assert itd == itr, (itd, itr, it2)
    assert max(rd) < 1e-12
    assert np.linalg.norm(Wd - Wr) / np.linalg.norm(Wr) < 1e-12
    if form == 1 and law == "inv1.5":
        assert sum(itd) < sum(it2), (itd, it2)  # the saved evaluation


def test_history_start_every_run_length(dev):
    """Runs of 1 .. 6 steps end with their state in each of the rotating buffers in turn; each
    is copied back to the caller's matrix and matches the oracle."""
    from paper_2206_05466_amd import Zeuler

    N, h = 80, 0.01
    W0 = O.assemble(N, omega_coeffs(N, 4, "inv1"))
    with Zeuler(N) as z:
        z.set_initial_guess(3)
        z.set_update_form(1)
        for steps in range(1, 7):
            Wr, itr, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3,
                                     update="difference", solution_differences=True)
            Wd, itd, _ = run_gpu(z, W0, h, steps)
            assert itd == itr, (steps, itd, itr)
            assert np.linalg.norm(Wd - Wr) / np.linalg.norm(Wr) < 1e-12, steps


def test_history_start_order4_is_mode2(dev):
    from paper_2206_05466_amd import Zeuler

    N, h = 64, 0.02
    W0 = O.assemble(N, omega_coeffs(N, 1, "inv1"))
    out = []
    with Zeuler(N) as z:
        z.set_order(4)
        z.set_update_form(1)
        for mode in (2, 3):
            z.set_initial_guess(mode)
            out.append(run_gpu(z, W0, h, 6))
    assert out[0][1] == out[1][1] and np.array_equal(out[0][0], out[1][0])


def test_history_start_device_stopping_and_graph(dev):
    """Device stopping gives the host loop's results bit for bit; a captured 6-step run replayed
    twice equals eager runs from the same state."""
    from paper_2206_05466_amd import Zeuler

    N, h, tol, maxit, steps = 192, 0.005, 1e-12, 5, 6
    W0 = O.assemble(N, omega_coeffs(N, 3, "inv1.5"))
    with Zeuler(N) as z:
        z.set_initial_guess(3)
        z.set_update_form(1)
        Wh, ith, rh = run_gpu(z, W0, h, steps, tol, maxit)
        z.set_stopping(1)
        Wd, itd, rd = run_gpu(z, W0, h, steps, tol, maxit)
    assert itd == ith and rd == rh and np.array_equal(Wd, Wh)
    s = torch.cuda.Stream()
    zg, ze = Zeuler(N, stream=s), Zeuler(N)
    for z in (zg, ze):
        z.set_stopping(1)
        z.set_initial_guess(3)
        z.set_update_form(1)
    Wg = torch.from_numpy(W0).cuda()
    We = Wg.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        zg.isomp_run_async(Wg, h, steps, tol, maxit)
    torch.cuda.synchronize()
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        its_g, res_g, st_g = zg.run_stats(steps)
        its_e, res_e = ze.isomp_run(We, h, steps, tol, maxit)
        torch.cuda.synchronize()
        assert its_g == its_e and res_g == res_e and st_g == 0, (rep, its_g, its_e)
        assert torch.equal(Wg, We), rep
    zg.close()
    ze.close()
