"""Parity at the workloads' full sizes, in the launch configurations bench.py times.

The oracle cannot build the full-spectrum W_0 at N = 4096 quickly (a full eigen-decomposition
of every block), so the step tests start from the oracle's own assembly of the same seeded
coefficients truncated to low degree (same N, same kernels and launch shapes on the GPU);
the full-spectrum GPU basis assembly is checked on sampled diagonals, which the oracle can
form one at a time.  Bars: 1e-10 relative Frobenius after the steps (the spec bar), the
same evaluation counts, and Casimir drift <= 1e-11.
"""

import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, ensemble_sizes, omega_coeffs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05466_amd import load_library

    load_library()
    return torch.device("cuda", 0)


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.complex128)).cuda()


def to_host(X):
    torch.cuda.synchronize()
    return X.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def casimir_ok(W0, W):
    c0, c1 = O.casimirs(W0, 4), O.casimirs(W, 4)
    r = np.abs(c1 - c0) / np.abs(c0)
    return r[1] < 1e-11 and r[3] < 1e-11 and abs(c1[2] - c0[2]) / np.linalg.norm(W0) ** 3 < 1e-11


def test_n4096_steps_fp64_and_split(dev):
    from paper_2206_05466_amd import PREC_CRT, PREC_FP64, PREC_MIXED, PREC_SPLIT, Zeuler

    cfg = WORKLOADS["n4096"]
    N, h, L, steps = cfg["N"], cfg["h"], 32, 5
    W0 = O.assemble(N, omega_coeffs(N, 0, cfg["law"], lmax=L), lmax=L)
    # the polynomial start of the timed runs: steps 3..5 use degrees 1, 2, 3
    Wr, it_ref, _ = O.isomp_run(W0, h, steps, cfg["tol"], cfg["maxit"], extrapolate=True, degree=3)
    z = Zeuler(N)
    z.set_initial_guess(2)
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, steps, cfg["tol"], cfg["maxit"], PREC_FP64)
    W = to_host(Wd)
    assert its == it_ref and max(res) < cfg["tol"], (its, it_ref)
    assert rel(W, Wr) < 1e-12, rel(W, Wr)
    assert np.abs(W + W.conj().T).max() == 0.0
    z.set_split_slices(5)
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, steps, cfg["tol"], cfg["maxit"], PREC_SPLIT)
    W = to_host(Wd)
    assert its == it_ref and rel(W, Wr) < 1e-10, (its, rel(W, Wr))
    z.set_split_slices(5)  # lower product: 4 slices
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, steps, cfg["tol"], cfg["maxit"], PREC_MIXED)
    W = to_host(Wd)
    assert its == it_ref and rel(W, Wr) < 1e-12, (its, rel(W, Wr))
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, steps, cfg["tol"], cfg["maxit"], PREC_CRT)
    W = to_host(Wd)
    assert its == it_ref and rel(W, Wr) < 1e-12, (its, rel(W, Wr))
    # the timed headline form: W_{n+1} = W_n + h (A - A^H)
    Wd_r, itd, _ = O.isomp_run(W0, h, steps, cfg["tol"], cfg["maxit"], extrapolate=True, degree=3,
                               update="difference")
    z.set_update_form(1)
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, steps, cfg["tol"], cfg["maxit"], PREC_FP64)
    W = to_host(Wd)
    assert its == itd and max(res) < cfg["tol"] and rel(W, Wd_r) < 1e-12, (its, itd)
    z.close()


@pytest.mark.parametrize("N", [4096, 3000, 2048])
def test_zgemm_crt_full_size_integers_exact_sampled_rows(dev, N):
    """The modular product at the full sizes on integer operands up to 2^19, where every
    modulus is needed and the exact sums (< 2^51) are FP64 integers: sampled rows equal numpy's
    exact row products.  N = 4096: one whole round of 256 x 256 tiles, XCD-ordered; N = 3000
    (ragged): 144 tiles over the whole K; N = 2048: 64 tiles, each split along K into 4 parts
    whose byte residues the combine adds."""
    from paper_2206_05466_amd import PREC_CRT, Zeuler

    rng = np.random.default_rng(N + 5)
    lim = 2 ** 19
    A = rng.integers(-lim, lim + 1, (N, N)) + 1j * rng.integers(-lim, lim + 1, (N, N))
    B = rng.integers(-lim, lim + 1, (N, N)) + 1j * rng.integers(-lim, lim + 1, (N, N))
    z = Zeuler(N)
    C = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_CRT))
    z.close()
    rows = np.concatenate([[0, N - 1], rng.integers(0, N, 6)])
    for r in rows:
        assert np.array_equal(C[r], A[r] @ B), r


def test_n4096_basis_sampled_diagonals(dev):
    from paper_2206_05466_amd import Zeuler

    N = 4096
    om = omega_coeffs(N, 0, "inv1.5")
    z = Zeuler(N)
    W = z.basis_assemble(om)
    for m in (0, 1, 1500, 4094, 4095):
        _, V = O.eigvecs(N, m)
        n = N - m
        i = np.arange(n)
        l = np.arange(m, N)
        ref = 1j * (V @ om[l * l + l + m])
        got = W[torch.arange(n) + m, torch.arange(n)].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), m
        if m > 0:
            refu = 1j * (-1) ** m * (V @ om[l * l + l - m])
            gotu = W[torch.arange(n), torch.arange(n) + m].cpu().numpy()
            assert np.abs(gotu - refu).max() <= 1e-11 * np.abs(refu).max(), m
    z.close()


def test_n4096_extract_sampled_and_spectrum_identity(dev):
    """The extraction at full size: the full-spectrum W_0 (GPU assembly) maps back to its
    coefficients; on sampled diagonals the oracle forms the projections one at a time from
    the GPU's W (bar 1e-11 of the largest, as for the assembly: the GPU's twisted-factorisation
    eigenvectors and LAPACK's agree to ~1e-12 at this size); and the spectrum obeys
    sum_l l(l+1) E_l = ||W||_F^2."""
    from paper_2206_05466_amd import Zeuler

    N = 4096
    om = omega_coeffs(N, 0, "inv1.5")
    z = Zeuler(N)
    W = z.basis_assemble(om)
    got = z.basis_extract(W)
    E = z.energy_spectrum(got).cpu().numpy()
    got = got.cpu().numpy()
    assert np.abs(got - om).max() <= 1e-12 * np.abs(om).max()
    for m in (0, 2, 2047, 4095):
        _, V = O.eigvecs(N, m)
        n = N - m
        l = np.arange(m, N)
        low = W[torch.arange(n) + m, torch.arange(n)].cpu().numpy()
        ref = -1j * (V.T @ low)
        assert np.abs(got[l * l + l + m] - ref).max() <= 1e-11 * np.abs(ref).max(), m
        if m > 0:
            up = W[torch.arange(n), torch.arange(n) + m].cpu().numpy()
            refu = -1j * (-1) ** m * (V.T @ up)
            assert np.abs(got[l * l + l - m] - refu).max() <= 1e-11 * np.abs(refu).max(), m
    nf2 = float(torch.linalg.norm(W).item()) ** 2
    ll = np.arange(N, dtype=np.float64)
    assert abs((ll * (ll + 1) * E).sum() - nf2) <= 1e-12 * nf2
    z.close()


def test_n2048_twenty_steps(dev):
    from paper_2206_05466_amd import Zeuler

    cfg = WORKLOADS["n2048"]
    N, h, L = cfg["N"], cfg["h"], 48
    W0 = O.assemble(N, omega_coeffs(N, 0, cfg["law"], lmax=L), lmax=L)
    Wr, it_ref, _ = O.isomp_run(W0, h, cfg["steps"], cfg["tol"], cfg["maxit"], extrapolate=True,
                                degree=3)
    z = Zeuler(N)
    z.set_initial_guess(2)
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, cfg["steps"], cfg["tol"], cfg["maxit"])
    W = to_host(Wd)
    assert its == it_ref and max(res) < cfg["tol"]
    assert rel(W, Wr) < 1e-10, rel(W, Wr)
    assert casimir_ok(W0, W)
    z.close()


def test_n512_hundred_steps(dev):
    from paper_2206_05466_amd import Zeuler

    cfg = WORKLOADS["n512"]
    N, h = cfg["N"], cfg["h"]
    W0 = O.assemble(N, omega_coeffs(N, 0, cfg["law"]))
    Wr, it_ref, _ = O.isomp_run(W0, h, cfg["steps"], cfg["tol"], cfg["maxit"])
    z = Zeuler(N)
    Wd = to_dev(W0)
    its, res = z.isomp_run(Wd, h, cfg["steps"], cfg["tol"], cfg["maxit"])
    W = to_host(Wd)
    assert its == it_ref and max(res) < cfg["tol"]
    assert rel(W, Wr) < 1e-10, rel(W, Wr)
    assert casimir_ok(W0, W)
    z.close()


@pytest.mark.parametrize("prec_name", ["fp64", "split"])
def test_ensemble64_sampled_members(dev, prec_name):
    """The full 64-simulation ensemble (bench.py's leg: polynomial start; FP64, and split with 5
    slices) for 6 steps, so the cubic start is reached; one member of each size class is checked
    against the oracle's run with the same start."""
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Ensemble, Zeuler

    cfg = WORKLOADS["ensemble64"]
    sizes = ensemble_sizes(cfg["nsim"], cfg["size_seed"], cfg["sizes"])
    h, tol, K, steps = cfg["h"], 1e-12, 8, 6
    picks = [sizes.index(n) for n in sorted(set(sizes))]
    # checked members start from the oracle's own assembly; the others from the GPU basis
    W0s = {j: O.assemble(sizes[j], omega_coeffs(sizes[j], cfg["seed0"] + j, cfg["law"])) for j in picks}
    ctxs = {n: Zeuler(n) for n in sorted(set(sizes))}
    Ws = [to_dev(W0s[j]) if j in W0s else
          ctxs[n].basis_assemble(omega_coeffs(n, cfg["seed0"] + j, cfg["law"])) for j, n in enumerate(sizes)]
    for z in ctxs.values():
        z.close()
    split = prec_name == "split"
    with Ensemble(sizes) as ens:
        if split:
            ens.set_split_slices(5)
        ens.set_initial_guess(2)
        ens.run(Ws, h, steps, tol, K, prec=PREC_SPLIT if split else PREC_FP64)
        its, res = ens.stats()
    assert max(res) < tol
    bar = 1e-10 if split else 1e-12
    for j in picks:
        Wr, it_ref, _ = O.isomp_run(W0s[j], h, steps, tol, K, extrapolate=True, degree=3)
        if not split:
            assert its[j] == it_ref[-1]
        assert rel(to_host(Ws[j]), Wr) < bar, (j, sizes[j])


def test_max_size_n16384_one_step_and_slice_limit(dev):
    """The largest N the library accepts: one FP64 step and one split-precision step (the
    default slice count there is the int32-exactness bound, 3) from a low-degree W_0 the
    oracle assembles.  The oracle cannot step at this size on the host; the checks are the
    properties every step has: convergence, exact skew-Hermitian output, conservation of
    C_2 = -||W||_F^2 (pinned at the start by the oracle's closed form), and the split result
    within the 3-slice error of the FP64 one."""
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Zeuler, ZeulerError

    N, h, L = 16384, 0.005, 6
    W0 = O.assemble(N, omega_coeffs(N, 3, "inv1", lmax=L), lmax=L)
    c2_ref = -np.linalg.norm(W0) ** 2  # C_2 = tr W^2 = -||W||_F^2 for skew-Hermitian W
    z = Zeuler(N)
    with pytest.raises(ZeulerError):
        z.set_split_slices(4)  # 4 * 2N * 128^2 >= 2^31: int32 sums could overflow
    Wd = to_dev(W0)
    del W0
    c0 = z.casimirs(Wd, 2)
    assert abs(c0[1] - c2_ref) <= 1e-13 * abs(c2_ref)
    Ws = Wd.clone()
    info = z.isomp_step(Wd, h, 1e-12, 8, prec=PREC_FP64)
    assert info.resid < 1e-12 and info.iters <= 4
    assert float((Wd + Wd.conj().T).abs().max().item()) == 0.0
    c1 = z.casimirs(Wd, 2)
    assert abs(c1[1] - c0[1]) <= 1e-12 * abs(c0[1])
    info = z.isomp_step(Ws, h, 1e-12, 8, prec=PREC_SPLIT)
    assert info.resid < 1e-12
    d = float((torch.linalg.norm(Ws - Wd) / torch.linalg.norm(Wd)).item())
    assert d < 1e-8, d
    z.close()
