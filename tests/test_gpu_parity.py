"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by element.

Tolerances (FP64 throughout):
* stream solve: each diagonal is a forward/backward recurrence of length <= N with
  multipliers below 1 in magnitude; relative error <~ N eps -> 1e-12 relative (max-norm).
* products: FP64 MFMA accumulates K = N terms; |C - C_ref| <= ~N eps |A||B| -> 1e-13
  relative to max|A| max|B| N; exact on small integers (all partial sums are integers
  below 2^53).
* IsoMP steps: the spec bar, 1e-10 relative Frobenius error after 10 steps, with the
  same iteration counts (the residuals differ only by rounding).
* basis assembly: the eigenvectors agree with LAPACK's to ~1e-13 (twisted factorisation
  with the exact eigenvalue); W is compared at 1e-11 relative.
"""

import ctypes

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

    load_library()  # must load: no fallback
    return torch.device("cuda", 0)


def ctx(N):
    from paper_2206_05466_amd import Zeuler

    return Zeuler(N)


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.complex128)).cuda()


def to_host(X):
    torch.cuda.synchronize()
    return X.cpu().numpy()


def rand_skew(N, seed, traceless=True):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    W = X - X.conj().T
    if traceless:
        W -= np.trace(W) / N * np.eye(N)
    return W


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ------------------------------------------------------------------ stream solve
# launch-shape limits of the band widths: 191/383/639 (one lane), 1150 (two lanes), 2172 (four)
@pytest.mark.parametrize("N", [1, 2, 3, 5, 63, 64, 65, 130, 191, 192, 257, 383, 384, 512, 639, 640,
                               1150, 1151, 2172, 2173])
@pytest.mark.parametrize("traceless", [True, False])
def test_stream_solve_parity(dev, N, traceless):
    W = rand_skew(N, N, traceless)
    with ctx(N) as z:
        P = to_host(z.stream_solve(to_dev(W)))
    P_ref = O.stream_solve(W)
    assert relmax(P, P_ref) < 1e-12, (N, relmax(P, P_ref))
    assert np.abs(P + P.conj().T).max() == 0.0


def test_stream_solve_single_degree(dev):
    N, l, m = 96, 7, 3
    om = np.zeros(N * N, complex)
    om[l * l + l + m] = 0.6 - 0.2j
    om[l * l + l - m] = (-1) ** m * np.conj(om[l * l + l + m])
    W = O.assemble(N, om)
    with ctx(N) as z:
        P = to_host(z.stream_solve(to_dev(W)))
    assert np.abs(P + W / (l * (l + 1))).max() < 1e-14


# ------------------------------------------------------------------ products
# sizes on both sides of the small kernel's limit (32 x 32 tiles, one per CU: N <= 512 on 256 CUs)
@pytest.mark.parametrize("N", [1, 7, 64, 100, 128, 129, 200, 256, 511, 512, 513])
def test_zgemm_small_integers_exact(dev, N):
    rng = np.random.default_rng(N)
    A = rng.integers(-8, 9, (N, N)) + 1j * rng.integers(-8, 9, (N, N))
    B = rng.integers(-8, 9, (N, N)) + 1j * rng.integers(-8, 9, (N, N))
    with ctx(N) as z:
        C = to_host(z.zgemm(to_dev(A), to_dev(B)))
    assert np.array_equal(C, A @ B)


# 1500: the split rule's whole tiles a multiple of the CU count (256 whole, 32 tiles in K ranges)
@pytest.mark.parametrize("N", [64, 131, 384, 512, 544, 1500])
def test_zgemm_random(dev, N):
    rng = np.random.default_rng(N + 1)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    B = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    with ctx(N) as z:
        C = to_host(z.zgemm(to_dev(A), to_dev(B)))
    err = np.abs(C - A @ B).max() / (N * np.abs(A).max() * np.abs(B).max())
    assert err < 1e-15, err


# ------------------------------------------------------------------ IsoMP step
def w0(N, seed, law="inv1", lmax=None):
    return O.assemble(N, omega_coeffs(N, seed, law, lmax))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_isomp_ten_steps_n64(dev, seed):
    N, h = 64, 0.01
    W0 = w0(N, seed)
    Wr, it_ref, res_ref = O.isomp_run(W0, h, 10, 1e-12, 50)
    Wd = to_dev(W0)
    with ctx(N) as z:
        its, res = z.isomp_run(Wd, h, 10, 1e-12, 50)
        W = to_host(Wd)
    assert its == it_ref, (its, it_ref)
    assert max(res) < 1e-12
    err = np.linalg.norm(W - Wr) / np.linalg.norm(Wr)
    assert err < 1e-10, err
    assert np.abs(W + W.conj().T).max() == 0.0
    c0, c1 = O.casimirs(W0, 4), O.casimirs(W, 4)
    rel = np.abs(c1 - c0) / np.abs(c0)
    assert rel[1] < 1e-11 and rel[3] < 1e-11
    assert abs(c1[2] - c0[2]) / np.linalg.norm(W0) ** 3 < 1e-11


@pytest.mark.parametrize("N", [1, 2, 3, 65, 130, 200])
def test_isomp_ragged_sizes(dev, N):
    h = 0.02
    W0 = w0(N, 5) if N > 1 else np.zeros((1, 1), complex)
    W1, k, r = O.isomp_step(W0, h, 1e-13, 50)
    Wd = to_dev(W0)
    with ctx(N) as z:
        info = z.isomp_step(Wd, h, 1e-13, 50)
        W = to_host(Wd)
    assert info.converged and info.iters == k
    assert np.linalg.norm(W - W1) <= 1e-12 * max(np.linalg.norm(W1), 1e-300) + 1e-300


def test_isomp_one_step_n512(dev):
    N, h = 512, 0.005
    W0 = w0(N, 0)
    W1, k, r = O.isomp_step(W0, h, 1e-12, 50)
    Wd = to_dev(W0)
    with ctx(N) as z:
        info = z.isomp_step(Wd, h, 1e-12, 50)
        W = to_host(Wd)
    assert info.iters == k and info.converged
    assert np.linalg.norm(W - W1) / np.linalg.norm(W1) < 1e-12


def test_isomp_fixed_iterations_and_errors(dev):
    from paper_2206_05466_amd import ZeulerError

    N = 32
    W0 = w0(N, 3)
    W1, k, r = O.isomp_step(W0, 0.05, 0.0, 3)
    Wd = to_dev(W0)
    with ctx(N) as z:
        info = z.isomp_step(Wd, 0.05, 0.0, 3)
        assert info.iters == 3 and not info.converged
        assert abs(info.resid - r) <= 1e-3 * r
        assert np.linalg.norm(to_host(Wd) - W1) / np.linalg.norm(W1) < 1e-13
        with pytest.raises(ZeulerError):
            z.isomp_step(Wd, float("nan"), 1e-12, 5)
        with pytest.raises(ZeulerError):
            z.isomp_step(Wd, 0.1, 1e-12, 0)
        bad = Wd.clone()
        bad[3, 1] = float("nan")
        with pytest.raises(ZeulerError, match="non-finite"):
            z.isomp_step(bad, 0.1, 1e-12, 5)
        with pytest.raises(ZeulerError):
            z.set_initial_guess(4)
        with pytest.raises(ZeulerError):
            z.set_split_slices(1)
        lib = z.lib
        p = ctypes.c_void_p(Wd.data_ptr())
        assert lib.ze_basis_extract(z._ctx, p, p) != 0  # omega aliasing W
        assert lib.ze_energy_spectrum(z._ctx, None, p) != 0
        assert lib.ze_basis_assemble(z._ctx, p, p) != 0


def test_ensemble_argument_errors(dev):
    from paper_2206_05466_amd import Ensemble, ZeulerError

    with Ensemble([16, 24]) as ens:
        with pytest.raises(ZeulerError):
            ens.set_initial_guess(-1)
        with pytest.raises(ZeulerError):
            ens.set_split_slices(99)
        with pytest.raises(ZeulerError):
            ens.run([to_dev(w0(16, 1)), to_dev(w0(24, 2))], 0.01, 1, 1e-12, 0)  # K < 1
        for bad in (-1, 4):
            with pytest.raises(ZeulerError):
                ens.set_initial_guess(bad)
        for bad in (-1, 2):
            with pytest.raises(ZeulerError):
                ens.set_update_form(bad)
        ens.set_split_slices(4)
        for bad in (1, 5):
            with pytest.raises(ZeulerError):
                ens.set_split_slices_lower(bad)
        # the ensemble runs FP64 or split products only; the single-context modes and
        # unknown codes are refused before any launch
        from paper_2206_05466_amd import PREC_CRT, PREC_MIXED

        for bad in (PREC_MIXED, PREC_CRT, 4, -1):
            with pytest.raises(ZeulerError):
                ens.run([to_dev(w0(16, 1)), to_dev(w0(24, 2))], 0.01, 1, 1e-12, 4, prec=bad)


def test_unknown_precision_codes_rejected(dev):
    from paper_2206_05466_amd import PREC_MIXED, Zeuler, ZeulerError

    W = to_dev(w0(20, 3))
    before = W.clone()
    with Zeuler(20) as z:
        with pytest.raises(ZeulerError):  # mixed precision applies to the step only
            z.zgemm(W, W, prec=PREC_MIXED)
        for bad in (4, -1):
            with pytest.raises(ZeulerError):
                z.zgemm(W, W, prec=bad)
            with pytest.raises(ZeulerError):
                z.isomp_step(W, 0.01, prec=bad)
    assert torch.equal(W, before)


# ------------------------------------------------------------------ Casimirs
@pytest.mark.parametrize("N,kmax", [(1, 3), (17, 5), (64, 8), (200, 4)])
def test_casimirs_parity(dev, N, kmax):
    W = w0(N, 7) if N > 1 else np.array([[0.3j]])
    with ctx(N) as z:
        c = z.casimirs(to_dev(W), kmax)
    c_ref = O.casimirs(W, kmax)
    scale = np.array([np.linalg.norm(W) ** k for k in range(1, kmax + 1)])
    assert np.all(np.abs(c - c_ref) <= 1e-13 * N * scale + 1e-300), (c, c_ref)


# ------------------------------------------------------------------ basis assembly
@pytest.mark.parametrize("N", [1, 2, 3, 8, 64, 129, 256])
def test_basis_assemble_parity(dev, N):
    om = omega_coeffs(N, 11, "inv1")
    with ctx(N) as z:
        W = to_host(z.basis_assemble(om))
    W_ref = O.assemble(N, om)
    assert np.abs(W - W_ref).max() <= 1e-11 * max(np.abs(W_ref).max(), 1e-300), relmax(W, W_ref)
    assert np.abs(W + W.conj().T).max() == 0.0


def test_basis_single_elements(dev):
    """Each single coefficient reproduces i T_lm (eigenvector of Delta_N, eq. (lap_prop))."""
    N = 24
    with ctx(N) as z:
        for l in (0, 1, 5, 23):
            for m in sorted({-l, 0, l // 2, l}):
                om = np.zeros(N * N, complex)
                om[l * l + l + m] = 1.0
                W = to_host(z.basis_assemble(om))
                assert np.abs(W - O.assemble(N, om)).max() < 1e-13


# ------------------------------------------------------------------ extraction and spectrum
# omega_lm = -i <T_lm, W> (the inverse of the assembly, Sec. 3.2) and E_l (Sec. 4).
@pytest.mark.parametrize("N", [1, 2, 7, 64, 129, 300])
def test_basis_extract_and_spectrum_match_oracle(dev, N):
    rng = np.random.default_rng(N + 11)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    W = X - X.conj().T  # skew-Hermitian (trace not removed: omega_00 != 0)
    with ctx(N) as z:
        om = to_host(z.basis_extract(to_dev(W)))
        E = to_host(z.energy_spectrum(om))
    ref = O.extract(W)
    assert np.abs(om - ref).max() <= 1e-12 * np.abs(ref).max(), relmax(om, ref)
    E_ref = O.energy_spectrum(ref, N)
    assert np.abs(E - E_ref).max() <= 1e-12 * max(E_ref.max(), 1e-300)


def test_basis_extract_general_matrix(dev):
    """For a W that is not skew-Hermitian the coefficients of m < 0 come from the upper
    diagonals: each one is -i <T_lm, W>_F against the oracle's basis elements one by one."""
    N = 7
    rng = np.random.default_rng(5)
    W = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    with ctx(N) as z:
        om = to_host(z.basis_extract(to_dev(W)))
    for l in range(N):
        for m in range(-l, l + 1):
            e = np.zeros(N * N, complex)
            e[l * l + l + m] = 1.0
            T = O.assemble(N, e) / 1j
            assert abs(om[l * l + l + m] - (-1j) * np.vdot(T, W)) < 1e-13


def test_basis_roundtrip(dev):
    N = 256
    om = omega_coeffs(N, 21, "inv1")
    with ctx(N) as z:
        back = to_host(z.basis_extract(z.basis_assemble(om)))
    assert np.abs(back - om).max() <= 1e-13 * np.abs(om).max()


# ------------------------------------------------------------------ split precision
# Ozaki splitting on INT8 MFMA with s balanced slices (7 bits, then 8 bits each) per
# row/column scale: small integers are exact (the first slices carry them); otherwise
# |C - AB| <~ 3 * 2^(-8 s) * 2N max|A| max|B| (the roundings of both operands plus the dropped
# slice products), tested with a factor 10.
# The sizes also cover every tile order of the full INT8 product: row-major (column-tile
# count not a multiple of 4, e.g. N = 129), the 2 x 4 XCD regions walked row by row (N = 256,
# 1000 ragged, 1024), and in 8 x 8 super-tiles (N = 2048).
@pytest.mark.parametrize("N", [1, 7, 64, 100, 129, 256, 1000, 1024, 2048])
def test_zgemm_split_small_integers_exact(dev, N):
    from paper_2206_05466_amd import PREC_SPLIT

    rng = np.random.default_rng(N + 7)
    A = rng.integers(-8, 9, (N, N)) + 1j * rng.integers(-8, 9, (N, N))
    B = rng.integers(-8, 9, (N, N)) + 1j * rng.integers(-8, 9, (N, N))
    with ctx(N) as z:
        C = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_SPLIT))
    assert np.array_equal(C, A @ B)


@pytest.mark.parametrize("N,s", [(64, 6), (131, 4), (131, 6), (200, 8), (384, 5)])
def test_zgemm_split_random_bound(dev, N, s):
    from paper_2206_05466_amd import PREC_SPLIT

    rng = np.random.default_rng(N + s)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    B = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    with ctx(N) as z:
        z.set_split_slices(s)
        C = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_SPLIT))
    scale = 2 * N * np.abs(A).max() * np.abs(B).max()
    err = np.abs(C - A @ B).max() / scale
    assert err < 10 * 3 * 2.0 ** (-8 * s) + 1e-16, (s, err)


def test_zgemm_split_error_decreases_with_slices(dev):
    from paper_2206_05466_amd import PREC_SPLIT

    N = 96
    rng = np.random.default_rng(5)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    B = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    errs = []
    with ctx(N) as z:
        for s in (2, 3, 4, 5, 6):
            z.set_split_slices(s)
            C = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_SPLIT))
            errs.append(np.abs(C - A @ B).max())
    assert all(errs[i + 1] < errs[i] / 20 for i in range(4)), errs


@pytest.mark.parametrize("s", [5, 6, 8])
def test_isomp_split_ten_steps_n64(dev, s):
    from paper_2206_05466_amd import PREC_SPLIT

    N, h = 64, 0.01
    W0 = w0(N, 0)
    Wr, it_ref, _ = O.isomp_run(W0, h, 10, 1e-12, 50)
    Wd = to_dev(W0)
    with ctx(N) as z:
        z.set_split_slices(s)
        its, res = z.isomp_run(Wd, h, 10, 1e-12, 50, prec=PREC_SPLIT)
        W = to_host(Wd)
    err = np.linalg.norm(W - Wr) / np.linalg.norm(Wr)
    assert err < 1e-10, (s, err)
    assert max(res) < 1e-12
    assert np.abs(W + W.conj().T).max() == 0.0
    c0, c1 = O.casimirs(W0, 4), O.casimirs(W, 4)
    rel = np.abs(c1 - c0) / np.abs(c0)
    assert rel[1] < 1e-11 and rel[3] < 1e-11


def test_isomp_split_step_ragged_n1000(dev):
    """One split-precision step (4 slices) at a ragged size whose INT8 products both end in a
    partial round of block slots, split along K with exact atomic sums (full product: 128
    tiles in 4 parts each; lower product: 72 tiles in 4 parts), against the oracle's step."""
    from paper_2206_05466_amd import PREC_SPLIT

    N, h = 1000, 0.005
    W0 = O.assemble(N, omega_coeffs(N, 3, "inv1", lmax=40), lmax=40)
    Wr, it_ref, _ = O.isomp_step(W0, h, 1e-12, 50)
    Wd = to_dev(W0)
    with ctx(N) as z:
        z.set_split_slices(4)
        info = z.isomp_step(Wd, h, 1e-12, 50, prec=PREC_SPLIT)
        W = to_host(Wd)
    err = np.linalg.norm(W - Wr) / np.linalg.norm(Wr)
    assert info.iters == it_ref and err < 1e-10, (info.iters, it_ref, err)
    assert np.abs(W + W.conj().T).max() == 0.0


# ------------------------------------------------------------------ ensemble (graph replays)
def test_ensemble_matches_oracle_and_eager_each_replay(dev):
    """One graph replay per step; between replays the eager single-context path runs on the
    same inputs (and the host synchronises); every replay must match it and the oracle."""
    from paper_2206_05466_amd import Ensemble

    sizes = [48, 64, 100, 128, 32, 96]
    h, tol, K = 0.01, 1e-12, 8
    W0s = [w0(n, 40 + j) for j, n in enumerate(sizes)]
    Wd = [to_dev(W) for W in W0s]
    We = [to_dev(W) for W in W0s]
    Wr = [W.copy() for W in W0s]
    ctxs = [ctx(n) for n in sizes]
    with Ensemble(sizes) as ens:
        for step in range(3):
            ens.run(Wd, h, 1, tol, K)
            its, res = ens.stats()
            for j, z in enumerate(ctxs):
                info = z.isomp_step(We[j], h, tol, K)
                Wr[j], k, _ = O.isomp_step(Wr[j], h, tol, K)
                assert its[j] == info.iters == k, (step, j, its[j], info.iters, k)
                assert res[j] < tol
            torch.cuda.synchronize()
            for j in range(len(sizes)):
                a, b = to_host(Wd[j]), to_host(We[j])
                assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b), (step, j)
                assert np.linalg.norm(a - Wr[j]) <= 1e-12 * np.linalg.norm(Wr[j]), (step, j)
        choice, ms = ens.tuning()
        assert 0 <= choice < 4 and min(ms) > 0
    for z in ctxs:
        z.close()


def test_ensemble_multi_step_run_and_fixed_K(dev):
    from paper_2206_05466_amd import Ensemble

    sizes = [64, 40]
    W0s = [w0(n, 7 + j) for j, n in enumerate(sizes)]
    Wd = [to_dev(W) for W in W0s]
    with Ensemble(sizes) as ens:
        ens.run(Wd, 0.02, 4, 0.0, 2)  # tol 0: exactly K = 2 evaluations per step
        its, _ = ens.stats()
        assert its == [2, 2]
    for j, n in enumerate(sizes):
        W = W0s[j]
        for _ in range(4):
            W, _, _ = O.isomp_step(W, 0.02, 0.0, 2)
        assert np.linalg.norm(to_host(Wd[j]) - W) <= 1e-12 * np.linalg.norm(W)


def test_ensemble_steady_cap_same_steps(dev):
    """The steady cap (2 evaluations from the fifth step of a run, polynomial start) gives the
    same steps, bit for bit, as the full cap whenever the later steps need at most 2, and an odd
    step count (the last W_{n+1} in the scratch buffer, copied back) matches the oracle."""
    from paper_2206_05466_amd import Ensemble

    sizes = [64, 96, 130]
    h, tol, K, steps = 0.01, 1e-12, 6, 9
    W0s = [w0(n, 80 + j) for j, n in enumerate(sizes)]
    out = {}
    for cap in (0, 2):
        Wd = [to_dev(W) for W in W0s]
        with Ensemble(sizes) as ens:
            ens.set_initial_guess(2)
            ens.set_update_form(1)
            ens.set_steady_cap(cap, 4)
            ens.run(Wd, h, steps, tol, K)
            its, res = ens.stats()
        assert max(res) < tol and max(its) <= 2, (cap, its)
        out[cap] = [to_host(W) for W in Wd]
    for j in range(len(sizes)):
        assert np.array_equal(out[0][j], out[2][j]), j
        Wr, _, _ = O.isomp_run(W0s[j], h, steps, tol, K, extrapolate=True, degree=3,
                               update="difference")
        assert np.linalg.norm(out[2][j] - Wr) <= 1e-12 * np.linalg.norm(Wr), j


@pytest.mark.parametrize("cap,from_step", [(5, 0), (3, 1), (2, 4)])
def test_ensemble_steady_cap_history_start(dev, cap, from_step):
    """Guess mode 3 with the difference form under a steady cap whose graph runs from step 0,
    1 or 4 of the call (from step 1 on it has no copy of the first evaluation's output, which
    only step 0 makes): the same steps, bit for bit, as without the cap, and the oracle's run
    with solution_differences."""
    from paper_2206_05466_amd import Ensemble

    sizes = [64, 96, 130]
    h, tol, K, steps = 0.01, 1e-12, 6, 7
    W0s = [w0(n, 80 + j) for j, n in enumerate(sizes)]
    out = {}
    for c in (0, cap):
        Wd = [to_dev(W) for W in W0s]
        with Ensemble(sizes) as ens:
            ens.set_initial_guess(3)
            ens.set_update_form(1)
            ens.set_steady_cap(c, from_step)
            ens.run(Wd, h, steps, tol, K)
            its, res = ens.stats()
        assert max(res) < tol, (c, its, res)
        out[c] = [to_host(W) for W in Wd]
    for j in range(len(sizes)):
        assert np.array_equal(out[0][j], out[cap][j]), j
        Wr, _, _ = O.isomp_run(W0s[j], h, steps, tol, K, extrapolate=True, degree=3,
                               update="difference", solution_differences=True)
        assert np.linalg.norm(out[cap][j] - Wr) <= 1e-12 * np.linalg.norm(Wr), j


def test_ensemble_extrapolated_guess(dev):
    """Guess mode 1 in the ensemble (steps after the first of a run start from 2 W_n - F_prev):
    every simulation matches the single-context run in the same mode and the oracle's
    extrapolated run, with the same iteration count on the last step."""
    from paper_2206_05466_amd import Ensemble

    sizes = [64, 40, 96]
    h, tol, K, steps = 0.01, 1e-12, 8, 4
    W0s = [w0(n, 60 + j) for j, n in enumerate(sizes)]
    Wd = [to_dev(W) for W in W0s]
    with Ensemble(sizes) as ens:
        ens.set_initial_guess(1)
        ens.run(Wd, h, steps, tol, K)
        its, res = ens.stats()
    for j, n in enumerate(sizes):
        We = to_dev(W0s[j])
        with ctx(n) as z:
            z.set_initial_guess(1)
            it1, _ = z.isomp_run(We, h, steps, tol, K)
        Wr, itr, _ = O.isomp_run(W0s[j], h, steps, tol, K, extrapolate=True)
        a, b = to_host(Wd[j]), to_host(We)
        assert its[j] == it1[-1] == itr[-1] and res[j] < tol, (j, its[j], it1, itr)
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b), j
        assert np.linalg.norm(a - Wr) <= 1e-12 * np.linalg.norm(Wr), j


def test_ensemble_split_matches_single_context_and_oracle(dev):
    """Split-precision ensemble (ragged N, slice count changed between replays): every step
    matches the single-context split path and the oracle."""
    from paper_2206_05466_amd import PREC_SPLIT, Ensemble

    sizes = [48, 64, 100, 128, 200, 32, 130]
    h, tol, K = 0.01, 1e-12, 8
    W0s = [w0(n, 60 + j) for j, n in enumerate(sizes)]
    Wd = [to_dev(W) for W in W0s]
    We = [to_dev(W) for W in W0s]
    Wr = [W.copy() for W in W0s]
    ctxs = [ctx(n) for n in sizes]
    with Ensemble(sizes) as ens:
        for step, ns in enumerate((6, 6, 5)):
            ens.set_split_slices(ns)
            ens.run(Wd, h, 1, tol, K, prec=PREC_SPLIT)
            its, res = ens.stats()
            for j, z in enumerate(ctxs):
                z.set_split_slices(ns)
                info = z.isomp_step(We[j], h, tol, K, prec=PREC_SPLIT)
                Wr[j], _, _ = O.isomp_step(Wr[j], h, tol, K)
                assert its[j] == info.iters, (step, j, its[j], info.iters)
                assert res[j] < tol
            torch.cuda.synchronize()
            for j in range(len(sizes)):
                a, b = to_host(Wd[j]), to_host(We[j])
                assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b), (step, j)
                assert np.linalg.norm(a - Wr[j]) <= 1e-10 * np.linalg.norm(Wr[j]), (step, j)
                assert np.abs(a + a.conj().T).max() == 0.0
        choice, ms = ens.tuning(PREC_SPLIT)
        assert choice in (0, 1) and len(ms) == 2 and min(ms) > 0
        choice64, _ = ens.tuning()
        assert choice64 == -1  # no FP64 run yet
    for z in ctxs:
        z.close()


@pytest.mark.parametrize("prec_name", ["fp64", "split"])
def test_isomp_run_extrapolated_guess(dev, prec_name):
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT

    N, h = 128, 0.005
    W0 = w0(N, 0)
    Wr, it_ref, _ = O.isomp_run(W0, h, 6, 1e-12, 50, extrapolate=True)
    Wd = to_dev(W0)
    with ctx(N) as z:
        z.set_initial_guess(1)
        its, res = z.isomp_run(Wd, h, 6, 1e-12, 50, prec=PREC_SPLIT if prec_name == "split" else PREC_FP64)
        W = to_host(Wd)
    assert its == it_ref and max(res) < 1e-12, (its, it_ref)
    assert np.linalg.norm(W - Wr) <= 1e-12 * np.linalg.norm(Wr)


# ------------------------------------------------------------------ long-run properties
def test_long_run_isospectral_n64(dev):
    """2000 steps (the paper's long run: degrees 2..20 only, unit spectral norm, Sec. 4) on the
    GPU: the spectrum of iW and the Casimirs stay those of W_0 (the scheme is isospectral up to
    the fixed-point tolerance), W stays exactly skew-Hermitian, and every step converges."""
    N, h, steps = 64, 0.01, 2000
    W0 = w0(N, 11, "paper")
    W0 = W0 / np.linalg.norm(W0, 2)
    Wd = to_dev(W0)
    with ctx(N) as z:
        z.set_initial_guess(1)
        its, res = z.isomp_run(Wd, h, steps, 1e-12, 20)
    W = to_host(Wd)
    assert max(res) < 1e-12 and max(its) <= 4
    assert np.abs(W + W.conj().T).max() == 0.0
    lam0 = np.linalg.eigvalsh(1j * W0)
    lam = np.linalg.eigvalsh(1j * W)
    assert np.abs(lam - lam0).max() <= 1e-10, np.abs(lam - lam0).max()
    c0, c1 = O.casimirs(W0, 4), O.casimirs(W, 4)
    assert abs(c1[1] - c0[1]) <= 1e-10 * abs(c0[1]) and abs(c1[3] - c0[3]) <= 1e-10 * abs(c0[3])
    assert np.linalg.norm(W - W0) > 1e-2 * np.linalg.norm(W0)  # the field did evolve


def test_reversibility(dev):
    """A step with h followed by a step with -h returns W_0 (the midpoint scheme is symmetric);
    the two fixed points are each met to the tolerance."""
    N, h = 128, 0.02
    W0 = w0(N, 12)
    Wd = to_dev(W0)
    with ctx(N) as z:
        a = z.isomp_step(Wd, h, 1e-13, 50)
        b = z.isomp_step(Wd, -h, 1e-13, 50)
    assert a.converged and b.converged
    W = to_host(Wd)
    assert np.linalg.norm(W - W0) <= 1e-12 * np.linalg.norm(W0), np.linalg.norm(W - W0) / np.linalg.norm(W0)


# ------------------------------------------------------------------ higher order (compositions)
@pytest.mark.parametrize("order,N,guess", [(4, 64, 0), (4, 100, 1), (6, 64, 1), (6, 33, 0)])
def test_isomp_composed_matches_oracle(dev, order, N, guess):
    """Order-4 and order-6 steps (3 and 9 midpoint substeps, one of each triple backwards):
    the same evaluation counts per step as the oracle's composition and the same W to 1e-12,
    from W_n or from the extrapolated substep starts; then one more step through the
    single-step entry point, from the oracle's W."""
    h, steps = 0.02, 3
    W0 = w0(N, 5)
    ex = bool(guess)
    Wr, it_ref, _ = O.isomp_composed_run(W0, h, steps, order, 1e-12, 50, extrapolate=ex)
    W1r, i1, _ = O.isomp_composed_run(Wr, h, 1, order, 1e-12, 50, extrapolate=ex)
    Wd = to_dev(W0)
    with ctx(N) as z:
        z.set_order(order)
        z.set_initial_guess(guess)
        its, res = z.isomp_run(Wd, h, steps, 1e-12, 50)
        W = to_host(Wd)
        Wd = to_dev(Wr)
        info = z.isomp_step(Wd, h, 1e-12, 50)
        W1 = to_host(Wd)
    assert its == it_ref and max(res) < 1e-12, (its, it_ref)
    assert np.linalg.norm(W - Wr) <= 1e-12 * np.linalg.norm(Wr)
    assert info.converged and info.iters == i1[0], (info, i1)
    assert np.linalg.norm(W1 - W1r) <= 1e-12 * np.linalg.norm(W1r)
    assert np.abs(W1 + W1.conj().T).max() == 0.0


def test_isomp_composed_split_and_fixed_iterations(dev):
    """Order 4 with the split-precision products (5 slices) against the oracle (1e-10); and
    the fixed-iteration mode (tol = 0, maxit = 2): every substep still runs its 2 evaluations,
    the step reports 6 and is not converged, and W matches the oracle's fixed-count run."""
    from paper_2206_05466_amd import PREC_SPLIT, ZeulerError

    N, h = 64, 0.02
    W0 = w0(N, 8)
    Wr, _, _ = O.isomp_composed_run(W0, h, 3, 4, 1e-12, 50, extrapolate=True)
    Wf, itf, _ = O.isomp_composed_run(W0, h, 1, 4, 0.0, 2)
    with ctx(N) as z:
        z.set_order(4)
        z.set_initial_guess(1)
        z.set_split_slices(5)
        Wd = to_dev(W0)
        its, res = z.isomp_run(Wd, h, 3, 1e-12, 50, prec=PREC_SPLIT)
        W = to_host(Wd)
        z.set_initial_guess(0)
        Wd = to_dev(W0)
        info = z.isomp_step(Wd, h, 0.0, 2)
        Wx = to_host(Wd)
        for bad in (0, 3, 5, 8):
            with pytest.raises(ZeulerError):
                z.set_order(bad)
    assert max(res) < 1e-12
    assert np.linalg.norm(W - Wr) <= 1e-10 * np.linalg.norm(Wr)
    assert not info.converged and info.iters == itf[0] == 6
    assert np.linalg.norm(Wx - Wf) <= 1e-12 * np.linalg.norm(Wf)


# ------------------------------------------------------------------ polynomial starting iterates
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("N,law,h,steps", [(64, "inv1", 0.01, 12), (130, "inv1.5", 0.005, 10),
                                           (256, "inv1.5", 0.005, 9)])
def test_isomp_run_polynomial_guess(dev, N, law, h, steps, form):
    """Mode 2 (cubic extrapolation of the run's midpoints), with either form of W_{n+1}: the
    same evaluation counts per step as the oracle's run of that form and the same W to 1e-12;
    a second run call restarts the history (its first step starts from W_n again)."""
    upd = ("second_line", "difference")[form]
    W0 = w0(N, 4, law)
    Wr, it_ref, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3, update=upd)
    W2r, it2, _ = O.isomp_run(Wr, h, 3, 1e-12, 50, extrapolate=True, degree=3, update=upd)
    Wd = to_dev(W0)
    with ctx(N) as z:
        z.set_update_form(form)
        z.set_initial_guess(2)
        its, res = z.isomp_run(Wd, h, steps, 1e-12, 50)
        W = to_host(Wd)
        Wd = to_dev(Wr)
        its2, _ = z.isomp_run(Wd, h, 3, 1e-12, 50)
        W2 = to_host(Wd)
    assert its == it_ref and max(res) < 1e-12, (its, it_ref)
    assert np.linalg.norm(W - Wr) <= 1e-12 * np.linalg.norm(Wr)
    assert its2 == it2 and np.linalg.norm(W2 - W2r) <= 1e-12 * np.linalg.norm(W2r)
    assert np.abs(W + W.conj().T).max() == 0.0


def test_isomp_polynomial_guess_split_and_mode_errors(dev):
    """Mode 2 with the split-precision products (5 slices) and the difference form of W_{n+1}
    against the oracle's FP64 run (1e-10), one evaluation per step at the end; update forms
    other than 0 and 1 and guess modes outside 0..3 are rejected."""
    from paper_2206_05466_amd import PREC_SPLIT, ZeulerError

    N, h = 128, 0.005
    W0 = w0(N, 0)
    Wr, _, _ = O.isomp_run(W0, h, 10, 1e-12, 50, extrapolate=True, degree=3, update="difference")
    with ctx(N) as z:
        z.set_split_slices(5)
        z.set_update_form(1)
        for bad in (-1, 2):
            with pytest.raises(ZeulerError):
                z.set_update_form(bad)
        z.set_initial_guess(2)
        Wd = to_dev(W0)
        its, res = z.isomp_run(Wd, h, 10, 1e-12, 50, prec=PREC_SPLIT)
        W = to_host(Wd)
        with pytest.raises(ZeulerError):
            z.set_initial_guess(4)
    assert max(res) < 1e-12 and its[-1] == 1, its
    assert np.linalg.norm(W - Wr) <= 1e-10 * np.linalg.norm(Wr)


@pytest.mark.parametrize("prec_name,form", [("fp64", 0), ("split", 0), ("fp64", 1), ("split", 1)])
def test_ensemble_polynomial_guess(dev, prec_name, form):
    """Guess mode 2 in the ensemble (one graph; the step index of the run read on the device):
    after 7 steps every simulation matches the oracle's run with the polynomial start (FP64:
    1e-12 and the same evaluation count on the last step; split, 5 slices: 1e-10), and a
    second run call starts its history again (its first step from W_n)."""
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Ensemble

    sizes = [64, 40, 96, 130]
    h, tol, K, steps = 0.005, 1e-12, 8, 7
    split = prec_name == "split"
    upd = ("second_line", "difference")[form]
    W0s = [w0(n, 70 + j) for j, n in enumerate(sizes)]
    refs = [O.isomp_run(W, h, steps, tol, K, extrapolate=True, degree=3, update=upd) for W in W0s]
    refs2 = [O.isomp_run(r[0], h, 2, tol, K, extrapolate=True, degree=3, update=upd) for r in refs]
    Wd = [to_dev(W) for W in W0s]
    with Ensemble(sizes) as ens:
        ens.set_update_form(form)
        if split:
            ens.set_split_slices(5)
        ens.set_initial_guess(2)
        prec = PREC_SPLIT if split else PREC_FP64
        ens.run(Wd, h, steps, tol, K, prec=prec)
        its, res = ens.stats()
        got = [to_host(W) for W in Wd]
        Wd2 = [to_dev(r[0]) for r in refs]
        ens.run(Wd2, h, 2, tol, K, prec=prec)
        its2, _ = ens.stats()
        got2 = [to_host(W) for W in Wd2]
    bar = 1e-10 if split else 1e-12
    for j in range(len(sizes)):
        Wr, itr, _ = refs[j]
        W2r, itr2, _ = refs2[j]
        assert res[j] < tol
        if not split:
            assert its[j] == itr[-1] and its2[j] == itr2[-1], (j, its[j], itr, its2[j], itr2)
        assert np.linalg.norm(got[j] - Wr) <= bar * np.linalg.norm(Wr), j
        assert np.linalg.norm(got2[j] - W2r) <= bar * np.linalg.norm(W2r), j


@pytest.mark.parametrize("prec_name,form", [("fp64", 1), ("fp64", 0), ("split", 1)])
def test_ensemble_history_start(dev, prec_name, form):
    """Guess mode 3 in the ensemble: runs of 1 .. 5 steps (each a call of its own from W_0, so
    each ends in another buffer of the states' rotation) end, for every simulation, where the
    oracle's run with solution_differences does (FP64: 1e-12 and the evaluation count of the
    run's last step, i.e. of every step in turn; split, 5 slices: 1e-10)."""
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Ensemble

    sizes = [64, 40, 96, 130]
    h, tol, K = 0.005, 1e-12, 8
    split = prec_name == "split"
    upd = ("second_line", "difference")[form]
    W0s = [w0(n, 90 + j) for j, n in enumerate(sizes)]
    refs = [O.isomp_run(W, h, 5, tol, K, extrapolate=True, degree=3, update=upd,
                        solution_differences=True)[1] for W in W0s]
    bar = 1e-10 if split else 1e-12
    with Ensemble(sizes) as ens:
        ens.set_update_form(form)
        if split:
            ens.set_split_slices(5)
        ens.set_initial_guess(3)
        prec = PREC_SPLIT if split else PREC_FP64
        for L in range(1, 6):
            Wd = [to_dev(W) for W in W0s]
            ens.run(Wd, h, L, tol, K, prec=prec)
            its, res = ens.stats()
            got = [to_host(W) for W in Wd]
            for j in range(len(sizes)):
                Wr, _, _ = O.isomp_run(W0s[j], h, L, tol, K, extrapolate=True, degree=3,
                                       update=upd, solution_differences=True)
                assert res[j] < tol, (L, j)
                if not split:
                    assert its[j] == refs[j][L - 1], (L, j, its[j], refs[j])
                assert np.linalg.norm(got[j] - Wr) <= bar * np.linalg.norm(Wr), (L, j)


def test_split_lower_slices(dev):
    """The lower product Q = A P with one slice fewer than A (the default) or with as many:
    both runs stay within 1e-10 of the oracle and within 1e-12 of each other at h = 0.005 (Q's
    term carries h^2/4), and the setters reject counts outside 2 .. s."""
    from paper_2206_05466_amd import PREC_SPLIT, ZeulerError

    N, h, steps = 128, 0.005, 6
    W0 = w0(N, 5)
    Wr, _, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3)
    out = []
    with ctx(N) as z:
        z.set_initial_guess(2)
        for sq in (None, 5):
            z.set_split_slices(5)
            if sq:
                z.set_split_slices_lower(sq)
            Wd = to_dev(W0)
            _, res = z.isomp_run(Wd, h, steps, 1e-12, 50, prec=PREC_SPLIT)
            assert max(res) < 1e-12
            out.append(to_host(Wd))
        for bad in (1, 6):
            with pytest.raises(ZeulerError):
                z.set_split_slices_lower(bad)
    for W in out:
        assert np.linalg.norm(W - Wr) <= 1e-10 * np.linalg.norm(Wr)
    assert np.linalg.norm(out[0] - out[1]) <= 1e-12 * np.linalg.norm(Wr)


@pytest.mark.parametrize("N,steps", [(128, 8), (1000, 5)])
def test_isomp_mixed_precision_meets_fp64_bar(dev, N, steps):
    """PREC_MIXED (FP64 product A, lower product Q on INT8 with 4 slices): the FP64 path's
    bar against the oracle (1e-12, the same evaluation counts), because Q's term carries
    h^2/4; ze_zgemm and the ensemble reject it."""
    from paper_2206_05466_amd import PREC_MIXED, Ensemble, ZeulerError

    h = 0.005
    W0 = w0(N, 9, "inv1.5")
    Wr, it_ref, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3)
    with ctx(N) as z:
        z.set_initial_guess(2)
        Wd = to_dev(W0)
        its, res = z.isomp_run(Wd, h, steps, 1e-12, 50, prec=PREC_MIXED)
        W = to_host(Wd)
        with pytest.raises(ZeulerError):
            z.zgemm(Wd, Wd.clone(), prec=PREC_MIXED)
    assert its == it_ref and max(res) < 1e-12, (its, it_ref)
    assert np.linalg.norm(W - Wr) <= 1e-12 * np.linalg.norm(Wr)
    assert np.abs(W + W.conj().T).max() == 0.0
    with Ensemble([16, 24]) as ens:
        with pytest.raises(ZeulerError):
            ens.run([to_dev(w0(16, 1)), to_dev(w0(24, 2))], h, 1, 1e-12, 4, prec=PREC_MIXED)


@pytest.mark.parametrize("N", [1, 2, 3, 17])
def test_tiny_sizes_every_mode(dev, N):
    """N = 1, 2, 3, 17 through the polynomial start, mixed precision and the order-4 step,
    each against the oracle's run of the same kind (1e-12 of ||W||, or exact zeros)."""
    from paper_2206_05466_amd import PREC_MIXED

    h = 0.01
    W0 = w0(N, 2)
    Wr, it_ref, _ = O.isomp_run(W0, h, 6, 1e-12, 50, extrapolate=True, degree=3)
    W4, it4, _ = O.isomp_composed_run(W0, h, 2, 4, 1e-12, 50)
    scale = max(np.linalg.norm(W0), 1e-300)
    with ctx(N) as z:
        z.set_initial_guess(2)
        for prec in (0, PREC_MIXED):
            Wd = to_dev(W0)
            its, res = z.isomp_run(Wd, h, 6, 1e-12, 50, prec=prec)
            assert its == it_ref, (prec, its, it_ref)
            assert np.linalg.norm(to_host(Wd) - Wr) <= 1e-12 * scale
        z.set_initial_guess(0)
        z.set_order(4)
        Wd = to_dev(W0)
        its, _ = z.isomp_run(Wd, h, 2, 1e-12, 50)
        assert its == it4
        assert np.linalg.norm(to_host(Wd) - W4) <= 1e-12 * scale


def test_ensemble_tiny_sizes_history_start(dev):
    """An ensemble of N = 1, 2, 3, 5, 17 and 40 with guess mode 3 and the difference form over 6
    steps (the start kernel's 1024-entry work items cover a whole small matrix in one, partly
    empty, item; the solve's bands, the products' and the update's tiles are ragged): every
    simulation ends where the oracle's run does (1e-12 of ||W||, exact zeros for N = 1), with
    its evaluation count in the last step."""
    from paper_2206_05466_amd import Ensemble

    sizes = [1, 2, 3, 5, 17, 40]
    h, tol, K, steps = 0.01, 1e-12, 50, 6
    W0s = [w0(n, 500 + j) for j, n in enumerate(sizes)]
    Wd = [to_dev(W) for W in W0s]
    with Ensemble(sizes) as ens:
        ens.set_initial_guess(3)
        ens.set_update_form(1)
        ens.run(Wd, h, steps, tol, K)
        its, res = ens.stats()
    for j, n in enumerate(sizes):
        Wr, it_ref, _ = O.isomp_run(W0s[j], h, steps, tol, K, extrapolate=True, degree=3,
                                    update="difference", solution_differences=True)
        scale = max(np.linalg.norm(W0s[j]), 1e-300)
        got = to_host(Wd[j])
        assert its[j] == it_ref[-1] and res[j] < tol, (n, its[j], it_ref)
        assert np.linalg.norm(got - Wr) <= 1e-12 * scale, (n, np.linalg.norm(got - Wr))
        assert np.abs(got + got.conj().T).max() == 0.0, n


@pytest.mark.parametrize("order,N,form,h", [(4, 64, 1, 0.01), (4, 100, 0, 0.01), (6, 48, 1, 0.005)])
def test_isomp_composed_polynomial_guess(dev, order, N, form, h):
    """Orders 4 and 6 with the per-substep polynomial starts (mode 2): the oracle's evaluation
    counts per step and its W to 1e-12, for either form of W_{n+1}; with the difference form
    every substep of the later steps takes one evaluation."""
    upd = ("second_line", "difference")[form]
    steps = 7
    W0 = w0(N, 5, "inv1.5")
    Wr, it_ref, _ = O.isomp_composed_run(W0, h, steps, order, 1e-12, 50, extrapolate=True,
                                         update=upd, degree=3)
    with ctx(N) as z:
        z.set_order(order)
        z.set_update_form(form)
        z.set_initial_guess(2)
        Wd = to_dev(W0)
        its, res = z.isomp_run(Wd, h, steps, 1e-12, 50)
        W = to_host(Wd)
    assert its == it_ref and max(res) < 1e-12, (its, it_ref)
    assert np.linalg.norm(W - Wr) <= 1e-12 * np.linalg.norm(Wr)
    if form == 1:
        assert its[-1] == len(O.composition_weights(order)), its


@pytest.mark.parametrize("N", [1, 33, 100])
def test_input_validation(dev, N):
    """ze_set_validation: a W in su(N) passes and steps as without the check; W with a
    Hermitian part of 1e-9 relative, with a trace of 1e-6, or with a NaN is refused with
    ZE_EINVAL and left unchanged; the check is off by default."""
    from paper_2206_05466_amd import ZeulerError

    W0 = w0(N, 3)
    scale = max(np.abs(W0).max(), 1.0)
    W1r, _, _ = O.isomp_step(W0, 0.01, 1e-12, 50)
    bad_h = W0.copy()
    bad_h[N - 1, 0] += 1e-9 * scale  # breaks W_rc = -conj(W_cr) (on the diagonal when N = 1)
    bad_t = W0 + 1e-6 * scale * 1j * np.eye(N)
    bad_n = W0.copy()
    bad_n[0, N - 1] = np.nan
    with ctx(N) as z:
        Wd = to_dev(bad_h)
        z.isomp_step(Wd, 0.01, 1e-12, 50)  # unchecked by default
        z.set_validation(True)
        Wd = to_dev(W0)
        info = z.isomp_step(Wd, 0.01, 1e-12, 50)
        assert info.converged
        assert np.linalg.norm(to_host(Wd) - W1r) <= 1e-12 * max(np.linalg.norm(W1r), 1e-300)
        for bad in (bad_h, bad_t, bad_n):
            Wd = to_dev(bad)
            with pytest.raises(ZeulerError, match="su"):
                z.isomp_step(Wd, 0.01, 1e-12, 50)
            with pytest.raises(ZeulerError):
                z.isomp_run(Wd, 0.01, 2, 1e-12, 50)
            got = to_host(Wd)
            assert np.array_equal(got[~np.isnan(got)], bad[~np.isnan(bad)])


# ------------------------------------------------------------------ modular (CRT) form
@pytest.mark.parametrize("N", [1, 7, 64, 129, 300, 1000])
def test_zgemm_crt_small_integers_exact(dev, N):
    """The modular form recovers integer products exactly (every input is a small integer, so
    the scaling rounds nothing and the CRT gives the exact sums), including values that need
    every modulus: entries up to 2^20."""
    from paper_2206_05466_amd import PREC_CRT

    rng = np.random.default_rng(N + 11)
    for lim in (9, 2 ** 20):
        A = rng.integers(-lim, lim + 1, (N, N)) + 1j * rng.integers(-lim, lim + 1, (N, N))
        B = rng.integers(-lim, lim + 1, (N, N)) + 1j * rng.integers(-lim, lim + 1, (N, N))
        with ctx(N) as z:
            C = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_CRT))
        exact = A @ B  # |entries| < 2^53: numpy's FP64 sums are exact here
        assert np.array_equal(C, exact), (N, lim)


@pytest.mark.parametrize("N", [64, 131, 384])
def test_zgemm_crt_random_fp64_level(dev, N):
    """Random complex operands with entries spread over 2^-20 .. 1: the modular form's error is
    the rounding of the scaled inputs to 55-bit integers, 2^-55 relative to the row / column
    maxima per term, i.e. at the level of the FP64 product itself: both within
    4 * 2N * 2^-52 max|A| max|B| of the exact product (from exact integer arithmetic on the
    FP64 inputs), and the CRT result no worse than 2x the FP64 product's own error."""
    from fractions import Fraction

    from paper_2206_05466_amd import PREC_CRT, PREC_FP64

    rng = np.random.default_rng(N)
    sc = 2.0 ** rng.integers(-20, 1, (N, N))
    A = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * sc
    B = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * sc.T
    with ctx(N) as z:
        C = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_CRT))
        F = to_host(z.zgemm(to_dev(A), to_dev(B), prec=PREC_FP64))
    # exact reference on sampled entries, in rational arithmetic of the FP64 inputs
    idx = rng.integers(0, N, (24, 2))
    bound = 4 * 2 * N * 2.0 ** -52 * np.abs(A).max() * np.abs(B).max()
    ec = ef = 0.0
    for r, c in idx:
        re = sum(Fraction(a.real) * Fraction(b.real) - Fraction(a.imag) * Fraction(b.imag)
                 for a, b in zip(A[r], B[:, c]))
        im = sum(Fraction(a.real) * Fraction(b.imag) + Fraction(a.imag) * Fraction(b.real)
                 for a, b in zip(A[r], B[:, c]))
        ec = max(ec, abs(float(Fraction(C[r, c].real) - re)), abs(float(Fraction(C[r, c].imag) - im)))
        ef = max(ef, abs(float(Fraction(F[r, c].real) - re)), abs(float(Fraction(F[r, c].imag) - im)))
    assert ec <= bound, (ec, bound)
    assert ec <= 2 * ef + 1e-300, (ec, ef)


@pytest.mark.parametrize("N,steps", [(128, 8), (1000, 5)])
def test_isomp_crt_meets_fp64_bar(dev, N, steps):
    """PREC_CRT (the product A = P W~ in the modular form, the lower product as PREC_MIXED):
    the FP64 path's bar against the oracle (1e-12, the same evaluation counts)."""
    from paper_2206_05466_amd import PREC_CRT

    h = 0.005
    W0 = w0(N, 9, "inv1.5")
    Wr, it_ref, _ = O.isomp_run(W0, h, steps, 1e-12, 50, extrapolate=True, degree=3)
    with ctx(N) as z:
        z.set_initial_guess(2)
        Wd = to_dev(W0)
        its, res = z.isomp_run(Wd, h, steps, 1e-12, 50, prec=PREC_CRT)
        W = to_host(Wd)
    assert its == it_ref and max(res) < 1e-12, (its, it_ref)
    assert np.linalg.norm(W - Wr) <= 1e-12 * np.linalg.norm(Wr)
