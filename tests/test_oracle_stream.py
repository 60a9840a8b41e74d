"""Pins of the oracle's stream solve P = Delta_N^+ W.

* brute force: the Moore-Penrose pseudo-inverse of the dense N^2 x N^2 Laplacian applied to
  vec(W), for every N up to 8 (pins the sign, the index map, the singular m = 0 block and
  the upper triangle at once);
* residual: Delta_N P = W - tr(W)/N I with the commutator form of Delta_N, at N = 64;
* eq. (lap_prop): a single-degree W gives P = -W / (l(l+1)) exactly;
* symmetry: P is skew-Hermitian and traceless; P commutes with SU(2) rotations,
  stream_solve(U W U^H) = U stream_solve(W) U^H.
"""

import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from workloads import omega_coeffs


def rand_skew(N, rng, traceless=True):
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    W = X - X.conj().T
    if traceless:
        W -= np.trace(W) / N * np.eye(N)
    return W


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("traceless", [True, False])
def test_matches_brute_pseudo_inverse(N, traceless):
    rng = np.random.default_rng(N)
    W = rand_skew(N, rng, traceless)
    P = O.stream_solve(W)
    Lp = np.linalg.pinv(O.brute_laplacian(N), rcond=1e-10)
    P_ref = (Lp @ W.reshape(-1)).reshape(N, N)
    assert np.abs(P - P_ref).max() < 1e-13 * max(1.0, np.abs(W).max())


def test_residual_and_symmetry_N64():
    rng = np.random.default_rng(7)
    N = 64
    W = rand_skew(N, rng, traceless=False)
    P = O.stream_solve(W)
    R = O.apply_laplacian(P) - (W - np.trace(W) / N * np.eye(N))
    assert np.abs(R).max() < 1e-11 * np.abs(W).max()
    assert np.abs(P + P.conj().T).max() == 0.0
    assert abs(np.trace(P)) < 1e-14 * np.abs(P).sum()


@pytest.mark.parametrize("N,l,m", [(8, 1, 0), (8, 3, 2), (12, 5, -3), (16, 15, 15), (16, 7, -7)])
def test_single_degree_is_eigenvector(N, l, m):
    om = np.zeros(N * N, complex)
    om[l * l + l + m] = 0.3 + 0.4j
    om[l * l + l - m] = (-1) ** m * np.conj(om[l * l + l + m])
    W = O.assemble(N, om)
    P = O.stream_solve(W)
    assert np.abs(P + W / (l * (l + 1))).max() < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_su2_equivariance(axis):
    N = 10
    rng = np.random.default_rng(11)
    W = rand_skew(N, rng)
    J = O.spin_matrices(N)[axis]
    U = expm(0.7j * J)
    P = O.stream_solve(W)
    P_rot = O.stream_solve(U @ W @ U.conj().T)
    assert np.abs(P_rot - U @ P @ U.conj().T).max() < 1e-13


def test_large_N_residual():
    N = 300
    W = O.assemble(N, omega_coeffs(N, 5, "inv1", lmax=40))
    P = O.stream_solve(W)
    R = O.apply_laplacian(P) - W
    assert np.abs(R).max() < 1e-10 * np.abs(W).max()
