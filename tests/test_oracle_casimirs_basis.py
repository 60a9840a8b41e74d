"""Pins of the oracle's Casimirs (eq. (W_pow)) and quantised basis (Sec. 3.2, eq. (W0)).

Casimirs: closed forms C_1 = Tr W, C_2 = -||W||_F^2, C_4 = ||W^2||_F^2 for skew-Hermitian
W, and the spectral route sum_j mu_j^k.
Basis: every assembled T_lm is an eigenvector of the dense Laplacian with eigenvalue
-l(l+1) (eq. (lap_prop)) and lies on diagonal m; the T_lm are orthonormal (extract inverts
assemble, assemble is an isometry); W is skew-Hermitian and traceless for omega_00 = 0;
the sign rule is deterministic.
"""

import numpy as np
import pytest

import oracle as O
from workloads import omega_coeffs


def test_casimir_closed_forms():
    N = 40
    W = O.assemble(N, omega_coeffs(N, 9, "inv1"))
    c = O.casimirs(W, 5)
    ce = O.casimirs_eig(W, 5)
    nf = np.linalg.norm(W)
    assert abs(c[0] - np.trace(W)) < 1e-14
    assert abs(c[1] + nf ** 2) < 1e-13 * nf ** 2
    assert abs(c[3] - np.linalg.norm(W @ W) ** 2) < 1e-13 * nf ** 4
    assert np.abs(c - ce).max() < 1e-12 * max(1, nf ** 5)
    # even k real, odd k imaginary for skew-Hermitian W
    assert abs(c[1].imag) < 1e-14 and abs(c[2].real) < 1e-14 * nf ** 3


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_basis_elements_are_laplacian_eigenvectors(N):
    L = O.brute_laplacian(N)
    for l in range(N):
        for m in range(-l, l + 1):
            om = np.zeros(N * N, complex)
            om[l * l + l + m] = 1.0
            W = O.assemble(N, om)  # = i T_lm (not skew-Hermitian for m != 0 alone)
            v = W.reshape(-1)
            assert abs(np.linalg.norm(v) - 1.0) < 1e-13
            assert np.abs(L @ v + l * (l + 1) * v).max() < 1e-12 * max(1, N * N)
            rows, cols = np.nonzero(np.abs(W) > 1e-300)
            assert np.all(rows - cols == m)


def test_orthonormal_and_roundtrip():
    N = 48
    om = omega_coeffs(N, 4, "inv1")
    W = O.assemble(N, om)
    assert np.abs(W + W.conj().T).max() == 0.0
    assert abs(np.trace(W)) < 1e-14
    assert abs(np.linalg.norm(W) - np.linalg.norm(om)) < 1e-13
    assert np.abs(O.extract(W) - om).max() < 1e-13


def test_sign_rule_and_eigvals():
    for N in (9, 64):
        for m in (0, 3, N - 1):
            w, V = O.eigvecs(N, m)
            n = N - m
            l = np.arange(m, N)
            assert np.abs(w - l * (l + 1)).max() < 1e-11 * N * N
            half = (n - 1) // 2 + 1
            a = np.abs(V[:half])
            for j in range(n):
                k = np.nonzero(a[:, j] >= (1 - 1e-8) * a[:, j].max())[0][0]
                assert V[k, j] > 0


def test_sign_rule_exact_tie():
    """N = 8, l = 3, m = 0: |v_0| = |v_2| exactly (opposite signs); the lowest index wins."""
    _, V = O.eigvecs(8, 0)
    v = V[:, 3]
    assert abs(abs(v[0]) - abs(v[2])) < 1e-15 and v[0] * v[2] < 0
    assert v[0] > 0


def test_generator_reality_and_law():
    N = 128
    om = omega_coeffs(N, 1, "inv1")
    l = np.floor(np.sqrt(np.arange(N * N))).astype(int)
    m = np.arange(N * N) - l * l - l
    mirror = l * l + l - m
    assert np.abs(om[mirror] - (-1.0) ** m * np.conj(om)).max() == 0.0
    assert om[0] == 0 and np.all(om[l * l + l].imag == 0)
    # E|omega_lm|^2 = sigma_l^2: average over the 2l+1 modes of each degree, then over l
    ratio = np.array([np.mean(np.abs(om[l0 * l0:(l0 + 1) ** 2]) ** 2) * (l0 + 1) ** 2
                      for l0 in range(1, N)])
    assert abs(ratio.mean() - 1.0) < 0.05
    assert np.array_equal(om, omega_coeffs(N, 1, "inv1"))
    p = omega_coeffs(64, 0, "paper")
    assert np.all(p[: 4] == 0) and np.all(p[21 * 21:] == 0) and np.any(p[4:21 * 21] != 0)


def test_truncated_assembly_matches_full():
    N, L = 80, 12
    om = omega_coeffs(N, 2, "inv1", lmax=L)
    assert np.abs(O.assemble(N, om, lmax=L) - O.assemble(N, om)).max() < 1e-13
    with pytest.raises(ValueError):
        O.assemble(N, omega_coeffs(N, 2, "inv1"), lmax=L)


def test_energy_spectrum_pins():
    """E_l (Sec. 4) against two independent routes: sum_l E_l = tr(P W) with P from the
    stream solve (eq. (sub_tria_W)), and sum_l l(l+1) E_l = ||W||_F^2 (orthonormal T_lm);
    a single-degree field puts all its energy at that degree."""
    N = 24
    om = omega_coeffs(N, 5, "inv1")
    W = O.assemble(N, om)
    E = O.energy_spectrum(om, N)
    P = O.stream_solve(W)
    tPW = np.trace(P @ W)
    assert E[0] == 0.0 and np.all(E >= 0)
    assert abs(tPW.imag) < 1e-14 and abs(E.sum() - tPW.real) < 1e-13 * E.sum()
    l = np.arange(N)
    assert abs((l * (l + 1) * E).sum() - np.linalg.norm(W) ** 2) < 1e-13 * np.linalg.norm(W) ** 2
    one = np.zeros(N * N, complex)
    one[7 * 7 + 7 - 3] = 0.5 - 0.25j
    E1 = O.energy_spectrum(one, N)
    assert np.count_nonzero(E1) == 1 and abs(E1[7] - 0.3125 / 56) < 1e-17
