"""Pins of the oracle's Laplacian against what the paper and the mathematics fix.

* eq. (lap_prop): Delta_N has eigenvalues -l(l+1), l = 0..N-1, multiplicity 2l+1
  (checked on the dense spin-representation operator, which is built independently);
* eq. (delta_tria): its restriction to the m-th diagonal (sub- and super-) is -Delta^m,
  entry for entry, and there is no coupling between diagonals;
* a hand-worked N = 3 example (tests/golden/laplacian_N3.txt).
"""

import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_brute_spectrum_is_minus_l_lplus1(N):
    L = O.brute_laplacian(N)
    assert np.abs(L - L.conj().T).max() < 1e-12
    ev = np.sort(np.linalg.eigvalsh(L))[::-1]
    expect = -np.sort(np.concatenate([[l * (l + 1.0)] * (2 * l + 1) for l in range(N)]))
    assert np.abs(ev - expect).max() < 1e-11 * max(1.0, N * N)


def test_spin_matrices_commutation():
    for N in (2, 3, 5, 8):
        J1, J2, J3 = O.spin_matrices(N)
        assert np.abs(J1 @ J2 - J2 @ J1 - 1j * J3).max() < 1e-12
        s = (N - 1) / 2
        C = J1 @ J1 + J2 @ J2 + J3 @ J3
        assert np.abs(C - s * (s + 1) * np.eye(N)).max() < 1e-12


@pytest.mark.parametrize("N", [2, 3, 4, 6, 9, 12])
def test_delta_tria_is_block_of_brute_laplacian(N):
    L = O.brute_laplacian(N)
    seen = np.zeros(N * N, dtype=bool)
    for m in range(N):
        d, e = O.delta_tridiag(N, m)
        n = N - m
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        lower = [(i + m) * N + i for i in range(n)]
        upper = [i * N + i + m for i in range(n)]
        for idx in (lower, upper):
            assert np.abs(-L[np.ix_(idx, idx)] - T).max() < 1e-12 * N * N
            seen[idx] = True
            others = np.setdiff1d(np.arange(N * N), idx)
            assert np.abs(L[np.ix_(others, idx)]).max(initial=0.0) < 1e-12 * N * N
    assert seen.all()


def test_golden_N3_hand_worked():
    rows = []
    with open(os.path.join(GOLDEN, "laplacian_N3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([p.split() for p in line.split("|")])
    assert len(rows) == 3
    for m_s, d_s, e_s, ev_s in rows:
        m = int(m_s[0])
        d, e = O.delta_tridiag(3, m)
        assert np.allclose(d, np.array(d_s, float), atol=1e-14)
        assert np.allclose(e, np.array(e_s, float), atol=1e-14)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        assert np.allclose(np.linalg.eigvalsh(T), np.array(ev_s, float), atol=1e-13)


@pytest.mark.parametrize("N", [16, 64, 257])
def test_block_eigenvalues_large_N(N):
    for m in sorted({0, 1, N // 3, N - 2, N - 1}):
        d, e = O.delta_tridiag(N, m)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        ev = np.linalg.eigvalsh(T)
        l = np.arange(m, N, dtype=float)
        assert np.abs(ev - l * (l + 1)).max() < 1e-10 * N * N


def test_apply_laplacian_matches_brute():
    rng = np.random.default_rng(3)
    for N in (3, 7):
        X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
        L = O.brute_laplacian(N)
        assert np.abs(O.apply_laplacian(X).reshape(-1) - L @ X.reshape(-1)).max() < 1e-11
